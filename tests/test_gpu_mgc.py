"""GPU parity of mg0 on the octree (composite-grid Poisson operator on the
leaves of a refined periodic mesh, V-cycles over the hierarchy of coarsened
meshes down to the uniform root grid) with the oracle, through the C ABI:
two- and three-level meshes with N = 8, 16 and 32, seeded standard-normal
right-hand sides, the solution within 1e-12 of the oracle relative to its
max norm, the residual norms within 1e-10 of the first (the means and norms
are two-stage sums on the GPU and sequential ones in the oracle, and a small
residual is the difference of two much larger terms).  The entry point without a
workspace gives the same bits on a refined mesh."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd.mesh import Mesh

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(msg):
    print(f"[gpu-mgc] {msg}", file=sys.stderr, flush=True)


CASES = [
    ("3 levels N=8", I.MeshSpec(root=(4, 4, 4), block_cells=8, max_level=2, refine=[(0, 1, 1, 1), (1, 2, 2, 2)])),
    ("2 levels N=16", I.MeshSpec(root=(2, 2, 2), block_cells=16, max_level=2, refine=[(0, 0, 0, 0), (1, 1, 1, 1)])),
    ("3 levels N=16 non-cubic roots", I.MeshSpec(root=(4, 2, 2), block_cells=16, max_level=2,
                                                 refine=[(0, 1, 0, 1), (1, 3, 1, 2)])),
    ("2 levels N=32", I.MeshSpec(root=(4, 4, 4), block_cells=32, max_level=1, refine=[(0, 2, 1, 1)])),
]


def solve_pair(spec, seed, ncycles):
    gm = Mesh(**spec.kwargs())
    om = O.OracleMesh(**spec.kwargs())
    idx = {tuple(k): s for s, k in enumerate(om.keys)}
    perm = np.array([idx[tuple(k)] for k in gm.keys])  # GPU leaf -> oracle leaf
    N = spec.block_cells
    f = np.random.default_rng(seed).standard_normal((gm.nleaf, N, N, N))
    fo = np.empty_like(f)
    fo[perm] = f
    want, want_res = O.mgc_solve(om, fo, ncycles)
    fg = torch.from_numpy(f).to(gm.device)
    phi = torch.zeros_like(fg)
    res = gm.poisson_solve(fg, phi, ncycles)
    torch.cuda.synchronize()
    return gm, fg, phi.cpu().numpy(), res.cpu().numpy(), want[perm], want_res


@pytest.mark.parametrize("name,spec", CASES, ids=[c[0] for c in CASES])
def test_composite_solve_matches_oracle(name, spec):
    say(f"{name}: root={spec.root} levels={spec.max_level}")
    gm, _, got, res, want, want_res = solve_pair(spec, seed=17, ncycles=4)
    assert len(set(gm.keys[:, 0])) >= 2
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    rerr = np.max(np.abs(res - want_res)) / want_res[0]
    say(f"{name}: {gm.nleaf} leaves, phi rel err {err:.3e}, residual norms rel err {rerr:.3e}, "
        f"contraction {res[-1] / res[-2]:.3f}")
    assert err <= TOL and rerr <= 1e-10
    assert res[-1] < 1e-3 * res[0]


def test_static_entry_equals_workspace_entry_on_a_refined_mesh():
    spec = CASES[0][1]
    say("static entry on the 3-level N=8 mesh")
    gm, fg, got, res, _, _ = solve_pair(spec, seed=18, ncycles=3)
    phi = torch.zeros_like(fg)
    r = torch.empty(4, dtype=torch.float64, device=gm.device)
    gm.poisson_solve_static(fg, phi, 3, resid=r)
    torch.cuda.synchronize()
    assert np.array_equal(phi.cpu().numpy(), got)
    assert np.array_equal(r.cpu().numpy(), res)


def gravity_state(spec, keys, seed):
    x, y, z = I.cell_centres(spec, keys)
    ph = np.random.default_rng(seed).uniform(0, 1, 3)
    rho = 1.0 + 0.1 * np.cos(2 * np.pi * (x + ph[0])) * np.cos(2 * np.pi * (y + ph[1]))
    g = spec.gamma
    u = 0.05 * np.sin(2 * np.pi * (z + ph[2]))
    v = 0.04 * np.sin(2 * np.pi * (x + ph[1]))
    w = 0.03 * np.cos(2 * np.pi * (y + ph[0]))
    act = I.conserved(g, rho, u, v, w, rho ** g)
    return I.with_internal_energy(act) if spec.dual_energy else act


@pytest.mark.parametrize("de", [False, True])
def test_self_gravity_steps_on_a_refined_mesh_match_oracle(de):
    """Kick-drift-kick with mg0 on the octree, 3 steps (the potential solved
    first, then carried) on a three-level mesh of 8^3 blocks: every field
    within 1e-12 of the oracle relative to its max norm, dt and the
    potential too."""
    from test_gpu_parity import TOL as PTOL, compare_active, load, pair

    spec = I.MeshSpec(root=(4, 4, 4), block_cells=8, max_level=2, gamma=5.0 / 3.0,
                      refine=[(0, 1, 1, 1), (1, 2, 2, 2)], dual_energy=de, eta1=1e-3, eta2=0.1)
    say(f"self-gravity on 3 levels, dual energy {de}")
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, gravity_state(spec, gm.keys, 3))
    N = 8
    phi_o = np.zeros((om.nleaf, N, N, N))
    phi_g = torch.zeros((gm.nleaf, N, N, N), dtype=torch.float64, device=gm.device)
    work = gm.poisson_workspace()
    dt = torch.zeros(1, dtype=torch.float64, device=gm.device)
    for k in range(3):
        gm.step_gravity(U, dt, k, 20.0, phi_g, k > 0, ncycles=3, work=work)
        dto = om.step_gravity_amr(k, 20.0, phi_o, k > 0, ncycles=3)
        dtg = float(dt.cpu()[0])
        assert abs(dtg - dto) <= 1e-12 * dto, (k, dtg, dto)
        err, bw = compare_active(gm, U, om, perm)
        pg = phi_g.cpu().numpy()
        perr = np.max(np.abs(pg - phi_o[perm])) / np.max(np.abs(phi_o))
        say(f"step {k}: state rel err {err:.2e} (bitwise {bw:.4f}), phi rel err {perr:.2e}")
        assert err <= PTOL and perr <= TOL
