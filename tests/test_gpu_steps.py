"""GPU tests of amr_hydro_steps, the multi-step entry whose CFL reduction is
fused into the previous step (last sweep plus the refluxed cells): the dt
sequence and the state equal the same number of single steps bit for bit,
and the dt sequence equals the oracle's, on AMR meshes with coarse-fine
faces (N = 8, 16, 32), with every sweep mode as the last sweep, with floors,
and on batched instances."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd.mesh import Mesh

from test_gpu_parity import load, pair

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-steps] {msg}", file=sys.stderr, flush=True)


def compare_steps(name, spec, act, n, modes=None):
    say(f"case {name}: root={spec.root} N={spec.block_cells} levels={spec.max_level} steps={n} modes={modes}")
    om, gm, perm = pair(spec)
    if modes is not None:
        gm.set_launch(sweep_mode=list(modes))
    a = act(spec, gm.keys)
    Ua = load(om, gm, perm, a)
    Ub = gm.state_from_active(a)
    dts = torch.zeros(n, gm.n_instances, dtype=torch.float64, device="cuda")
    dt1 = gm.dt_tensor()
    gm.steps(Ua, dts, n, 0)
    seq = []
    for k in range(n):
        gm.step(Ub, dt1, k)
        seq.append(dt1.clone())
    torch.cuda.synchronize()
    assert torch.equal(dts, torch.stack(seq)), f"{name}: dt sequences differ"
    assert torch.equal(Ua, Ub), f"{name}: states differ"
    do = [om.step(k) for k in range(n)]
    assert dts[:, 0].cpu().numpy().tolist() == do, f"{name}: dt differs from the oracle"
    say(f"case {name}: {n} steps bitwise equal, nreflux faces present: {int(np.any(np.asarray(gm.keys)[:, 0] > 0))}")


@pytest.mark.parametrize("N,levels,seed", [(8, 3, 1), (16, 2, 2), (32, 1, 3)])
def test_steps_equal_single_steps_on_amr(N, levels, seed):
    root = (2, 2, 2)
    spec = I.MeshSpec(root=root, block_cells=N, max_level=levels, gamma=1.4,
                      refine=I.random_refine_list(root, levels, 5, seed))
    compare_steps(f"smooth N={N}", spec, lambda s, k: I.smooth_state(s, k, seed=50 + seed, vel=1.0), 5)


@pytest.mark.parametrize("modes", [(0, 0, 0), (1, 1, 1), (1, 0, 0)])
def test_steps_with_every_last_sweep_kind(modes):
    spec = I.sedov_spec(root=2, block_cells=16, levels=2)
    compare_steps("sedov", spec, I.sedov_state, 4, modes)


def test_steps_with_floors():
    spec = I.MeshSpec(root=(4, 1, 1), block_cells=8, gamma=1.4, p_floor=1e-3, rho_floor=1e-6)

    def act(s, keys):
        x = I.cell_centres(s, keys)[0]
        u = np.where(x < 0.5, -4.0, 4.0)
        return I.conserved(1.4, np.ones_like(x), u, 0.0, 0.0, np.full(x.shape, 2e-3))

    compare_steps("floors", spec, act, 6)


def test_steps_on_batched_instances():
    specs, cents = zip(*[I.batch_instance(i) for i in range(6)])
    gm = Mesh.batch([s.kwargs() for s in specs])
    act = np.concatenate([I.batch_state(sp, gm.keys[gm.first_leaf[i]:gm.first_leaf[i + 1]], c)
                          for i, (sp, c) in enumerate(zip(specs, cents))])
    Ua, Ub = gm.state_from_active(act), gm.state_from_active(act)
    n = 4
    dts = torch.zeros(n, gm.n_instances, dtype=torch.float64, device="cuda")
    dt1 = gm.dt_tensor()
    gm.steps(Ua, dts, n, 0)
    seq = []
    for k in range(n):
        gm.step(Ub, dt1, k)
        seq.append(dt1.clone())
    torch.cuda.synchronize()
    assert torch.equal(dts, torch.stack(seq))
    assert torch.equal(Ua, Ub)


def test_fresh_steps_after_a_refresh_equal_steps():
    """amr_hydro_steps_fresh skips the first step's refresh: after an explicit
    refresh it gives amr_hydro_steps' dt sequence and state bit for bit."""
    spec = I.sedov_spec(root=2, block_cells=16, levels=2)
    gm = Mesh(**spec.kwargs())
    act = I.sedov_state(spec, gm.keys)
    Ua, Ub = gm.state_from_active(act), gm.state_from_active(act)
    da = torch.zeros(4, 1, dtype=torch.float64, device="cuda")
    db = torch.zeros_like(da)
    gm.refresh(Ua)
    gm.steps(Ua, da, 4, 0, ghosts_fresh=True)
    gm.steps(Ub, db, 4, 0)
    torch.cuda.synchronize()
    assert torch.equal(da, db) and torch.equal(Ua, Ub)


def test_fresh_steps_after_an_unchanged_remesh_equal_steps():
    """A remesh that refines and coarsens nothing returns the same mesh and
    state with the ghosts refreshed: the next run of steps may skip its first
    refresh (as the adaptive benchmark does) and matches plain steps bit for
    bit."""
    spec = I.blasts_spec(root=2, block_cells=16, levels=2)
    gm = Mesh(**spec.kwargs())
    U = gm.state_from_active(I.blasts_state(spec, gm.keys))
    d = torch.zeros(4, 1, dtype=torch.float64, device="cuda")
    gm.steps(U, d, 4, 0)
    Ub = U.clone()
    new, Un, st = gm.remesh(U, 1e300, 0.0, gm.nleaf + 100)
    assert new is gm and Un is U and st["refined"] == 0 and st["coarsened"] == 0
    da = torch.zeros(4, 1, dtype=torch.float64, device="cuda")
    db = torch.zeros_like(da)
    gm.steps(U, da, 4, 4, ghosts_fresh=True)
    gm.steps(Ub, db, 4, 4)
    torch.cuda.synchronize()
    assert torch.equal(da, db) and torch.equal(U, Ub)
