"""GPU parity of the dual-energy step (sixth field rho e, Bryan et al. 1995)
with the oracle, through the C ABI.  The states are hypersonic, cold flows
whose internal energy falls on both sides of eta1 E (Mach ~ 30-60), so both
pressure sources and the resynchronisation are exercised; also Sedov, floors
of rho e, every sweep-kernel combination, fused runs of steps, batched
instances with different thresholds, remesh, comoving steps, the two-step
graph, and the recomputing adjoint's refusal (the recorded adjoint of the
dual-energy step has its own tests).  Bar: dt and every field bitwise
(the floating-point bar of 1e-12 is the tolerance, bitwise the observed and
designed result)."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd._lib import AmrError
from paper_1810_01319_amd.mesh import Mesh

from test_gpu_parity import TOL, compare_active, load, pair

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


def say(msg):
    print(f"[gpu-dual] {msg}", file=sys.stderr, flush=True)


def cold_flow(spec, keys, seed=0):
    """rho e = E - ke at t = 0; the x velocity 40..90 puts E - ke of cells on
    both sides of 1e-3 E."""
    x, y, z = I.cell_centres(spec, keys)
    ph = np.random.default_rng(seed).uniform(0.0, 1.0, 6)
    tw = 2.0 * np.pi
    rho = 1.0 + 0.3 * np.sin(tw * (x + ph[0])) * np.sin(tw * (y + ph[1]))
    u = 65.0 + 25.0 * np.sin(tw * (y + ph[2]))
    v = 0.5 * np.sin(tw * (z + ph[3]))
    w = 0.3 * np.cos(tw * (x + ph[4]))
    p = 1.0 + 0.5 * np.sin(tw * (z + ph[5]))
    return I.with_internal_energy(I.conserved(spec.gamma, rho, u, v, w, p))


def amr(N, levels, seed, **kw):
    root = (2, 2, 2)
    return I.MeshSpec(root=root, block_cells=N, max_level=levels, gamma=GAMMA,
                      refine=I.random_refine_list(root, levels, 4, seed), dual_energy=True, **kw)


def run(name, spec, act_fn, steps, modes=None):
    say(f"case {name}: root={spec.root} N={spec.block_cells} levels={spec.max_level} "
        f"eta=({spec.eta1}, {spec.eta2}) steps={steps} modes={modes}")
    om, gm, perm = pair(spec)
    assert gm.nf == 6 and om.nf == 6
    if modes is not None:
        gm.set_launch(sweep_mode=list(modes))
    U = load(om, gm, perm, act_fn(spec, gm.keys))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(steps):
        gm.step(U, dt, k)
        dto = om.step(k)
        assert float(dt.cpu()[0]) == dto, f"{name}: dt differs at step {k}"
        err, bw = compare_active(gm, U, om, perm)
        assert err <= TOL and bw == 1.0, f"{name}: step {k} rel err {err:.3e}, bitwise {bw}"
    assert gm.floor_count() == om.floors, f"{name}: floor counts {gm.floor_count()} vs {om.floors}"
    return om, gm, perm, U


@pytest.mark.parametrize("N,levels,seed,eta", [
    (8, 2, 1, (1e-3, 0.1)), (16, 2, 2, (1e-3, 0.1)), (32, 1, 3, (1e-3, 0.1)),
    (16, 2, 4, (1.0, 1.0)), (8, 2, 5, (0.0, 0.0)), (16, 1, 6, (0.05, 0.5)),
])
def test_dual_energy_amr_steps_match_oracle(N, levels, seed, eta):
    spec = amr(N, levels, seed, eta1=eta[0], eta2=eta[1])
    run(f"cold flow N={N}", spec, lambda s, k: cold_flow(s, k, seed), 4)


def test_dual_energy_sedov_matches_oracle():
    spec = I.with_(I.sedov_spec(root=2, block_cells=16, levels=2), dual_energy=True)
    run("sedov", spec, lambda s, k: I.with_internal_energy(I.sedov_state(s, k)), 4)


@pytest.mark.parametrize("modes", [(0, 0, 0), (1, 1, 1), (0, 1, 1), (1, 0, 1)])
def test_dual_energy_sweep_kernels_match_oracle(modes):
    """The walk and the staged tile along every axis."""
    for N in (8, 32):
        run(f"modes N={N}", amr(N, 1 if N == 32 else 2, 7 + N), lambda s, k: cold_flow(s, k, N), 2, modes)


def test_dual_energy_floors_match_oracle():
    """A diverging cold flow drives E and rho e under the pressure floor."""
    spec = I.MeshSpec(root=(4, 1, 1), block_cells=8, gamma=GAMMA, p_floor=1e-3, rho_floor=1e-6,
                      dual_energy=True, eta1=0.5, eta2=0.6)

    def act(s, keys):
        x = I.cell_centres(s, keys)[0]
        u = np.where(x < 0.5, -4.0, 4.0)
        return I.with_internal_energy(I.conserved(GAMMA, np.ones_like(x), u, 0.0, 0.0, np.full(x.shape, 2e-3)))

    om, gm, perm, U = run("floors", spec, act, 6)
    assert om.floors > 0


def test_dual_energy_fused_steps_equal_single_steps():
    spec = amr(16, 2, 11)
    gm = Mesh(**spec.kwargs())
    act = cold_flow(spec, gm.keys, 11)
    Ua, Ub = gm.state_from_active(act), gm.state_from_active(act)
    dts = torch.zeros(5, dtype=torch.float64, device="cuda")
    gm.steps(Ua, dts, 5, 0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    one = []
    for k in range(5):
        gm.step(Ub, dt, k)
        one.append(float(dt.cpu()[0]))
    assert dts.cpu().tolist() == one
    assert torch.equal(Ua, Ub) or np.array_equal(gm.active(Ua), gm.active(Ub))


def test_dual_energy_batched_instances_match_oracle():
    specs = [amr(16, 2, 20 + i, eta1=e1, eta2=e2) for i, (e1, e2) in
             enumerate([(1e-3, 0.1), (1.0, 1.0), (0.0, 0.0), (0.02, 0.3)])]
    gm = Mesh.batch([s.kwargs() for s in specs])
    assert gm.nf == 6
    acts, oms = [], []
    for i, sp in enumerate(specs):
        keys = gm.keys[gm.first_leaf[i]:gm.first_leaf[i + 1]]
        acts.append(cold_flow(sp, keys, 30 + i))
        om = O.OracleMesh(**sp.kwargs())
        idx = {tuple(k): s for s, k in enumerate(om.keys)}
        perm = np.array([idx[tuple(k)] for k in keys])
        o = np.empty_like(acts[-1])
        o[perm] = acts[-1]
        om.set_active(o)
        oms.append((om, perm))
    U = gm.state_from_active(np.concatenate(acts))
    dt = gm.dt_tensor()
    for k in range(3):
        gm.step(U, dt, k)
        d = dt.cpu().numpy()
        for i, (om, perm) in enumerate(oms):
            assert d[i] == om.step(k), (i, k)
    act = gm.active(U)
    for i, (om, perm) in enumerate(oms):
        assert np.array_equal(act[gm.first_leaf[i]:gm.first_leaf[i + 1]], om.active()[perm]), i


def test_dual_energy_batch_must_agree():
    with pytest.raises(AmrError):
        Mesh.batch([amr(8, 1, 1).kwargs(), I.MeshSpec(root=(2, 2, 2), block_cells=8).kwargs()])


def test_dual_energy_remesh_matches_oracle():
    spec = amr(8, 3, 40)
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, cold_flow(spec, gm.keys, 40))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(2):
        gm.step(U, dt, k)
        om.step(k)
    gm2, U2, st = gm.remesh(U, 0.05, 0.01, 10 ** 6)
    om2, ost = om.remesh(0.05, 0.01, 10 ** 6)
    say(f"remesh: {gm.nleaf} -> {gm2.nleaf} leaves, stats {st}")
    assert [st["refined"], st["coarsened"], st["refused"]] == [int(v) for v in ost]
    assert st["refined"] + st["coarsened"] > 0
    idx = {tuple(k): s for s, k in enumerate(om2.keys)}
    perm2 = np.array([idx[tuple(k)] for k in gm2.keys])
    assert gm2.nf == 6
    assert compare_active(gm2, U2, om2, perm2)[1] == 1.0
    dt2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    gm2.step(U2, dt2, 2)
    assert float(dt2.cpu()[0]) == om2.step(2)
    assert compare_active(gm2, U2, om2, perm2)[1] == 1.0


def test_dual_energy_comoving_matches_oracle():
    spec = amr(16, 2, 50)
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, cold_flow(spec, gm.keys, 50))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 1.0
    for k in range(3):
        a = t ** (2.0 / 3.0)
        gm.cfl_dt_comoving(U, a, dt)
        d = float(dt.cpu()[0])
        assert d == om.cfl_dt_comoving(a)
        tm = t + 0.5 * d
        gm.step_comoving(U, dt, k, tm ** (2.0 / 3.0), 2.0 / (3.0 * tm))
        om.step_comoving(k, d, tm ** (2.0 / 3.0), 2.0 / (3.0 * tm))
        assert compare_active(gm, U, om, perm)[1] == 1.0
        t += d
    assert gm.floor_count() == om.floors


def test_dual_energy_graph_replays_equal_eager_steps():
    spec = amr(8, 2, 60)
    gm = Mesh(**spec.kwargs())
    act = cold_flow(spec, gm.keys, 60)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        Ue, dte = gm.state_from_active(act), gm.dt_tensor()
        for k in range(4):
            gm.step(Ue, dte, k)
        Ug, dtg = gm.state_from_active(act), gm.dt_tensor()
        side.synchronize()
        g = gm.graph(Ug, dtg, first_step=0)
        for _ in range(2):
            g.launch()
            side.synchronize()
    assert np.array_equal(gm.active(Ug), gm.active(Ue))
    assert torch.equal(dtg, dte)


def test_recomputing_adjoint_equals_recorded_adjoint():
    """With the dual-energy field the adjoint that recomputes the sweep
    inputs from a checkpoint equals the one from the recorded inputs (up to
    the order of the refresh transpose's atomic sums), in both threshold
    regimes, and leaves the mesh's floor-reset count unchanged."""
    for eta1, eta2 in ((1e-3, 0.1), (1e-3, 0.99)):
        spec = amr(8, 1, 70, eta1=eta1, eta2=eta2)
        m = Mesh(**spec.kwargs())
        N = spec.block_cells
        U = m.state_from_active(cold_flow(spec, m.keys, 70))
        rng = np.random.default_rng(71)
        act = torch.zeros(U.shape[2:], dtype=torch.bool, device=U.device)
        act[3:3 + N, 3:3 + N, 3:3 + N] = True
        for k in range(3):
            ck = U.clone()
            dt = m.dt_tensor()
            S1, S2, Uo = (torch.empty_like(U) for _ in range(3))
            floors = torch.empty(1, dtype=torch.int64, device=U.device)
            m.step_record(U, dt, S1, S2, Uo, floors, k)
            lam0 = torch.zeros_like(U)
            lam0[:, :, act] = torch.from_numpy(rng.normal(size=(m.nleaf, 6, N ** 3))).to(U.device)
            la, lb = lam0.clone(), lam0.clone()
            m.step_adjoint_recorded(U, S1, S2, dt, floors, la, m.adjoint_face_scratch(), k)
            before = m.floor_count()
            m.step_adjoint(ck, dt, lb, m.adjoint_scratch(), k)
            assert m.floor_count() == before
            err = float((la - lb).abs().max()) / float(lb.abs().max())
            say(f"eta2 {eta2} step {k}: max |recorded - recomputed| / max {err:.3e}")
            assert err <= 1e-13, (eta2, k, err)
            U = Uo
