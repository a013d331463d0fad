"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Bar: dt sequences bitwise equal; every active cell within 1e-12 of the oracle
relative to max(|b|, ||b_field||_inf) (the FP64 parity tolerance; momenta
cross zero so the field max-norm scales it).  Refresh is compared on every
cell, ghosts included, bitwise.  The design target is bitwise equality, and
the tests report the fraction of bitwise-equal values.
"""
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
    print(f"[gpu-parity] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU parity tests need an MI355X"


def pair(spec):
    om = O.OracleMesh(**spec.kwargs())
    gm = Mesh(**spec.kwargs())
    idx = {tuple(k): s for s, k in enumerate(om.keys)}
    perm = np.array([idx[tuple(k)] for k in gm.keys])  # gpu order -> oracle index
    assert len(perm) == om.nleaf == gm.nleaf
    return om, gm, perm


def load(om, gm, perm, act):
    """act in GPU order; the oracle receives the same blocks."""
    o = np.empty_like(act)
    o[perm] = act
    om.set_active(o)
    return gm.state_from_active(act)


def compare_active(gm, U, om, perm, tol=TOL):
    a = gm.active(U)
    b = om.active()[perm]
    assert np.all(np.isfinite(a)), "non-finite values on the GPU"
    scale = np.max(np.abs(b), axis=(0, 2, 3, 4))  # per field max-norm
    den = np.maximum(np.abs(b), scale[None, :, None, None, None])
    with np.errstate(divide="ignore", invalid="ignore"):
        err = np.where(a == b, 0.0, np.abs(a - b) / np.where(den > 0, den, np.inf))
    err = np.where((a != b) & (den == 0), np.inf, err)
    bitwise = np.mean(a == b)
    return float(np.max(err)), float(bitwise)


def run_case(name, spec, act_fn, steps, fixed_dt=None, compare_every=1):
    say(f"case {name}: root={spec.root} N={spec.block_cells} levels={spec.max_level} steps={steps}")
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, act_fn(spec, gm.keys))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    worst = 0.0
    for k in range(steps):
        if fixed_dt is None:
            gm.step(U, dt, k)
            dto = om.step(k)
            dtg = float(dt.cpu()[0])
            assert dtg == dto, f"{name}: dt differs at step {k}: {dtg!r} vs {dto!r}"
        else:
            dt.fill_(fixed_dt)
            gm.step_dt(U, dt, k)
            om.step_dt(k, fixed_dt)
        torch.cuda.synchronize()
        if (k + 1) % compare_every and k + 1 < steps:
            continue
        err, bw = compare_active(gm, U, om, perm)
        worst = max(worst, err)
        say(f"case {name}: step {k}, rel err {err:.3e}, bitwise fraction {bw:.6f}")
        assert err <= TOL, f"{name}: step {k} rel err {err:.3e}"
    assert gm.floor_count() == om.floors, f"{name}: floor counts differ"
    say(f"case {name}: worst rel err {worst:.3e}, bitwise fraction {bw:.6f}")
    return worst, bw


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,levels,seed", [(8, 3, 1), (16, 2, 2), (32, 1, 3)])
def test_refresh_matches_oracle_bitwise(N, levels, seed):
    root = (2, 3, 2)
    spec = I.MeshSpec(root=root, block_cells=N, max_level=levels,
                      refine=I.random_refine_list(root, levels, 4, seed) if levels else [])
    say(f"refresh N={N} levels={levels}")
    om, gm, perm = pair(spec)
    rng = np.random.default_rng(seed)
    U = load(om, gm, perm, rng.uniform(0.5, 1.5, (gm.nleaf, 5, N, N, N)))
    gm.refresh(U)
    om.refresh()
    torch.cuda.synchronize()
    a = U.cpu().numpy()
    b = om.U[perm]
    assert np.array_equal(a, b)


def test_refresh_large_mesh_bitwise():
    """A mesh above the large-mesh threshold of the phase-1 refresh (4,096
    leaves and more: XCD-contiguous workgroup order, non-temporal ghost
    stores): 16^3 roots of 8^3, two of them refined (4,110 leaves), every cell
    bitwise against the oracle."""
    root = (16, 16, 16)
    spec = I.MeshSpec(root=root, block_cells=8, max_level=1, refine=[(0, 3, 4, 5), (0, 11, 7, 2)])
    om, gm, perm = pair(spec)
    assert gm.nleaf >= 4096
    say(f"refresh large mesh: {gm.nleaf} leaves of 8^3")
    rng = np.random.default_rng(17)
    U = load(om, gm, perm, rng.uniform(0.5, 1.5, (gm.nleaf, 5, 8, 8, 8)))
    gm.refresh(U)
    om.refresh()
    torch.cuda.synchronize()
    assert np.array_equal(U.cpu().numpy(), om.U[perm])


def test_refresh_outflow_uniform_bitwise():
    spec = I.MeshSpec(root=(3, 1, 2), block_cells=8, bc="outflow")
    om, gm, perm = pair(spec)
    rng = np.random.default_rng(9)
    U = load(om, gm, perm, rng.uniform(0.5, 1.5, (gm.nleaf, 5, 8, 8, 8)))
    gm.refresh(U)
    om.refresh()
    torch.cuda.synchronize()
    assert np.array_equal(U.cpu().numpy(), om.U[perm])


def test_cfl_dt_bitwise():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=16, max_level=2, gamma=5 / 3,
                      refine=[(0, 0, 0, 0), (1, 1, 1, 1)])
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, I.smooth_state(spec, gm.keys, seed=4, vel=1.5))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(2):  # the accumulator resets itself
        gm.cfl_dt(U, dt)
        assert float(dt.cpu()[0]) == om.cfl_dt()


def test_sod_config_parity():
    spec = I.sod_spec()
    run_case("sod 4^3 x 16^3 outflow, 20 steps", spec, I.sod_state, 20)


def test_sedov_small_amr_parity():
    spec = I.sedov_spec(root=4, block_cells=8, levels=2)
    run_case("sedov 4^3 x 8^3, 2 levels", spec, I.sedov_state, 12)


@pytest.mark.parametrize("N", [8, 16, 32])
def test_random_amr_smooth_parity(N):
    root = (2, 2, 2)
    levels = 3 if N == 8 else 2
    spec = I.MeshSpec(root=root, block_cells=N, max_level=levels, gamma=5 / 3,
                      refine=I.random_refine_list(root, levels, 5, 100 + N))
    run_case(f"random amr N={N}", spec, lambda s, k: I.smooth_state(s, k, seed=N, amp=0.3, vel=0.8), 4)


@pytest.mark.parametrize("root,bc", [((1, 1, 1), "periodic"), ((3, 1, 2), "periodic"), ((2, 3, 1), "outflow")])
def test_edge_meshes_parity(root, bc):
    spec = I.MeshSpec(root=root, block_cells=8, bc=bc, gamma=1.4)
    run_case(f"edge mesh {root} {bc}", spec, lambda s, k: I.smooth_state(s, k, seed=7, vel=0.7), 3)


def test_fixed_dt_step_parity():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=16, max_level=1, gamma=1.4, refine=[(0, 1, 0, 1)])
    run_case("fixed dt", spec, lambda s, k: I.smooth_state(s, k, seed=12), 3, fixed_dt=1e-3)


def test_floor_triggers_match():
    """Diverging supersonic streams empty the centre: the post-update
    pressure floor fires on both sides in the same cells."""
    spec = I.MeshSpec(root=(4, 1, 1), block_cells=8, gamma=1.4, p_floor=1e-3, rho_floor=1e-6)

    def act(s, keys):
        x = I.cell_centres(s, keys)[0]
        u = np.where(x < 0.5, -4.0, 4.0)
        return I.conserved(1.4, np.ones_like(x), u, 0.0, 0.0, np.full(x.shape, 2e-3))

    run_case("floors", spec, act, 6)


def test_sedov_full_size_parity():
    """The static two-level Sedov workload at its full size (8^3 roots of
    32^3 cells, 624 leaves, 20.4M cells) for its 50 steps against the
    oracle: every step's dt exactly, every field every 10 steps."""
    spec = I.sedov_spec(root=8, block_cells=32, levels=2)
    run_case("sedov full 8^3 x 32^3", spec, I.sedov_state, 50, compare_every=10)


def test_repeat_runs_are_bitwise_identical():
    spec = I.sedov_spec(root=4, block_cells=16, levels=2)
    gm = Mesh(**spec.kwargs())
    act = I.sedov_state(spec, gm.keys)
    outs = []
    for _ in range(2):
        U = gm.state_from_active(act)
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        for k in range(3):
            gm.step(U, dt, k)
        outs.append(gm.active(U))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("modes", [(0, 0, 0), (1, 1, 1), (1, 0, 1), (0, 1, 0)])
def test_sweep_variants_are_bitwise_identical_to_oracle(modes):
    """Both sweep kernels (lane-per-pencil walk, LDS-staged tile) in every
    per-axis combination give the oracle's result bitwise."""
    for N in (8, 16, 32):
        root = (2, 2, 2)
        spec = I.MeshSpec(root=root, block_cells=N, max_level=2, gamma=5 / 3,
                          refine=I.random_refine_list(root, 2, 3, 7 + N))
        say(f"sweep modes {modes} N={N}")
        om, gm, perm = pair(spec)
        gm.set_launch(sweep_mode=list(modes))
        U = load(om, gm, perm, I.smooth_state(spec, gm.keys, seed=N + 1, amp=0.3, vel=0.8))
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        for k in range(2):
            gm.step(U, dt, k)
            assert float(dt.cpu()[0]) == om.step(k)
        err, bw = compare_active(gm, U, om, perm)
        assert bw == 1.0, (modes, N, err)


def test_autotuned_launch_is_bitwise_identical():
    from paper_1810_01319_amd import autotune

    spec = I.sedov_spec(root=4, block_cells=16, levels=2)
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, I.sedov_state(spec, gm.keys))
    cfg = autotune.tune(gm, U, steps=1, use_cache=False)
    say(f"autotuned {cfg['sweep_mode']} block {cfg['sweep_block']}")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(3):
        gm.step(U, dt, k)
        assert float(dt.cpu()[0]) == om.step(k)
    assert compare_active(gm, U, om, perm)[1] == 1.0


def _oracle_adaptive(om, steps, thr_r, thr_c, cap, interval=4):
    dts, stats = [], []
    for k in range(steps):
        if k > 0 and k % interval == 0:
            om, st = om.remesh(thr_r, thr_c, cap)
            stats.append([int(v) for v in st])
        dts.append(om.step(k))
    return om, dts, stats


@pytest.mark.parametrize("root,N,levels,cap_extra,steps", [
    (3, 8, 2, 10 ** 6, 13), (3, 16, 3, 10 ** 6, 13), (3, 8, 3, 60, 13),
    (4, 32, 3, 10 ** 6, 9),  # the large adaptive workload's 4^3-octree tile: remesh before steps 4 and 8
])
def test_adaptive_blasts_parity(root, N, levels, cap_extra, steps):
    """Blasts with remesh every 4 steps: indicator, decisions, migrated data
    and the following steps all bitwise equal to the oracle."""
    from paper_1810_01319_amd import adaptive

    spec = I.blasts_spec(root=root, block_cells=N, levels=levels)
    say(f"adaptive blasts root={root} N={N} levels={levels} steps={steps}")
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, I.blasts_state(spec, gm.keys))
    cap = gm.nleaf + cap_extra
    gm2, U2, dts, gst = adaptive.run(gm, U, steps, max_blocks=cap)
    om2, odts, ost = _oracle_adaptive(om, steps, 0.3, 0.1, cap)
    assert [float(d.cpu()[0]) for d in dts] == odts
    assert [[s["refined"], s["coarsened"], s["refused"]] for s in gst] == ost
    idx = {tuple(k): s for s, k in enumerate(om2.keys)}
    perm2 = np.array([idx[tuple(k)] for k in gm2.keys])
    err, bw = compare_active(gm2, U2, om2, perm2)
    say(f"adaptive: leaves {gm.nleaf} -> {gm2.nleaf}, stats {ost}, bitwise {bw}")
    assert bw == 1.0, err


@pytest.mark.parametrize("seed", [0, 1 << 40])
def test_kernel_reciprocal_and_sqrt_are_ieee_bitwise(seed):
    """The kernels' reciprocal and square root of positive operands (the IEEE
    sequences without operand scaling and special-value fix-ups) equal IEEE
    1/x and sqrt(x) bit for bit on 2^26 operands spread over the exponent
    range [-767, 1022] that floors >= 1e-100 guarantee."""
    from paper_1810_01319_amd.mesh import arith_selftest
    n = 1 << 26
    bad_rcp, bad_sqrt = arith_selftest(n, seed)
    say(f"arith self-test seed {seed}: {n} operands, {bad_rcp} reciprocal and {bad_sqrt} sqrt mismatches")
    assert bad_rcp == 0 and bad_sqrt == 0


def test_indicator_bitwise():
    spec = I.blasts_spec(root=3, block_cells=16, levels=2)
    om, gm, perm = pair(spec)
    U = load(om, gm, perm, I.blasts_state(spec, gm.keys))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(3):
        gm.step(U, dt, k)
        om.step(k)
    gm.refresh(U)
    om.refresh()
    assert np.array_equal(gm.indicator(U).cpu().numpy(), om.indicator()[perm])


def test_batched_instances_match_oracle_bitwise():
    """16 uneven instances of the batched workload in one worklist: every
    instance's dt sequence and state equal its own oracle run bitwise over
    10 steps."""
    specs, cents = zip(*[I.batch_instance(i) for i in range(16)])
    gm = Mesh.batch([s.kwargs() for s in specs])
    say(f"batch of 16: {gm.nleaf} leaves")
    acts = []
    oms = []
    for i, (sp, c) in enumerate(zip(specs, cents)):
        keys = gm.keys[gm.first_leaf[i]:gm.first_leaf[i + 1]]
        acts.append(I.batch_state(sp, keys, c))
        om = O.OracleMesh(**sp.kwargs())
        idx = {tuple(k): s for s, k in enumerate(om.keys)}
        perm = np.array([idx[tuple(k)] for k in keys])
        o = np.empty_like(acts[-1])
        o[perm] = acts[-1]
        om.set_active(o)
        oms.append((om, perm))
    U = gm.state_from_active(np.concatenate(acts))
    dt = gm.dt_tensor()
    for k in range(10):
        gm.step(U, dt, k)
        dts = dt.cpu().numpy()
        for i, (om, perm) in enumerate(oms):
            assert dts[i] == om.step(k), (i, k)
    act = gm.active(U)
    for i, (om, perm) in enumerate(oms):
        a = act[gm.first_leaf[i]:gm.first_leaf[i + 1]]
        assert np.array_equal(a, om.active()[perm]), i


def test_graph_replays_equal_eager_steps():
    """Two captured steps (the second's CFL fused into the first) replayed
    several times, with eager work and synchronisations in between, equal
    the same steps run eagerly one by one, state and dt."""
    specs, cents = zip(*[I.batch_instance(i) for i in range(6)])
    gm = Mesh.batch([s.kwargs() for s in specs])
    acts = [I.batch_state(sp, gm.keys[gm.first_leaf[i]:gm.first_leaf[i + 1]], c)
            for i, (sp, c) in enumerate(zip(specs, cents))]
    act = np.concatenate(acts)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        Ue = gm.state_from_active(act)
        dte = gm.dt_tensor()
        for k in range(6):
            gm.step(Ue, dte, k)
        ref = gm.active(Ue)
        Ug = gm.state_from_active(act)
        dtg = gm.dt_tensor()
        side.synchronize()
        g = gm.graph(Ug, dtg, first_step=0)
        for rep in range(3):
            g.launch()
            junk = torch.ones(1000, device="cuda").sum()  # eager work between replays
            side.synchronize()
            assert float(junk) == 1000.0
        got = gm.active(Ug)
    assert np.array_equal(got, ref)
    assert torch.equal(dtg, dte)  # both hold the sixth step's dt


def _floor_spec_state():
    spec = I.MeshSpec(root=(4, 1, 1), block_cells=8, gamma=1.4, p_floor=1e-3, rho_floor=1e-6)
    m = Mesh(**spec.kwargs())
    x = I.cell_centres(spec, m.keys)[0]
    u = np.where(x < 0.5, -4.0, 4.0)
    act = I.conserved(1.4, np.ones_like(x), u, 0.0, 0.0, np.full(x.shape, 2e-3))
    return spec, m, act


@pytest.mark.parametrize("case", ["random-amr", "floors"])
def test_recorded_steps_equal_plain_steps(case):
    """The recording step (out-of-place sweeps into S1, S2 and a new state)
    gives bitwise the plain step's dt and active cells, leaves its input's
    active cells unchanged, and counts the step's floor resets."""
    if case == "random-amr":
        spec = I.MeshSpec(root=(2, 2, 2), block_cells=16, max_level=2, gamma=5 / 3,
                          refine=I.random_refine_list((2, 2, 2), 2, 4, 7))
        m = Mesh(**spec.kwargs())
        act = I.smooth_state(spec, m.keys, seed=8, amp=0.2, vel=0.4)
    else:
        spec, m, act = _floor_spec_state()
    say(f"recorded steps: {case}, {m.nleaf} leaves")
    Up = m.state_from_active(act)
    dtp = m.dt_tensor()
    U = m.state_from_active(act)
    dt = m.dt_tensor()
    total = 0
    for k in range(5):
        before = m.floor_count()
        m.step(Up, dtp, k)
        plain_resets = m.floor_count() - before
        S1, S2, Uo = (torch.empty_like(U) for _ in range(3))
        floors = torch.empty(1, dtype=torch.int64, device=U.device)
        a0 = m.active(U)
        before = m.floor_count()
        m.step_record(U, dt, S1, S2, Uo, floors, k)
        assert int(floors.cpu()[0]) == m.floor_count() - before == plain_resets
        total += plain_resets
        assert np.array_equal(m.active(U), a0)
        assert float(dt.cpu()[0]) == float(dtp.cpu()[0])
        assert np.array_equal(m.active(Uo), m.active(Up)), k
        U = Uo
    if case == "floors":
        assert total > 0
