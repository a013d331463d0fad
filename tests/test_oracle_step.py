"""Pins of the oracle's full timestep (refresh + CFL + three PPM sweeps +
reflux) against exact solutions, conservation laws and symmetries."""
import os
import subprocess
import sys

import numpy as np
import pytest

import physics_ref as P
from oracle import oracle as O
from paper_1810_01319_amd import inputs as I

G = 3


def run(spec, U0, steps, mesh=None):
    m = mesh or O.OracleMesh(**spec.kwargs())
    m.set_active(U0 if not callable(U0) else U0(spec, m.keys))
    dts = [m.step(k) for k in range(steps)]
    return m, dts


def totals(m, spec):
    act = m.active()
    vol = np.array([spec.dx(int(l)) ** 3 for l in m.keys[:, 0]])
    return (act.reshape(act.shape[0], 5, -1).sum(-1) * vol[:, None]).sum(0)


def test_free_stream_is_preserved_bitwise_on_amr():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=2, gamma=5 / 3,
                      refine=[(0, 0, 0, 0), (1, 1, 1, 1)])
    m = O.OracleMesh(**spec.kwargs())
    U0 = I.conserved(spec.gamma, np.full((m.nleaf, 8, 8, 8), 1.3), 0.7, -0.4, 0.25,
                     np.full((m.nleaf, 8, 8, 8), 0.9))
    m.set_active(U0)
    for k in range(4):
        m.step(k)
    assert np.array_equal(m.active(), U0)


@pytest.fixture(scope="module")
def sod_run():
    spec = I.sod_spec()
    m, dts = run(spec, I.sod_state, 20)
    return spec, m, float(np.sum(dts))


def sod_profile(spec, m):
    """rho along x from the row of blocks at y, z index 0 (all rows agree)."""
    N = spec.block_cells
    act = m.active()
    x = np.zeros(spec.root[0] * N)
    rho = np.zeros_like(x)
    for s, k in enumerate(m.keys):
        if k[2] == 0 and k[3] == 0:
            sl = slice(k[1] * N, (k[1] + 1) * N)
            rho[sl] = act[s, 0, 0, 0, :]
            x[sl] = (np.arange(N) + k[1] * N + 0.5) * spec.dx(0)
    return x, rho


def test_sod_rows_are_identical_bitwise(sod_run):
    spec, m, t = sod_run
    act = m.active()
    for f in range(5):
        a = act[:, f]
        assert np.all(a == a[:, :1, :1, :]), "every (y,z) row of a 1-D problem must agree"


def test_sod_matches_exact_solution(sod_run):
    spec, m, t = sod_run
    x, rho = sod_profile(spec, m)
    WL, WR = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ex = np.array([P.exact_sample(WL, WR, 1.4, (xi - 0.5) / t)[0] for xi in x])
    l1 = np.mean(np.abs(rho - ex))
    assert l1 <= 0.02
    dx = spec.dx(0)
    ps, us = P.exact_star(WL, WR, 1.4)
    S = P.shock_speed_right(WR, ps, 1.4)
    rsl = P.exact_sample(WL, WR, 1.4, us - 1e-9)[0]
    rsr = P.exact_sample(WL, WR, 1.4, us + 1e-9)[0]

    def crossing(level, lo, hi):
        sel = np.where((x > lo) & (x < hi))[0]
        i = sel[np.argmax(np.diff(np.sign(rho[sel] - level)) != 0)]
        return x[i] + dx * (level - rho[i]) / (rho[i + 1] - rho[i])

    xs = crossing(0.5 * (rsr + 0.125), 0.5 + us * t + 2 * dx, 0.99)
    xc = crossing(0.5 * (rsl + rsr), 0.5, 0.5 + (us + S) * t / 2 + 2 * dx)
    assert abs(xs - (0.5 + S * t)) <= 2 * dx
    assert abs(xc - (0.5 + us * t)) <= 2 * dx


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_blocked_mesh_equals_single_block_bitwise(bc):
    big = I.MeshSpec(root=(1, 1, 1), block_cells=16, bc=bc, gamma=1.4)
    small = I.MeshSpec(root=(2, 2, 2), block_cells=8, bc=bc, gamma=1.4)
    mb = O.OracleMesh(**big.kwargs())
    Ub = I.smooth_state(big, mb.keys, seed=11)
    mb.set_active(Ub)
    ms = O.OracleMesh(**small.kwargs())
    # the same global field cut into 8 blocks
    Us = np.zeros((ms.nleaf, 5, 8, 8, 8))
    for s, k in enumerate(ms.keys):
        Us[s] = Ub[0][:, k[3] * 8:(k[3] + 1) * 8, k[2] * 8:(k[2] + 1) * 8, k[1] * 8:(k[1] + 1) * 8]
    ms.set_active(Us)
    for k in range(4):
        db, ds = mb.step(k), ms.step(k)
        assert db == ds
    ab, as_ = mb.active(), ms.active()
    for s, k in enumerate(ms.keys):
        blk = ab[0][:, k[3] * 8:(k[3] + 1) * 8, k[2] * 8:(k[2] + 1) * 8, k[1] * 8:(k[1] + 1) * 8]
        assert np.array_equal(blk, as_[s])


def test_rotated_one_dimensional_problems_agree_bitwise():
    """The same 1-D wave along x, y and z gives the same profile: checks the
    sweep's axis strides and the normal/transverse momentum roles."""
    N, n = 8, 4
    outs = []
    for ax in range(3):
        root = [1, 1, 1]
        root[ax] = n
        spec = I.MeshSpec(root=tuple(root), block_cells=N, gamma=1.4)
        m = O.OracleMesh(**spec.kwargs())
        coords = I.cell_centres(spec, m.keys)
        s = coords[ax] / (n * spec.dx(0) * N)  # position along the wave, in [0,1)
        rho = 1.0 + 0.3 * np.sin(2 * np.pi * s) + 0.4 * (s > 0.5)
        vel = [0.0, 0.0, 0.0]
        un = 0.3 * np.cos(2 * np.pi * s)
        p = 1.0 + 0.2 * (s < 0.3)
        U = I.conserved(1.4, rho, *(un if a == ax else 0.0 for a in range(3)), p)
        m.set_active(U)
        dx = spec.dx(0)
        for k in range(6):
            m.step_dt(k, 0.05 * dx)
        act = m.active()
        prof = np.zeros((5, n * N))
        for si, key in enumerate(m.keys):
            blk = np.moveaxis(act[si], 3 - ax, -1)[:, 0, 0, :]
            prof[:, key[1 + ax] * N:(key[1 + ax] + 1) * N] = blk
        # put the normal momentum in slot 1, transverse ones are zero
        prof = prof[[0, 1 + ax, 4]]
        outs.append(prof)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_conservation_to_round_off_on_periodic_amr():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=2, gamma=5 / 3,
                      refine=[(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 1, 0)])
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(I.smooth_state(spec, m.keys, seed=5, amp=0.3, vel=0.6))
    t0 = totals(m, spec)
    for k in range(6):
        m.step(k)
    t1 = totals(m, spec)
    assert m.floors == 0
    scale = np.array([t0[0], t0[0], t0[0], t0[0], t0[4]])
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t1 - t0) / scale


def test_conservation_check_detects_a_missing_reflux():
    """With the reflux switched off (a mistake planted in the oracle) the
    same run loses conservation far above round-off."""
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=2, gamma=5 / 3,
                      refine=[(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 1, 0)])
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(I.smooth_state(spec, m.keys, seed=5, amp=0.3, vel=0.6))
    t0 = totals(m, spec)
    O.set_debug(O.DEBUG_SKIP_REFLUX)
    try:
        for k in range(3):
            m.step(k)
    finally:
        O.set_debug(0)
    assert np.max(np.abs(totals(m, spec) - t0)[[0, 4]] / t0[[0, 4]]) > 1e-8


def test_blast_on_symmetric_amr_mesh_is_mirror_symmetric_bitwise():
    spec = I.sedov_spec(root=4, block_cells=8, levels=2)
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(I.sedov_state(spec, m.keys))
    for k in range(6):
        m.step(k)
    act = m.active()
    N = 8
    idx = {tuple(k): s for s, k in enumerate(m.keys)}
    for ax in range(3):
        for s, k in enumerate(m.keys):
            l = int(k[0])
            mk = list(k)
            mk[1 + ax] = (spec.root[ax] << l) - 1 - k[1 + ax]
            t = idx[tuple(mk)]
            mirrored = np.flip(act[t], axis=3 - ax)
            sign = np.ones(5)
            sign[1 + ax] = -1
            assert np.array_equal(act[s], mirrored * sign[:, None, None, None])


def _wave_error(n_cells, kind, mach=0.0):
    """L1 error (relative to the amplitude) of a smooth wave on a background
    flow of Mach number `mach` along x, after T = 0.25, at fixed dt."""
    N = 8
    spec = I.MeshSpec(root=(n_cells // N, 1, 1), block_cells=N, gamma=1.4)
    m = O.OracleMesh(**spec.kwargs())
    x = I.cell_centres(spec, m.keys)[0]
    dx = spec.dx(0)
    c0 = np.sqrt(1.4)
    u0 = mach * c0
    if kind == "entropy":
        amp = 0.2
        rho = 1.0 + amp * np.sin(2 * np.pi * x)
        U = I.conserved(1.4, rho, u0 if mach else 1.0, 0.0, 0.0, np.ones_like(x))
        speed = u0 if mach else 1.0
    else:  # linear acoustic wave running with speed u0 + s c0
        amp = 1e-6  # small enough that nonlinear steepening is below the error
        s = 1.0 if kind == "acoustic" else -1.0
        d = amp * np.sin(2 * np.pi * x)
        U = I.conserved(1.4, 1.0 + d, u0 + s * c0 * d, 0.0, 0.0, 1.0 + 1.4 * d)
        speed = u0 + s * c0
    m.set_active(U)
    T = 0.25
    vmax = abs(u0) + c0
    nsteps = int(np.ceil(T / (0.4 * dx / vmax)))
    dt = T / nsteps
    for k in range(nsteps):
        m.step_dt(k, dt)
    rho = m.active()[:, 0]
    ex = 1.0 + amp * np.sin(2 * np.pi * (x - speed * T))
    return np.mean(np.abs(rho - ex)) / amp


@pytest.mark.parametrize("kind,mach", [("entropy", 0.0), ("acoustic", 0.0), ("entropy", 0.5),
                                       ("acoustic", 0.5), ("acoustic_left", 0.5),
                                       ("acoustic", 2.0), ("acoustic_left", 2.0),
                                       ("acoustic", -2.0), ("acoustic_left", -2.0)])
def test_smooth_waves_converge_at_second_order(kind, mach):
    """Sub- and supersonic background flows exercise every branch of the
    characteristic tracing (each family reaching either edge)."""
    e1, e2 = _wave_error(32, kind, mach), _wave_error(64, kind, mach)
    order = np.log2(e1 / e2)
    assert order > 1.6, (e1, e2, order)


@pytest.mark.slow
def test_sedov_radius_and_peak_density():
    spec = I.sedov_spec(root=4, block_cells=8, levels=2)
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(I.sedov_state(spec, m.keys))
    t = 0.0
    k = 0
    target = 0.06
    g = spec.gamma
    while P.sedov_radius(1.0, t, 1.0, g) < target:
        t += m.step(k)
        k += 1
    assert m.floors == 0
    act = m.active()
    dx2 = spec.dx(2)
    x, y, z = I.cell_centres(spec, m.keys)
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2)
    fine = (m.keys[:, 0] == 2)
    rr, rho = r[fine].ravel(), act[fine][:, 0].ravel()
    bins = np.arange(0, 0.125, dx2)
    which = np.digitize(rr, bins)
    prof = np.array([rho[which == i].mean() if np.any(which == i) else 0 for i in range(1, len(bins))])
    Rnum = 0.5 * (bins[np.argmax(prof)] + bins[np.argmax(prof) + 1])
    R = P.sedov_radius(1.0, t, 1.0, g)
    assert abs(Rnum - R) <= max(0.05 * R, 2 * dx2), (Rnum, R, k)
    assert act[:, 0].max() <= (g + 1) / (g - 1)
    assert R < 0.125  # the shock is still inside the finest region


def test_results_do_not_depend_on_thread_count(tmp_path):
    code = r"""
import sys, numpy as np
sys.path.insert(0, %r)
from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=2, gamma=5/3, refine=[(0,0,0,0),(1,1,1,1)])
m = O.OracleMesh(**spec.kwargs())
m.set_active(I.smooth_state(spec, m.keys, seed=3))
for k in range(2): m.step(k)
np.save(sys.argv[1], m.active())
""" % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for th in ("1", "5"):
        f = tmp_path / f"o{th}.npy"
        env = dict(os.environ, OMP_NUM_THREADS=th)
        subprocess.check_call([sys.executable, "-c", code, str(f)], env=env)
        outs.append(np.load(f))
    assert np.array_equal(outs[0], outs[1])
