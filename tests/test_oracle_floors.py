"""Pins of the oracle's positivity floors and of its 3-D CFL time step.

The floors and the CFL rule are readings (the paper names the PPM Method of
Sec. II-C but none of its safeguards), so each is pinned against what the
reading itself fixes, independently of the oracle's code:

* post-update floors: after a sweep no active cell has rho below rho_floor
  or pressure below p_floor; a pressure reset changes E alone (momenta are
  untouched, so total momentum stays conserved on a periodic mesh while mass
  and energy can only grow); the reset count is the number of cells reset;
* the dual-energy field's floor: rho e is never left with (gamma-1) rho e
  below p_floor;
* the edge-state floors in the characteristic tracing keep every Riemann
  input positive, so any pencil of positive states gives finite fluxes;
* the comoving expansion source raises an internal energy that it lowered
  below the floor to exactly the floor, scales every momentum by the same
  factor, and counts each raised cell once;
* the CFL step is C min_cells dx_l / (max_d |u_d| + c), checked against a
  closed form and a brute-force minimum over an AMR mesh.

Each check has a planted mistake in the oracle (``DEBUG_*``) that fails it.
"""
import numpy as np
import pytest

import physics_ref as P
from oracle import oracle as O
from paper_1810_01319_amd import inputs as I

GAMMA = 1.4


def planted(flags, fn, *a, **kw):
    O.set_debug(flags)
    try:
        return fn(*a, **kw)
    finally:
        O.set_debug(0)


def kinetic(a):
    """Kinetic energy density of active cells, in the order the step's floor
    test evaluates it."""
    rho = a[:, 0]
    ir = 1.0 / rho
    u, v, w = a[:, 1] * ir, a[:, 2] * ir, a[:, 3] * ir
    return (0.5 * rho) * ((u * u + v * v) + w * w)


# ---------------------------------------------------------------------------
# Post-update floors
# ---------------------------------------------------------------------------

# Floors well inside the state's range: a diverging flow pulls the centre
# below both within one sweep, while the initial state satisfies them.
FLOOR_SPEC = I.MeshSpec(root=(4, 1, 1), block_cells=8, gamma=GAMMA, rho_floor=0.97, p_floor=0.95)


def diverging(spec, keys, dual=False):
    """1-D along x: streams leaving x = 1/2 at +-0.5 on a bulk flow of 0.15,
    transverse velocities 0.2 and -0.1 (so a floor that touched the momenta
    would show in every component), density 1 + 0.02 sin(2 pi x), p = 1."""
    x = I.cell_centres(spec, keys)[0]
    u = np.where(x < 0.5, -0.5, 0.5) + 0.15
    rho = 1.0 + 0.02 * np.sin(2 * np.pi * x)
    U = I.conserved(spec.gamma, rho, u, 0.2 + 0 * x, -0.1 + 0 * x, np.ones_like(x))
    return I.with_internal_energy(U) if dual else U


def floor_step_violations(spec, k, dual=False):
    """One step of index k from the diverging state; returns (list of
    violated statements, floor count, number of reset cells seen)."""
    m = O.OracleMesh(**spec.kwargs())
    a0 = diverging(spec, m.keys, dual)
    m.set_active(a0)
    m.step(k)
    a = m.active()
    bad = []
    rho, E = a[:, 0], a[:, 4]
    ke = kinetic(a)
    ig = 1.0 / (spec.gamma - 1.0)
    if np.any(rho < spec.rho_floor):
        bad.append("rho below its floor")
    p = (spec.gamma - 1.0) * (E - ke)
    E_reset = E == spec.p_floor * ig + ke  # the reset's own value, bit for bit
    if np.any(~E_reset & (p < spec.p_floor)):
        bad.append("pressure below its floor in a cell the floor did not reset")
    if np.any(E_reset & (np.abs(p - spec.p_floor) > 1e-12 * np.abs(E))):
        bad.append("reset cell's (gamma-1)(E-ke) is not p_floor to rounding")
    seen = int(np.sum(rho == spec.rho_floor) + np.sum(E_reset))
    if dual:
        ge = a[:, 5]
        ge_floor = ge == spec.p_floor * ig
        if np.any(~ge_floor & ((spec.gamma - 1.0) * ge < spec.p_floor)):
            bad.append("rho e below its floor")
        seen += int(np.sum(ge_floor))
    return bad, m.floors, seen


@pytest.mark.parametrize("dual", [False, True])
def test_floors_on_a_last_sweep_reset_exactly_the_counted_cells(dual):
    """Step 1 sweeps z, y, x: the 1-D flow leaves the first two sweeps
    bitwise unchanged (identical fluxes on both faces), so every reset
    happens in the last sweep, on active cells only, and stays visible: the
    count must equal the cells at their floor values."""
    spec = I.with_(FLOOR_SPEC, dual_energy=True, p_floor=0.94) if dual else FLOOR_SPEC
    if dual:  # a resynchronised rho e equal to the floor value is itself reset
        assert (spec.gamma - 1.0) * (spec.p_floor * (1.0 / (spec.gamma - 1.0))) < spec.p_floor
    bad, count, seen = floor_step_violations(spec, 1, dual)
    assert not bad, bad
    assert seen > 0
    assert count == seen


@pytest.mark.parametrize("p_floor", [0.95, 0.94])
def test_floors_in_a_first_sweep_count_every_swept_row(p_floor):
    """Step 0 sweeps x first, over the active cells along x and over every
    row of the block including the ghost rows along y and z (they are
    swept to give the later sweeps their ghosts).  All M^2 rows of the 1-D
    flow reset the same cells, so the first sweep counts the active resets
    times M^2 / N^2.  A reset cell whose (gamma-1)(E - ke) rounds below
    p_floor again (p_floor 0.94 here, not 0.95) is reset to the same bits by
    the y sweep (active x and y, all z: M/N of the active count) and by the
    z sweep (active cells), and counted each time."""
    spec = I.with_(FLOOR_SPEC, p_floor=p_floor)
    bad, count, seen = floor_step_violations(spec, 0)
    assert not bad, bad
    N, M = spec.block_cells, spec.block_cells + 6
    assert seen > 0 and seen % (N * N) == 0
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(diverging(spec, m.keys))
    m.step(0)
    a = m.active()
    ke = kinetic(a)
    E_reset = a[:, 4] == spec.p_floor * (1.0 / (spec.gamma - 1.0)) + ke
    again = int(np.sum(E_reset & ((spec.gamma - 1.0) * (a[:, 4] - ke) < spec.p_floor)))
    assert (again > 0) == (p_floor == 0.94)
    assert count == seen // (N * N) * (M * M) + again * M // N + again


def test_floors_conserve_momentum_and_only_add_mass_and_energy():
    """Six steps on the periodic mesh with floors firing every step: the
    floors change rho and E only, so total momentum (all three components
    nonzero) stays constant to round-off, mass and energy never decrease,
    and rho and p stay at or above their floors."""
    spec = FLOOR_SPEC
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(diverging(spec, m.keys))
    vol = spec.dx(0) ** 3

    def tot(a):
        return a.reshape(a.shape[0], 5, -1).sum(-1).sum(0) * vol

    t0 = tot(m.active())
    scale = np.abs(m.active()[:, 1:4]).sum() * vol
    prev = t0
    for k in range(6):
        before = m.floors
        m.step(k)
        a = m.active()
        t = tot(a)
        assert m.floors > before
        assert np.max(np.abs(t[1:4] - t0[1:4])) <= 1e-14 * scale, "momentum changed"
        assert t[0] >= prev[0] and t[4] >= prev[4]
        assert np.all(a[:, 0] >= spec.rho_floor)
        p = (spec.gamma - 1.0) * (a[:, 4] - kinetic(a))
        assert np.all(p >= spec.p_floor * (1 - 1e-12))
        prev = t


def test_planted_floor_mistakes_fail_the_pins():
    spec = FLOOR_SPEC
    # E reset to p_floor/(gamma-1) without the kinetic energy
    bad, _, _ = planted(O.DEBUG_FLOOR_E_NO_KE, floor_step_violations, spec, 1)
    assert bad
    # a density floor that keeps the velocity changes the momenta
    with pytest.raises(AssertionError, match="momentum"):
        planted(O.DEBUG_FLOOR_KEEP_VEL, test_floors_conserve_momentum_and_only_add_mass_and_energy)
    # density resets left uncounted
    bad, count, seen = planted(O.DEBUG_FLOOR_NO_COUNT, floor_step_violations, spec, 1)
    assert count != seen
    # rho e floored to p_floor instead of p_floor/(gamma-1)
    bad, _, _ = planted(O.DEBUG_DE_FLOOR_NO_IG, floor_step_violations,
                        I.with_(spec, dual_energy=True, p_floor=0.94), 1, True)
    assert bad


# ---------------------------------------------------------------------------
# Edge-state floors of the characteristic tracing
# ---------------------------------------------------------------------------

def random_pencils(n_pencils, seed=1, n=12):
    """Pencils of positive states over many decades of density and pressure
    and supersonic velocities, each with nu at CFL 0.4 of its own fastest
    signal."""
    rng = np.random.default_rng(seed)
    for _ in range(n_pencils):
        rho = np.exp(rng.uniform(-8, 0, n))
        u = rng.uniform(-3, 3, n)
        p = np.exp(rng.uniform(-10, 0, n))
        nu = 0.4 / np.max(np.abs(u) + np.sqrt(GAMMA * p / rho))
        U = np.stack([rho, rho * u, 0 * u, 0 * u, p / (GAMMA - 1) + 0.5 * rho * u * u])
        yield U, nu


def count_nonfinite_pencils(n_pencils):
    return sum(not np.all(np.isfinite(O.pencil_flux(U, nu, GAMMA))) for U, nu in random_pencils(n_pencils))


def test_edge_floors_keep_every_pencil_flux_finite():
    """Tracing can carry an edge pressure or density below zero in a strong
    rarefaction; the floors keep the Riemann inputs positive, so every
    pencil of positive states has finite fluxes.  Without them the same
    seeded set holds pencils whose fluxes are NaN."""
    n = 11000
    assert count_nonfinite_pencils(n) == 0
    assert planted(O.DEBUG_EDGE_NO_FLOOR, count_nonfinite_pencils, n) > 0


def double_rarefaction(U, steps_to=0.15, N=8, root=8, floors=(1e-20, 1e-20)):
    spec = I.MeshSpec(root=(root, 1, 1), block_cells=N, gamma=GAMMA, bc="outflow",
                      rho_floor=floors[0], p_floor=floors[1])
    m = O.OracleMesh(**spec.kwargs())
    x = I.cell_centres(spec, m.keys)[0]
    m.set_active(I.conserved(GAMMA, np.ones_like(x), np.where(x < 0.5, -U, U), 0.0, 0.0, np.full(x.shape, 0.4)))
    t, k = 0.0, 0
    while t < steps_to - 1e-14:
        dt = min(m.cfl_dt(), steps_to - t)
        m.step_dt(k, dt)
        t += dt
        k += 1
    a = m.active()
    xs = np.zeros(root * N)
    prof = np.zeros((3, root * N))
    for s, key in enumerate(m.keys):
        sl = slice(key[1] * N, (key[1] + 1) * N)
        xs[sl] = (np.arange(N) + key[1] * N + 0.5) * spec.dx(0)
        r, mu, E = a[s, 0, 0, 0], a[s, 1, 0, 0], a[s, 4, 0, 0]
        prof[:, sl] = r, mu / r, (GAMMA - 1) * (E - 0.5 * mu * mu / r)
    return xs, prof, t, m.floors


def test_near_vacuum_double_rarefaction_matches_exact_solution():
    """Toro's '123' problem (rho 1, u -+2, p 0.4, gamma 1.4) at t = 0.15 on
    64 cells: density within an L1 error of 0.02 of the exact solution, the
    centre's near-vacuum resolved with positive density and pressure and no
    floor reset."""
    xs, prof, t, floors = double_rarefaction(2.0)
    ex = np.array([P.exact_sample((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), GAMMA, (x - 0.5) / t)[0] for x in xs])
    assert np.mean(np.abs(prof[0] - ex)) <= 0.02
    assert np.all(prof[0] > 0) and np.all(prof[2] > 0)
    assert floors == 0
    # the exact minimum density is 0.0219 at the centre; the scheme's is
    # smaller (numerical diffusion of a vacuum-like state), not negative
    assert prof[0].min() < 0.05


def test_vacuum_forming_rarefaction_stays_positive():
    """Streams at -+4 open a true vacuum (2 c / (gamma - 1) < 4): with the
    floors at 1e-8 the run stays finite, rho positive and p at or above the
    floor to rounding, with the floors firing."""
    xs, prof, t, floors = double_rarefaction(4.0, floors=(1e-8, 1e-8))
    assert np.all(np.isfinite(prof))
    assert np.all(prof[0] > 0)
    assert np.all(prof[2] >= 1e-8 * (1 - 1e-6))
    assert floors > 0


# ---------------------------------------------------------------------------
# Expansion source floor (comoving coordinates)
# ---------------------------------------------------------------------------

EXP_SPEC = I.MeshSpec(root=(2, 1, 1), block_cells=8, gamma=5.0 / 3.0, p_floor=1e-3, rho_floor=1e-6)


def cold_hot(spec, keys):
    x = I.cell_centres(spec, keys)[0]
    p = np.where(x < 0.5, 1.2e-3, 1.0)
    return I.conserved(spec.gamma, np.ones_like(x), 0.1 * np.sin(2 * np.pi * x), 0.05, -0.03, p)


def expansion_violations(spec, dt, a, hubble):
    """The comoving step against the plain step with dt / a on the same
    input (the expansion source runs after it): returns violated
    statements."""
    mc = O.OracleMesh(**spec.kwargs())
    mp = O.OracleMesh(**spec.kwargs())
    act = cold_hot(spec, mc.keys)
    mc.set_active(act)
    mp.set_active(act)
    mc.step_comoving(0, dt, a, hubble)
    mp.step_dt(0, dt / a)
    ac, ap = mc.active(), mp.active()
    bad = []
    # every momentum component scaled by one common factor, below 1
    ratio = ac[:, 1:4] / ap[:, 1:4]
    f = ratio.flat[0]
    if not (0.0 < f < 1.0) or np.max(np.abs(ratio - f)) > 1e-15:
        bad.append("momenta not scaled by one factor")
    if not np.array_equal(ac[:, 0], ap[:, 0]):
        bad.append("density changed")
    ie_c = ac[:, 4] - kinetic(ac)
    ie_p = ap[:, 4] - kinetic(ap)
    gm1 = spec.gamma - 1.0
    raised = np.abs(gm1 * ie_c - spec.p_floor) <= 1e-9 * spec.p_floor
    if np.any(gm1 * ie_c < spec.p_floor * (1 - 1e-9)):
        bad.append("internal energy left below the floor")
    # cells not raised follow the Crank-Nicolson factor of the adiabatic
    # decay rate 3 (gamma - 1) H: ie'/ie = (1 - 3 (gamma-1) c) / (1 + 3 (gamma-1) c)
    c = 0.5 * dt * hubble
    fe = (1 - 3 * gm1 * c) / (1 + 3 * gm1 * c)
    keep = ~raised
    if np.any(np.abs(ie_c[keep] - fe * ie_p[keep]) > 1e-9 * np.abs(ie_p[keep])):
        bad.append("unraised cell's internal energy not decayed by the source factor")
    if mc.floors - mp.floors != int(raised.sum()):
        bad.append(f"count {mc.floors - mp.floors} != raised cells {int(raised.sum())}")
    return bad, int(raised.sum())


def test_expansion_floor_raises_to_the_floor_and_counts_once():
    """A strong expansion rate (c = dt H / 2 = 0.25) cools the cold half
    below the pressure floor and leaves the hot half above it."""
    bad, raised = expansion_violations(EXP_SPEC, 1e-3, 1.0, 500.0)
    assert not bad, bad
    N = EXP_SPEC.block_cells
    assert 0 < raised < 2 * N ** 3


def test_planted_expansion_floor_mistake_fails_the_pin():
    bad, _ = planted(O.DEBUG_EXP_FLOOR_NO_IG, expansion_violations, EXP_SPEC, 1e-3, 1.0, 500.0)
    assert bad


# ---------------------------------------------------------------------------
# CFL time step in three dimensions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("vel", [(0.7, 0.3, -0.5), (0.3, -0.7, 0.5), (0.2, 0.5, -0.7)])
def test_cfl_of_a_uniform_3d_flow_is_the_closed_form(vel):
    """Uniform rho 1, p 0.5, velocity with its largest component on x, y or
    z in turn: dt = C dx / (max_d |u_d| + c) (a sum over the components
    would give C dx / (1.5 + c))."""
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, gamma=GAMMA, cfl=0.4)
    m = O.OracleMesh(**spec.kwargs())
    shape = (m.nleaf, 8, 8, 8)
    m.set_active(I.conserved(GAMMA, np.ones(shape), *vel, np.full(shape, 0.5)))
    c = np.sqrt(GAMMA * 0.5)
    want = 0.4 * spec.dx(0) / (0.7 + c)
    assert abs(m.cfl_dt() - want) <= 1e-15 * want


def brute_force_cfl(spec, keys, act):
    best = np.inf
    for s, key in enumerate(keys):
        a = act[s]
        rho = a[0]
        u, v, w = a[1] / rho, a[2] / rho, a[3] / rho
        p = (spec.gamma - 1) * (a[4] - 0.5 * rho * (u * u + v * v + w * w))
        c = np.sqrt(spec.gamma * np.maximum(p, spec.p_floor) / rho)
        vmax = np.maximum(np.maximum(np.abs(u), np.abs(v)), np.abs(w))
        best = min(best, float(np.min(spec.dx(int(key[0])) / (vmax + c))))
    return spec.cfl * best


def test_cfl_on_an_amr_mesh_is_the_brute_force_minimum():
    """A random smooth 3-D state on a three-level mesh: the oracle's dt
    equals the minimum over every active cell of its own level's dx over
    its largest velocity component plus sound speed, to rounding; the
    planted sum of components misses it."""
    spec = I.MeshSpec(root=(4, 4, 4), block_cells=8, max_level=2, gamma=5.0 / 3.0, cfl=0.3,
                      refine=[(0, 0, 0, 0), (1, 0, 0, 0)])
    m = O.OracleMesh(**spec.kwargs())
    act = I.smooth_state(spec, m.keys, seed=13, amp=0.3, vel=0.9)
    m.set_active(act)
    assert len(set(m.keys[:, 0])) == 3
    want = brute_force_cfl(spec, m.keys, act)
    assert abs(m.cfl_dt() - want) <= 1e-14 * want
    got = planted(O.DEBUG_CFL_SUM, m.cfl_dt)
    assert abs(got - want) > 1e-3 * want
