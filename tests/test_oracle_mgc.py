"""Pins of the oracle's mg0 on the octree (composite-grid Poisson operator on
the leaves of a refined periodic mesh and its multigrid V-cycle).

* an unrefined mesh is the uniform mg0 solver, bit for bit (pinned in
  test_oracle_mg.py against the textbook properties);
* constants are in the operator's null space exactly;
* the volume-weighted sum of L phi over a periodic refined mesh vanishes
  (fluxes through a coarse-fine face agree on both sides): a planted coarse
  side that keeps its own two-point flux breaks it;
* a manufactured periodic solution is reached at second order in the cell
  size across a coarse-fine interface: a planted constant (slope-free)
  interpolation at the interface drops it to first order;
* V(2,2) cycles contract the residual by about 0.09 per cycle on a
  three-level mesh, as on a uniform grid, and the solve satisfies
  L phi = f - mean(f) to its residual;
* self-gravity on a refined mesh: on an unrefined mesh it is the uniform
  self-gravity step bit for bit; a growing and an oscillating Jeans mode
  through a refined region follow linear theory within 1%, converging with
  resolution; the planted g = +grad(phi) fails that.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I


def weights(om):
    return 8.0 ** (-om.keys[:, 0].astype(float))


def planted(flags, fn, *a, **kw):
    O.mgc_set_debug(flags)
    try:
        return fn(*a, **kw)
    finally:
        O.mgc_set_debug(0)


THREE_LEVELS = I.MeshSpec(root=(4, 4, 4), block_cells=8, max_level=2, refine=[(0, 1, 1, 1), (1, 2, 2, 2)])


def test_unrefined_mesh_is_the_uniform_solver_bitwise():
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8)
    om = O.OracleMesh(**spec.kwargs())
    f = np.random.default_rng(1).standard_normal((om.nleaf, 8, 8, 8))
    phi, res = O.mgc_solve(om, f, 3)
    g = np.zeros((16, 16, 16))
    for s, k in enumerate(om.keys):
        g[k[3] * 8:(k[3] + 1) * 8, k[2] * 8:(k[2] + 1) * 8, k[1] * 8:(k[1] + 1) * 8] = f[s]
    pu, ru = O.mg_solve(g, spec.dx(0), 3)
    pb = np.stack([pu[k[3] * 8:(k[3] + 1) * 8, k[2] * 8:(k[2] + 1) * 8, k[1] * 8:(k[1] + 1) * 8] for k in om.keys])
    assert np.array_equal(phi, pb) and np.array_equal(res, ru)


def conservation_defect(spec, seed=2):
    om = O.OracleMesh(**spec.kwargs())
    phi = np.random.default_rng(seed).standard_normal((om.nleaf,) + (spec.block_cells,) * 3)
    L = O.mgc_apply(om, phi)
    w = weights(om)[:, None, None, None]
    return abs(np.sum(w * L)) / np.sum(w * np.abs(L)), om


def test_constants_are_in_the_null_space_and_fluxes_match():
    om = O.OracleMesh(**THREE_LEVELS.kwargs())
    assert set(om.keys[:, 0]) == {0, 1, 2}
    assert np.all(O.mgc_apply(om, np.full((om.nleaf, 8, 8, 8), 0.7)) == 0.0)
    d, _ = conservation_defect(THREE_LEVELS)
    assert d <= 1e-15
    d_bad, _ = planted(O.MGC_DEBUG_NO_MATCH, conservation_defect, THREE_LEVELS)
    assert d_bad > 1e-6


def manufactured_error(N):
    """Max error of the solve against a smooth periodic solution on a
    two-level mesh (levels 1 and 2 after balancing the 2^3 roots)."""
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=N, max_level=2, refine=[(0, 0, 0, 0), (1, 1, 1, 1)])
    om = O.OracleMesh(**spec.kwargs())
    assert set(om.keys[:, 0]) == {1, 2}
    x, y, z = I.cell_centres(spec, om.keys)
    k = 2 * np.pi
    exact = np.sin(k * x) * np.cos(k * y) * np.sin(2 * k * z) + 0.5 * np.cos(k * x + 0.3)
    f = -6 * k * k * np.sin(k * x) * np.cos(k * y) * np.sin(2 * k * z) - 0.5 * k * k * np.cos(k * x + 0.3)
    phi, _ = O.mgc_solve(om, f, 12)
    w = weights(om)[:, None, None, None]
    exact = exact - np.sum(w * exact) / np.sum(w * np.ones_like(exact))
    return float(np.max(np.abs(phi - exact)))


def test_manufactured_solution_converges_at_second_order():
    e8, e16 = manufactured_error(8), manufactured_error(16)
    assert e8 < 2e-2
    assert e8 / e16 > 3.5
    f8, f16 = (planted(O.MGC_DEBUG_FLAT, manufactured_error, n) for n in (8, 16))
    assert f8 / f16 < 2.5


def test_v_cycles_contract_like_uniform_multigrid():
    om = O.OracleMesh(**THREE_LEVELS.kwargs())
    f = np.random.default_rng(3).standard_normal((om.nleaf, 8, 8, 8))
    phi, res = O.mgc_solve(om, f, 8)
    rates = res[1:] / res[:-1]
    assert np.all(rates[:8] < 0.12), rates
    # the solve answers the operator it applies
    L = O.mgc_apply(om, phi)
    w = weights(om)[:, None, None, None]
    fm = f - np.sum(w * f) / np.sum(w * np.ones_like(f))
    assert np.sqrt(np.sum(w * (fm - L) ** 2)) <= 1.0000001 * res[-1]
    assert np.sum(w * phi) == pytest.approx(0.0, abs=1e-12 * np.sum(w * np.abs(phi)))


# ---------------------------------------------------------------------------
# Self-gravity on a refined mesh
# ---------------------------------------------------------------------------

GAMMA = 5.0 / 3.0


def test_gravity_step_on_an_unrefined_mesh_is_the_uniform_step_bitwise():
    spec = I.MeshSpec(root=(2, 2, 1), block_cells=8, gamma=GAMMA)
    a, b = O.OracleMesh(**spec.kwargs()), O.OracleMesh(**spec.kwargs())
    U = I.smooth_state(spec, a.keys, seed=5, amp=0.1, vel=0.2)
    a.set_active(U)
    b.set_active(U)
    pa = np.zeros((a.nleaf, 8, 8, 8))
    pg = np.zeros((8, 16, 16))
    for k in range(3):
        assert a.step_gravity_amr(k, 3.0, pa, k > 0) == b.step_gravity(k, 3.0, pg, k > 0)
        assert np.array_equal(a.active(), b.active())
    blocks = np.stack([pg[kk * 8:(kk + 1) * 8, j * 8:(j + 1) * 8, i * 8:(i + 1) * 8] for _, i, j, kk in a.keys])
    assert np.array_equal(pa, blocks)


def jeans_amr(level0_cells, ratio, T, eps=1e-4):
    """Jeans mode cos(2 pi x) on a periodic row of roots with the roots in
    the middle third refined once: density amplitude (volume-weighted
    projection, relative to eps) at time t >= T and linear theory there."""
    N = 8
    R = level0_cells // N
    refine = [(0, i, 0, 0) for i in range(R // 3, 2 * R // 3)]
    spec = I.MeshSpec(root=(R, 1, 1), block_cells=N, max_level=1, gamma=GAMMA, refine=refine)
    m = O.OracleMesh(**spec.kwargs())
    assert set(m.keys[:, 0]) == {0, 1}
    x = I.cell_centres(spec, m.keys)[0]
    k = 2.0 * np.pi
    fpg = ratio * GAMMA * k * k
    m.set_active(I.conserved(GAMMA, 1.0 + eps * np.cos(k * x), 0.0, 0.0, 0.0, 1.0 + GAMMA * eps * np.cos(k * x)))
    phi = np.zeros((m.nleaf, N, N, N))
    t, s = 0.0, 0
    while t < T:
        t += m.step_gravity_amr(s, fpg, phi, s > 0, ncycles=4)
        s += 1
    w = (8.0 ** (-m.keys[:, 0].astype(float)))[:, None, None, None]
    amp = 2.0 * np.sum(w * (m.active()[:, 0] - 1.0) * np.cos(k * x)) / np.sum(w * np.ones_like(x)) / eps
    w2 = GAMMA * k * k * (1.0 - ratio)
    return amp, (np.cosh(np.sqrt(-w2) * t) if w2 < 0 else np.cos(np.sqrt(w2) * t))


@pytest.mark.parametrize("ratio,T", [(2.0, 0.2), (0.5, 0.3)])
def test_jeans_mode_across_a_refined_region_matches_linear_theory(ratio, T):
    """The growing and the oscillating Jeans mode run through coarse-fine
    interfaces: within 1% of linear theory at 48 level-0 cells per
    wavelength (96 in the refined third), the error falling at about second
    order from 24; the planted g = +grad(phi) fails it."""
    a1, x1 = jeans_amr(24, ratio, T)
    a2, x2 = jeans_amr(48, ratio, T)
    e1, e2 = abs(a1 - x1) / abs(x1), abs(a2 - x2) / abs(x2)
    assert e2 < 0.01 and e1 / e2 > 2.5, (e1, e2)
    O.set_debug(O.DEBUG_GRAVITY_SIGN)
    try:
        a3, x3 = jeans_amr(48, ratio, T)
    finally:
        O.set_debug(0)
    assert abs(a3 - x3) / abs(x3) > 0.05
