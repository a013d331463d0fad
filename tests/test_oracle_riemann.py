"""Pins of the oracle's two-shock Riemann solver and PPM pencil.

The two-shock solver is exact when both waves are shocks, converges to the
two-shock root, and agrees with the exact solver to third order in the jump
for weak waves.  The pencil preserves constant states and is mirror
symmetric.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import physics_ref as P
from oracle import oracle as O

G14 = 1.4


def euler_flux(W, gamma):
    r, u, v, w, p = W
    E = p / (gamma - 1) + 0.5 * r * (u * u + v * v + w * w)
    return np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)])


def test_identical_states_give_the_flux_of_that_state():
    rng = np.random.default_rng(1)
    for _ in range(50):
        W = np.array([rng.uniform(0.1, 3), rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(-1, 1),
                      rng.uniform(0.1, 3)])
        st, fl, ps, us = O.riemann(W, W, gamma=G14)
        np.testing.assert_allclose(st, W, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(fl, euler_flux(W, G14), rtol=1e-12, atol=1e-13)
        assert ps == pytest.approx(W[4], rel=1e-13)


def test_symmetric_collision_has_zero_contact_speed_and_exact_pressure():
    for u0 in (0.1, 1.0, 3.0):
        WL = np.array([1.0, u0, 0.0, 0.0, 1.0])
        WR = np.array([1.0, -u0, 0.0, 0.0, 1.0])
        st, fl, ps, us = O.riemann(WL, WR, gamma=G14)
        assert us == 0.0
        assert fl[0] == 0.0
        # two shocks: the two-shock approximation is the exact solution
        pe, ue = P.exact_star((1.0, u0, 1.0), (1.0, -u0, 1.0), G14)
        assert ps == pytest.approx(pe, rel=1e-10)


def test_double_shock_states_match_exact_solution():
    rng = np.random.default_rng(2)
    for _ in range(40):
        rL, rR = rng.uniform(0.2, 2, 2)
        pL, pR = rng.uniform(0.2, 2, 2)
        uL, uR = rng.uniform(1.0, 3.0), rng.uniform(-3.0, -1.0)
        pe, ue = P.exact_star((rL, uL, pL), (rR, uR, pR), G14)
        if pe <= max(pL, pR):
            continue
        st, fl, ps, us = O.riemann([rL, uL, 0.3, -0.2, pL], [rR, uR, 0.1, 0.4, pR], gamma=G14)
        assert ps == pytest.approx(pe, rel=1e-9)
        assert us == pytest.approx(ue, rel=1e-9, abs=1e-9)
        ex = P.exact_sample((rL, uL, pL), (rR, uR, pR), G14, 0.0)
        np.testing.assert_allclose(st[[0, 1, 4]], ex, rtol=1e-8, atol=1e-9)


def _two_shock_root(WL, WR, g):
    """The two-shock p*: root of u*_R(p) - u*_L(p), each side's velocity
    behind a shock of pressure p (Rankine-Hugoniot mass flux), by bracketing."""
    def W(p, r, pk):
        C = math.sqrt(g * pk * r)
        return C * math.sqrt(1 + (g + 1) / (2 * g) * (p / pk - 1))

    def h(p):
        (rL, uL, pL), (rR, uR, pR) = WL, WR
        return (uR + (p - pR) / W(p, rR, pR)) - (uL - (p - pL) / W(p, rL, pL))

    return brentq(h, 1e-8, 100.0, xtol=1e-15, rtol=1e-15)


@pytest.mark.parametrize("WL,WR", [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
                                   ((1.0, 0.5, 2.0), (0.5, -0.2, 0.7)),
                                   ((2.0, -0.3, 0.4), (1.0, 0.4, 1.2))])
def test_five_newton_steps_reach_the_two_shock_root(WL, WR):
    root = _two_shock_root(WL, WR, G14)
    _, _, ps, _ = O.riemann([WL[0], WL[1], 0, 0, WL[2]], [WR[0], WR[1], 0, 0, WR[2]], gamma=G14)
    assert ps == pytest.approx(root, rel=1e-10)


def test_weak_waves_agree_with_exact_to_third_order():
    errs = []
    for eps in (1e-1, 5e-2, 2.5e-2):
        WL, WR = (1.0, 0.0, 1.0 + eps), (1.0, 0.0, 1.0)  # rarefaction + shock
        pe, _ = P.exact_star(WL, WR, G14)
        _, _, ps, _ = O.riemann([1.0, 0, 0, 0, 1 + eps], [1.0, 0, 0, 0, 1.0], gamma=G14)
        errs.append(abs(ps - pe))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 6.0 and r2 > 6.0, errs


def test_supersonic_and_fan_sampling():
    # supersonic to the right: interface sees the left state unchanged
    WL = np.array([1.0, 5.0, 0.2, 0.1, 1.0])
    WR = np.array([0.9, 5.1, -0.1, 0.3, 0.9])
    st, fl, _, _ = O.riemann(WL, WR, gamma=G14)
    np.testing.assert_array_equal(st, WL)
    # transonic rarefaction: the sampled state lies strictly between the
    # left state and the two-shock star state (linear fan)
    WL = np.array([1.0, 0.0, 0.0, 0.0, 1.0])
    WR = np.array([0.01, 0.0, 0.0, 0.0, 0.01])
    st, fl, ps, us = O.riemann(WL, WR, gamma=G14)
    assert 0.0 < st[1] < us
    assert ps < st[4] < 1.0
    # a weak transonic fan is close to the exact solution
    WL = np.array([1.0, 0.8, 0.0, 0.0, 1.0])
    WR = np.array([0.8, 1.0, 0.0, 0.0, 0.7])
    st, fl, ps, us = O.riemann(WL, WR, gamma=G14)
    ex = P.exact_sample((1, 0.8, 1), (0.8, 1.0, 0.7), G14, 0.0)
    np.testing.assert_allclose(st[[0, 1, 4]], ex, rtol=2e-2)


def test_riemann_mirror_symmetry_is_bitwise():
    rng = np.random.default_rng(3)
    for _ in range(200):
        WL = np.array([rng.uniform(0.1, 2), rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(-1, 1),
                       rng.uniform(0.05, 2)])
        WR = np.array([rng.uniform(0.1, 2), rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(-1, 1),
                       rng.uniform(0.05, 2)])
        st, fl, ps, us = O.riemann(WL, WR, gamma=G14)
        mL = WR * np.array([1, -1, 1, 1, 1])
        mR = WL * np.array([1, -1, 1, 1, 1])
        st2, fl2, ps2, us2 = O.riemann(mL, mR, gamma=G14)
        assert ps2 == ps and us2 == -us
        if us != 0.0:
            assert fl2[0] == -fl[0] and fl2[1] == fl[1] and fl2[4] == -fl[4]


def _pencil_state(n, rng):
    x = np.arange(n)
    rho = 1 + 0.3 * np.sin(0.7 * x + rng.uniform(0, 6)) + 0.2 * (x > n // 2)
    u = 0.4 * np.cos(0.5 * x + rng.uniform(0, 6))
    v = 0.2 * np.sin(0.3 * x)
    w = -0.1 * np.cos(0.9 * x)
    p = 1 + 0.5 * (x < n // 3) + 0.1 * np.sin(x)
    E = p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)
    return np.array([rho, rho * u, rho * v, rho * w, E])


def test_pencil_preserves_constant_state_bitwise():
    n = 22
    U = np.empty((5, n))
    U[:] = np.array([1.3, 1.3 * 0.7, 1.3 * -0.2, 1.3 * 0.4, 2.9])[:, None]
    F = O.pencil_flux(U, nu=0.3)
    assert np.all(F == F[:, :1])


def test_pencil_mirror_symmetry_is_bitwise():
    rng = np.random.default_rng(4)
    for _ in range(20):
        U = _pencil_state(22, rng)
        F = O.pencil_flux(U, nu=0.35)
        Um = U[:, ::-1] * np.array([1, -1, 1, 1, 1])[:, None]
        Fm = O.pencil_flux(np.ascontiguousarray(Um), nu=0.35)
        # interface j+1/2 maps to interface (n-2-j)+1/2; odd fields flip sign
        Fback = Fm[:, ::-1] * np.array([-1, 1, -1, -1, -1])[:, None]
        np.testing.assert_array_equal(F, Fback)


def _entropy_pencil(n, a, b, c, u, gamma=1.4):
    """Cell averages of rho(x) = a + b x + c x^2 (cell j spans [j-1/2, j+1/2]),
    uniform u and p = 1."""
    j = np.arange(n, dtype=np.float64)
    rho = a + b * j + c * (j * j + 1.0 / 12.0)
    E = 1.0 / (gamma - 1.0) + 0.5 * rho * u * u
    return np.array([rho, rho * u, 0 * rho, 0 * rho, E])


def _quad_mean(a, b, c, x0, x1):
    F = lambda x: a * x + b * x * x / 2 + c * x ** 3 / 3
    return (F(x1) - F(x0)) / (x1 - x0)


@pytest.mark.parametrize("u", [0.7, -0.6])
def test_parabolic_reconstruction_and_tracing_are_exact_on_quadratics(u):
    """PPM reproduces a quadratic exactly (4th-order interface values, the
    parabola of each cell is the quadratic itself), and the traced state of
    the contact is the mean of the quadratic over the upwind domain of
    dependence, so the mass flux is u times that mean."""
    n, nu = 22, 0.4
    a, b, c = 1.0, 0.05, 0.004
    U = _entropy_pencil(n, a, b, c, u)
    F = O.pencil_flux(U, nu=nu)
    sig = abs(u) * nu
    for k in range(n - 5):
        x0 = 2 + k + 0.5
        mean = _quad_mean(a, b, c, x0 - sig, x0) if u > 0 else _quad_mean(a, b, c, x0, x0 + sig)
        assert F[0, k] == pytest.approx(u * mean, rel=1e-12)


def test_full_flattening_at_a_compressive_jump_gives_godunov_flux():
    """A jump spread over one intermediate cell J gives pressure ratio r = 1
    there, so with converging flow the flattening coefficient of cell J is 1:
    its parabola becomes the constant cell value (its neighbours are flat by
    the monotonicity constraint) and the flux at J+1/2 is the Riemann flux of
    the cell states.  Diverging flow across the same jump is not flattened
    and the traced parabola gives a different flux."""
    n, J = 22, 10
    x = np.arange(n)
    gm1 = 0.4
    for conv, expect_godunov in ((+1, True), (-1, False)):
        rho = np.where(x < J, 1.0, np.where(x == J, 0.8, 0.5))
        u = conv * np.where(x < J, 0.3, np.where(x == J, 0.0, -0.3))
        p = np.where(x < J, 2.0, np.where(x == J, 1.2, 0.5))
        E = p / gm1 + 0.5 * rho * u * u
        U = np.array([rho, rho * u, 0 * rho, 0 * rho, E])
        F = O.pencil_flux(U, nu=0.3)

        def prim(j):
            uu = U[1, j] * (1.0 / U[0, j])
            return np.array([U[0, j], uu, 0, 0, gm1 * (U[4, j] - (0.5 * U[0, j]) * (uu * uu))])

        _, Fg, _, _ = O.riemann(prim(J), prim(J + 1), gamma=1.4)
        k = J - 2
        if expect_godunov:
            np.testing.assert_allclose(F[:, k], Fg, rtol=1e-12, atol=1e-13)
        else:
            assert np.max(np.abs(F[:, k] - Fg)) > 1e-3
