"""Pins of the oracle's mg0 Poisson solver (geometric multigrid V-cycle on a
uniform periodic grid; the paper's self-gravity solver, Sec. II-C and III).

What fixes the results:
  * a discrete eigenmode of the 7-point Laplacian (products of sines and
    cosines, whose eigenvalue is a closed form) is solved to round-off;
  * on a tiny grid the result equals the dense least-squares solve of the
    periodic Laplacian (mean-free);
  * the converged solution does not depend on the cycle parameters, and is
    mirror-symmetric for a mirror-symmetric right-hand side;
  * V(2,2) cycles reduce a random residual by a factor below 0.12 each,
    V(1,1) below 0.25 (textbook multigrid rates for this smoother);
  * the prolongation and the residual restriction are second-order accurate
    on smooth periodic fields (error ratio near 4 per halving);
  * each planted mistake (piecewise-constant prolongation, a summing
    restriction, the smoother's sign) fails one of these pins.
"""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(autouse=True)
def _no_planted_mistake():
    O.mg_set_debug(0)
    yield
    O.mg_set_debug(0)


def centres(shape, h):
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h, (np.arange(nx) + 0.5) * h,
                          indexing="ij")
    return x, y, z


@pytest.mark.parametrize("shape,modes", [((32, 32, 32), (1, 2, 1)), ((16, 32, 64), (3, 1, 2))])
def test_discrete_eigenmode_is_solved_to_round_off(shape, modes):
    nz, ny, nx = shape
    h = 1.0 / nx
    x, y, z = centres(shape, h)
    L = (nx * h, ny * h, nz * h)
    k = [2.0 * np.pi * m / l for m, l in zip(modes, L)]
    s = np.sin(k[0] * x) * np.sin(k[1] * y) * np.cos(k[2] * z)
    lam = -(4.0 / h ** 2) * sum(np.sin(0.5 * kk * h) ** 2 for kk in k)
    phi, res = O.mg_solve(lam * s, h, 25)
    assert np.max(np.abs(phi - s)) < 1e-11
    assert res[-1] < 1e-11 * res[0]


def periodic_laplacian(shape, h):
    nz, ny, nx = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    idx = np.arange(n).reshape(shape)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = idx[k, j, i]
                A[c, c] = -6.0
                for dk, dj, di in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
                    A[c, idx[(k + dk) % nz, (j + dj) % ny, (i + di) % nx]] += 1.0
    return A / h ** 2


def test_tiny_grid_equals_the_dense_solve():
    shape, h = (4, 8, 8), 0.125
    assert O.mg_levels(shape) == 2
    f = np.random.default_rng(3).standard_normal(shape)
    f0 = f - f.mean()
    sol = np.linalg.lstsq(periodic_laplacian(shape, h), f0.ravel(), rcond=None)[0]
    sol = (sol - sol.mean()).reshape(shape)
    phi, _ = O.mg_solve(f, h, 30)
    assert np.max(np.abs(phi - sol)) < 1e-12 * np.max(np.abs(sol))


def test_converged_solution_is_independent_of_cycle_parameters_and_symmetric():
    shape, h = (16, 32, 32), 1.0 / 32
    rng = np.random.default_rng(5)
    f = rng.standard_normal(shape)
    f = f + f[:, :, ::-1]  # mirror-symmetric in x (cells i and nx-1-i)
    a, _ = O.mg_solve(f, h, 30, 1, 1)
    b, _ = O.mg_solve(f, h, 20, 2, 2)
    c, _ = O.mg_solve(f, h, 25, 3, 1)
    scale = np.max(np.abs(a))
    assert np.max(np.abs(a - b)) < 1e-12 * scale and np.max(np.abs(a - c)) < 1e-12 * scale
    assert np.max(np.abs(b - b[:, :, ::-1])) < 1e-12 * scale


def rate(nu1, nu2, cycles=8):
    f = np.random.default_rng(11).standard_normal((64, 64, 64))
    _, res = O.mg_solve(f, 1.0 / 64, cycles, nu1, nu2)
    fac = res[1:] / res[:-1]
    return float(np.exp(np.mean(np.log(fac[1:])))), res


def test_v_cycle_convergence_rates():
    r22, res = rate(2, 2)
    r11, _ = rate(1, 1)
    assert r22 < 0.12 and r11 < 0.25, (r22, r11)
    assert res[-1] < 1e-7 * res[0]


def _transfer_errors(n):
    """Max errors of the prolongation of a smooth periodic field sampled on an
    n^3 coarse grid, and of the residual restriction of f = g with phi = 0
    from a 2n^3 grid, against the field at the target cell centres."""
    def g(x, y, z):
        return np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.5 * np.sin(4 * np.pi * z)
    hc = 1.0 / n
    xc, yc, zc = centres((n, n, n), hc)
    xf, yf, zf = centres((2 * n, 2 * n, 2 * n), hc / 2)
    ep = np.max(np.abs(O.mg_prolong(g(xc, yc, zc)) - g(xf, yf, zf)))
    er = np.max(np.abs(O.mg_restrict_residual(g(xf, yf, zf), np.zeros((2 * n,) * 3), hc / 2) - g(xc, yc, zc)))
    return ep, er


def test_transfer_operators_are_second_order():
    p1, r1 = _transfer_errors(16)
    p2, r2 = _transfer_errors(32)
    assert 3.5 < p1 / p2 < 4.5 and 3.5 < r1 / r2 < 4.5, (p1 / p2, r1 / r2)


@pytest.mark.parametrize("flag", ["inject", "restrict_sum", "smooth_sign"])
def test_planted_mistakes_fail_a_pin(flag):
    if flag == "inject":
        O.mg_set_debug(O.MG_DEBUG_INJECT)
        with pytest.raises(AssertionError):
            test_transfer_operators_are_second_order()
    else:
        O.mg_set_debug(O.MG_DEBUG_RESTRICT_SUM if flag == "restrict_sum" else O.MG_DEBUG_SMOOTH_SIGN)
        with pytest.raises(AssertionError):
            test_v_cycle_convergence_rates()
