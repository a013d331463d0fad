"""Pins of the oracle's frozen-branch forward (the adjoint's reading: the
dt sequence and every discrete choice of the scheme held at the base run's).

The replayed function is the scheme restricted to one smooth branch, so:
* its unperturbed run is the plain run (same loss);
* where no choice changes under the perturbation its central differences
  are the plain oracle's central differences, bit for bit;
* its central differences converge at second order in eps even at a size of
  eps that flips limiter, parabola or Riemann choices in the plain scheme
  (there the plain differences jump by O(1) relative amounts).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I

SPEC = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=1, gamma=5.0 / 3.0, refine=[(0, 0, 0, 0)])


@pytest.fixture(scope="module")
def tiny():
    m = O.OracleMesh(**SPEC.kwargs())
    act = I.grf_state(SPEC, m.keys, seed=4)
    tgt = I.grf_density(SPEC, m.keys, seed=40)
    m.set_active(act)
    p = O.OracleMesh(**SPEC.kwargs())
    p.set_active(act)
    dts = [p.step(0), p.step(1)]
    return m, act, tgt, dts


def plain_loss(act, tgt, dts):
    o = O.OracleMesh(**SPEC.kwargs())
    o.set_active(act)
    for k, dt in enumerate(dts):
        o.step_dt(k, dt)
    a = o.active()[:, 0]
    w = 8.0 ** (-o.keys[:, 0].astype(float))
    return float(np.sum(w * np.sum((a - tgt.reshape(a.shape)) ** 2, axis=(1, 2, 3))))


def perturbed(act, i, d):
    N = SPEC.block_cells
    s, r = divmod(int(i), N ** 3)
    out = act.copy()
    out[s, 0, r // (N * N), (r // N) % N, r % N] += d
    return out


def test_unperturbed_replay_is_the_plain_run(tiny):
    m, act, tgt, dts = tiny
    _, L = m.frozen_fd_density_grad(0, dts, tgt, 1e-6, idx=np.array([0]))
    assert abs(L - plain_loss(act, tgt, dts)) <= 1e-14 * L
    # the mesh's own state is left as it was
    assert np.array_equal(m.active(), act)


def test_small_eps_differences_equal_the_plain_ones(tiny):
    """Equal up to the last bit of the two losses' sums (the oracle sums
    leaf by leaf, this test with numpy): |difference| <= 4 ulp(L) / eps."""
    m, act, tgt, dts = tiny
    idx = np.arange(3, SPEC.block_cells ** 3 * m.nleaf, 613)
    g, L = m.frozen_fd_density_grad(0, dts, tgt, 1e-7, idx=idx)
    for q, i in enumerate(idx):
        fd = (plain_loss(perturbed(act, i, 1e-7), tgt, dts) - plain_loss(perturbed(act, i, -1e-7), tgt, dts)) / 2e-7
        assert abs(fd - g[q]) <= 4 * np.spacing(L) / 1e-7, (i, fd, g[q])


def shocked(m):
    """A shock tube along x (rho 1 | 0.125 with 5% y ripple, p 1 | 0.1, a
    z-varying u) on the two-level mesh: limiters, parabola cases,
    flattening and the Riemann sampling all switch near x = 1/2."""
    x, y, z = I.cell_centres(SPEC, m.keys)
    rho = np.where(x < 0.5, 1.0, 0.125) * (1 + 0.05 * np.sin(2 * np.pi * y))
    return I.conserved(SPEC.gamma, rho, 0.1 * np.sin(2 * np.pi * z), 0.0, 0.0, np.where(x < 0.5, 1.0, 0.1))


def test_frozen_differences_converge_at_second_order_where_plain_ones_jump():
    """Near the shock, eps = 1e-2, 5e-3, 2.5e-3: the frozen differences
    change by factors of 4 (smooth: error ~ eps^2), while the plain scheme's
    differences change choices between these eps and do not."""
    m = O.OracleMesh(**SPEC.kwargs())
    act = shocked(m)
    m.set_active(act)
    p = O.OracleMesh(**SPEC.kwargs())
    p.set_active(act)
    dts = [p.step(0), p.step(1)]
    tgt = np.full((m.nleaf,) + (SPEC.block_cells,) * 3, 0.5)
    N = SPEC.block_cells
    idx = []
    for s, k in enumerate(m.keys):
        for c in range(0, N, 3):
            for b in range(0, N, 3):
                for a in range(N):
                    if abs((k[1] * N + a + 0.5) * SPEC.dx(int(k[0])) - 0.5) < 3 * SPEC.dx(int(k[0])):
                        idx.append(s * N ** 3 + (c * N + b) * N + a)
    idx = np.array(idx)
    eps = [1e-2, 5e-3, 2.5e-3]
    g = [m.frozen_fd_density_grad(0, dts, tgt, e, idx=idx)[0] for e in eps]
    d1, d2 = np.abs(g[0] - g[1]), np.abs(g[1] - g[2])
    scale = np.max(np.abs(g[2]))
    assert np.all(d1 > 1e-8 * scale)
    ratio = d1 / d2
    assert np.all((ratio > 3.5) & (ratio < 4.5)), (ratio.min(), ratio.max())

    def loss(a):
        o = O.OracleMesh(**SPEC.kwargs())
        o.set_active(a)
        for k, dt in enumerate(dts):
            o.step_dt(k, dt)
        w = 8.0 ** (-o.keys[:, 0].astype(float))
        return float(np.sum(w * np.sum((o.active()[:, 0] - tgt) ** 2, axis=(1, 2, 3))))

    irregular = 0
    for q in range(0, len(idx), 7):
        fd = [(loss(perturbed(act, idx[q], e)) - loss(perturbed(act, idx[q], -e))) / (2 * e) for e in eps]
        r = abs(fd[0] - fd[1]) / max(abs(fd[1] - fd[2]), 1e-300)
        irregular += not (3.5 < r < 4.5)
    assert irregular >= 5
