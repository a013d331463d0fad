"""Pins of the oracle's tracer particles (positions in level-0 cell units):
point location against brute-force box containment, exact translation in a
uniform flow, exact trilinear interpolation of a linear velocity field across
refinement jumps, periodic wrap, removal through outflow faces, and the
ownership invariant over full steps."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I


def amr_spec(N=8, seed=3, root=(2, 2, 2), bc="periodic"):
    return I.MeshSpec(root=root, block_cells=N, max_level=2, gamma=1.4, bc=bc,
                      refine=I.random_refine_list(root, 2, 4, seed) if bc == "periodic" else [])


def boxes(spec, keys):
    """[leaf, axis, lo/hi] in level-0 cell units."""
    keys = np.asarray(keys, dtype=np.float64)
    N = spec.block_cells
    w = N / np.power(2.0, keys[:, 0])
    lo = keys[:, 1:4] * w[:, None]
    return lo, lo + w[:, None]


def brute_owner(spec, keys, P):
    lo, hi = boxes(spec, keys)
    inside = np.all((P[:, None, :] >= lo[None]) & (P[:, None, :] < hi[None]), axis=2)
    assert np.all(inside.sum(axis=1) == 1), "leaves must tile the domain"
    return inside.argmax(axis=1)


def state_from(spec, keys, rho, m):
    """Conserved cells from callables of the level-0 cell-unit centre X[n, 3]."""
    keys = np.asarray(keys)
    N = spec.block_cells
    act = np.empty((len(keys), 5, N, N, N))
    c = (np.arange(N) + 0.5)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    for s, (l, i, j, k) in enumerate(keys):
        X = np.stack([x + i * N, y + j * N, z + k * N], axis=-1) / float(1 << int(l))
        r = rho(X)
        mv = m(X)
        act[s, 0] = r
        act[s, 1:4] = mv
        act[s, 4] = 1.0 / 0.4 + 0.5 * (mv ** 2).sum(axis=0) / r
    return act


def test_locate_matches_box_containment():
    spec = amr_spec(8, 5)
    om = O.OracleMesh(**spec.kwargs())
    rng = np.random.default_rng(1)
    E = np.array(spec.root, dtype=float) * spec.block_cells
    P = rng.uniform(0, 1, size=(400, 3)) * E
    # points exactly on block faces of every level, and on the domain's low faces
    on = np.array([[4.0, 8.0, 2.0], [0.0, 0.0, 0.0], [8.0, 4.0, 12.0], [2.0, 6.0, 4.0]])
    P = np.concatenate([P, on])
    assert np.array_equal(om.locate(P), brute_owner(spec, om.keys, P))
    assert np.all(om.locate(np.array([[-1e-9, 1.0, 1.0], [E[0], 1.0, 1.0]])) == -1)


def test_uniform_flow_translates_every_particle():
    spec = amr_spec(8, 6)
    om = O.OracleMesh(**spec.kwargs())
    vel = np.array([0.3, -0.2, 0.45])
    om.set_active(state_from(spec, om.keys, lambda X: np.ones(X.shape[:-1]),
                             lambda X: np.broadcast_to(vel[:, None, None, None], (3,) + X.shape[:-1]).copy()))
    om.refresh()
    pos, ids = I.tracer_positions(spec, om.keys, 1, jitter_seed=2)
    tr = O.Tracers(*pos.reshape(-1, 3).T, ids.ravel())
    dt = 0.01
    n0 = spec.root[0] * spec.block_cells
    assert om.tracers_drift(dt, tr) == 0
    E = np.array(spec.root, dtype=float) * spec.block_cells
    want = np.mod(pos.reshape(-1, 3) + dt * vel * n0, E)
    got = tr.positions()
    d = np.abs(got - want)
    d = np.minimum(d, E - d)  # across the periodic seam
    assert d.max() <= 1e-12, d.max()


def test_linear_velocity_is_interpolated_exactly_across_refinement():
    """u = a + B X (each component depends on a different axis): cell-centred
    values of a linear field, their restriction and their (equal-slope)
    prolongation are exact, and trilinear interpolation of a linear field is
    exact, so every particle away from the periodic seam moves by exactly
    dt u(X) n0 (to rounding).  A half-cell slip of the interpolation stencil
    or a swapped axis moves it by B/2 or more."""
    spec = amr_spec(8, 7)
    om = O.OracleMesh(**spec.kwargs())
    n0 = spec.root[0] * spec.block_cells
    a = np.array([0.1, -0.05, 0.2])
    B = np.array([[0.0, 0.02, 0.0], [0.0, 0.0, -0.03], [0.025, 0.0, 0.0]])  # u_d = a_d + B[d] . X

    def mom(X):
        return np.moveaxis(a + X @ B.T, -1, 0)

    om.set_active(state_from(spec, om.keys, lambda X: np.ones(X.shape[:-1]), mom))
    om.refresh()
    rng = np.random.default_rng(3)
    E = np.array(spec.root, dtype=float) * spec.block_cells
    P = rng.uniform(3.0, E - 3.0, size=(600, 3))
    tr = O.Tracers(*P.T, np.arange(len(P)))
    dt = 0.02
    om.tracers_drift(dt, tr)
    want = P + dt * (a + P @ B.T) * n0
    err = np.abs(tr.positions() - want).max()
    assert err <= 1e-12, err


def test_periodic_wrap_conserves_particles():
    spec = I.MeshSpec(root=(2, 1, 1), block_cells=8, gamma=1.4)
    om = O.OracleMesh(**spec.kwargs())
    vel = np.array([-0.5, 0.4, 0.3])
    om.set_active(state_from(spec, om.keys, lambda X: np.ones(X.shape[:-1]),
                             lambda X: np.broadcast_to(vel[:, None, None, None], (3,) + X.shape[:-1]).copy()))
    om.refresh()
    E = np.array([16.0, 8.0, 8.0])
    P = np.array([[0.01, 7.99, 7.995], [15.99, 0.0, 0.5], [3.0, 4.0, 5.0]])
    tr = O.Tracers(*P.T, np.arange(3))
    dt = 0.05
    assert om.tracers_drift(dt, tr) == 0
    got = tr.positions()
    assert np.all((got >= 0) & (got < E))
    want = np.mod(P + dt * vel * 16.0, E)
    assert np.abs(got - want).max() <= 1e-12


def test_outflow_faces_remove_exactly_the_leavers():
    spec = I.MeshSpec(root=(2, 1, 1), block_cells=8, gamma=1.4, bc="outflow")
    om = O.OracleMesh(**spec.kwargs())
    vel = np.array([0.6, -0.6, 0.0])
    om.set_active(state_from(spec, om.keys, lambda X: np.ones(X.shape[:-1]),
                             lambda X: np.broadcast_to(vel[:, None, None, None], (3,) + X.shape[:-1]).copy()))
    om.refresh()
    rng = np.random.default_rng(4)
    P = rng.uniform(0, 1, size=(300, 3)) * np.array([16.0, 8.0, 8.0])
    tr = O.Tracers(*P.T, np.arange(len(P)))
    dt = 0.05
    moved = P + dt * vel * 16.0
    leave = np.any((moved < 0) | (moved >= np.array([16.0, 8.0, 8.0])), axis=1)
    assert leave.sum() > 10
    assert om.tracers_drift(dt, tr) == leave.sum()
    assert np.array_equal(tr.alive == 0, leave)


def test_full_steps_keep_particles_inside_their_leaves():
    spec = I.sedov_spec(root=2, block_cells=8, levels=1)
    om = O.OracleMesh(**spec.kwargs())
    om.set_active(I.sedov_state(spec, om.keys))
    pos, ids = I.tracer_positions(spec, om.keys, 1, jitter_seed=5)
    tr = O.Tracers(*pos.reshape(-1, 3).T, ids.ravel())
    P0 = tr.positions().copy()
    for k in range(6):
        om.step_tracers(k, tr)
    assert tr.alive.all()
    P = tr.positions()
    own = om.locate(P)
    assert np.array_equal(own, brute_owner(spec, om.keys, P))
    assert np.abs(P - P0).max() > 1e-3  # the blast moved them


def test_linear_velocity_with_varying_density_on_a_uniform_mesh():
    """The interpolated quantity is the cell velocity m / rho: with rho varying
    and m = rho u for a linear u, particles still move by exactly dt u(X) n0
    (no refinement jump here: restriction and prolongation act on rho and m
    separately, which would not keep m / rho linear)."""
    spec = I.MeshSpec(root=(2, 2, 1), block_cells=8, gamma=1.4)
    om = O.OracleMesh(**spec.kwargs())
    n0 = spec.root[0] * spec.block_cells
    a = np.array([0.05, 0.1, -0.02])
    B = np.array([[0.0, 0.0, 0.03], [0.015, 0.0, 0.0], [0.0, -0.02, 0.0]])

    def rho(X):
        return 1.0 + 0.3 * np.sin(0.7 * X[..., 0] + 0.4 * X[..., 1]) * np.cos(0.5 * X[..., 2])

    om.set_active(state_from(spec, om.keys, rho, lambda X: rho(X)[None] * np.moveaxis(a + X @ B.T, -1, 0)))
    om.refresh()
    rng = np.random.default_rng(6)
    E = np.array(spec.root, dtype=float) * spec.block_cells
    P = rng.uniform(2.0, E - 2.0, size=(500, 3))
    tr = O.Tracers(*P.T, np.arange(len(P)))
    dt = 0.02
    om.tracers_drift(dt, tr)
    want = P + dt * (a + P @ B.T) * n0
    err = np.abs(tr.positions() - want).max()
    assert err <= 1e-12, err
