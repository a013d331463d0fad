"""Pins of the oracle's array-of-octrees mesh and its ghost refresh.

Mesh: leaves tile the domain and obey 2:1 balance across faces, edges and
corners (checked geometrically here, by box contact, not by the oracle's own
neighbour walk).  Refresh: constants are reproduced exactly; a linear field
is reproduced in every ghost cell (copies, means of 8 children and the
limited linear prolongation are all exact on linear data); same-level and
outflow ghosts equal the cell found by plain global indexing; prolonged
ghosts conserve the coarse cell's mean.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I

G = 3


def boxes(keys, max_level):
    """Leaf boxes in finest-level block units: lo, hi (exclusive)."""
    s = (1 << (max_level - keys[:, 0]))[:, None]
    lo = keys[:, 1:] * s
    return lo, lo + s


def check_tiling_and_balance(keys, root, max_level, periodic=True):
    lo, hi = boxes(keys, max_level)
    ext = np.array(root) << max_level
    cover = np.zeros(ext[::-1], dtype=np.int32)
    for a, b in zip(lo, hi):
        cover[a[2]:b[2], a[1]:b[1], a[0]:b[0]] += 1
    assert np.all(cover == 1), "leaves must tile the domain exactly once"
    n = len(keys)
    shifts = list(itertools.product(*[(-e, 0, e) for e in ext])) if periodic else [(0, 0, 0)]
    for i in range(n):
        for j in range(i + 1, n):
            if abs(int(keys[i, 0]) - int(keys[j, 0])) <= 1:
                continue
            for sh in shifts:
                l2, h2 = lo[j] + sh, hi[j] + sh
                if np.all(lo[i] <= h2) and np.all(l2 <= hi[i]):
                    raise AssertionError(f"leaves {keys[i]} and {keys[j]} touch across >1 level")


def test_sedov_mesh_leaf_counts():
    spec = I.sedov_spec(root=8, block_cells=32, levels=2)
    m = O.OracleMesh(**spec.kwargs())
    counts = np.bincount(m.keys[:, 0])
    assert list(counts) == [504, 56, 64]
    check_tiling_and_balance(m.keys, spec.root, spec.max_level)


@pytest.mark.parametrize("seed", range(6))
def test_random_refinement_is_balanced_and_tiles(seed):
    root = (3, 2, 2) if seed % 2 else (2, 2, 2)
    refine = I.random_refine_list(root, 3, 6, seed)
    m = O.OracleMesh(root=root, block_cells=8, max_level=3, refine=refine)
    check_tiling_and_balance(m.keys, root, 3)
    # every requested node is refined: none of the requests is a leaf
    leaves = {tuple(k) for k in m.keys}
    for r in refine:
        assert tuple(r) not in leaves


def test_leaf_list_round_trip_and_rejections():
    spec = I.sedov_spec(root=4, block_cells=8, levels=2)
    m = O.OracleMesh(**spec.kwargs())
    m2 = O.OracleMesh(root=spec.root, block_cells=8, max_level=2, leaves=m.keys)
    assert sorted(map(tuple, m.keys)) == sorted(map(tuple, m2.keys))
    with pytest.raises(ValueError):  # a gap
        O.OracleMesh(root=spec.root, block_cells=8, max_level=2, leaves=m.keys[1:])
    # refine one level-2 leaf next to level-1 leaves away from the centre is
    # fine; refining a level-1 leaf adjacent to level-0 leaves to level 2
    # without balance must be rejected
    bad = [k for k in map(tuple, m.keys) if not (k[0] == 0 and k[1:] == (0, 0, 0))]
    bad += [(1, a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1) if (a, b, c) != (0, 0, 0)]
    bad += [(2, a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    with pytest.raises(ValueError):
        O.OracleMesh(root=spec.root, block_cells=8, max_level=2, leaves=bad)


def amr_mesh(N=8):
    spec = I.MeshSpec(root=(4, 4, 4), block_cells=N, max_level=2,
                      refine=[(0, 1, 1, 1), (1, 3, 3, 3), (0, 2, 1, 1)])
    return spec, O.OracleMesh(**spec.kwargs())


def ghost_mask(N):
    M = N + 2 * G
    act = np.zeros((M, M, M), bool)
    act[G:G + N, G:G + N, G:G + N] = True
    return ~act


def test_constant_field_fills_every_ghost_exactly():
    spec, m = amr_mesh()
    vals = np.array([1.25, -0.5, 0.75, 3.0, 7.5])
    act = np.broadcast_to(vals[None, :, None, None, None], (m.nleaf, 5, 8, 8, 8))
    m.set_active(act)
    m.refresh()
    gm = ghost_mask(8)
    for f in range(5):
        assert np.all(m.U[:, f][:, gm] == vals[f])


def cell_centres_padded(spec, keys, N):
    M = N + 2 * G
    out = []
    for ax in range(3):
        dx = np.array([spec.dx(int(l)) for l in keys[:, 0]])
        r = np.arange(M) - G + 0.5
        c = (keys[:, 1 + ax][:, None] * N + r[None, :]) * dx[:, None]
        shape = [len(keys), 1, 1, 1]
        shape[3 - ax] = M
        out.append(np.broadcast_to(c.reshape(shape), (len(keys), M, M, M)))
    return out


def test_linear_field_is_reproduced_in_ghosts_away_from_the_wrap():
    spec, m = amr_mesh()
    coef = np.array([0.3, 1.7, -0.9, 0.4])
    x, y, z = cell_centres_padded(spec, m.keys, 8)
    lin = coef[0] + coef[1] * x + coef[2] * y + coef[3] * z
    act = np.stack([lin[:, G:-G, G:-G, G:-G] * (f + 1) for f in range(5)], axis=1)
    m.set_active(act)
    m.refresh()
    # ghost cells whose prolongation stencil (up to one coarse cell, 2 dx of
    # its level) stays inside the domain see no periodic wrap
    dx = np.array([spec.dx(int(l)) for l in m.keys[:, 0]])[:, None, None, None]
    inside = (x > 4 * dx) & (x < 1 - 4 * dx) & (y > 4 * dx) & (y < 1 - 4 * dx) & \
             (z > 4 * dx) & (z < 1 - 4 * dx)
    sel = inside & ghost_mask(8)[None]
    assert sel.sum() > 1000
    for f in range(5):
        np.testing.assert_allclose(m.U[:, f][sel], (lin * (f + 1))[sel], rtol=0, atol=2e-14 * (f + 1))


def global_array(m, N, ext):
    """Assemble a uniform level-0 mesh into one global array [5, z, y, x]."""
    out = np.zeros((5, ext[2] * N, ext[1] * N, ext[0] * N))
    act = m.active()
    for s, k in enumerate(m.keys):
        out[:, k[3] * N:(k[3] + 1) * N, k[2] * N:(k[2] + 1) * N, k[1] * N:(k[1] + 1) * N] = act[s]
    return out


@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_same_level_ghosts_match_global_indexing(bc):
    root, N = (3, 2, 2), 8
    m = O.OracleMesh(root=root, block_cells=N, bc=bc)
    rng = np.random.default_rng(7)
    m.set_active(rng.uniform(0.5, 1.5, (m.nleaf, 5, N, N, N)))
    m.refresh()
    glob = global_array(m, N, root)
    M = N + 2 * G
    for s, k in enumerate(m.keys):
        idx = []
        for ax in range(3):
            g = k[1 + ax] * N + np.arange(M) - G
            n = root[ax] * N
            idx.append(np.mod(g, n) if bc == "periodic" else np.clip(g, 0, n - 1))
        expect = glob[:, idx[2][:, None, None], idx[1][None, :, None], idx[0][None, None, :]]
        np.testing.assert_array_equal(m.U[s], expect)


def test_restricted_ghosts_are_child_means_and_prolonged_ghosts_conserve():
    spec, m = amr_mesh()
    rng = np.random.default_rng(8)
    m.set_active(rng.uniform(0.5, 1.5, (m.nleaf, 5, 8, 8, 8)))
    m.refresh()
    N, M = 8, 14
    keyidx = {tuple(k): s for s, k in enumerate(m.keys)}
    act = m.active()
    checked_r = checked_p = 0
    for s, k in enumerate(m.keys):
        l = int(k[0])
        for c, b, a in itertools.product(range(M), repeat=3):
            if G <= a < G + N and G <= b < G + N and G <= c < G + N:
                continue
            p = [(int(k[1 + ax]) * N + (a, b, c)[ax] - G) % ((spec.root[ax] << l) * N) for ax in range(3)]
            bp = tuple(q // N for q in p)
            if (l, *bp) in keyidx:
                continue
            # restriction: the 8 children of a refined same-level position
            fine = [(2 * p[0] + ox, 2 * p[1] + oy, 2 * p[2] + oz) for oz in (0, 1) for oy in (0, 1) for ox in (0, 1)]
            fb = tuple(q // N for q in fine[0])
            if (l + 1, *fb) in keyidx and checked_r < 400:
                fs = keyidx[(l + 1, *fb)]
                vals = [act[fs, :, q[2] - fb[2] * N, q[1] - fb[1] * N, q[0] - fb[0] * N] for q in fine]
                np.testing.assert_allclose(m.U[s, :, c, b, a], np.mean(vals, axis=0), rtol=1e-15)
                checked_r += 1
    assert checked_r > 100
    # prolongation: every complete 2x2x2 group of prolonged ghosts averages
    # to its coarse parent (fine ghosts at padded indices 1,2 and N+3,N+4)
    for s, k in enumerate(m.keys):
        l = int(k[0])
        if l == 0:
            continue
        for cz, cy, cx in itertools.product((1, 3, 5, 7, 9, 11), repeat=3):
            if all(3 <= q < 3 + N for q in (cx, cy, cz)):
                continue
            if 3 <= cx < 11 and 3 <= cy < 11 and 3 <= cz < 11:
                continue
            if not all(q in (1, N + 3) or 3 <= q < N + 3 for q in (cx, cy, cz)):
                continue
            p = [int(k[1 + ax]) * N + (cx, cy, cz)[ax] - G for ax in range(3)]
            p = [q % ((spec.root[ax] << l) * N) for ax, q in enumerate(p)]
            if (l, *[q // N for q in p]) in keyidx:
                continue
            pc = [q >> 1 for q in p]
            cb = tuple(q // N for q in pc)
            if (l - 1, *cb) not in keyidx:
                continue
            grp = m.U[s, :, cz:cz + 2, cy:cy + 2, cx:cx + 2].reshape(5, 8)
            cs = keyidx[(l - 1, *cb)]
            parent = act[cs, :, pc[2] - cb[2] * N, pc[1] - cb[1] * N, pc[0] - cb[0] * N]
            np.testing.assert_allclose(grp.mean(axis=1), parent, rtol=1e-14)
            checked_p += 1
    assert checked_p > 50
