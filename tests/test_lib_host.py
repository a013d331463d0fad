"""CPU tests of the HIP library's host side: the C ABI loads and exports every
symbol include/amr.h declares, and the host mesh builder (hash-map octree,
level-by-level balance) produces the same leaf sets as the oracle's
independent builder (dense per-level arrays, fixed-point balance).  No kernel
is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_01319_amd import _lib, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "amr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amr_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def host_mesh(**kw):
    L = _lib.lib()
    refine = kw.pop("refine", ())
    leaves = kw.pop("leaves", None)
    d, keep = _lib.make_desc(refine=refine, **kw)
    h = ctypes.c_void_p()
    if leaves is not None:
        lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
        rc = L.amr_mesh_create_from_leaves(ctypes.byref(d), lv.shape[0], lv.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(h))
    else:
        rc = L.amr_mesh_create(ctypes.byref(d), ctypes.byref(h))
    if rc != 0:
        return rc, None, None
    info = _lib.MeshInfo()
    assert L.amr_mesh_info(h, ctypes.byref(info)) == 0
    keys = np.zeros((info.n_leaves, 4), dtype=np.int32)
    assert L.amr_mesh_blocks(h, keys.ctypes.data_as(ctypes.c_void_p), info.n_leaves) == 0
    L.amr_mesh_destroy(h)
    return 0, info, keys


@pytest.mark.parametrize("seed", range(8))
def test_host_mesh_matches_oracle_mesh(seed):
    root = [(2, 2, 2), (3, 2, 2), (1, 2, 3), (4, 4, 4)][seed % 4]
    refine = I.random_refine_list(root, 3, 5 + seed, seed)
    rc, info, keys = host_mesh(root=root, block_cells=8, max_level=3, refine=refine)
    assert rc == 0
    om = O.OracleMesh(root=root, block_cells=8, max_level=3, refine=refine)
    assert sorted(map(tuple, keys)) == sorted(map(tuple, om.keys))
    assert info.n_leaves == om.nleaf
    assert list(info.levels[:4]) == list(np.bincount(om.keys[:, 0], minlength=4)[:4])


def test_storage_order_is_morton_within_each_root():
    spec = I.sedov_spec(root=2, block_cells=16, levels=2)
    rc, info, keys = host_mesh(**spec.kwargs())
    assert rc == 0
    L = spec.max_level

    def morton(k):
        l, i, j, kk = map(int, k)
        s = L - l
        i, j, kk = i << s, j << s, kk << s
        r = (i >> L) + spec.root[0] * ((j >> L) + spec.root[1] * (kk >> L))
        code = 0
        for b in range(L - 1, -1, -1):
            code = code * 8 + ((i >> b) & 1) + 2 * ((j >> b) & 1) + 4 * ((kk >> b) & 1)
        return (r, code)

    codes = [morton(k) for k in keys]
    assert codes == sorted(codes)


def test_info_sizes():
    spec = I.sedov_spec(root=8, block_cells=32, levels=2)
    rc, info, keys = host_mesh(**spec.kwargs())
    assert rc == 0
    assert info.n_leaves == 624
    assert info.padded == 38
    assert info.block_stride == 5 * 38 ** 3
    assert info.field_bytes == 624 * 5 * 38 ** 3 * 8
    assert info.workspace_bytes % 256 == 0
    assert info.n_cf_faces > 0
    assert info.n_fields == 5
    rc, de, _ = host_mesh(**I.with_(spec, dual_energy=True).kwargs())
    assert rc == 0 and de.n_fields == 6
    assert de.block_stride == 6 * 38 ** 3
    assert de.field_bytes == 624 * 6 * 38 ** 3 * 8
    assert de.workspace_bytes > info.workspace_bytes  # six face fluxes per coarse-fine face cell


@pytest.mark.parametrize("bad,code", [
    (dict(ghost=2), _lib.STATUS and -1),
    (dict(block_cells=12), -1),
    (dict(max_level=9), -1),
    (dict(gamma=1.0), -1),
    (dict(rho_floor=1e-120), -1),
    (dict(p_floor=0.0), -1),
    (dict(bc="outflow", refine=[(0, 0, 0, 0)], max_level=1), -1),
    (dict(refine=[(1, 0, 0, 0)], max_level=1), -1),
    (dict(dual_energy=2), -1),
    (dict(dual_energy=True, eta1=-0.1), -1),
    (dict(dual_energy=True, eta2=1.5), -1),
])
def test_invalid_descriptors_are_rejected(bad, code):
    kw = dict(root=(2, 2, 2), block_cells=8)
    kw.update(bad)
    rc, _, _ = host_mesh(**kw)
    assert rc == code


def test_unbalanced_or_gapped_leaf_sets_are_rejected():
    spec = I.sedov_spec(root=4, block_cells=8, levels=2)
    rc, info, keys = host_mesh(**spec.kwargs())
    assert rc == 0
    rc2, _, keys2 = host_mesh(root=spec.root, block_cells=8, max_level=2, leaves=keys)
    assert rc2 == 0 and sorted(map(tuple, keys2)) == sorted(map(tuple, keys))
    rc3, _, _ = host_mesh(root=spec.root, block_cells=8, max_level=2, leaves=keys[1:])
    assert rc3 == -2
    bad = [k for k in map(tuple, keys) if not (k[0] == 0 and k[1:] == (0, 0, 0))]
    bad += [(1, a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1) if (a, b, c) != (0, 0, 0)]
    bad += [(2, a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    rc4, _, _ = host_mesh(root=spec.root, block_cells=8, max_level=2, leaves=bad)
    assert rc4 == -2


def _blast_oracle(root, N, levels, seed, steps=4):
    spec = I.MeshSpec(root=(root,) * 3, block_cells=N, max_level=levels, gamma=5 / 3)
    m = O.OracleMesh(**spec.kwargs())
    rng = np.random.default_rng(seed)
    w = 1.0 / root
    centres = [np.array([(i + 0.5) * w, (j + 0.5) * w, (k + 0.5) * w]) + rng.uniform(-0.25, 0.25, 3) * w
               for k in range(root) for j in range(root) for i in range(root)]
    m.set_active(I.blast_state(spec, m.keys, centres, energy=1.0, rho0=1.0, p0=1e-5, radius_cells=2.0, level=0))
    for k in range(steps):
        m.step(k)
    return spec, m


def _new_leaves(L, h, h2, st):
    """Leaf keys of the remeshed mesh h2; a remesh that changed nothing
    returns no mesh, and the leaves are h's."""
    src = h2 if h2.value else h
    if not h2.value:
        assert st.refined == 0 and st.coarsened == 0
    info = _lib.MeshInfo()
    L.amr_mesh_info(src, ctypes.byref(info))
    assert info.n_leaves == st.n_leaves
    k2 = np.zeros((info.n_leaves, 4), dtype=np.int32)
    L.amr_mesh_blocks(src, k2.ctypes.data_as(ctypes.c_void_p), info.n_leaves)
    return k2


def test_remesh_that_changes_nothing_returns_no_mesh():
    L = _lib.lib()
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=2, gamma=1.4,
                      refine=I.random_refine_list((2, 2, 2), 2, 4, 1))
    d, keep = _lib.make_desc(**spec.kwargs())
    h = ctypes.c_void_p()
    assert L.amr_mesh_create(ctypes.byref(d), ctypes.byref(h)) == 0
    info = _lib.MeshInfo()
    L.amr_mesh_info(h, ctypes.byref(info))
    n = int(info.n_leaves)
    S = np.full(n, 0.5)
    for prm, refused in [(_lib.RemeshParams(1e300, 0.0, n), 0),  # nothing is a candidate
                         (_lib.RemeshParams(0.3, 0.0, n + 6), None)]:  # every candidate refused at the cap
        st = _lib.RemeshStats()
        h2 = ctypes.c_void_p(1)
        assert L.amr_remesh_plan_host(h, S.ctypes.data_as(ctypes.c_void_p), ctypes.byref(prm), ctypes.byref(h2),
                                      ctypes.byref(st)) == 0
        assert not h2.value and st.refined == 0 and st.coarsened == 0 and st.n_leaves == n
        assert st.refused > 0 if refused is None else st.refused == refused
    L.amr_mesh_destroy(h)


@pytest.mark.parametrize("seed,cap_extra,levels", [(5, 10 ** 6, 2), (6, 40, 2), (7, 10 ** 6, 3), (8, 90, 3)])
def test_host_remesh_decisions_match_oracle(seed, cap_extra, levels):
    """Same indicator in, same leaf set and counters out: the library's local
    ripple closure with an undo journal against the oracle's global
    fixed-point balance, including refusals at a tight capacity and a second
    remesh that coarsens."""
    spec, m = _blast_oracle(3, 8, levels, seed)
    L = _lib.lib()
    for rnd in range(2):
        m.refresh()
        S_or = m.indicator()
        d, keep = _lib.make_desc(refine=(), **{k: v for k, v in spec.kwargs().items() if k != "refine"})
        h = ctypes.c_void_p()
        lv = np.ascontiguousarray(m.keys)
        assert L.amr_mesh_create_from_leaves(ctypes.byref(d), lv.shape[0], lv.ctypes.data_as(ctypes.c_void_p),
                                             ctypes.byref(h)) == 0
        info = _lib.MeshInfo()
        L.amr_mesh_info(h, ctypes.byref(info))
        keys = np.zeros((info.n_leaves, 4), dtype=np.int32)
        L.amr_mesh_blocks(h, keys.ctypes.data_as(ctypes.c_void_p), info.n_leaves)
        idx = {tuple(k): s for s, k in enumerate(m.keys)}
        S = np.ascontiguousarray([S_or[idx[tuple(k)]] for k in keys])
        cap = m.nleaf + cap_extra
        prm = _lib.RemeshParams(0.3, 0.1 if rnd else 0.0, cap)
        st = _lib.RemeshStats()
        h2 = ctypes.c_void_p()
        assert L.amr_remesh_plan_host(h, S.ctypes.data_as(ctypes.c_void_p), ctypes.byref(prm), ctypes.byref(h2),
                                      ctypes.byref(st)) == 0
        k2 = _new_leaves(L, h, h2, st)
        m2, ost = m.remesh(0.3, 0.1 if rnd else 0.0, cap)
        assert sorted(map(tuple, k2)) == sorted(map(tuple, m2.keys))
        assert (st.refined, st.coarsened, st.refused) == tuple(int(v) for v in ost)
        L.amr_mesh_destroy(h2)
        L.amr_mesh_destroy(h)
        m = m2
        for k in range(3):
            m.step(k)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_host_coarsening_decisions_match_oracle(seed):
    root = (3, 2, 2)
    spec = I.MeshSpec(root=root, block_cells=8, max_level=3, gamma=1.4,
                      refine=I.random_refine_list(root, 3, 10, seed))
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(I.smooth_state(spec, m.keys, seed=seed, amp=0.2, vel=0.3))
    m.refresh()
    S_or = m.indicator()
    thr = float(np.median(S_or))
    L = _lib.lib()
    d, keep = _lib.make_desc(**spec.kwargs())
    h = ctypes.c_void_p()
    assert L.amr_mesh_create(ctypes.byref(d), ctypes.byref(h)) == 0
    info = _lib.MeshInfo()
    L.amr_mesh_info(h, ctypes.byref(info))
    keys = np.zeros((info.n_leaves, 4), dtype=np.int32)
    L.amr_mesh_blocks(h, keys.ctypes.data_as(ctypes.c_void_p), info.n_leaves)
    idx = {tuple(k): s for s, k in enumerate(m.keys)}
    S = np.ascontiguousarray([S_or[idx[tuple(k)]] for k in keys])
    for rs in (1e9, thr * 2):
        prm = _lib.RemeshParams(rs, thr, 10 ** 6)
        st = _lib.RemeshStats()
        h2 = ctypes.c_void_p()
        assert L.amr_remesh_plan_host(h, S.ctypes.data_as(ctypes.c_void_p), ctypes.byref(prm), ctypes.byref(h2),
                                      ctypes.byref(st)) == 0
        k2 = _new_leaves(L, h, h2, st)
        m2, ost = m.remesh(rs, thr, 10 ** 6)
        assert st.coarsened > 0
        assert sorted(map(tuple, k2)) == sorted(map(tuple, m2.keys))
        assert (st.refined, st.coarsened, st.refused) == tuple(int(v) for v in ost)
        L.amr_mesh_destroy(h2)
    L.amr_mesh_destroy(h)


def test_batch_leaf_sets_equal_single_meshes():
    L = _lib.lib()
    specs = [I.batch_instance(i)[0] for i in range(12)]
    descs = (_lib.MeshDesc * len(specs))()
    keep = []
    for i, sp in enumerate(specs):
        d, k = _lib.make_desc(**sp.kwargs())
        descs[i] = d
        keep.append(k)
    h = ctypes.c_void_p()
    assert L.amr_batch_create(descs, len(specs), ctypes.byref(h)) == 0
    info = _lib.MeshInfo()
    L.amr_mesh_info(h, ctypes.byref(info))
    assert info.n_instances == len(specs)
    keys = np.zeros((info.n_leaves, 4), dtype=np.int32)
    L.amr_mesh_blocks(h, keys.ctypes.data_as(ctypes.c_void_p), info.n_leaves)
    off = np.zeros(len(specs) + 1, dtype=np.int64)
    assert L.amr_mesh_instance_offsets(h, off.ctypes.data_as(ctypes.c_void_p), off.size) == 0
    for i, sp in enumerate(specs):
        rc, inf1, k1 = host_mesh(**sp.kwargs())
        assert rc == 0
        assert np.array_equal(keys[off[i]:off[i + 1]], k1)  # same storage order too
        om = O.OracleMesh(**sp.kwargs())
        assert sorted(map(tuple, k1)) == sorted(map(tuple, om.keys))
    L.amr_mesh_destroy(h)
    # mixed block sizes are rejected
    d2, k2 = _lib.make_desc(**dict(specs[1].kwargs(), block_cells=8))
    descs[1] = d2
    h = ctypes.c_void_p()
    assert L.amr_batch_create(descs, 2, ctypes.byref(h)) == -1


def _poisson_bytes(**kw):
    L = _lib.lib()
    refine = kw.pop("refine", ())
    d, keep = _lib.make_desc(refine=refine, **kw)
    h = ctypes.c_void_p()
    assert L.amr_mesh_create(ctypes.byref(d), ctypes.byref(h)) == 0
    n = ctypes.c_int64(-1)
    rc = L.amr_poisson_workspace_bytes(h, ctypes.byref(n))
    L.amr_mesh_destroy(h)
    return rc, n.value


def test_poisson_workspace_and_refusals_on_the_host():
    """The mg0 workspace holds phi and f of every level (each 256-byte
    rounded) and the reduction scratch; on a refined mesh (mg0 on the
    octree) it also holds the hierarchy of coarsened meshes and their
    arrays, so it is larger than the root grid's; outflow axes and coarsest
    levels above 4096 cells are refused before any GPU work."""
    rc, nbytes = _poisson_bytes(root=(2, 2, 2), block_cells=16)  # 32^3: levels 32, 16, 8, 4, 2
    assert rc == 0
    levels = [32 ** 3, 16 ** 3, 8 ** 3, 4 ** 3, 2 ** 3]
    want = sum(2 * ((c * 8 + 255) // 256 * 256) for c in levels) + (1024 + 64) * 8
    assert nbytes == want
    rc, refined = _poisson_bytes(root=(4, 4, 4), block_cells=8, max_level=2, refine=[(0, 1, 1, 1), (1, 2, 2, 2)])
    _, root_only = _poisson_bytes(root=(4, 4, 4), block_cells=8)
    assert rc == 0 and refined > 3 * root_only
    assert _poisson_bytes(root=(2, 2, 2), block_cells=8, bc="outflow")[0] == -1
    # 9^3 roots of 32^3: 288 -> 144 -> 72 -> 36 -> 18 (not a multiple of 4): coarsest 18^3 = 5832 cells
    assert _poisson_bytes(root=(9, 9, 9), block_cells=32)[0] == -1
    assert _poisson_bytes(root=(7, 7, 7), block_cells=32)[0] == 0  # coarsest 14^3 = 2744 cells
    assert _poisson_bytes(root=(3, 2, 1), block_cells=16)[0] == 0  # coarsest 6 x 4 x 2


def test_launch_size_limit():
    """A dispatch counts its work items in 32 bits: the library rejects a
    mesh with more leaves than its largest launch over the leaves can cover
    (at 32^3 the first x sweep's and the transposes' ceil(38^2 / 3) tiles of
    128 lanes per leaf: 69,615 leaves), and a remesh refuses growth beyond it
    like growth beyond max_blocks."""
    L = _lib.lib()
    per_leaf = -(-38 * 38 // 3) * 128
    limit = (2 ** 32 - 1) // per_leaf
    assert limit == 69615
    for root, ok in (((40, 40, 43), True), ((41, 41, 42), False)):
        d, keep = _lib.make_desc(refine=(), root=root, block_cells=32, max_level=1)
        h = ctypes.c_void_p()
        rc = L.amr_mesh_create(ctypes.byref(d), ctypes.byref(h))
        assert (rc == 0) == ok, (root, rc)
        if not ok:
            assert _lib.STATUS[rc] == "AMR_E_INVALID"
            continue
        n = 40 * 40 * 43
        S = np.zeros(n)
        S[:200] = 1.0  # 200 root refinements of 7 new leaves each (one level: no balancing)
        prm = _lib.RemeshParams(0.3, 0.0, 10 ** 9)
        h2, st = ctypes.c_void_p(), _lib.RemeshStats()
        assert L.amr_remesh_plan_host(h, S.ctypes.data_as(ctypes.c_void_p), ctypes.byref(prm), ctypes.byref(h2),
                                      ctypes.byref(st)) == 0
        assert st.n_leaves <= limit and st.refused > 0 and st.refined == (limit - n) // 7
        assert st.n_leaves == n + 7 * st.refined
        L.amr_mesh_destroy(h2)
        L.amr_mesh_destroy(h)
