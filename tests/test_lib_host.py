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


@pytest.mark.parametrize("bad,code", [
    (dict(ghost=2), _lib.STATUS and -1),
    (dict(block_cells=12), -1),
    (dict(max_level=9), -1),
    (dict(gamma=1.0), -1),
    (dict(bc="outflow", refine=[(0, 0, 0, 0)], max_level=1), -1),
    (dict(refine=[(1, 0, 0, 0)], max_level=1), -1),
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
