"""Checkpoint and restart of an adaptive run: the leaf set (amr_mesh_blocks)
and the active cells of the state, written to disk and read back into a mesh
built from that leaf set (amr_mesh_create_from_leaves), continue the run bit
for bit.  Ten steps of the blast array with remeshes every four steps in one
run equal six steps, a save and a restore, and four more steps: leaf set,
every active value and every step's dt."""
import sys

import numpy as np
import pytest
import torch

from paper_1810_01319_amd import adaptive
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd.mesh import Mesh

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-restart] {msg}", file=sys.stderr, flush=True)


def by_key(keys_from, blocks, keys_to):
    """blocks (one per leaf of keys_from) reordered to the leaf order keys_to"""
    idx = {tuple(k): s for s, k in enumerate(np.asarray(keys_from).tolist())}
    return blocks[np.array([idx[tuple(k)] for k in np.asarray(keys_to).tolist()])]


def test_save_and_restore_continue_the_adaptive_run_bitwise(tmp_path):
    spec = I.blasts_spec(root=2, block_cells=16, levels=2)
    cap = 2048

    def start():
        m = Mesh(**spec.kwargs())
        return m, m.state_from_active(I.blasts_state(spec, m.keys))

    say("uninterrupted run: 10 steps")
    m, U = start()
    ma, Ua, dta, sta = adaptive.run(m, U, 10, max_blocks=cap)
    assert sum(s["refined"] for s in sta) > 0
    say(f"restarted run: 6 steps, save, restore, 4 steps ({ma.nleaf} leaves at the end)")
    m, U = start()
    mb, Ub, dtb, _ = adaptive.run(m, U, 6, max_blocks=cap)
    path = tmp_path / "checkpoint.npz"
    np.savez(path, keys=mb.keys, active=mb.active(Ub), step=6)
    del mb, Ub
    ck = np.load(path)
    mc = Mesh(leaves=ck["keys"], **spec.kwargs())
    Uc = mc.state_from_active(by_key(ck["keys"], ck["active"], mc.keys))
    mc, Uc, dtc, _ = adaptive.run(mc, Uc, 4, start=int(ck["step"]), max_blocks=cap)
    torch.cuda.synchronize()
    assert sorted(map(tuple, mc.keys.tolist())) == sorted(map(tuple, ma.keys.tolist()))
    assert np.array_equal(by_key(mc.keys, mc.active(Uc), ma.keys), ma.active(Ua))
    seq_a = torch.stack(dta).cpu().numpy()
    seq_b = torch.stack(dtb + dtc).cpu().numpy()
    assert np.array_equal(seq_a, seq_b)
