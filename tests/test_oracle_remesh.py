"""Pins of the oracle's remesh: indicator values, the new mesh's tiling and
2:1 balance, the capacity policy, conservation across migration, and
restrict(prolong(U)) = U through a refine-then-coarsen round trip."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
from test_oracle_mesh_refresh import check_tiling_and_balance


def totals(m, spec):
    act = m.active()
    vol = np.array([spec.dx(int(l)) ** 3 for l in m.keys[:, 0]])
    return (act.reshape(act.shape[0], 5, -1).sum(-1) * vol[:, None]).sum(0)


def test_indicator_values():
    spec = I.MeshSpec(root=(2, 1, 1), block_cells=8)
    m = O.OracleMesh(**spec.kwargs())
    x = I.cell_centres(spec, m.keys)[0]
    # uniform density: zero; a jump 1 -> 2 inside block 0 between cells 3|4:
    # the cell with rho=1 next to it sees |2-1|/(2*1) = 0.5
    rho = np.where((x > 4 / 16) & (x < 12 / 16), 2.0, 1.0)
    rho[1] = 1.0  # block 1 uniform
    m.set_active(I.conserved(1.4, rho, 0.0, 0.0, 0.0, np.ones_like(x)))
    m.refresh()
    S = m.indicator()
    assert S[0] == 0.5
    # block 1 (cells 8..15) is uniform, but its cell 8 sees block 0's rho=2
    # cell 7 through the refreshed ghost: |1-2|/(2*1) = 0.5
    assert S[1] == 0.5
    m.set_active(I.conserved(1.4, np.ones_like(x), 0.0, 0.0, 0.0, np.ones_like(x)))
    m.refresh()
    assert np.all(m.indicator() == 0.0)


def blast_mesh(root=4, N=8, levels=2, seed=5):
    spec = I.MeshSpec(root=(root, root, root), block_cells=N, max_level=levels, gamma=5 / 3)
    m = O.OracleMesh(**spec.kwargs())
    rng = np.random.default_rng(seed)
    w = 1.0 / root
    centres = [np.array([(i + 0.5) * w, (j + 0.5) * w, (k + 0.5) * w]) + rng.uniform(-0.25, 0.25, 3) * w
               for k in range(root) for j in range(root) for i in range(root)]
    m.set_active(I.blast_state(spec, m.keys, centres, energy=1.0, rho0=1.0, p0=1e-5, radius_cells=2.0, level=0))
    return spec, m


def test_remesh_keeps_balance_conservation_and_capacity():
    spec, m = blast_mesh()
    for k in range(4):
        m.step(k)
    t0 = totals(m, spec)
    n0 = m.nleaf
    m2, st = m.remesh(0.3, 0.1, max_blocks=10 ** 6)
    check_tiling_and_balance(m2.keys, spec.root, spec.max_level)
    assert st[0] > 0
    assert m2.nleaf == n0 + 7 * st[0] - 7 * st[1]
    np.testing.assert_allclose(totals(m2, spec), t0, rtol=1e-13, atol=1e-13 * abs(t0[0]))
    # a tight capacity refuses refinements and is respected
    cap = n0 + 7 * 4
    m3, st3 = m.remesh(0.3, 0.1, max_blocks=cap)
    assert m3.nleaf <= cap and st3[2] > 0
    check_tiling_and_balance(m3.keys, spec.root, spec.max_level)


def test_refined_leaves_are_the_high_indicator_ones():
    spec, m = blast_mesh()
    for k in range(4):
        m.step(k)
    m.refresh()
    S = m.indicator()
    m2, st = m.remesh(0.3, 0.0, max_blocks=10 ** 6)
    old = {tuple(k): s for s, k in enumerate(m.keys)}
    new = {tuple(k) for k in m2.keys}
    for key, s in old.items():
        if S[s] > 0.3 and key[0] < spec.max_level:
            assert key not in new, "a candidate above threshold must be refined when capacity allows"


def test_refine_then_coarsen_round_trip_restores_the_state():
    """Refining every root (prolongation) and merging them back (restriction)
    returns the original data to round-off: restrict o prolong = identity."""
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=1, gamma=1.4)
    m = O.OracleMesh(**spec.kwargs())
    U0 = I.smooth_state(spec, m.keys, seed=21, amp=0.3, vel=0.5)
    m.set_active(U0)
    fine, st = m.remesh(-1.0, -1.0, max_blocks=10 ** 6)  # every leaf refines, none coarsens
    assert st[0] == 8 and fine.nleaf == 64
    back, st2 = fine.remesh(1e300, 1e300, max_blocks=10 ** 6)  # nothing refines, all octets merge
    assert st2[1] == 8 and back.nleaf == 8
    order = {tuple(k): s for s, k in enumerate(back.keys)}
    got = back.active()[[order[tuple(k)] for k in m.keys]]
    np.testing.assert_allclose(got, U0, rtol=4e-16, atol=4e-16)


def test_one_level_per_remesh():
    spec, m = blast_mesh(levels=3)
    for k in range(4):
        m.step(k)
    m2, st = m.remesh(0.3, 0.1, max_blocks=10 ** 6)
    assert int(m2.keys[:, 0].max()) <= int(m.keys[:, 0].max()) + 1


def test_blockwise_blast_inputs_equal_the_generic_deposit():
    """The per-block fast path of the blast-array inputs gives the same bytes
    as the generic deposit over all cells."""
    spec = I.blasts_spec(root=3, block_cells=16, levels=2)
    m = O.OracleMesh(**spec.kwargs())
    fast = I.blasts_state(spec, m.keys)
    slow = I.blast_state(spec, m.keys, I.blast_centres(3), energy=1.0, rho0=1.0, p0=1e-5, radius_cells=2.0,
                         level=0)
    assert np.array_equal(fast, slow)
    # a subset of blocks in another order gives the matching slices
    sub = m.keys[::-3]
    assert np.array_equal(I.blasts_state(spec, sub), fast[::-3])
