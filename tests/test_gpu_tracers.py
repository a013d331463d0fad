"""GPU tracer particles against the oracle: after several full steps every
particle (by id) is held by the same leaf with a bitwise-equal position, the
hydro state and dt sequence stay bitwise equal, removals through outflow
faces match, batched instances match their own oracle runs, and a capacity
overflow is counted, not written out of bounds.  The order of particles
inside a leaf is not unique (arrivals), so leaves are compared as id sets."""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_01319_amd import inputs as I
from paper_1810_01319_amd.mesh import Mesh
from paper_1810_01319_amd.tracers import Tracers

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-tracers] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tracer tests need an MI355X"


def oracle_pair(spec, gm, act):
    om = O.OracleMesh(**spec.kwargs())
    idx = {tuple(k): s for s, k in enumerate(om.keys)}
    perm = np.array([idx[tuple(k)] for k in gm.keys])
    o = np.empty_like(act)
    o[perm] = act
    om.set_active(o)
    return om, perm


def compare(gm, tr, om, otr, perm):
    leaf, pos, ids = tr.to_host()
    alive = otr.alive.astype(bool)
    assert len(ids) == alive.sum(), (len(ids), alive.sum(), tr.counters())
    order = np.argsort(ids)
    leaf, pos, ids = leaf[order], pos[order], ids[order]
    oid = otr.ids[alive]
    oo = np.argsort(oid)
    opos = otr.positions()[alive][oo]
    assert np.array_equal(ids, oid[oo])
    assert np.array_equal(pos, opos), np.abs(pos - opos).max()
    own = om.locate(opos)
    assert np.array_equal(perm[leaf], own)  # same leaf (oracle index of the GPU leaf)


def run(spec, act, per_axis, steps, capacity=None, jitter=7):
    gm = Mesh(**spec.kwargs())
    om, perm = oracle_pair(spec, gm, act)
    pos, ids = I.tracer_positions(spec, gm.keys, per_axis, jitter_seed=jitter)
    tr = Tracers.from_positions(gm, pos, ids, capacity)
    otr = O.Tracers(*pos.reshape(-1, 3).T, ids.ravel())
    U = gm.state_from_active(act)
    dt = gm.dt_tensor()
    for k in range(steps):
        tr.step(U, dt, k)
        odt = om.step_tracers(k, otr)
        assert float(dt.cpu()[0]) == odt, k
    assert np.array_equal(gm.active(U), om.active()[perm])
    compare(gm, tr, om, otr, perm)
    return gm, tr, otr


@pytest.mark.parametrize("N", [8, 16])
def test_tracers_match_oracle_on_random_amr(N):
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=N, max_level=2, gamma=5 / 3,
                      refine=I.random_refine_list((2, 2, 2), 2, 4, 11))
    keys = Mesh(**spec.kwargs()).keys
    act = I.smooth_state(spec, keys, seed=12, amp=0.2, vel=0.5)
    say(f"random AMR N={N}: {len(keys)} leaves")
    gm, tr, otr = run(spec, act, 1, 8)
    assert tr.counters() == {"overflow": 0, "removed": 0, "lost": 0}


def test_tracers_cross_blocks_and_levels():
    """A fast bulk flow over a three-level mesh of 8^3 blocks: particles cross
    same-level, coarse-to-fine and fine-to-coarse block faces and the
    periodic seam; all of them stay bitwise equal to the oracle."""
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=2, gamma=1.4,
                      refine=I.random_refine_list((2, 2, 2), 2, 5, 21))
    keys = Mesh(**spec.kwargs()).keys
    x, y, z = I.cell_centres(spec, keys)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    act = I.conserved(1.4, rho, 1.5, -1.0, 0.7, np.ones_like(x))
    say(f"bulk-flow tracers: {len(keys)} leaves")
    gm, tr, otr = run(spec, act, 1, 20, capacity=8 * 512)
    assert tr.counters() == {"overflow": 0, "removed": 0, "lost": 0}
    leaf, pos, ids = tr.to_host()
    start = np.repeat(np.arange(gm.nleaf), spec.block_cells ** 3)  # placement leaf of each id
    lv = gm.keys[:, 0]
    changed = start[ids] != leaf
    up = int((lv[start[ids]] < lv[leaf]).sum())
    down = int((lv[start[ids]] > lv[leaf]).sum())
    say(f"bulk-flow tracers: {int(changed.sum())} changed leaf, {up} to a finer one, {down} to a coarser one")
    assert changed.sum() > 1000 and up > 10 and down > 10


def test_tracers_removed_through_outflow_faces():
    spec = I.MeshSpec(root=(3, 1, 2), block_cells=8, gamma=1.4, bc="outflow")
    keys = Mesh(**spec.kwargs()).keys
    x = I.cell_centres(spec, keys)[0]
    u = np.where(x < 0.5, -2.0, 2.0)
    act = I.conserved(1.4, np.ones_like(x), u, 0.5, 0.0, np.ones_like(x))
    gm, tr, otr = run(spec, act, 1, 12)
    c = tr.counters()
    assert c["removed"] == int((otr.alive == 0).sum()) > 0, c


def test_tracers_on_batched_instances():
    specs, cents = zip(*[I.batch_instance(i) for i in range(5)])
    gm = Mesh.batch([s.kwargs() for s in specs])
    acts, oms, otrs, poss, idss = [], [], [], [], []
    for i, (sp, c) in enumerate(zip(specs, cents)):
        keys = gm.keys[gm.first_leaf[i]:gm.first_leaf[i + 1]]
        a = I.batch_state(sp, keys, c)
        acts.append(a)
        om = O.OracleMesh(**sp.kwargs())
        idx = {tuple(k): s for s, k in enumerate(om.keys)}
        perm = np.array([idx[tuple(k)] for k in keys])
        o = np.empty_like(a)
        o[perm] = a
        om.set_active(o)
        pos, ids = I.tracer_positions(sp, keys, 1, jitter_seed=20 + i)
        ids = ids + 10 ** 7 * i
        oms.append((om, perm))
        otrs.append(O.Tracers(*pos.reshape(-1, 3).T, ids.ravel()))
        poss.append(pos)
        idss.append(ids)
    say(f"batched tracers: {gm.nleaf} leaves")
    tr = Tracers.from_positions(gm, np.concatenate(poss), np.concatenate(idss))
    U = gm.state_from_active(np.concatenate(acts))
    dt = gm.dt_tensor()
    for k in range(4):
        tr.step(U, dt, k)
        d = dt.cpu().numpy()
        for i, (om, perm) in enumerate(oms):
            assert d[i] == om.step_tracers(k, otrs[i])
    leaf, pos, ids = tr.to_host()
    for i, (om, perm) in enumerate(oms):
        sel = (leaf >= gm.first_leaf[i]) & (leaf < gm.first_leaf[i + 1])
        order = np.argsort(ids[sel])
        lo, po, io = leaf[sel][order] - gm.first_leaf[i], pos[sel][order], ids[sel][order]
        ot = otrs[i]
        oo = np.argsort(ot.ids)
        assert np.array_equal(io, ot.ids[oo])
        assert np.array_equal(po, ot.positions()[oo])
        assert np.array_equal(perm[lo], om.locate(po))


def test_capacity_overflow_is_counted():
    """A uniform flow pushes a full row of particles into a leaf that is
    already near capacity: the excess is dropped and counted."""
    spec = I.MeshSpec(root=(2, 1, 1), block_cells=8, gamma=1.4)
    gm = Mesh(**spec.kwargs())
    x = I.cell_centres(spec, gm.keys)[0]
    act = I.conserved(1.4, np.ones_like(x), 0.9, 0.0, 0.0, np.ones_like(x))
    rng = np.random.default_rng(3)
    n = 250
    pos = np.empty((2, n, 3))
    for s, (l, i, j, k) in enumerate(gm.keys):
        lo = np.array([i, j, k], dtype=float) * 8
        pos[s] = lo + rng.uniform([7.0, 0, 0], [8.0, 8, 8], size=(n, 3))  # near each leaf's +x face
    ids = np.arange(2 * n).reshape(2, n)
    tr = Tracers.from_positions(gm, pos, ids, capacity=256)
    U = gm.state_from_active(act)
    dt = gm.dt_tensor()
    tr.step(U, dt, 0)
    c = tr.counters()
    say(f"overflow counters {c}, kept {tr.count}")
    assert c["overflow"] > 0 and c["lost"] == 0
    assert tr.count == 2 * n - c["overflow"]
    assert int(tr.sets[tr.cur][2].max()) <= 256


@pytest.mark.parametrize("root,N,levels,cap_extra", [(3, 8, 2, 10 ** 6), (3, 8, 3, 60)])
def test_tracers_through_remesh(root, N, levels, cap_extra):
    """Blast tiles with a remesh every 4 steps: the tracers follow their
    leaves through refinement and coarsening (and refusals at a tight
    capacity) and stay bitwise equal to the oracle, whose particles are
    located by position in whatever mesh it holds."""
    spec = I.blasts_spec(root=root, block_cells=N, levels=levels)
    gm = Mesh(**spec.kwargs())
    act = I.blasts_state(spec, gm.keys)
    om, perm = oracle_pair(spec, gm, act)
    pos, ids = I.tracer_positions(spec, gm.keys, 1, jitter_seed=31)
    tr = Tracers.from_positions(gm, pos, ids, capacity=8 * N ** 3)
    otr = O.Tracers(*pos.reshape(-1, 3).T, ids.ravel())
    U = gm.state_from_active(act)
    cap = gm.nleaf + cap_extra
    say(f"tracers through remesh: root={root} N={N} levels={levels}, {gm.nleaf} leaves")
    remeshes = 0
    for k in range(13):
        if k > 0 and k % 4 == 0:
            new, U, st = gm.remesh(U, 0.3, 0.1, cap)
            tr = tr.remesh(new)
            remeshes += new is not gm
            gm = new
            om, _ = om.remesh(0.3, 0.1, cap)
        dt = gm.dt_tensor()
        tr.step(U, dt, k)
        assert float(dt.cpu()[0]) == om.step_tracers(k, otr), k
    assert remeshes > 0
    idx = {tuple(kk): s for s, kk in enumerate(om.keys)}
    perm = np.array([idx[tuple(kk)] for kk in gm.keys])
    assert np.array_equal(gm.active(U), om.active()[perm])
    compare(gm, tr, om, otr, perm)
    assert tr.counters() == {"overflow": 0, "removed": 0, "lost": 0}
    say(f"tracers through remesh: {remeshes} remeshes, now {gm.nleaf} leaves, {tr.count} particles")


def test_tracers_on_a_dual_energy_mesh():
    """Six-field state (rho e, thresholds 1e-3 and 0.1): the drift reads the
    velocity through the six-field block stride; particles and state bitwise
    equal to the oracle."""
    spec = I.MeshSpec(root=(2, 2, 2), block_cells=8, max_level=2, gamma=5 / 3,
                      refine=I.random_refine_list((2, 2, 2), 2, 4, 13), dual_energy=True)
    keys = Mesh(**spec.kwargs()).keys
    act = I.with_internal_energy(I.smooth_state(spec, keys, seed=14, amp=0.2, vel=0.5))
    say(f"dual energy: {len(keys)} leaves")
    gm, tr, otr = run(spec, act, 1, 6)
    assert gm.nf == 6
