"""Mean FP64 operations per pencil sweep that the oracle executes on the
benchmark's workloads: the algorithmic flop count of the FP64 roof.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  The counts come from the oracle's own
pencil and cell update compiled with a counting number type (``opcount.cpp``):
every +, -, *, / and sqrt the oracle's formulas evaluate on the pencil's data,
with the fixed Newton count, so branches not taken (limiters that return zero,
flat parabolas, waves moving away from an edge, the Riemann sampling region)
count nothing.  The states are the oracle's own runs of the workloads
(``paper_1810_01319_amd.inputs``); pencils are drawn with a seeded generator
along all three axes over every transverse position of a leaf (ghost rows
included, as a step's first sweep sees them) from the refreshed state, with
the next step's dt.

Run ``python -m oracle.sweep_ops`` from the repository root to rewrite
``tests/golden/sweep_ops_mean.json``; ``paper_1810_01319_amd.costs`` carries
the same numbers and a CPU test keeps the two equal.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "tests", "golden", "sweep_ops_mean.json")
PENCILS_PER_AXIS = 1000


def sample_pencils(m, spec, rng, per_axis=PENCILS_PER_AXIS):
    """Counted operations of `per_axis` random pencils along each axis of the
    refreshed state of oracle mesh `m`, with nu from the mesh's next dt."""
    G, N, M = O.GHOST, m.N, m.M
    kw = spec.kwargs()
    m.refresh()
    dt = m.cfl_dt()
    totals = []
    for d in range(3):
        fields = [0, 1 + d, 1 + (d + 1) % 3, 1 + (d + 2) % 3, 4]  # rho, m_normal, m_t1, m_t2, E
        for _ in range(per_axis):
            s = int(rng.integers(m.nleaf))
            a, b = (int(v) for v in rng.integers(0, M, 2))
            dx = 1.0 / (spec.root[0] * N * 2 ** int(m.keys[s][0]))
            B = m.U[s]
            pen = (B[:, b, a, :], B[:, b, :, a], B[:, :, b, a])[d][fields]
            c = O.count_sweep_ops(pen, dt / dx, gamma=kw["gamma"], rho_floor=kw["rho_floor"],
                                  p_floor=kw["p_floor"], iters=kw["riemann_iters"])
            totals.append(c["total"])
    return totals


def sedov(rng):
    from paper_1810_01319_amd import inputs as I

    spec = I.sedov_spec(root=8, block_cells=32, levels=2)
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(I.sedov_state(spec, m.keys))
    totals, at = [], []
    for k in range(11):
        if k in (1, 10):
            totals += sample_pencils(m, spec, rng)
            at.append(k)
        m.step(k)
    return spec, totals, (f"sedov-static-amr (624 leaves x 32^3), states before steps {at}, "
                          f"{PENCILS_PER_AXIS} pencils per axis each")


def blasts(rng):
    from paper_1810_01319_amd import inputs as I

    spec = I.blasts_spec(root=4, block_cells=32, levels=3)
    m = O.OracleMesh(**spec.kwargs())
    m.set_active(I.blasts_state(spec, m.keys))
    totals, at = [], []
    for k in range(10):
        if k > 0 and k % 4 == 0:
            m, _ = m.remesh(0.3, 0.1, 10 ** 9)
        if k in (5, 9):
            totals += sample_pencils(m, spec, rng)
            at.append(k)
        m.step(k)
    return spec, totals, (f"4^3-octree tile of the blast-array-adaptive workload (32^3 blocks, 3 levels, remesh "
                          f"every 4 steps), states before steps {at} ({m.nleaf} leaves at the end), "
                          f"{PENCILS_PER_AXIS} pencils per axis each")


def main() -> int:
    from paper_1810_01319_amd import costs

    out = {}
    for name, fn, seed in (("sedov", sedov, 11), ("blasts", blasts, 12)):
        rng = np.random.default_rng(seed)
        spec, totals, sample = fn(rng)
        t = np.asarray(totals, dtype=np.float64)
        out[name] = {"block_cells": spec.block_cells, "riemann_iters": spec.kwargs()["riemann_iters"],
                     "mean_ops_per_pencil": round(float(t.mean()), 1), "min": int(t.min()), "max": int(t.max()),
                     "pencils": int(t.size), "seed": seed,
                     "bound_ops_per_pencil": costs.sweep_flops_per_pencil(spec.block_cells, 5),
                     "sample": sample}
        print(name, out[name], flush=True)
    with open(GOLDEN, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
