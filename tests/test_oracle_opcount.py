"""The FP64 operation counts behind the FP64 roof, pinned to the oracle's
instrumented build (``oracle/opcount.cpp``: the oracle's own pencil and cell
update compiled with a counting number type).

* Each block's longest path, as the cost model states it, is the largest count
  the instrumented oracle reaches for that block over many seeded inputs, and
  its shorter paths are the counts the formulas give for the branch taken.
* A whole pencil sweep counts exactly its blocks plus the inline face values
  and flattening (uniform states at rest and in supersonic flow, where every
  branch is known), and no pencil exceeds the cost model's bound.
* The counting build changes no value: its Riemann fluxes equal the oracle's
  bit for bit.
* The per-workload means the benchmark uses equal the stored measurement.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_01319_amd import costs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sweep_ops_mean.json")
GAMMA = 5.0 / 3.0


def random_state(rng, supersonic=False):
    rho, p = rng.uniform(0.1, 3.0), rng.uniform(0.05, 3.0)
    c = np.sqrt(GAMMA * p / rho)
    u = rng.uniform(-3.0, 3.0) * c if supersonic else rng.uniform(-0.9, 0.9) * c
    return np.array([rho, u, rng.uniform(-1, 1), rng.uniform(-1, 1), p])


@pytest.mark.parametrize("iters", [0, 1, 3, 5, 6])
def test_riemann_longest_path_is_the_cost_model(iters):
    rng = np.random.default_rng(100 + iters)
    seen = set()
    for _ in range(3000):
        WL, WR = random_state(rng, True), random_state(rng, True)
        seen.add(O.count_riemann_ops(WL, WR, gamma=GAMMA, iters=iters)["total"])
    # sampled inside a rarefaction fan is the longest arm (23 operations);
    # the star or outer state beside a rarefaction skips the fan's
    # interpolation (11), the sampling beside a shock takes 4
    assert max(seen) == costs.riemann_flops(iters)
    assert costs.riemann_flops(iters) - 11 in seen


def test_counting_changes_no_value():
    rng = np.random.default_rng(7)
    for _ in range(200):
        WL, WR = random_state(rng, True), random_state(rng, True)
        _, flux, _, _ = O.riemann(WL, WR, gamma=GAMMA, p_floor=1e-20, iters=5)
        assert np.array_equal(O.count_riemann_ops(WL, WR, gamma=GAMMA, iters=5)["flux"], flux)


def test_block_longest_paths_are_the_cost_model():
    rng = np.random.default_rng(8)
    prim = {O.count_block_ops("primitives", np.r_[rng.uniform(0.1, 2), rng.uniform(-1, 1, 3), rng.uniform(2, 4)],
                              gamma=GAMMA)["total"] for _ in range(50)}
    assert prim == {costs.PRIMITIVES}
    assert O.count_block_ops("slope", [1.0, 2.0, 3.5])["total"] == costs.SLOPES // 5
    assert O.count_block_ops("slope", [1.0, 2.0, 1.5])["total"] == costs.SLOPES // 5 - 2  # extremum: zero
    par = {O.count_block_ops("parabola", [1.0, *rng.uniform(0.0, 2.0, 2), rng.choice([0.0, 0.4])])["total"]
           for _ in range(400)}
    # flat (an extremum), no steepening or the first case, the second case
    assert par == {16, costs.PARABOLAS // 5 - 3, costs.PARABOLAS // 5}

    def trace(u_over_c):
        rho, p = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
        c = np.sqrt(GAMMA * p / rho)
        u = u_over_c * c
        q = [rho, u, 0.3, -0.2, p]
        vals = [rho, rho * u, rho * 0.3, rho * -0.2, p / (GAMMA - 1) + 0.5 * rho * (u * u + 0.13)]
        for v in range(5):
            vals += [q[v] - 0.1, q[v] + 0.2, 0.0]
        return O.count_block_ops("trace", vals, nu=0.3, gamma=GAMMA)["total"]

    counts = {s: trace(s) for s in (-3.0, -0.5, 0.0, 0.5, 3.0)}
    assert max(counts.values()) == costs.TRACE
    assert counts[3.0] == counts[-3.0] == costs.TRACE
    assert counts[0.5] == counts[-0.5] < costs.TRACE
    upd = O.count_block_ops("update", [1, 0, 0, 0, 2] + [0] * 10, nu=0.1, gamma=GAMMA)["total"]
    both = O.count_block_ops("update", [1e-30, 0, 0, 0, 1e-30] + [0] * 10, nu=0.1, gamma=GAMMA,
                             rho_floor=1e-20, p_floor=1e-20)["total"]
    assert both == costs.UPDATE and upd == costs.UPDATE - 2  # the energy floor adds p_floor/(g-1) + ke


@pytest.mark.parametrize("mach", [0.0, 3.0])
def test_uniform_pencil_counts_its_blocks(mach):
    """Every branch of a uniform pencil is known: slopes are zero, parabolas
    flat, the flattening finds no shock and no pressure difference.  The
    sweep's count is its blocks' counts on that path plus the inline face
    values (5 per primitive) and flattening (5 on this path)."""
    N, M = 32, 38
    rho, p = 1.3, 0.7
    u = mach * np.sqrt(GAMMA * p / rho)
    E = p / (GAMMA - 1) + 0.5 * rho * u * u
    U = np.array([[rho] * M, [rho * u] * M, [0.0] * M, [0.0] * M, [E] * M])
    got = O.count_sweep_ops(U, 0.2, gamma=GAMMA)["total"]
    W = [rho, u, 0.0, 0.0, p]
    blk = {
        "prim": O.count_block_ops("primitives", U[:, 0], gamma=GAMMA)["total"],
        "slope": O.count_block_ops("slope", [p, p, p])["total"],
        "para": O.count_block_ops("parabola", [p, p, p, 0.0])["total"],
        "trace": O.count_block_ops("trace", list(U[:, 0]) + sum(([w, w, 0.0] for w in W), []), nu=0.2,
                                   gamma=GAMMA)["total"],
        "riemann": O.count_riemann_ops(W, W, gamma=GAMMA, iters=5)["total"],
        "update": O.count_block_ops("update", list(U[:, 0]) + [1.0] * 10, nu=0.2, gamma=GAMMA)["total"],
    }
    want = (M * blk["prim"] + (M - 2) * 5 * blk["slope"] + (M - 3) * 5 * 5
            + (M - 4) * (5 + 5 * blk["para"] + blk["trace"]) + (N + 1) * blk["riemann"] + N * blk["update"])
    assert got == want
    assert blk["trace"] == (costs.TRACE if mach > 1 else 97)


def test_no_pencil_exceeds_the_bound():
    rng = np.random.default_rng(9)
    N, M = 32, 38
    x = np.arange(M) / M
    bound = costs.sweep_flops_per_pencil(N, 5)
    worst = 0
    for t in range(150):
        rho = 1.0 + 0.5 * np.sin(2 * np.pi * (x * rng.integers(1, 6) + rng.uniform()))
        p = 1.0 + 0.5 * np.cos(2 * np.pi * (x * rng.integers(1, 6) + rng.uniform()))
        if t % 3 == 0:  # a jump
            j = rng.integers(8, M - 8)
            rho[j:] *= rng.uniform(0.1, 0.5)
            p[j:] *= rng.uniform(0.01, 0.2)
        u = rng.uniform(-3, 3) * np.sqrt(GAMMA * p / rho) * (0.5 + 0.5 * np.sin(2 * np.pi * x))
        v, w = rng.uniform(-1, 1, (2, M))
        U = np.array([rho, rho * u, rho * v, rho * w, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)])
        c = O.count_sweep_ops(U, 0.1, gamma=GAMMA)["total"]
        assert c <= bound
        worst = max(worst, c)
    assert worst > 0.85 * bound


def test_workload_means_are_the_stored_measurement():
    with open(GOLDEN) as f:
        g = json.load(f)
    for name in ("sedov", "blasts"):
        rec = g[name]
        key = (name, rec["block_cells"], rec["riemann_iters"])
        assert costs.SWEEP_OPS_MEAN[key] == rec["mean_ops_per_pencil"]
        assert rec["bound_ops_per_pencil"] == costs.sweep_flops_per_pencil(rec["block_cells"], rec["riemann_iters"])
        assert rec["min"] <= rec["mean_ops_per_pencil"] <= rec["max"] <= rec["bound_ops_per_pencil"]
        assert costs.sweep_ops_per_pencil(name, 32, 5) == rec["mean_ops_per_pencil"]
    assert costs.sweep_ops_per_pencil("sod", 16, 5) == costs.sweep_flops_per_pencil(16, 5)
