"""Algorithmic operation and byte counts of the step's kernels.

Flops are FP64 operations (+, -, *, /, sqrt; comparisons, selects, |x| and
negation not counted) of the sweep's formulas as the oracle writes them.  Two
counts: the per-block constants below give each block's longest path (the
branch arms that evaluate the most operations), so `sweep_flops_per_pencil`
bounds any pencil; `SWEEP_OPS_MEAN` holds the mean the oracle actually
executes per pencil on a benchmark workload's states (branches as the data
take them), measured by the oracle's instrumented build and used for the FP64
roof.  The CPU tests pin both against that instrumented count.  Bytes are the
FP64 values a kernel must read and write in HBM at minimum (each input once,
each output once).
"""
from __future__ import annotations

FIELDS = 5
GHOST = 3
DOUBLE = 8

# per unit of the sweep, longest path (see the formulas of the PPM pencil)
PRIMITIVES = 16          # 1/rho, u v w, kinetic sum, p, c
SLOPES = 5 * 7           # MC-limited slope of 5 primitives (5 where it is zero)
FACE_VALUES = 5 * 5      # fourth-order face value of 5 primitives
FLATTEN = 7              # shock detector and pressure-ratio ramp
# flattening blend 8, monotonicity test 3, D and the first case test 7, the
# second case test 3, steepening 3, dq 1, q6 4
PARABOLAS = 5 * 29
# eigen-quantities 9 (one reciprocal of c); the edge all three waves move
# towards: 3 Courant numbers, 9 parabola means of 7, the two projections 5 + 4,
# the edge state 6 = 81; the other edge then has none moving towards it: 3, 3
# means at zero speed 21, the edge state 6, the transverse means 14 = 44
TRACE = 9 + 81 + 44
TRACED_CELL = FLATTEN + PARABOLAS + TRACE


def riemann_flops(iters: int) -> int:
    """Two-shock solve and flux at one interface: setup 17 (C_K, 1/p_K, first
    p*), (iters+1) evaluations of mass fluxes, their reciprocals, star
    velocities and reciprocal impedances (30 each), iters Newton updates (4
    each), u* 5, star density 6, sampling 23 (fan arm), flux 15."""
    return 17 + (iters + 1) * 30 + iters * 4 + 5 + 6 + 23 + 15


UPDATE = 5 * 3 + 15      # conservative update; 1/rho, u v w, ke, p and the energy floor


def sweep_flops_per_pencil(N: int, iters: int = 5) -> int:
    M = N + 2 * GHOST
    return (M * PRIMITIVES + (M - 2) * SLOPES + (M - 3) * FACE_VALUES + (M - 4) * TRACED_CELL
            + (N + 1) * riemann_flops(iters) + N * UPDATE)


# Mean FP64 operations per pencil sweep (fluxes, update and floors) that the
# oracle executes on states of a workload, (workload, N, Newton steps) ->
# mean; the sample (states, pencils, seed) is recorded with the same numbers
# in the golden file the measurement writes.
SWEEP_OPS_MEAN = {
    ("sedov", 32, 5): 17882.5,   # Sedov static mesh, states before steps 1 and 10
    ("blasts", 32, 5): 18095.2,  # 4^3-octree tile of the blast array, states before steps 5 and 9
}


def sweep_ops_per_pencil(workload: str, N: int, iters: int = 5) -> float:
    """The oracle's mean executed operations per pencil on `workload`, or the
    longest-path bound where no measurement exists."""
    m = SWEEP_OPS_MEAN.get((workload, N, iters))
    return float(m) if m is not None else float(sweep_flops_per_pencil(N, iters))


def sweep_pencils_per_block(N: int) -> dict:
    """Pencils of each sweep of a step, in sweep order: the first sweep runs
    over all transverse cells, the second over active cells of the first
    axis, the third over active cells only."""
    M = N + 2 * GHOST
    return {"first": M * M, "second": N * M, "third": N * N}


def sweep_flops_per_block_step(N: int, iters: int = 5) -> int:
    return sum(sweep_pencils_per_block(N).values()) * sweep_flops_per_pencil(N, iters)


def sweep_bytes_per_pencil(N: int) -> int:
    """Read the pencil's M cells and write its N updated cells, 5 fields."""
    M = N + 2 * GHOST
    return FIELDS * DOUBLE * (M + N)


def sweep_bytes_per_block_step(N: int) -> int:
    return sum(sweep_pencils_per_block(N).values()) * sweep_bytes_per_pencil(N)


def refresh_bytes_per_block(N: int) -> int:
    """Same-level refresh: read and write every ghost cell's 5 fields."""
    M = N + 2 * GHOST
    return 2 * FIELDS * DOUBLE * (M ** 3 - N ** 3)


def cfl_bytes_per_block(N: int) -> int:
    return FIELDS * DOUBLE * N ** 3
