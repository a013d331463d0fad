"""Algorithmic operation and byte counts of the step's kernels.

Flops are the distinct FP64 operations (+, -, *, /, sqrt; comparisons,
selects, |x| and negation not counted) that the sweep's formulas evaluate,
each common subexpression once, taking the longer arm where the formulas
branch.  Bytes are the FP64 values a kernel must read and write in HBM at
minimum (each input once, each output once).
"""
from __future__ import annotations

FIELDS = 5
GHOST = 3
DOUBLE = 8

# per unit of the sweep (see the formulas of the PPM pencil)
PRIMITIVES = 16          # 1/rho, u v w, kinetic sum, p, floor, c
SLOPES = 5 * 7           # MC-limited slope of 5 primitives
FACE_VALUES = 5 * 5      # fourth-order face value of 5 primitives
FLATTEN = 7              # shock detector and pressure-ratio ramp
PARABOLAS = 5 * 24       # flattening blend, monotonicity, dq and q6
TRACE = 9 + 2 * 63       # eigen-quantities (one reciprocal of c), then both edges
TRACED_CELL = FLATTEN + PARABOLAS + TRACE


def riemann_flops(iters: int) -> int:
    """Two-shock solve and flux at one interface: setup 17 (C_K, 1/p_K, first
    p*), (iters+1) evaluations of mass fluxes, their reciprocals, star
    velocities and reciprocal impedances (30 each), iters Newton updates (4
    each), u* 5, star density 6, sampling 23 (fan arm), flux 15."""
    return 17 + (iters + 1) * 30 + iters * 4 + 5 + 6 + 23 + 15


UPDATE = 5 * 3 + 13      # conservative update, post-update floor test


def sweep_flops_per_pencil(N: int, iters: int = 5) -> int:
    M = N + 2 * GHOST
    return (M * PRIMITIVES + (M - 2) * SLOPES + (M - 3) * FACE_VALUES + (M - 4) * TRACED_CELL
            + (N + 1) * riemann_flops(iters) + N * UPDATE)


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
