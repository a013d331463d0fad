"""Adaptive time stepping: hydro steps with a remesh every few steps.

The remesh (indicator, refine/coarsen with balance and capacity, migration)
runs in the HIP library; this loop only swaps the mesh and state objects."""
from __future__ import annotations

import torch

from .mesh import Mesh


def capacity_from_memory(mesh: Mesh, reserve_bytes: int = 24 << 30) -> int:
    """Largest leaf count such that an old and a new state of that size fit in
    the device's HBM together (a remesh holds both while it migrates)."""
    total = torch.cuda.get_device_properties(mesh.device).total_memory
    per_block = mesh.info.block_stride * 8
    return max(mesh.nleaf, int((total - reserve_bytes) // (2 * per_block)))


class StatePool:
    """Two fixed state arenas of `capacity` blocks each, allocated once: a
    remesh migrates from the arena holding the current state into the other,
    so an adaptive run allocates no device memory after start-up and the
    allocator cannot fragment the 288 GB of HBM."""

    def __init__(self, mesh: Mesh, capacity: int):
        n = capacity * mesh.info.block_stride
        self.capacity = capacity
        self.bufs = [torch.empty(n, dtype=torch.float64, device=mesh.device) for _ in range(2)]
        self.cur = 0

    def initial(self, mesh: Mesh, fn) -> torch.Tensor:
        return mesh.state_from_blocks(fn, out=self.bufs[self.cur])

    def other(self) -> torch.Tensor:
        return self.bufs[1 - self.cur]

    def swap(self) -> None:
        self.cur = 1 - self.cur


def run(mesh: Mesh, U: torch.Tensor, steps: int, refine_slope=0.3, coarsen_slope=0.1, interval=4,
        max_blocks=None, start=0, on_remesh=None, pool: StatePool = None):
    """Advance `steps` steps from step index `start`, remeshing before every
    step index that is a positive multiple of `interval`.  The steps between
    two remeshes run as one multi-step call; after a remesh that changed
    nothing (which refreshed the state's ghosts) that call skips its first
    refresh, unless `on_remesh` is given: the callback may write U's
    active cells (sources, re-seeding), so its ghosts are refreshed again.
    Returns (mesh, U, dt list (device tensors of n_instances
    doubles, one per step), remesh stats list)."""
    dts, stats = [], []
    k, end = start, start + steps
    while k < end:
        fresh = False
        if interval and k > 0 and k % interval == 0:
            cap = max_blocks if max_blocks is not None else capacity_from_memory(mesh)
            if pool is not None:
                cap = min(cap, pool.capacity)
                new, Un, st = mesh.remesh(U, refine_slope, coarsen_slope, cap, out=pool.other())
                if new is not mesh:
                    pool.swap()
            else:
                new, Un, st = mesh.remesh(U, refine_slope, coarsen_slope, cap)
            fresh = new is mesh and on_remesh is None
            mesh, U = new, Un
            stats.append(st)
            if on_remesh is not None:
                on_remesh(k, mesh, U, st)
        n = min(end, (k // interval + 1) * interval) - k if interval else end - k
        seg = torch.zeros(n, mesh.n_instances, dtype=torch.float64, device=mesh.device)
        mesh.steps(U, seg, n, k, ghosts_fresh=fresh)
        dts.extend(seg[i] for i in range(n))
        k += n
    return mesh, U, dts, stats
