"""Adaptive time stepping: hydro steps with a remesh every few steps.

The remesh (indicator, refine/coarsen with balance and capacity, migration)
runs in the HIP library; this loop only swaps the mesh and state objects."""
from __future__ import annotations

import torch

from .mesh import Mesh


def capacity_from_memory(mesh: Mesh, reserve_bytes: int = 8 << 30) -> int:
    """Largest leaf count whose old and new state fit in free HBM together
    (a remesh holds both while it migrates)."""
    free, _ = torch.cuda.mem_get_info(mesh.device)
    per_block = mesh.info.block_stride * 8
    return max(mesh.nleaf, int((free - reserve_bytes) // (2 * per_block)))


def run(mesh: Mesh, U: torch.Tensor, steps: int, refine_slope=0.3, coarsen_slope=0.1, interval=4,
        max_blocks=None, start=0, on_remesh=None):
    """Advance `steps` steps from step index `start`, remeshing before every
    step index that is a positive multiple of `interval`.  Returns
    (mesh, U, dt list (device tensors), remesh stats list)."""
    dts, stats = [], []
    for k in range(start, start + steps):
        if interval and k > 0 and k % interval == 0:
            cap = max_blocks if max_blocks is not None else capacity_from_memory(mesh)
            new, Un, st = mesh.remesh(U, refine_slope, coarsen_slope, cap)
            mesh, U = new, Un
            stats.append(st)
            if on_remesh is not None:
                on_remesh(k, mesh, U, st)
        dt = torch.zeros(1, dtype=torch.float64, device=mesh.device)
        mesh.step(U, dt, k)
        dts.append(dt)
    return mesh, U, dts, stats
