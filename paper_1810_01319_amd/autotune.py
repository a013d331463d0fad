"""Autotuner of the sweep launch shapes.

For each sweep axis it times the candidate kernels (lane-per-pencil walk at
several workgroup sizes, LDS-staged tile) with HIP events on a scratch copy
of the state and keeps the fastest.  Every candidate computes bitwise the
same result, so tuning never changes answers.  Results are cached in JSON
keyed by device name, block size and mesh shape.
"""
from __future__ import annotations

import json
import os

import torch

CANDIDATES = [(0, 64), (0, 128), (0, 256), (1, 128)]  # (sweep_mode, sweep_block)


def _cache_path() -> str:
    return os.environ.get("AMR_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "amr_mi355x", "tune.json"))


def _key(mesh) -> str:
    name = torch.cuda.get_device_name(mesh.device)
    lv = list(mesh.info.levels[:8])
    return f"{name}|N{mesh.N}|leaves{mesh.nleaf}|levels{lv}"


def _time_axis(mesh, U, dt, axis, steps, scratch=None):
    """Mean ms of the given axis' sweep over `steps` steps (both parities)."""
    if scratch is not None:
        work = scratch[:U.numel()].view(U.shape)
        work.copy_(U)
    else:
        work = U.clone()
    mesh.step(work, dt, 0)  # warm-up
    mesh.profile(True)
    for k in range(steps):
        mesh.step(work, dt, k + 1)
    prof = mesh.profile_read()
    mesh.profile(False)
    ms, n = prof[("sweep_x", "sweep_y", "sweep_z")[axis]]
    return ms / max(n, 1)


def tune(mesh, U, steps: int = 2, use_cache: bool = True, scratch=None) -> dict:
    """Choose per-axis sweep kernels for this mesh; applies and returns the
    launch configuration."""
    key = _key(mesh)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        cfg = cache[key]
        mesh.set_launch(sweep_mode=cfg["sweep_mode"], sweep_block=cfg["sweep_block"])
        return cfg
    dt = torch.zeros(1, dtype=torch.float64, device=mesh.device)
    base = mesh.get_launch()
    best_mode = list(base["sweep_mode"])
    best_block = base["sweep_block"]
    timings = {}
    for axis in range(3):
        best = None
        for mode, block in CANDIDATES:
            modes = list(best_mode)
            modes[axis] = mode
            mesh.set_launch(sweep_mode=modes, sweep_block=block if mode == 0 else best_block)
            t = _time_axis(mesh, U, dt, axis, steps, scratch)
            timings[f"axis{axis}_mode{mode}_block{block}"] = t
            if best is None or t < best[0]:
                best = (t, mode, block)
        best_mode[axis] = best[1]
        if best[1] == 0:
            best_block = best[2]
    # one workgroup size serves every walk axis: re-check it against the others
    mesh.set_launch(sweep_mode=best_mode, sweep_block=best_block)
    cfg = {"sweep_mode": best_mode, "sweep_block": best_block, "timings_ms": timings}
    if use_cache:
        cache[key] = cfg
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return cfg
