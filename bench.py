#!/usr/bin/env python3
"""Throughput of the AMR hydro step on one MI355X.

Headline workload (the default): the large adaptive blast array, one GPU's
share of the paper's weak-scaling shape -- 24^3 root octrees of 32^3-cell
blocks (453M cells at start), one Sedov blast per octree at a seeded offset,
up to 3 levels by density slope (refine > 0.3, coarsen < 0.1), remesh every
4 steps, gamma 5/3, FP64, periodic.  One step = CFL reduction + two-phase
ghost refresh + three PPM sweeps + reflux over every leaf; the remesh
(indicator, host decisions, migration) is inside the timed region.  Inputs
are generated on the host, uploaded once and resident in HBM before timing.

Prints one JSON line: cell-updates/s, the dominant kernel's roofline (live
HIP-event timing of every kernel over the timed region, HBM and FP64
fractions, the higher one binding), the FP64 CPU oracle on a bounded tile
of the same workload, and sub-objects for the other workloads: the static
two-level Sedov mesh, the batched uneven meshes, the adjoint, tracers,
comoving and dual-energy steps, mg0 and self-gravity.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per PPM step incl. ghost refresh (plain vs batched); adjoint/fwd"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector, published
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, published


def kernel_source_hash() -> str:
    """sha256 over the sources the sweep kernels are compiled from."""
    import hashlib

    h = hashlib.sha256()
    for f in ("kernels.hip", "ppm_core.hpp", "layout.hpp", "ghost.hpp", "xcd.hpp"):
        with open(os.path.join(ROOT, "paper_1810_01319_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_counters(kernel: str, workload_name: str, what: str) -> dict:
    """key: value lines of the committed rocprofv3 counter summary
    profiles/<kernel>_<workload>_<what>.txt, or {} if there is none or the
    kernel sources changed since the counters were taken."""
    name = kernel.replace("<", "_").replace(">", "").replace(",", "_")
    path = os.path.join(ROOT, "profiles", f"{name}_{workload_name}_{what}.txt")
    if not os.path.exists(path):
        return {}
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return kv


def measured_traffic(kernel: str, workload_name: str):
    """HBM bytes per launch of `kernel` (FETCH_SIZE and WRITE_SIZE per
    dispatch, scaled by the same counters' reading for a copy of known size),
    or None."""
    kv = committed_counters(kernel, workload_name, "traffic")
    return float(kv["hbm_bytes_per_launch"]) if kv else None


def workload(name):
    from paper_1810_01319_amd import inputs as I

    if name == "sedov":
        spec = I.sedov_spec(root=8, block_cells=32, levels=2)
        desc = ("sedov-static-amr: 8^3 root octrees x 32^3 cells, 2 refinement levels at the centre "
                "(624 leaves, 20.4M cells), gamma 5/3, periodic, E=1 in r<2 finest cells")
        return spec, I.sedov_state, desc
    if name == "blasts":
        spec = I.blasts_spec(root=24, block_cells=32, levels=3)
        desc = ("blast-array-adaptive: 24^3 root octrees x 32^3 cells (453M cells at start), one blast per "
                "octree at seeded offsets, up to 3 levels by density slope (refine > 0.3, coarsen < 0.1), "
                "remesh every 4 steps, gamma 5/3, periodic")
        return spec, I.blasts_state, desc
    if name == "sod":
        spec = I.sod_spec()
        return spec, I.sod_state, "sod-uniform: 4^3 x 16^3 cells, outflow, gamma 1.4"
    raise SystemExit(f"unknown workload {name}")


def sweep_roofline(prof, step_leaves, N, nf, launch, workload_name, iters=5):
    """Roofline of the three sweep kernels over a timed region.

    step_leaves: (step index, leaf count) of every timed step; a sweep's
    pencils per leaf depend on its place in that step's order (x, y, z on
    even steps, z, y, x on odd ones).  Per launch: algorithmic bytes (read
    the pencil's M cells and write its N cells, 5 fields of 8 B) and
    algorithmic flops (the oracle's mean executed operations per pencil on
    this workload, else the cost model's longest-path count), divided by the
    kernel's mean launch time from the library's HIP events.  Returns
    (per-axis table, dominant axis)."""
    from paper_1810_01319_amd import costs

    pen = costs.sweep_pencils_per_block(N)
    fpp = costs.sweep_ops_per_pencil(workload_name, N, iters)
    bpp = costs.sweep_bytes_per_pencil(N)
    axes = ("x", "y", "z")
    per_axis = {}
    for a in range(3):
        pencils = 0
        for k, leaves in step_leaves:
            order = (0, 1, 2) if k % 2 == 0 else (2, 1, 0)
            pencils += leaves * (pen["first"], pen["second"], pen["third"])[order.index(a)]
        ms, n = prof["sweep_" + axes[a]]
        sec = ms / n * 1e-3
        flops = fpp * pencils / n
        byts = bpp * pencils / n
        kname = ("sweep_staged" if launch["sweep_mode"][a] == 1 else "sweep_kernel") + f"<{N},{a},{nf}>"
        per_axis[axes[a]] = {"kernel": kname, "avg_launch_ms": ms / n, "launches": n,
                             "flops_per_launch": flops, "TFLOP/s": flops / sec / 1e12,
                             "fp64_frac": flops / sec / 1e12 / PEAK_FP64_TFLOPS,
                             "algorithmic_bytes_per_launch": byts, "GB/s": byts / sec / 1e9,
                             "hbm_frac": byts / sec / 1e9 / PEAK_HBM_GBS}
    dom = max(per_axis, key=lambda a: per_axis[a]["avg_launch_ms"])
    return per_axis, dom


def roofline_object(d: dict, workload_name: str) -> dict:
    """The dominant kernel's roofline: its algorithmic HBM rate and its
    algorithmic FP64 rate against the published peaks; the binding roof is
    the one with the higher fraction.  `traffic` is the committed rocprofv3
    FETCH_SIZE + WRITE_SIZE per launch (scaled by a plain copy's reading),
    or None once the kernel sources have changed since it was taken."""
    traffic = measured_traffic(d["kernel"], workload_name)
    hbm = {"bound": "hbm", "achieved": d["GB/s"], "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": d["hbm_frac"]}
    alu = {"bound": "alu", "achieved": d["TFLOP/s"], "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
           "frac": d["fp64_frac"]}
    top, other = (hbm, alu) if hbm["frac"] >= alu["frac"] else (alu, hbm)
    out = dict(top)
    out.update({"traffic": traffic, "kernel": d["kernel"], "avg_launch_ms": d["avg_launch_ms"],
                "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"],
                "flops_per_launch": d["flops_per_launch"],
                "other_roof": other})
    sec = d["avg_launch_ms"] * 1e-3
    if traffic is not None:
        out["traffic_over_algorithmic"] = traffic / d["algorithmic_bytes_per_launch"]
        out["traffic_hbm_frac"] = traffic / sec / 1e9 / PEAK_HBM_GBS  # measured bytes, not algorithmic
    valu = committed_counters(d["kernel"], workload_name, "valu")
    if valu:
        out["valu_busy"] = float(valu["valu_busy"])
        out["valu_issue_frac"] = float(valu["valu_insts_per_launch"]) * 4 / (sec * 1024 * 2.4e9)
        if "fp64_flops_executed_per_launch" in valu:
            # executed FP64 operations (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes): divisions and square
            # roots as their Newton-Raphson / Goldschmidt sequences, divergent branches both arms
            ex = float(valu["fp64_flops_executed_per_launch"]) / sec / 1e12
            out["fp64_executed"] = {"TFLOP/s": ex, "frac": ex / PEAK_FP64_TFLOPS}
    return out


def cpu_baseline(spec, act_fn, min_seconds, max_steps=200):
    """The oracle as it stands, on this host's cores: whole steps of the same
    workload after one warm-up step, until at least `min_seconds` have passed
    (a bounded sample of the timed workload)."""
    from oracle import oracle as O

    m = O.OracleMesh(**spec.kwargs())
    m.set_active(act_fn(spec, m.keys))
    m.step(0)
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_seconds):
        steps += 1
        m.step(steps)
    t = time.perf_counter() - t0
    cells = m.nleaf * spec.block_cells ** 3
    return {"value": cells * steps / t, "unit": "cell-updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of the same workload ({m.nleaf} leaves, {cells} cells) after 1 warm-up "
                      f"step, {t:.1f} s"}


def batched_compare(steps: int, n_inst: int = 256):
    """The batched workload: n_inst independent meshes of uneven size in one
    flat worklist (two steps, the second's CFL fused into the first,
    captured in a HIP graph) against the same meshes stepped one mesh per
    launch sequence (two fused steps per call)."""
    import numpy as np
    import torch

    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh

    inst = [I.batch_instance(i) for i in range(n_inst)]
    bm = Mesh.batch([sp.kwargs() for sp, _ in inst])
    acts = [I.batch_state(sp, bm.keys[bm.first_leaf[i]:bm.first_leaf[i + 1]], c) for i, (sp, c) in enumerate(inst)]
    cells = bm.nleaf * bm.N ** 3
    side = torch.cuda.Stream()
    out = {"instances": n_inst, "leaves": int(bm.nleaf), "cells": int(cells), "steps": steps}
    with torch.cuda.stream(side):
        U = torch.empty((bm.nleaf, 5, bm.M, bm.M, bm.M), dtype=torch.float64, device=bm.device)
        g3 = 3
        for i, a in enumerate(acts):
            U[bm.first_leaf[i]:bm.first_leaf[i + 1], :, g3:g3 + bm.N, g3:g3 + bm.N, g3:g3 + bm.N] = \
                torch.from_numpy(a).to(bm.device)
        dt = bm.dt_tensor()
        dt2 = torch.zeros(2 * bm.n_instances, dtype=torch.float64, device=bm.device)
        # eager batched steps, two per call as in the graph (fewer: for reference only)
        eager = max(2, min(steps, 20)) // 2 * 2
        bm.steps(U, dt2, 2, 0)
        side.synchronize()
        t0 = time.perf_counter()
        for k in range(2, eager + 2, 2):
            bm.steps(U, dt2, 2, k)
        side.synchronize()
        out["batched_eager"] = cells * eager / (time.perf_counter() - t0)
        # graph of two steps
        g = bm.graph(U, dt, first_step=0)
        g.launch()
        side.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // 2):
            g.launch()
        side.synchronize()
        out["batched_graph"] = cells * 2 * (steps // 2) / (time.perf_counter() - t0)
        del g
        # one mesh per launch sequence, two fused steps per call
        meshes = []
        for i, (sp, _) in enumerate(inst):
            m = Mesh(**sp.kwargs())
            um = m.state_from_active(acts[i])
            meshes.append((m, um, torch.zeros(2, dtype=torch.float64, device=m.device)))
        for m, um, dtm in meshes:
            m.steps(um, dtm, 2, 0)
        side.synchronize()
        t0 = time.perf_counter()
        for k in range(2, 2 * (steps // 2) + 2, 2):
            for m, um, dtm in meshes:
                m.steps(um, dtm, 2, k)
        side.synchronize()
        out["per_mesh_launch"] = cells * 2 * (steps // 2) / (time.perf_counter() - t0)
    out["speedup_graph_vs_per_mesh"] = out["batched_graph"] / out["per_mesh_launch"]
    return out


def adjoint_compare(steps: int = 10, reps: int = 3):
    """The differentiation workload (4^3 root octrees of 32^3 cells, the
    central 2^3 roots refined once: 120 leaves, 3.9M cells; density misfit
    after `steps` steps): wall time of the plain forward, and of the
    differentiable forward and the hand-written adjoint in both modes
    (recording the sweep inputs, or checkpointing and recomputing them),
    best of `reps`.  adjoint_over_forward divides the adjoint by the plain
    forward; adjoint_over_own_forward by the differentiable forward it
    follows."""
    import torch

    from paper_1810_01319_amd import adjoint as A
    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh

    spec = I.grf_spec(root=4, block_cells=32)
    m = Mesh(**spec.kwargs())
    N, g3 = spec.block_cells, 3
    base = m.state_from_active(I.grf_state(spec, m.keys, seed=4))
    target = torch.from_numpy(I.grf_density(spec, m.keys, seed=40)).to(m.device)

    def plain():
        U = base.clone()
        for k in range(steps):
            m.step(U, m.dt_tensor(), k)
        return U

    def timed(fn):
        best = None
        for _ in range(reps + 1):  # first call warms up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        return best, r

    t_plain, _ = timed(plain)
    out = {"workload": "grf-density-misfit: 4^3 root octrees x 32^3 cells, central 2^3 roots refined once "
                       f"(120 leaves, 3.9M cells), {steps} steps, gamma 5/3, periodic",
           "steps": steps, "forward_ms": t_plain * 1e3}
    for record in (True, False):
        state = {}

        def fwd():
            r = base[:, 0, g3:g3 + N, g3:g3 + N, g3:g3 + N].clone().requires_grad_(True)
            L = A.density_misfit(m, A.run_steps(A.with_density(base, r), m, steps, record=record), target)
            state["L"], state["r"] = L, r
            return L

        best_f = best_b = None
        for i in range(reps + 1):  # first pass warms up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fwd()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            state["L"].backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if i > 0:
                best_f = t1 - t0 if best_f is None else min(best_f, t1 - t0)
                best_b = t2 - t1 if best_b is None else min(best_b, t2 - t1)
        # one more adjoint pass with per-phase events
        fwd()
        torch.cuda.synchronize()
        m.profile(True)
        state["L"].backward()
        prof = m.profile_read()
        m.profile(False)
        res = {"forward_ms": best_f * 1e3, "adjoint_ms": best_b * 1e3,
               "adjoint_over_forward": best_b / t_plain,
               "adjoint_over_own_forward": best_b / best_f,
               "forward_and_adjoint_over_forward": (best_f + best_b) / t_plain,
               "adjoint_phases_ms_per_step": {p: round(v[0] / steps, 4) for p, v in prof.items()
                                              if p.startswith("adj_")}}
        if record:
            out["adjoint_ms"] = res["adjoint_ms"]
            out["adjoint_over_forward"] = res["adjoint_over_forward"]
            out["adjoint_over_own_forward"] = res["adjoint_over_own_forward"]
            out["recording"] = res
        else:
            out["recomputing"] = res
        del state
    out["dual_energy"] = adjoint_compare_de(steps)
    return out


def adjoint_compare_de(steps: int):
    """The same workload with the dual-energy field (eta1 1e-3, eta2 0.1):
    plain forward, recording forward and adjoint (one timed pass after a
    warm-up)."""
    import dataclasses

    import torch

    from paper_1810_01319_amd import adjoint as A
    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh

    spec = dataclasses.replace(I.grf_spec(root=4, block_cells=32), dual_energy=True, eta1=1e-3, eta2=0.1)
    m = Mesh(**spec.kwargs())
    N, g3 = spec.block_cells, 3
    base = m.state_from_active(I.with_internal_energy(I.grf_state(spec, m.keys, seed=4)))
    target = torch.from_numpy(I.grf_density(spec, m.keys, seed=40)).to(m.device)
    t = {}
    for i in range(2):  # the first pass warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U = base.clone()
        for k in range(steps):
            m.step(U, m.dt_tensor(), k)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = base[:, 0, g3:g3 + N, g3:g3 + N, g3:g3 + N].clone().requires_grad_(True)
        L = A.density_misfit(m, A.run_steps(A.with_density(base, r), m, steps), target)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t = {"forward_ms": (t1 - t0) * 1e3, "recording_forward_ms": (t2 - t1) * 1e3, "adjoint_ms": (t3 - t2) * 1e3}
    t["adjoint_over_forward"] = t["adjoint_ms"] / t["forward_ms"]
    t["workload"] = "the same mesh and state with the dual-energy field (eta1 1e-3, eta2 0.1), recording mode"
    return t


def tracer_compare(steps: int = 20):
    """Tracer particles on the Sedov workload: one particle per active cell
    (20.4M, jittered inside the cell), hydro steps that also advance them,
    against plain steps of the same mesh.  The tracer phase (drift and
    migration kernels) is timed with HIP events."""
    import torch

    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh
    from paper_1810_01319_amd.tracers import Tracers

    spec = I.sedov_spec(root=8, block_cells=32, levels=2)
    m = Mesh(**spec.kwargs())
    U = m.state_from_active(I.sedov_state(spec, m.keys))
    pos, ids = I.tracer_positions(spec, m.keys, 1, jitter_seed=9)
    n = int(ids.size)
    tr = Tracers.from_positions(m, pos, ids, capacity=2 * spec.block_cells ** 3)
    del pos, ids
    dt = m.dt_tensor()
    tr.step(U, dt, 0)
    torch.cuda.synchronize()
    m.profile(True)
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        tr.step(U, dt, k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = m.profile_read()
    m.profile(False)
    tr_ms = prof["tracers"][0] / steps
    c = tr.counters()
    # algorithmic bytes per particle and step: drift reads X, Y, Z and writes
    # them and the destination (52 B); migration reads destination, position,
    # id and writes position and id (68 B); the interpolation reads 4 fields of
    # the cells around it, about one cell per particle at this density (32 B)
    bytes_pp = 52 + 68 + 32
    return {"workload": "sedov-static-amr with one tracer per active cell (20.4M particles)",
            "particles": n, "steps": steps, "ms_per_step_with_tracers": wall * 1e3 / steps,
            "tracer_ms_per_step": tr_ms, "particle_updates_per_s": n / (tr_ms * 1e-3),
            "tracer_hbm": {"algorithmic_bytes_per_particle": bytes_pp,
                           "GB/s": n * bytes_pp / (tr_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS},
            "counters": c, "particles_end": tr.count}


def comoving_compare(steps: int = 20):
    """Comoving steps on the Sedov workload in an Einstein-de Sitter expansion
    (a = t^(2/3), H = 2 / (3 t), from t = 1e-3, a = 0.01), two ways: (1) the
    device-resident run (amr_hydro_steps_comoving: a(t), the comoving CFL dt,
    a and H at the step's mid time all on the device, nothing read back);
    (2) host-driven steps, each reading its CFL dt back to place a and H at
    the step's mid time.  Reports the time per step of both and the
    expansion-source kernel's HBM rate (per active cell: 5 fields read, 4
    written)."""
    import torch

    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh

    spec = I.sedov_spec(root=8, block_cells=32, levels=2)
    m = Mesh(**spec.kwargs())
    U0 = m.state_from_active(I.sedov_state(spec, m.keys))
    cells = m.nleaf * spec.block_cells ** 3
    H0, t_start = 2.0 / 3.0, 1e-3  # a = (3/2 H0 t)^(2/3) = t^(2/3)

    # (1) device-resident
    U = U0.clone()
    cosmo = torch.tensor([t_start, 0.0, 0.0, 0.0], dtype=torch.float64, device=m.device)
    dts = torch.zeros(max(steps, 2), dtype=torch.float64, device=m.device)
    m.steps_comoving(U, dts, 2, 0, cosmo, H0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.steps_comoving(U, dts, steps, 2, cosmo, H0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_end = float(cosmo.cpu()[0])
    m.profile(True)  # per-phase times from one more run
    m.steps_comoving(U, dts, steps, 2 + steps, cosmo, H0)
    prof = m.profile_read()
    m.profile(False)

    # (2) host-driven
    U = U0.clone()
    dt = m.dt_tensor()

    def run(k0, n, t):
        for k in range(k0, k0 + n):
            a = t ** (2.0 / 3.0)
            m.cfl_dt_comoving(U, a, dt)
            d = float(dt.cpu()[0])
            tm = t + 0.5 * d
            m.step_comoving(U, dt, k, tm ** (2.0 / 3.0), 2.0 / (3.0 * tm))
            t += d
        return t

    t = run(0, 2, t_start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(2, steps, t)
    torch.cuda.synchronize()
    wall_host = time.perf_counter() - t0
    ex_ms = prof["expansion"][0] / steps
    bytes_pc = 72
    return {"workload": "sedov-static-amr, comoving, Einstein-de Sitter expansion from a = 0.01",
            "steps": steps, "a_end": t_end ** (2.0 / 3.0), "ms_per_step": wall * 1e3 / steps,
            "cell_updates_per_s": cells * steps / wall, "host_driven_ms_per_step": wall_host * 1e3 / steps,
            "expansion_ms_per_step": ex_ms,
            "expansion_hbm": {"algorithmic_bytes_per_cell": bytes_pc,
                              "GB/s": cells * bytes_pc / (ex_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS},
            "phases_ms_per_step": {p: round(v[0] / steps, 4) for p, v in prof.items() if v[1] > 0}}


def dual_energy_compare(steps: int = 50):
    """The dual-energy variant: (1) the Sedov workload with the sixth field
    rho e (thresholds 1e-3, 0.1), fused runs of steps as in the main line,
    against the same run without it; (2) accuracy on a cold stream: a
    density wave on a Mach 1e5 flow at uniform pressure (E - ke keeps about
    six of the thermal energy's sixteen digits), 20 steps, maximum relative
    deviation of the pressure from the exact uniform value, plain (from E -
    ke) against dual energy (from rho e)."""
    import numpy as np
    import torch

    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh

    out = {}
    spec = I.sedov_spec(root=8, block_cells=32, levels=2)
    for name, sp in (("plain", spec), ("dual_energy", I.with_(spec, dual_energy=True))):
        m = Mesh(**sp.kwargs())
        act = I.sedov_state(sp, m.keys)
        U = m.state_from_active(I.with_internal_energy(act) if sp.dual_energy else act)
        cells = m.nleaf * sp.block_cells ** 3
        dt = torch.zeros(steps * m.n_instances, dtype=torch.float64, device=m.device)
        m.steps(U, dt, 2, 0)
        torch.cuda.synchronize()
        m.profile(True)
        t0 = time.perf_counter()
        m.steps(U, dt, steps, 2)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = m.profile_read()
        m.profile(False)
        out[name] = {"ms_per_step": wall * 1e3 / steps, "cell_updates_per_s": cells * steps / wall,
                     "phases_ms_per_step": {p: round(v[0] / steps, 4) for p, v in prof.items() if v[1] > 0}}
        del U, m
        torch.cuda.empty_cache()
    out["workload"] = "sedov-static-amr (624 leaves x 32^3), gamma 5/3, eta1 1e-3, eta2 0.1"
    out["steps"] = steps
    out["dual_over_plain_time"] = out["dual_energy"]["ms_per_step"] / out["plain"]["ms_per_step"]
    # cold stream accuracy
    cs = I.MeshSpec(root=(4, 4, 1), block_cells=32, gamma=5.0 / 3.0)
    acc = {}
    for name, sp in (("plain", cs), ("dual_energy", I.with_(cs, dual_energy=True))):
        m = Mesh(**sp.kwargs())
        act = I.cold_stream_state(sp, m.keys, mach=1e5)
        U = m.state_from_active(act if sp.dual_energy else act[:, :5])
        dt = torch.zeros(1, dtype=torch.float64, device=m.device)
        for k in range(20):
            m.step(U, dt, k)
        a = m.active(U)
        rho, mom, E = a[:, 0], a[:, 1:4], a[:, 4]
        ke = 0.5 * (mom ** 2).sum(axis=1) / rho
        p = (sp.gamma - 1.0) * (a[:, 5] if sp.dual_energy else E - ke)
        acc[name] = float(np.max(np.abs(p - 1.0)))
        del U, m
    out["cold_stream"] = {"workload": "density wave on a uniform Mach 1e5 stream, 16 leaves x 32^3, 20 steps",
                          "max_rel_pressure_error": acc}
    return out


def mg0_compare(cycles: int = 10):
    """The mg0 Poisson solver on a uniform periodic mesh of 16^3 root octrees x
    32^3 cells (512^3 cells; the paper's uniform-mesh self-gravity shape on
    one GPU): V(2,2) cycles on a seeded standard-normal right-hand side, time
    per cycle and residual reduction per cycle.  Algorithmic HBM bytes per
    cycle and finest cell: 4 red-black sweeps x 2 colour passes x 12 B (read
    the other colour's phi and the own f, write the own phi, half the cells
    each), residual restriction 18 B, prolongation 17 B, all levels
    (x 8/7): 150 B."""
    import numpy as np
    import torch

    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh

    spec = I.MeshSpec(root=(16, 16, 16), block_cells=32)
    m = Mesh(**spec.kwargs())
    shape = (m.nleaf, m.N, m.N, m.N)
    g = torch.Generator(device=m.device)
    g.manual_seed(1234)
    f = torch.randn(shape, generator=g, dtype=torch.float64, device=m.device)
    phi = torch.zeros_like(f)
    work = m.poisson_workspace()
    m.poisson_solve(f, phi, 1, work=work, resid=False)  # warm-up
    phi.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.poisson_solve(f, phi, cycles, work=work, resid=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phi.zero_()
    res = m.poisson_solve(f, phi, cycles, work=work).cpu().tolist()
    n = m.nleaf * m.N ** 3
    fac = [res[i + 1] / res[i] for i in range(1, len(res) - 1)]
    ms = wall * 1e3 / cycles
    bytes_pc = 150
    out = {"workload": "uniform periodic mesh, 16^3 root octrees x 32^3 cells (512^3), V(2,2) cycles, "
                       "seeded standard-normal right-hand side",
           "cells": n, "cycles": cycles, "ms_per_vcycle": ms, "cell_vcycles_per_s": n * cycles / wall,
           "residual_factor_per_cycle": float(np.exp(np.mean(np.log(fac)))) if fac else None,
           "residual_first_last": [res[0], res[-1]],
           "hbm": {"algorithmic_bytes_per_cell_per_vcycle": bytes_pc, "GB/s": n * bytes_pc / (ms * 1e-3) / 1e9,
                   "peak": PEAK_HBM_GBS}}
    del f, phi, work, m
    torch.cuda.empty_cache()
    return out


def gravity_compare(steps: int = 10, ncycles: int = 2):
    """Self-gravity steps (kick-drift-kick with the mg0 potential, ncycles
    V(2,2) cycles per solve warm-started from the previous potential) on a
    uniform periodic mesh of 8^3 root octrees x 32^3 cells (256^3): a
    Jeans-unstable gas (4 pi G rho0 = 60, density 1 + 0.1 cos cos, adiabatic
    pressure).  Reports the time per step, the hydro and gravity shares, and
    the same mesh's plain step."""
    import numpy as np
    import torch

    from paper_1810_01319_amd import inputs as I
    from paper_1810_01319_amd.mesh import Mesh

    gamma = 5.0 / 3.0
    spec = I.MeshSpec(root=(8, 8, 8), block_cells=32, gamma=gamma)
    m = Mesh(**spec.kwargs())

    def act(keys):
        x, y, z = I.cell_centres(spec, keys)
        rho = 1.0 + 0.1 * np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y)
        return I.conserved(gamma, rho, 0.0, 0.0, 0.0, rho ** gamma)

    U = m.state_from_blocks(act)
    phi = torch.zeros((m.nleaf, m.N, m.N, m.N), dtype=torch.float64, device=m.device)
    work = m.poisson_workspace()
    dt = torch.zeros(1, dtype=torch.float64, device=m.device)
    m.step_gravity(U, dt, 0, 60.0, phi, False, ncycles, work=work)
    torch.cuda.synchronize()
    m.profile(True)
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        m.step_gravity(U, dt, k, 60.0, phi, True, ncycles, work=work)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = m.profile_read()
    m.profile(False)
    cells = m.nleaf * m.N ** 3
    grav = prof["poisson"][0] / steps
    hydro = sum(v[0] for p, v in prof.items() if p != "poisson") / steps
    U2 = m.state_from_blocks(act)
    m.step(U2, dt, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        m.step(U2, dt, k)
    torch.cuda.synchronize()
    plain = (time.perf_counter() - t0) * 1e3 / steps
    # the comoving step on the same gas in an Einstein-de Sitter universe
    # (a = t^(2/3) from t = 1, H = 2 / (3 t), 4 pi G mean rho = 2/3 with mean
    # rho = 1): dt from the comoving CFL, read back each step for a(t)
    U3 = m.state_from_blocks(act)
    phi.zero_()
    t = 1.0

    def co_step(k, current):
        nonlocal t
        m.cfl_dt_comoving(U3, t ** (2.0 / 3.0), dt)
        d = float(dt.cpu()[0])
        tm = t + 0.5 * d
        m.step_gravity_comoving(U3, dt, k, t ** (2.0 / 3.0), tm ** (2.0 / 3.0), (t + d) ** (2.0 / 3.0),
                                2.0 / (3.0 * tm), 2.0 / 3.0, phi, current, ncycles, work=work)
        t += d

    co_step(0, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        co_step(k, True)
    torch.cuda.synchronize()
    co_wall = time.perf_counter() - t0
    out = {"workload": "uniform periodic mesh, 8^3 root octrees x 32^3 cells (256^3), Jeans-unstable gas, "
                       f"4 pi G rho0 = 60, {ncycles} V(2,2) cycles per solve",
           "steps": steps, "ms_per_step": wall * 1e3 / steps, "cell_updates_per_s": cells * steps / wall,
           "gravity_ms_per_step": grav, "hydro_ms_per_step": hydro, "plain_step_ms": plain,
           "comoving": {"workload": "the same gas and mesh, comoving, Einstein-de Sitter from a = 1, "
                                    "4 pi G mean rho = 2/3, dt from the comoving CFL read back each step",
                        "ms_per_step": co_wall * 1e3 / steps, "a_end": t ** (2.0 / 3.0)}}
    del U, U2, U3, phi, work, m
    torch.cuda.empty_cache()
    return out


def step_bytes_per_block(N: int) -> int:
    """Algorithmic HBM bytes of one step of one block in a run of steps:
    refresh and three sweeps (the CFL candidates are taken from the values
    the last sweep writes, so the CFL reads nothing of its own; reflux is
    negligible)."""
    from paper_1810_01319_amd import costs

    return costs.refresh_bytes_per_block(N) + costs.sweep_bytes_per_block_step(N)


def cpu_baseline_adaptive(spec_tile, min_seconds: float):
    """The oracle on a 4^3-octree tile of the adaptive workload (same block
    size, levels, thresholds and interval, remesh before every fourth step),
    whole steps until at least `min_seconds` have passed."""
    from oracle import oracle as O
    from paper_1810_01319_amd import inputs as I

    m = O.OracleMesh(**spec_tile.kwargs())
    m.set_active(I.blasts_state(spec_tile, m.keys))
    cells = 0
    k = remeshes = 0
    t0 = time.perf_counter()
    while k < 200 and (k < 9 or time.perf_counter() - t0 < min_seconds):
        if k > 0 and k % 4 == 0:
            m, _ = m.remesh(0.3, 0.1, 10 ** 9)
            remeshes += 1
        m.step(k)
        cells += m.nleaf * spec_tile.block_cells ** 3
        k += 1
    t = time.perf_counter() - t0
    return {"value": cells / t, "unit": "cell-updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{k} steps incl. {remeshes} remeshes of a 4^3-octree tile of the same workload "
                      f"({m.nleaf} leaves at the end, {cells} cell-updates), {t:.1f} s"}


def run_adaptive(args, spec, desc):
    """The large adaptive workload: remesh included in the timed region."""
    import torch

    from paper_1810_01319_amd import _lib, adaptive, autotune
    from paper_1810_01319_amd.mesh import Mesh
    from paper_1810_01319_amd import inputs as I

    mesh = Mesh(**spec.kwargs())
    cap = adaptive.capacity_from_memory(mesh)
    pool = adaptive.StatePool(mesh, cap)
    U = pool.initial(mesh, lambda keys: I.blasts_state(spec, keys))
    if args.tune:
        # tune on the initial mesh, with the second arena as scratch
        autotune.tune(mesh, U, steps=1, use_cache=False, scratch=pool.other())
    mesh, U, _, _ = adaptive.run(mesh, U, args.warmup, max_blocks=cap, pool=pool)
    torch.cuda.synchronize()
    leaves_start = int(mesh.nleaf)
    step_leaves = []
    stats = []
    phases = {p: [0.0, 0] for p in _lib.PHASES if not p.startswith("adj_")}

    def collect(mm):
        prof = mm.profile_read()
        mm.profile(False)
        for p in phases:
            phases[p][0] += prof[p][0]
            phases[p][1] += prof[p][1]

    def total_mass(mm, uu):
        # sum over leaves of the cell volumes (root-cell units) times rho
        g, n = 3, spec.block_cells
        lev = torch.as_tensor(mm.keys[:, 0], device=uu.device, dtype=torch.float64)
        per_leaf = uu[:mm.nleaf, 0, g:g + n, g:g + n, g:g + n].sum(dim=(1, 2, 3))
        return float((per_leaf * torch.pow(0.125, lev)).sum())

    mass0 = total_mass(mesh, U)
    t_remesh = 0.0
    N = spec.block_cells
    m, u = mesh, U
    del mesh, U  # a remesh may hold only the old and the new state
    m.profile(True)
    t0 = time.perf_counter()
    dts = torch.zeros(4, 1, dtype=torch.float64, device=m.device)
    k, end = args.warmup, args.warmup + args.steps
    while k < end:
        fresh = False
        if k > 0 and k % 4 == 0:
            torch.cuda.synchronize()
            tr = time.perf_counter()
            new, un, st = m.remesh(u, 0.3, 0.1, cap, out=pool.other())
            if new is not m:
                pool.swap()
                collect(m)
                new.profile(True)
            else:
                fresh = True  # the remesh refreshed u's ghosts and changed nothing
            m, u = new, un
            stats.append(st)
            torch.cuda.synchronize()
            t_remesh += time.perf_counter() - tr
        # the steps up to the next remesh in one multi-step call
        n = min(end, (k // 4 + 1) * 4) - k
        m.steps(u, dts, n, k, ghosts_fresh=fresh)
        for j in range(n):
            step_leaves.append((k + j, int(m.nleaf)))
            if (k + j - args.warmup) % 10 == 0:
                print(f"[bench] step {k + j} leaves {m.nleaf}", file=sys.stderr, flush=True)
        k += n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    collect(m)
    if m.floor_count() != 0:
        print("warning: floors triggered", file=sys.stderr)
    mass1 = total_mass(m, u)
    total = float(sum(l for _, l in step_leaves)) * N ** 3
    hydro_s = wall - t_remesh
    step_bytes = sum(l for _, l in step_leaves) * step_bytes_per_block(N)
    prof = {p: (v[0], v[1]) for p, v in phases.items()}
    per_axis, dom = sweep_roofline(prof, step_leaves, N, m.nf, m.get_launch(), "blasts", spec.riemann_iters)
    out = {
        "metric": METRIC, "value": total / wall, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "leaves_start": leaves_start, "leaves_end": int(m.nleaf),
                   "cells_end": int(m.nleaf) * N ** 3, "block_cells": N, "max_blocks": cap,
                   "timed_steps": f"{args.warmup}..{end - 1}", "parallelism": "single GPU"},
        "roofline": roofline_object(per_axis[dom], "blasts"),
        "sweeps": per_axis,
        "without_remesh": total / hydro_s,
        "remesh_s": t_remesh,
        "remeshes": len(stats),
        "remesh_stats_last": stats[-1] if stats else None,
        "refused_total": int(sum(s["refused"] for s in stats)),
        "mass_relative_change": (mass1 - mass0) / mass0,
        "phases_ms_per_step": {p: round(v[0] / args.steps, 3) for p, v in phases.items() if v[1] > 0},
        "step_hbm_algorithmic": {"bytes_per_cell_update": step_bytes_per_block(N) / N ** 3,
                                 "GB/s": step_bytes / hydro_s / 1e9, "peak": PEAK_HBM_GBS,
                                 "frac": step_bytes / hydro_s / 1e9 / PEAK_HBM_GBS},
        "launch": m.get_launch(),
    }
    del m, u, pool
    torch.cuda.empty_cache()
    return out


def run_static(args, spec, act_fn, desc, workload_name):
    """A static mesh (the two-level Sedov blast by default): runs of steps
    through the multi-step entry (each step's CFL reduction fused into its
    predecessor; the same results as single steps)."""
    import torch

    from paper_1810_01319_amd import _lib, costs
    from paper_1810_01319_amd.mesh import Mesh

    mesh = Mesh(**spec.kwargs())
    N = spec.block_cells
    U = mesh.state_from_active(act_fn(spec, mesh.keys))
    tuned = None
    if args.tune:
        from paper_1810_01319_amd import autotune

        tuned = autotune.tune(mesh, U, use_cache=False)
    steps, warmup = args.static_steps, 2
    dts = torch.zeros(max(warmup, steps), mesh.n_instances, dtype=torch.float64, device=mesh.device)
    mesh.steps(U, dts, warmup, 0)
    torch.cuda.synchronize()
    mesh.profile(True)
    t0 = time.perf_counter()
    mesh.steps(U, dts, steps, warmup)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = mesh.profile_read()
    mesh.profile(False)
    if mesh.floor_count() != 0:
        print("warning: floors triggered", file=sys.stderr)
    cells = mesh.nleaf * N ** 3
    per_axis, dom = sweep_roofline(prof, [(k, mesh.nleaf) for k in range(warmup, warmup + steps)], N, mesh.nf,
                                   mesh.get_launch(), workload_name, spec.riemann_iters)
    refresh_bytes = mesh.nleaf * costs.refresh_bytes_per_block(N)
    refresh_ms = (prof["refresh1"][0] + prof["refresh2"][0]) / steps
    out = {
        "workload": desc, "leaves": mesh.nleaf, "cells": cells, "steps": steps, "warmup": warmup,
        "value": cells * steps / wall, "unit": "cell-updates/s", "ms_per_step": wall * 1e3 / steps,
        "roofline": roofline_object(per_axis[dom], workload_name),
        "sweeps": per_axis,
        "phases_ms_per_step": {p: round(prof[p][0] / steps, 4) for p in _lib.PHASES
                               if not p.startswith("adj_") and prof[p][1] > 0},
        "launch": mesh.get_launch(),
        "refresh_hbm": {"GB/s": refresh_bytes / (refresh_ms * 1e-3) / 1e9 if refresh_ms > 0 else None,
                        "peak": PEAK_HBM_GBS},
    }
    if tuned is not None:
        out["autotune"] = tuned
    del U, mesh
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before them (remeshes included)")
    ap.add_argument("--workload", default="blasts", choices=["blasts", "sedov", "sod"],
                    help="headline workload: the large adaptive blast array (default), the static "
                         "two-level Sedov mesh or the uniform Sod tube")
    ap.add_argument("--static-steps", type=int, default=50,
                    help="steps of the static Sedov sub-measurement (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum length of the oracle's timed sample (whole steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true", help="autotune the sweep launch shapes first")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="steps of the batched comparison, graph and one-mesh-per-launch (0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=10, help="steps of the adjoint comparison (0: skip)")
    ap.add_argument("--tracer-steps", type=int, default=20, help="steps of the tracer measurement (0: skip)")
    ap.add_argument("--comoving-steps", type=int, default=20,
                    help="steps of the comoving measurement (0: skip)")
    ap.add_argument("--dual-steps", type=int, default=50,
                    help="steps of the dual-energy measurement (0: skip)")
    ap.add_argument("--mg-cycles", type=int, default=10,
                    help="V-cycles of the mg0 Poisson measurement (0: skip)")
    ap.add_argument("--gravity-steps", type=int, default=10,
                    help="steps of the self-gravity measurement (0: skip)")
    ap.add_argument("--subs-only", action="store_true",
                    help="skip the headline workload (profiling runs of the sub-measurements)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    spec, act_fn, desc = workload(args.workload)
    out = {}
    if not args.subs_only:
        if args.workload == "blasts":
            out = run_adaptive(args, spec, desc)
        else:
            st = run_static(argparse.Namespace(**{**vars(args), "static_steps": args.steps}), spec, act_fn, desc,
                            args.workload)
            out = {"metric": METRIC, "value": st["value"], "unit": "cell-updates/s", "n_gpus": 1,
                   "steps": args.steps, "warmup": 2, "ms_per_step": st["ms_per_step"], "higher_is_better": True,
                   "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                   "config": {"workload": desc, "leaves": st["leaves"], "cells": st["cells"],
                              "block_cells": spec.block_cells, "parallelism": "single GPU"},
                   "roofline": st["roofline"], "sweeps": st["sweeps"],
                   "phases_ms_per_step": st["phases_ms_per_step"], "launch": st["launch"]}
    if args.workload == "blasts" and args.static_steps > 0:
        sspec, sfn, sdesc = workload("sedov")
        out["static_amr"] = run_static(argparse.Namespace(**{**vars(args), "tune": False}), sspec, sfn, sdesc,
                                       "sedov")
    if args.batch_steps > 0:
        out["batched"] = batched_compare(args.batch_steps)
    if args.adjoint_steps > 0:
        out["adjoint"] = adjoint_compare(args.adjoint_steps)
    if args.tracer_steps > 0:
        out["tracers"] = tracer_compare(args.tracer_steps)
    if args.comoving_steps > 0:
        out["comoving"] = comoving_compare(args.comoving_steps)
    if args.dual_steps > 0:
        out["dual_energy"] = dual_energy_compare(args.dual_steps)
    if args.mg_cycles > 0:
        out["mg0"] = mg0_compare(args.mg_cycles)
    if args.gravity_steps > 0:
        out["self_gravity"] = gravity_compare(args.gravity_steps)
    if not args.no_cpu_baseline and not args.subs_only:
        if args.workload == "blasts":
            from paper_1810_01319_amd import inputs as I

            tile = I.blasts_spec(root=4, block_cells=spec.block_cells, levels=spec.max_level)
            out["cpu_baseline"] = cpu_baseline_adaptive(tile, args.cpu_seconds)
        else:
            out["cpu_baseline"] = cpu_baseline(spec, act_fn, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
