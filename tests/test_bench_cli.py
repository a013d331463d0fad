"""The benchmark's command-line contract that holds without a GPU: more than
one GPU is refused with a message, and the algorithmic byte and flop models
the roofline figures use are consistent with their definitions."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sweep_cost_model():
    sys.path.insert(0, ROOT)
    from paper_1810_01319_amd import costs

    N, M = 32, 38
    pen = costs.sweep_pencils_per_block(N)
    assert (pen["first"], pen["second"], pen["third"]) == (M * M, N * M, N * N)
    # per pencil: 5 fields of M cells read and N cells written (40 B per cell and field group)
    assert costs.sweep_bytes_per_block_step(N) == 40 * (M + N) * (M * M + N * M + N * N)
    assert costs.sweep_flops_per_pencil(N, 5) > costs.sweep_flops_per_pencil(N, 1) > 0


def test_roofline_binds_on_the_higher_fraction():
    sys.path.insert(0, ROOT)
    import bench

    d = {"kernel": "k<32,0,5>", "avg_launch_ms": 1.0, "algorithmic_bytes_per_launch": 4e9, "GB/s": 4000.0,
         "hbm_frac": 0.5, "flops_per_launch": 1e10, "TFLOP/s": 10.0, "fp64_frac": 10.0 / 78.6}
    r = bench.roofline_object(d, "none")
    assert r["bound"] == "hbm" and r["frac"] == 0.5 and r["unit"] == "GB/s"
    assert r["other_roof"]["bound"] == "alu"
    d.update({"TFLOP/s": 60.0, "fp64_frac": 60.0 / 78.6})
    r = bench.roofline_object(d, "none")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["other_roof"]["frac"] == 0.5


def test_sweep_roofline_counts_pencils_by_place_in_the_order():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1810_01319_amd import costs

    N, M = 32, 38
    prof = {"sweep_x": (2.0, 2), "sweep_y": (1.0, 2), "sweep_z": (1.0, 2)}
    per, dom = bench.sweep_roofline(prof, [(0, 10), (1, 10)], N, 5, {"sweep_mode": [1, 0, 0]}, "none")
    assert dom == "x" and per["x"]["kernel"] == "sweep_staged<32,0,5>"
    # x is first on even steps (M^2 pencils) and last on odd ones (N^2)
    assert per["x"]["algorithmic_bytes_per_launch"] == 10 * (M * M + N * N) / 2 * costs.sweep_bytes_per_pencil(N)
    assert per["y"]["algorithmic_bytes_per_launch"] == 10 * N * M * costs.sweep_bytes_per_pencil(N)
