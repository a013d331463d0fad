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
