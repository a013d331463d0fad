"""The CPU suite under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle (plain C) and the library's host half (octree and balance,
FlatMap hash tables, plan tables, remesh decisions and capacity policy,
leaf-set and descriptor checks, the C ABI's argument handling) are built
with both sanitizers, aborting on the first report; then every
``-m "not gpu"`` test except this file runs in a child process that loads
those builds (AMR_LIBRARY, AMR_ORACLE_LIBRARY) with the sanitizer runtimes
preloaded.  Device code is not sanitized (there is no GPU here)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def test_cpu_suite_is_clean_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_1810_01319_amd import _build

    orc = O.build_sanitized(str(tmp_path / "liboracle_san.so"))
    lib = _build.build_host_sanitized(str(tmp_path / "libamr_san.so"))
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime("libasan.so") + " " + runtime("libubsan.so"),
        # the interpreter and torch are not instrumented: leak reports would be theirs
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "AMR_LIBRARY": lib,
        "AMR_ORACLE_LIBRARY": orc,
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        "--deselect", "tests/test_sanitizers.py", "tests/"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
