"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds sanitized variants of the two CPU oracles (oracle/rd_oracle.cpp,
oracle/rd3_oracle.cpp), of the host tile builder (through
tests/cpp/tiling_shim.cpp) and of the Delaunay flip and refinement bodies
(through tests/cpp/delaunay_shim.cpp), and runs their CPU pins against them
in a child process that preloads the sanitizer runtime. Any invalid access,
overflow or undefined operation aborts the child and fails this test."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SUITES = ["tests/test_oracle_pins.py", "tests/test_oracle3_pins.py", "tests/test_tiling.py",
          "tests/test_refine_cpu.py"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_pins_run_clean_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no libasan runtime next to gcc")
    env = dict(os.environ)
    env.update(RD_HOST_SANITIZE="1",
               RDO_LIB=str(tmp_path / "liboracle_san.so"),
               RDO3_LIB=str(tmp_path / "liboracle3_san.so"),
               LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               OMP_NUM_THREADS="4")
    # -s: the sanitizers report on the child's stderr, which pytest would otherwise capture and lose
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu"] + SUITES
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1800)
    tail = (r.stdout[-4000:] + "\n" + r.stderr[-4000:])
    assert r.returncode == 0, tail
    # the sanitized builds were the ones loaded
    assert os.path.exists(env["RDO_LIB"]) and os.path.exists(env["RDO3_LIB"]), tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
