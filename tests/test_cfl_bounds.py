"""Host run of the per-vertex CFL bound code of the CFL vertex pass
(rd::cfl_vertex_bounds) against a plain sum, with AddressSanitizer on the
host build (tests/cpp/cfl_bounds_check.cpp says what it checks). CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_cfl_vertex_bounds_on_the_host(tmp_path):
    exe = str(tmp_path / "cfl_bounds_check")
    cmd = ["hipcc", "-std=c++17", "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_1705_02028_amd", "csrc"), os.path.join(HERE, "cpp", "cfl_bounds_check.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-3000:])
