"""The library's host-side logic (FFT padding and plans, the Runge-Kutta
tableaux against Butcher's order conditions, reduced-unit coefficients),
compiled with the address and undefined-behaviour sanitizers on the host
and run without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "host_logic.hip")
OUT = os.path.join(ROOT, "paper_1102_3069_amd", "_build", "host_logic_sanitized")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None, reason="no hipcc")
def test_host_logic_under_sanitizers():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    if not os.path.exists(OUT) or os.path.getmtime(OUT) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(ROOT, "paper_1102_3069_amd", "csrc",
                                                                 "host_common.hpp"))):
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all",
               "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1102_3069_amd", "csrc"),
               SRC, "-o", OUT]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([OUT], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host logic ok" in r.stdout
