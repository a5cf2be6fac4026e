"""The request server's host code on the CPU (no GPU): server.hip built against
the host-runtime stand-in of tests/cpu_emulation/host, its engine thread
running rounds while the main thread submits and polls the server tests'
request patterns (real states beside complex ones, float64 storage,
automatic real storage, no graph, a slot limit), under AddressSanitizer and
under ThreadSanitizer.  Any sanitizer report, or a request that never comes
back, fails the test.
"""
import pathlib
import subprocess
import sys

import pytest

HERE = pathlib.Path(__file__).resolve().parent
RUN = HERE / "cpu_emulation" / "run.py"
CLANG = pathlib.Path("/opt/rocm/llvm/bin/clang++")


@pytest.mark.skipif(not CLANG.exists(), reason="needs the ROCm clang++")
@pytest.mark.parametrize("sanitizer,iters", [("address", 4), ("thread", 2)])
def test_server_host_code_under_sanitizer(sanitizer, iters):
    cmd = [sys.executable, str(RUN), "--server", "--iters", str(iters)] + (["--tsan"] if sanitizer == "thread" else [])
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert f"iterations {iters}, scenarios failing 0" in res.stdout
