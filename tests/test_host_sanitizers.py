"""The host code of the request server and of the batch on the CPU (no GPU),
built against the host-runtime stand-in of tests/cpu_emulation/host with the
kernels stubbed.  The server's engine thread runs rounds while the main
thread submits and polls the server tests' request patterns (real states
beside complex ones, float64 storage, automatic real storage, no graph, a
slot limit), under AddressSanitizer and under ThreadSanitizer; batches of
every storage type run steps, masks, rebinding, the tuner, the FP64 finish
and the stopping rule under AddressSanitizer.  Any sanitizer report, or a
request or call that fails, fails the test.
"""
import pathlib
import subprocess
import sys

import pytest

HERE = pathlib.Path(__file__).resolve().parent
RUN = HERE / "cpu_emulation" / "run.py"
CLANG = pathlib.Path("/opt/rocm/llvm/bin/clang++")


@pytest.mark.skipif(not CLANG.exists(), reason="needs the ROCm clang++")
@pytest.mark.parametrize("what,flags,iters,done", [
    ("server", ["--server"], 4, "scenarios failing 0"),
    ("server-tsan", ["--server", "--tsan"], 2, "scenarios failing 0"),
    ("batch", ["--batch"], 2, "cases failing 0"),
])
def test_host_code_under_sanitizer(what, flags, iters, done):
    cmd = [sys.executable, str(RUN), *flags, "--iters", str(iters)]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert f"iterations {iters}, {done}" in res.stdout
