"""Build and run one_launch_step.cpp: the batch kernels of the library on the
CPU, per class and in one launch over every class, under AddressSanitizer;
or, with --server, server_host.cpp: the request server's host code against
the host-runtime stand-in of host/, its engine thread running rounds while
the main thread submits and polls, under AddressSanitizer or (--tsan)
ThreadSanitizer; or, with --batch, batch_host.cpp: the batch's host code
against the same stand-in, under AddressSanitizer.

    python tests/cpu_emulation/run.py [--all] [--real] [--mask]
    python tests/cpu_emulation/run.py --server [--tsan] [--iters N]
    python tests/cpu_emulation/run.py --batch [--iters N]

The kernel sources are taken from paper_1206_1361_amd/csrc with two textual
changes (dynamic LDS becomes a per-block heap buffer, static LDS a static
array) and compiled with clang++ against the stand-in hip/hip_runtime.h of
this directory, which runs every GPU thread of a block as a host thread.  A
manual check, not a pytest test: with --all the full step takes about an hour
on 8 cores (every x block costs dozens of thread barriers).
"""
import argparse
import os
import pathlib
import re
import subprocess
import sys
import tempfile

HERE = pathlib.Path(__file__).resolve().parent
ROOT = HERE.parents[1]
CSRC = ROOT / "paper_1206_1361_amd" / "csrc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--all", action="store_true", help="every block (needed for the bitwise comparison)")
    ap.add_argument("--real", action="store_true", help="real time instead of imaginary time")
    ap.add_argument("--mask", action="store_true", help="the test's mask of active solves")
    ap.add_argument("--server", action="store_true", help="the server's host code instead")
    ap.add_argument("--batch", action="store_true", help="the batch's host code instead")
    ap.add_argument("--tsan", action="store_true", help="with --server: ThreadSanitizer")
    ap.add_argument("--iters", type=int, default=20, help="with --server: rounds of the scenarios")
    args = ap.parse_args()
    if args.server or args.batch:
        return run_host(args)
    with tempfile.TemporaryDirectory() as tmp:
        tmp = pathlib.Path(tmp)
        for h in CSRC.glob("*.h"):
            (tmp / h.name).write_text(h.read_text())
        for name in ("sweep_x", "sweep_yz", "reduce"):
            src = (CSRC / f"{name}.hip").read_text()
            src = re.sub(r"extern __shared__ unsigned char (\w+)\[\];", r"unsigned char *\1 = g_lds;", src)
            src = src.replace("__shared__", "static")
            (tmp / f"{name}.cpp").write_text(src)
        exe = tmp / "one_launch_step"
        cmd = [CLANG, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", f"-I{tmp}",
               f"-I{HERE}", f"-I{ROOT / 'include'}", str(HERE / "one_launch_step.cpp"), "-o", str(exe), "-lpthread"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode:
            print(res.stderr[-4000:])
            return 1
        env = dict(os.environ)
        if args.all:
            env["ALL"] = "1"
        run = [str(exe), "real" if args.real else "imag"] + (["mask"] if args.mask else [])
        res = subprocess.run(run, env=env, text=True, capture_output=True)
        sys.stdout.write(res.stdout)
        sys.stderr.write(res.stderr[-4000:])
        if res.returncode or "ERROR: AddressSanitizer" in res.stderr:
            return 1
        if args.all and "solves differing: 0, partials equal: 1" not in res.stdout:
            return 1
        return 0


def run_host(args) -> int:
    prog = "server_host" if args.server else "batch_host"
    with tempfile.TemporaryDirectory() as tmp:
        exe = pathlib.Path(tmp) / prog
        san = "-fsanitize=thread" if args.tsan and args.server else "-fsanitize=address"
        cmd = [CLANG, "-std=c++20", "-O1", "-g", san, "-fno-omit-frame-pointer", f"-I{HERE / 'host'}",
               f"-I{ROOT / 'include'}", f"-I{CSRC}", str(HERE / f"{prog}.cpp"), "-o", str(exe), "-lpthread"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode:
            print(res.stderr[-4000:])
            return 1
        res = subprocess.run([str(exe), str(args.iters)], text=True, capture_output=True)
        sys.stdout.write(res.stdout)
        sys.stderr.write(res.stderr[-4000:])
        good = "scenarios failing 0" if args.server else "cases failing 0"
        if res.returncode or "Sanitizer" in res.stderr or good not in res.stdout:
            return 1
        return 0


if __name__ == "__main__":
    sys.exit(main())
