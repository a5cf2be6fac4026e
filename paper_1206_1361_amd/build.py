"""Build libgpssc.so (the HIP kernels and the C ABI) for gfx950, in-tree.

    python -m paper_1206_1361_amd.build

Each .hip file under csrc/ is compiled to an object in parallel, then linked
into paper_1206_1361_amd/libgpssc.so.  Always recompiles.
"""
from __future__ import annotations

import concurrent.futures
import os
import pathlib
import subprocess
import sys

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
BUILD = PKG / "_build"
LIBRARY = PKG / "libgpssc.so"
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # never emit packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def sources() -> list[pathlib.Path]:
    return sorted(CSRC.glob("*.hip"))


def _compile(src: pathlib.Path) -> pathlib.Path:
    obj = BUILD / (src.stem + ".o")
    cmd = [HIPCC, *COMMON, "-c", str(src), "-o", str(obj)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src.name} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


PROBES = ["pattern_copy", "grid_sync"]   # measurement tools in probe/, not part of the library
PROBE_BIN = PKG / "probe" / "pattern_copy"


def build_probe() -> pathlib.Path:
    """The measurement probes: probe/<name>.hip -> probe/<name>."""
    for name in PROBES:
        src = PKG / "probe" / f"{name}.hip"
        binary = PKG / "probe" / name
        cmd = [HIPCC, *[f for f in COMMON if f != "-fPIC"], "-o", str(binary), str(src)]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"building the probe {name} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return PROBE_BIN


def build(verbose: bool = False) -> pathlib.Path:
    BUILD.mkdir(exist_ok=True)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIBRARY.with_suffix(".so.tmp")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIBRARY)
    build_probe()
    if verbose:
        print(f"built {LIBRARY} and the probes " + ", ".join(PROBES), file=sys.stderr)
    return LIBRARY


if __name__ == "__main__":
    build(verbose=True)
