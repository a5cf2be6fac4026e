"""CPU FP64 oracle for the 3D split-step Crank-Nicolson Gross-Pitaevskii step.

TEST INFRASTRUCTURE ONLY: this package is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import it.  It shares no code with the GPU
library and never calls it.

The arithmetic lives in ``gpo.c`` and, for the circularly, spherically and
axially symmetric forms, ``gpo_radial.c`` (plain C99, ``double complex``), which
follows the paper's description of the method (Vudragovic et al., Comput.
Phys. Commun. 183 (2012) 2021: program summaries (v) and (xiv), "Method of
solution"; "Summary of revisions" for the routine decomposition calcnu ->
calclux -> calcluy -> calcluz -> calcnorm and the physical quantities
calcmuen / calcrms).  This module only marshals numpy arrays through ctypes.

Arrays are complex128, C-contiguous, shape (Nz, Ny, Nx) (x fastest).
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
SOURCE = _HERE / "gpo.c"
SOURCE_RADIAL = _HERE / "gpo_radial.c"
LIBRARY = _HERE / "libgpo.so"

IMAG = 0
REAL = 1

OK = 0
ERR_INVALID = 1
ERR_NOMEM = 2
ERR_NONFINITE = 4

OBS_NAMES = (
    "norm", "mu", "energy",
    "rms_x", "rms_y", "rms_z", "rms_r",
    "mean_x", "mean_y", "mean_z",
    "kinetic", "potential", "interaction",
)

SUBSTEP = {"calcnu": 0, "calclux": 1, "calcluy": 2, "calcluz": 3, "calcnorm": 4}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build_command() -> list[str]:
    # No -ffast-math and no -march: IEEE semantics, portable to any x86-64 host.
    return ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared",
            "-Wall", "-Wextra", "-o", str(LIBRARY), str(SOURCE), str(SOURCE_RADIAL), "-lm"]


def build() -> pathlib.Path:
    """Compile gpo.c into libgpo.so (always recompiles)."""
    tmp = LIBRARY.with_suffix(".so.tmp")
    cmd = build_command()
    cmd[cmd.index(str(LIBRARY))] = str(tmp)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIBRARY)
    return LIBRARY


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgpo.so, compiling it first only if it is not there."""
    global _lib
    if _lib is None:
        if not LIBRARY.exists():
            build()
        L = ctypes.CDLL(str(LIBRARY))
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        L.gpo_validate.argtypes = [i64p, dp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_int]
        L.gpo_step.argtypes = [i64p, dp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_int,
                               dp, ctypes.c_int64]
        L.gpo_substep.argtypes = [i64p, dp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_int,
                                  dp, ctypes.c_int]
        L.gpo_observables.argtypes = [i64p, dp, dp, ctypes.c_double, dp, dp]
        L.gpo_norm.argtypes = [i64p, dp, dp, dp]
        L.gpo_step_nd.argtypes = [ctypes.c_int] + L.gpo_step.argtypes
        L.gpo_observables_nd.argtypes = [ctypes.c_int] + L.gpo_observables.argtypes
        L.gpo_norm_nd.argtypes = [ctypes.c_int] + L.gpo_norm.argtypes
        L.gpo_radial_step.argtypes = [ctypes.c_int] + L.gpo_step.argtypes
        L.gpo_radial_observables.argtypes = [ctypes.c_int] + L.gpo_observables.argtypes
        L.gpo_radial_step.restype = ctypes.c_int
        L.gpo_radial_observables.restype = ctypes.c_int
        L.gpo_thomas.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, dp, dp]
        L.gpo_coord.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int64]
        L.gpo_coord.restype = ctypes.c_double
        L.gpo_set_threads.argtypes = [ctypes.c_int]
        L.gpo_get_threads.restype = ctypes.c_int
        for f in (L.gpo_validate, L.gpo_step, L.gpo_substep, L.gpo_observables,
                  L.gpo_norm, L.gpo_thomas, L.gpo_step_nd, L.gpo_observables_nd, L.gpo_norm_nd):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _grid_args(psi: np.ndarray, dx, omega=(0.0, 0.0, 0.0)):
    if psi.dtype != np.complex128 or psi.ndim != 3 or not psi.flags.c_contiguous:
        raise ValueError("psi must be a C-contiguous complex128 array of shape (Nz, Ny, Nx)")
    nz, ny, nx = psi.shape
    n = (ctypes.c_int64 * 3)(nx, ny, nz)
    d = (ctypes.c_double * 3)(*[float(v) for v in dx])
    w = (ctypes.c_double * 3)(*[float(v) for v in omega])
    return n, d, w


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(nthreads: int) -> None:
    lib().gpo_set_threads(int(nthreads))


def get_threads() -> int:
    return int(lib().gpo_get_threads())


def validate(grid, dx, dt, omega, g, mode) -> int:
    n = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    d = (ctypes.c_double * 3)(*[float(v) for v in dx])
    w = (ctypes.c_double * 3)(*[float(v) for v in omega])
    return int(lib().gpo_validate(n, d, float(dt), w, float(g), int(mode)))


def step(psi: np.ndarray, dx, dt: float, omega, g: float, mode: int, nsteps: int = 1,
         ndim: int = 3) -> np.ndarray:
    """Advance psi in place by ``nsteps`` SSCN steps; returns psi.  ndim 1 or
    2: the equation in x (and y) only; psi then has shape (1, 1, Nx) or
    (1, Ny, Nx)."""
    n, d, w = _grid_args(psi, dx, omega)
    st = lib().gpo_step_nd(int(ndim), n, d, float(dt), w, float(g), int(mode), _ptr(psi), int(nsteps))
    if st != OK:
        raise OracleError(st, "step")
    return psi


def substep(psi: np.ndarray, which: str, dx, dt: float, omega, g: float, mode: int) -> np.ndarray:
    """Apply one named sub-step (calcnu, calclux, calcluy, calcluz, calcnorm) in place."""
    n, d, w = _grid_args(psi, dx, omega)
    st = lib().gpo_substep(n, d, float(dt), w, float(g), int(mode), _ptr(psi), SUBSTEP[which])
    if st != OK:
        raise OracleError(st, which)
    return psi


def norm(psi: np.ndarray, dx, ndim: int = 3) -> float:
    n, d, _ = _grid_args(psi, dx)
    out = ctypes.c_double()
    st = lib().gpo_norm_nd(int(ndim), n, d, _ptr(psi), ctypes.byref(out))
    if st != OK:
        raise OracleError(st, "norm")
    return out.value


def observables(psi: np.ndarray, dx, omega, g: float, ndim: int = 3) -> dict:
    n, d, w = _grid_args(psi, dx, omega)
    out = (ctypes.c_double * len(OBS_NAMES))()
    st = lib().gpo_observables_nd(int(ndim), n, d, w, float(g), _ptr(psi), out)
    if st != OK:
        raise OracleError(st, "observables")
    return {k: out[i] for i, k in enumerate(OBS_NAMES)}


def thomas(diag: complex, off: complex, rhs: np.ndarray) -> np.ndarray:
    """Solve diag*x_i + off*(x_{i-1}+x_{i+1}) = rhs_i (x_{-1}=x_N=0) by the oracle's recursion."""
    r = np.ascontiguousarray(rhs, dtype=np.complex128)
    x = np.empty_like(r)
    st = lib().gpo_thomas(r.size, complex(diag).real, complex(diag).imag,
                          complex(off).real, complex(off).imag, _ptr(r), _ptr(x))
    if st != OK:
        raise OracleError(st, "thomas")
    return x


def coord(n: int, dx: float) -> np.ndarray:
    """The oracle's node coordinates along one axis."""
    L = lib()
    return np.array([L.gpo_coord(int(n), float(dx), i) for i in range(int(n))])


GEOMETRIES = {"circular": 1, "spherical": 2, "axial": 3}


def radial_step(psi: np.ndarray, geom: str, dx, dt: float, omega, g: float, mode: int,
                nsteps: int = 1) -> np.ndarray:
    """Advance a symmetric-trap state in place (gpo_radial.c).  psi has shape
    (1, 1, N) (circular, spherical: r along the last axis) or (1, Nz, Nrho)
    (axial); dx = (h_r, dz, unused); omega = (w or gamma, unused, lambda)."""
    n, d, w = _grid_args(psi, dx, omega)
    st = lib().gpo_radial_step(GEOMETRIES[geom], n, d, float(dt), w, float(g), int(mode), _ptr(psi), int(nsteps))
    if st != OK:
        raise OracleError(st, "radial step")
    return psi


def radial_observables(psi: np.ndarray, geom: str, dx, omega, g: float) -> dict:
    n, d, w = _grid_args(psi, dx, omega)
    out = (ctypes.c_double * len(OBS_NAMES))()
    st = lib().gpo_radial_observables(GEOMETRIES[geom], n, d, w, float(g), _ptr(psi), out)
    if st != OK:
        raise OracleError(st, "radial observables")
    return {k: out[i] for i, k in enumerate(OBS_NAMES)}
