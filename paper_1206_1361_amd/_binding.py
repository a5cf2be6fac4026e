"""ctypes binding over libgpssc.so (include/gpssc.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libgpssc.  PyTorch supplies device memory (psi tensors) and the
stream work is queued on.  If the library is missing, every entry point
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import pathlib

PKG = pathlib.Path(__file__).resolve().parent
LIBRARY = PKG / "libgpssc.so"

IMAG = 0
REAL = 1
C128 = 0
C64 = 1
C64_F64 = 2
R64 = 3
R32 = 4

OK = 0
ERR_INVALID = 1
ERR_NOMEM = 2
ERR_DEVICE = 3
ERR_NONFINITE = 4
ERR_UNSUPPORTED = 5

KERNELS = ("nu_x", "y", "z", "norm", "scale", "obs")

# Every symbol include/gpssc.h declares.
EXPORTS = (
    "gp_plan_create", "gp_plan_create_nd", "gp_plan_create_radial", "gp_plan_destroy", "gp_set_g", "gp_set_trap", "gp_set_stream", "gp_step",
    "gp_step_schedule", "gp_step_noalloc", "gp_sync", "gp_plan_set_sweep",
    "gp_observables", "gp_density_profiles", "gp_plan_footprint_bytes", "gp_plan_describe", "gp_status_string",
    "gp_last_error", "gp_profile_enable", "gp_profile_read", "gp_sweep_shape", "gp_sweep_tables",
    "gp_batch_create", "gp_batch_destroy", "gp_batch_set_psi", "gp_batch_set_active", "gp_batch_step",
    "gp_batch_observables", "gp_batch_solve_imag", "gp_batch_describe",
    "gp_server_request_bytes", "gp_server_create", "gp_server_destroy", "gp_server_submit", "gp_server_poll",
    "gp_server_drain", "gp_server_stats",
)

BATCH_GRAPH = 1
BATCH_TUNE = 2
BATCH_FINISH_F64 = 4
BATCH_ONE_LAUNCH = 8
SERVER_GRAPH = 1
SERVER_REAL_AUTO = 2


class GPError(RuntimeError):
    """A libgpssc call returned a status other than GP_OK."""

    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


class GPInvalid(GPError, ValueError):
    pass


class GPNoMemory(GPError, MemoryError):
    pass


class GPNonFinite(GPError, FloatingPointError):
    pass


class GPObs(ctypes.Structure):
    _fields_ = [
        ("norm", ctypes.c_double), ("mu", ctypes.c_double), ("energy", ctypes.c_double),
        ("rms", ctypes.c_double * 3), ("rms_r", ctypes.c_double), ("mean", ctypes.c_double * 3),
        ("kinetic", ctypes.c_double), ("potential", ctypes.c_double),
        ("interaction", ctypes.c_double), ("steps_done", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {
            "norm": self.norm, "mu": self.mu, "energy": self.energy,
            "rms_x": self.rms[0], "rms_y": self.rms[1], "rms_z": self.rms[2], "rms_r": self.rms_r,
            "mean_x": self.mean[0], "mean_y": self.mean[1], "mean_z": self.mean[2],
            "kinetic": self.kinetic, "potential": self.potential,
            "interaction": self.interaction, "steps_done": self.steps_done,
        }


class GPRequest(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_int64 * 3), ("dx", ctypes.c_double * 3), ("dt", ctypes.c_double),
        ("trap", ctypes.c_double * 3), ("g", ctypes.c_double), ("mode", ctypes.c_int),
        ("steps", ctypes.c_int64), ("tol", ctypes.c_double), ("psi_in", ctypes.c_void_p),
        ("psi_out", ctypes.c_void_p), ("tag", ctypes.c_uint64), ("real_state", ctypes.c_int),
    ]


class GPResult(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("converged", ctypes.c_int),
        ("steps", ctypes.c_int64), ("obs", GPObs), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class GPServerCounters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "queued", "resident", "max_resident",
                                                "quanta", "graph_captures", "solve_steps")] + \
               [(n, ctypes.c_uint64) for n in ("bytes_in_use", "bytes_peak", "bytes_budget")] + \
               [(n, ctypes.c_double) for n in ("seconds_copy_in", "seconds_copy_out", "seconds_rounds")]


_lib = None


def library_path() -> pathlib.Path:
    return LIBRARY


def lib() -> ctypes.CDLL:
    """Load libgpssc.so.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIBRARY.exists():
        raise ImportError(
            f"{LIBRARY} is missing: build it with `python -m paper_1206_1361_amd.build` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(str(LIBRARY))
    vp, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    L.gp_plan_create.argtypes = [i64p, dp, dbl, dbl, dbl, dbl, dbl, ctypes.c_int, ctypes.c_int, vp,
                                 ctypes.POINTER(vp)]
    L.gp_plan_create_nd.argtypes = [ctypes.c_int] + L.gp_plan_create.argtypes
    L.gp_plan_create_nd.restype = ctypes.c_int
    L.gp_plan_create_radial.argtypes = [ctypes.c_int] + L.gp_plan_create.argtypes
    L.gp_plan_create_radial.restype = ctypes.c_int
    L.gp_plan_destroy.argtypes = [vp]
    L.gp_set_g.argtypes = [vp, dbl]
    L.gp_set_trap.argtypes = [vp, dbl, dbl, dbl]
    L.gp_step_schedule.argtypes = [vp, vp, i64, i64, dp, dp]
    L.gp_set_stream.argtypes = [vp, vp]
    L.gp_step.argtypes = [vp, vp, i64, i64]
    L.gp_plan_set_sweep.argtypes = [vp, ctypes.c_int]
    L.gp_step_noalloc.argtypes = [i64p, dp, dbl, dbl, dbl, dbl, dbl, ctypes.c_int, ctypes.c_int, vp, vp, i64, i64]
    L.gp_sync.argtypes = [vp]
    L.gp_observables.argtypes = [vp, vp, i64, ctypes.POINTER(GPObs)]
    L.gp_density_profiles.argtypes = [vp, vp, i64, dp, dp, dp]
    L.gp_density_profiles.restype = ctypes.c_int
    L.gp_plan_footprint_bytes.argtypes = [i64p, ctypes.c_int]
    L.gp_plan_footprint_bytes.restype = sz
    L.gp_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
    L.gp_status_string.argtypes = [ctypes.c_int]
    L.gp_status_string.restype = ctypes.c_char_p
    L.gp_last_error.argtypes = []
    L.gp_last_error.restype = ctypes.c_char_p
    L.gp_profile_enable.argtypes = [vp, ctypes.c_int]
    L.gp_profile_read.argtypes = [vp, dp, i64p]
    L.gp_sweep_shape.argtypes = [i64, ctypes.c_int, ctypes.c_int, ip, ip]
    L.gp_sweep_tables.argtypes = [i64, dbl, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  dp, sz, dp, sz, dp, sz]
    up = ctypes.POINTER(ctypes.c_ubyte)
    L.gp_batch_create.argtypes = [ctypes.c_int, i64p, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  vp, ctypes.POINTER(vp)]
    L.gp_batch_destroy.argtypes = [vp]
    L.gp_batch_set_psi.argtypes = [vp, ctypes.POINTER(vp), i64p]
    L.gp_batch_set_active.argtypes = [vp, up]
    L.gp_batch_step.argtypes = [vp, i64]
    L.gp_batch_observables.argtypes = [vp, ctypes.POINTER(GPObs)]
    L.gp_batch_solve_imag.argtypes = [vp, dbl, i64, i64, ctypes.POINTER(GPObs), i64p, up]
    L.gp_batch_describe.argtypes = [vp, ctypes.c_char_p, sz]
    L.gp_server_request_bytes.argtypes = [i64p, ctypes.c_int, ctypes.c_int]
    L.gp_server_request_bytes.restype = sz
    L.gp_server_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, i64, ctypes.c_int,
                                   ctypes.POINTER(vp)]
    L.gp_server_destroy.argtypes = [vp]
    L.gp_server_submit.argtypes = [vp, ctypes.POINTER(GPRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.gp_server_poll.argtypes = [vp, ctypes.POINTER(GPResult), ctypes.c_int, dbl, ip]
    L.gp_server_drain.argtypes = [vp, dbl, ip]
    L.gp_server_stats.argtypes = [vp, ctypes.POINTER(GPServerCounters)]
    for name in ("gp_server_create", "gp_server_destroy", "gp_server_submit", "gp_server_poll",
                 "gp_server_drain", "gp_server_stats"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("gp_batch_create", "gp_batch_destroy", "gp_batch_set_psi", "gp_batch_set_active",
                 "gp_batch_step", "gp_batch_observables", "gp_batch_solve_imag", "gp_batch_describe"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("gp_plan_create", "gp_plan_destroy", "gp_set_g", "gp_set_trap", "gp_step_schedule",
                 "gp_set_stream", "gp_step", "gp_step_noalloc", "gp_plan_set_sweep",
                 "gp_sync", "gp_observables", "gp_plan_describe", "gp_profile_enable",
                 "gp_profile_read", "gp_sweep_shape", "gp_sweep_tables"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int, what: str) -> None:
    if status == OK:
        return
    L = lib()
    msg = f"{what}: {L.gp_status_string(status).decode()} ({L.gp_last_error().decode()})"
    cls = {ERR_INVALID: GPInvalid, ERR_NOMEM: GPNoMemory, ERR_NONFINITE: GPNonFinite}.get(status, GPError)
    raise cls(status, msg)


def _mode(mode) -> int:
    if mode in (IMAG, "imag", "imaginary"):
        return IMAG
    if mode in (REAL, "real"):
        return REAL
    raise ValueError(f"unknown mode {mode!r}")


def _dtype(dtype) -> int:
    if isinstance(dtype, (int, str)):
        if dtype in (C128, "c128", "complex128"):
            return C128
        if dtype in (C64, "c64", "complex64"):
            return C64
        if dtype in (C64_F64, "c64_f64"):
            return C64_F64
        if dtype in (R64, "r64", "float64"):
            return R64
        if dtype in (R32, "r32", "float32"):
            return R32
        raise ValueError(f"unknown dtype {dtype!r}")
    import torch

    if dtype == torch.complex128:
        return C128
    if dtype == torch.complex64:
        return C64
    if dtype == torch.float64:
        return R64
    if dtype == torch.float32:
        return R32
    raise ValueError(f"unknown dtype {dtype!r}")


def torch_dtype_of(dtype: int):
    """Element type of psi tensors for a library dtype."""
    import torch

    return {C128: torch.complex128, C64: torch.complex64, C64_F64: torch.complex64, R64: torch.float64,
            R32: torch.float32}[dtype]


def numpy_dtype_of(dtype: int):
    import numpy as np

    return {C128: np.complex128, C64: np.complex64, C64_F64: np.complex64, R64: np.float64, R32: np.float32}[dtype]


def footprint_bytes(grid, dtype="c128") -> int:
    g = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    return int(lib().gp_plan_footprint_bytes(g, _dtype(dtype)))


def sweep_shape(n: int, axis: int, dtype="c128") -> tuple[int, int]:
    c, l = ctypes.c_int(), ctypes.c_int()
    _check(lib().gp_sweep_shape(int(n), int(axis), _dtype(dtype), ctypes.byref(c), ctypes.byref(l)),
           "gp_sweep_shape")
    return c.value, l.value


def sweep_tables(n: int, dx: float, dt: float, mode, chunk: int, lanes: int) -> dict:
    """Host-only copy of the constant sweep coefficients (see gp_sweep_tables)."""
    import numpy as np

    coef = np.zeros(14)
    stage = np.zeros(12)
    zt = np.zeros(2 * n)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().gp_sweep_tables(int(n), float(dx), float(dt), _mode(mode), int(chunk), int(lanes),
                                 coef.ctypes.data_as(dp), coef.size, stage.ctypes.data_as(dp), stage.size,
                                 zt.ctypes.data_as(dp), zt.size),
           "gp_sweep_tables")
    c = lambda a: a[0::2] + 1j * a[1::2]  # noqa: E731
    k = c(coef)
    return {"kappa": k[0], "b": k[1], "o": k[2], "c": k[3], "beta": k[4], "m": k[5], "a": k[6],
            "stage": c(stage), "zt": c(zt)}


def step_noalloc(psi, dx, dt, gamma, nu, lam, g, mode="imag", dtype="c128", nsteps: int = 1, stream=None):
    """gp_step_noalloc: nsteps steps on psi (in place, queued on the current
    torch stream) without a plan and without allocating device memory; the
    grid is psi's shape (Nz, Ny, Nx)."""
    import torch

    dt_code = _dtype(dtype)
    if not isinstance(psi, torch.Tensor) or psi.dtype != torch_dtype_of(dt_code) or psi.device.type != "cuda" \
            or psi.dim() != 3 or not psi.is_contiguous():
        raise ValueError(f"psi must be a contiguous {torch_dtype_of(dt_code)} CUDA tensor (Nz, Ny, Nx)")
    nz, ny, nx = psi.shape
    n = (ctypes.c_int64 * 3)(nx, ny, nz)
    d = (ctypes.c_double * 3)(*[float(v) for v in (dx if hasattr(dx, "__len__") else (dx, dx, dx))])
    _check(lib().gp_step_noalloc(n, d, float(dt), float(gamma), float(nu), float(lam), float(g), _mode(mode),
                                 dt_code, Plan._stream_handle(stream), ctypes.c_void_p(psi.data_ptr()),
                                 psi.numel(), int(nsteps)), "gp_step_noalloc")
    return psi


class Plan:
    """One grid, step size, trap, coupling, mode and dtype.

    psi tensors are torch.complex128 (dtype "c128") or torch.complex64
    ("c64": FP32 arithmetic, "c64_f64": FP64 arithmetic on FP32 storage), or,
    for imaginary time, real torch.float64 ("r64") or torch.float32 ("r32");
    CUDA (HIP) device, contiguous, shape (Nz, Ny, Nx).  ndim = 1 or 2 solves
    the equation in x (and y) only, on a grid with Nz = 1 (and Ny = 1).
    geometry = "circular" | "spherical" (radial variable along x, grid
    (N, 1, 1), trap gamma) or "axial" (rho along x, z along y, grid
    (N_rho, N_z, 1), traps gamma and lam) selects a symmetric trap.
    """

    GEOMETRIES = {"circular": 1, "spherical": 2, "axial": 3}

    def __init__(self, grid, dx, dt, gamma, nu, lam, g, mode="imag", dtype="c128", stream=None, ndim=3,
                 geometry=None):
        import torch

        L = lib()
        self.grid = tuple(int(v) for v in grid)
        self.dx = tuple(float(v) for v in (dx if hasattr(dx, "__len__") else (dx, dx, dx)))
        self.dt = float(dt)
        self.omega = (float(gamma), float(nu), float(lam))
        self.g = float(g)
        self.mode = _mode(mode)
        self.dtype = _dtype(dtype)
        self.torch_dtype = torch_dtype_of(self.dtype)
        self._handle = ctypes.c_void_p()
        n = (ctypes.c_int64 * 3)(*self.grid)
        d = (ctypes.c_double * 3)(*self.dx)
        self.ndim = int(ndim)
        self.geometry = geometry
        if geometry is not None:
            _check(L.gp_plan_create_radial(self.GEOMETRIES[geometry], n, d, self.dt, *self.omega, self.g, self.mode,
                                           self.dtype, self._stream_handle(stream), ctypes.byref(self._handle)),
                   "gp_plan_create_radial")
        else:
            _check(L.gp_plan_create_nd(self.ndim, n, d, self.dt, *self.omega, self.g, self.mode, self.dtype,
                                       self._stream_handle(stream), ctypes.byref(self._handle)),
                   "gp_plan_create_nd")

    @staticmethod
    def _stream_handle(stream):
        import torch

        if stream is None:
            if not torch.cuda.is_available():
                return None
            stream = torch.cuda.current_stream()
        return ctypes.c_void_p(stream.cuda_stream)

    def _psi(self, psi):
        import torch

        if not isinstance(psi, torch.Tensor):
            raise TypeError("psi must be a torch tensor")
        if psi.dtype != self.torch_dtype:
            raise TypeError(f"psi must be {self.torch_dtype}, got {psi.dtype}")
        if psi.device.type != "cuda":
            raise ValueError("psi must live on the GPU")
        if tuple(psi.shape) != self.grid[::-1]:
            raise ValueError(f"psi must have shape (Nz, Ny, Nx) = {self.grid[::-1]}, got {tuple(psi.shape)}")
        if not psi.is_contiguous():
            raise ValueError("psi must be contiguous")
        return ctypes.c_void_p(psi.data_ptr()), psi.numel()

    def _use_current_stream(self):
        _check(lib().gp_set_stream(self._handle, self._stream_handle(None)), "gp_set_stream")

    def step(self, psi, nsteps: int = 1):
        """Queue nsteps SSCN steps on psi (in place) on the current torch stream."""
        ptr, n = self._psi(psi)
        self._use_current_stream()
        _check(lib().gp_step(self._handle, ptr, n, int(nsteps)), "gp_step")
        return psi

    def observables(self, psi) -> dict:
        ptr, n = self._psi(psi)
        self._use_current_stream()
        out = GPObs()
        _check(lib().gp_observables(self._handle, ptr, n, ctypes.byref(out)), "gp_observables")
        return out.as_dict()

    def sync(self) -> None:
        _check(lib().gp_sync(self._handle), "gp_sync")

    def set_g(self, g: float) -> None:
        _check(lib().gp_set_g(self._handle, float(g)), "gp_set_g")
        self.g = float(g)

    def set_trap(self, gamma: float, nu: float, lam: float) -> None:
        _check(lib().gp_set_trap(self._handle, float(gamma), float(nu), float(lam)), "gp_set_trap")
        self.omega = (float(gamma), float(nu), float(lam))

    def density_profiles(self, psi):
        """(px, py, pz): |psi|^2 integrated over the other two axes."""
        import numpy as np

        ptr, n = self._psi(psi)
        self._use_current_stream()
        out = [np.zeros(v) for v in self.grid]
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().gp_density_profiles(self._handle, ptr, n, *[o.ctypes.data_as(dp) for o in out]),
               "gp_density_profiles")
        return tuple(out)

    def step_schedule(self, psi, g_steps=None, trap_steps=None):
        """Queue one step per entry of g_steps (and/or rows of trap_steps,
        shape (n, 3)), each with its own g and trap."""
        import numpy as np

        ptr, n = self._psi(psi)
        g_arr = None if g_steps is None else np.ascontiguousarray(g_steps, dtype=np.float64).reshape(-1)
        t_arr = None if trap_steps is None else np.ascontiguousarray(trap_steps, dtype=np.float64).reshape(-1, 3)
        if g_arr is None and t_arr is None:
            raise ValueError("give g_steps, trap_steps or both")
        nsteps = len(g_arr) if g_arr is not None else len(t_arr)
        if t_arr is not None and len(t_arr) != nsteps:
            raise ValueError("g_steps and trap_steps must have the same length")
        dp = ctypes.POINTER(ctypes.c_double)
        gp_ = None if g_arr is None else g_arr.ctypes.data_as(dp)
        tp_ = None if t_arr is None else t_arr.ctypes.data_as(dp)
        self._use_current_stream()
        _check(lib().gp_step_schedule(self._handle, ptr, n, nsteps, gp_, tp_), "gp_step_schedule")
        if g_arr is not None and nsteps:
            self.g = float(g_arr[-1])
        if t_arr is not None and nsteps:
            self.omega = tuple(float(v) for v in t_arr[-1])
        return psi

    SWEEPS = {"auto": 0, "chunked": 1, "stream": 2}

    def set_sweep(self, strategy: str) -> None:
        """y/z strategy of later steps: "auto", "chunked" or "stream"."""
        _check(lib().gp_plan_set_sweep(self._handle, self.SWEEPS[strategy]), "gp_plan_set_sweep")

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _check(lib().gp_plan_describe(self._handle, buf, len(buf)), "gp_plan_describe")
        return buf.value.decode()

    def profile(self, on: bool = True) -> None:
        _check(lib().gp_profile_enable(self._handle, int(bool(on))), "gp_profile_enable")

    def profile_read(self) -> dict:
        """{kernel class: (total ms, launches)} since the last read."""
        ms = (ctypes.c_double * len(KERNELS))()
        cnt = (ctypes.c_int64 * len(KERNELS))()
        _check(lib().gp_profile_read(self._handle, ms, cnt), "gp_profile_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}

    def close(self) -> None:
        if getattr(self, "_handle", None) and self._handle.value:
            lib().gp_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Independent solves advanced together (gp_batch_*).

    specs: sequence of dicts with keys grid (Nx, Ny, Nz), dx (scalar or
    3-tuple), dt, trap (gamma, nu, lambda), g.  All share mode and dtype.
    """

    def __init__(self, specs, mode="imag", dtype="c128", graph=True, tune=False, stream=None, finish_f64=False,
                 one_launch=False):
        import numpy as np
        import torch

        L = lib()
        self.specs = [dict(sp) for sp in specs]
        n = len(self.specs)
        if n < 1:
            raise ValueError("a batch needs at least one solve")
        grids = np.array([[int(v) for v in sp["grid"]] for sp in self.specs], dtype=np.int64)
        dxs = np.array([[float(v) for v in (sp["dx"] if hasattr(sp["dx"], "__len__") else (sp["dx"],) * 3)]
                        for sp in self.specs], dtype=np.float64)
        dts = np.array([float(sp["dt"]) for sp in self.specs], dtype=np.float64)
        traps = np.array([[float(v) for v in sp["trap"]] for sp in self.specs], dtype=np.float64)
        gs = np.array([float(sp["g"]) for sp in self.specs], dtype=np.float64)
        self.grids = [tuple(int(v) for v in row) for row in grids]
        self.mode = _mode(mode)
        self.dtype = _dtype(dtype)
        self.torch_dtype = torch_dtype_of(self.dtype)
        flags = ((BATCH_GRAPH if graph else 0) | (BATCH_TUNE if tune else 0) | (BATCH_FINISH_F64 if finish_f64 else 0)
                 | (BATCH_ONE_LAUNCH if one_launch else 0))
        self._handle = ctypes.c_void_p()
        self._psis = None
        dp = ctypes.POINTER(ctypes.c_double)
        _check(L.gp_batch_create(n, grids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 dxs.ctypes.data_as(dp), dts.ctypes.data_as(dp), traps.ctypes.data_as(dp),
                                 gs.ctypes.data_as(dp), self.mode, self.dtype, flags,
                                 Plan._stream_handle(stream), ctypes.byref(self._handle)),
               "gp_batch_create")
        self.n = n

    def bind(self, psis):
        """Bind solve i to the torch tensor psis[i] (kept referenced)."""
        if len(psis) != self.n:
            raise ValueError(f"need {self.n} tensors")
        for t, g in zip(psis, self.grids):
            if t.dtype != self.torch_dtype or t.device.type != "cuda" or tuple(t.shape) != g[::-1] \
                    or not t.is_contiguous():
                raise ValueError(f"each psi must be a contiguous {self.torch_dtype} CUDA tensor of shape (Nz, Ny, Nx)")
        ptrs = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in psis])
        elems = (ctypes.c_int64 * self.n)(*[t.numel() for t in psis])
        _check(lib().gp_batch_set_psi(self._handle, ptrs, elems), "gp_batch_set_psi")
        self._psis = list(psis)

    def set_active(self, mask=None):
        arr = None if mask is None else (ctypes.c_ubyte * self.n)(*[1 if m else 0 for m in mask])
        _check(lib().gp_batch_set_active(self._handle, arr), "gp_batch_set_active")

    def step(self, nsteps: int = 1):
        _check(lib().gp_batch_step(self._handle, int(nsteps)), "gp_batch_step")

    def observables(self):
        out = (GPObs * self.n)()
        _check(lib().gp_batch_observables(self._handle, out), "gp_batch_observables")
        return [o.as_dict() for o in out]

    def solve_imag(self, tol: float, check_every: int, max_steps: int):
        """Per-solve |dmu| < tol stopping; returns (observables, steps, converged)."""
        out = (GPObs * self.n)()
        steps = (ctypes.c_int64 * self.n)()
        conv = (ctypes.c_ubyte * self.n)()
        _check(lib().gp_batch_solve_imag(self._handle, float(tol), int(check_every), int(max_steps), out,
                                         steps, conv), "gp_batch_solve_imag")
        return [o.as_dict() for o in out], list(steps), [bool(c) for c in conv]

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(4096)
        _check(lib().gp_batch_describe(self._handle, buf, len(buf)), "gp_batch_describe")
        return buf.value.decode()

    def close(self) -> None:
        if getattr(self, "_handle", None) and self._handle.value:
            lib().gp_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def request_bytes(grid, dtype="c64", mode="imag") -> int:
    """Device bytes a served request of this grid holds while resident (0:
    unsupported grid)."""
    g = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    return int(lib().gp_server_request_bytes(g, _dtype(dtype), _mode(mode)))


_servers = None


def _close_servers():
    for srv in list(_servers or ()):
        srv.close()


class Server:
    """Continuous-batching request server (gp_server_*).

    Requests carry host (numpy) states of the server's dtype, shaped
    (Nz, Ny, Nx); the engine thread in the library admits them by device
    footprint, advances all resident solves together and writes each final
    state to the request's output array before reporting it.
    """

    def __init__(self, dtype="c64", hbm_budget: int = 8 << 30, max_slots: int = 64, check_every: int = 10,
                 graph: bool = True, real_auto: bool = False):
        import atexit
        import weakref

        import numpy as np

        global _servers
        L = lib()
        self.dtype = _dtype(dtype)
        self.np_dtype = numpy_dtype_of(self.dtype)
        self.check_every = int(check_every)
        self._handle = ctypes.c_void_p()
        self._held = {}
        _check(L.gp_server_create(self.dtype, int(hbm_budget), int(max_slots), self.check_every,
                                  (SERVER_GRAPH if graph else 0) | (SERVER_REAL_AUTO if real_auto else 0),
                                  ctypes.byref(self._handle)), "gp_server_create")
        if _servers is None:
            _servers = weakref.WeakSet()
            atexit.register(_close_servers)
        _servers.add(self)

    def submit(self, psi_in, *, dx, dt, trap, g, mode="imag", steps, tol=0.0, psi_out=None, tag=0) -> int:
        """Queue one request; returns its id.  psi_in (and psi_out, default a
        new array) are kept referenced until the result is polled.  A real
        psi_in (float64 on a c128 server, float32 on a c64 one) asks for an
        imaginary-time solve on real storage."""
        import numpy as np

        real_dt = {C128: np.float64, C64: np.float32}.get(self.dtype)
        real_state = real_dt is not None and isinstance(psi_in, np.ndarray) and psi_in.dtype == real_dt \
            and self.np_dtype != real_dt
        if not isinstance(psi_in, np.ndarray) or (psi_in.dtype != self.np_dtype and not real_state) \
                or psi_in.ndim != 3 or not psi_in.flags.c_contiguous:
            raise ValueError(f"psi_in must be a C-contiguous {np.dtype(self.np_dtype).name} array (Nz, Ny, Nx)")
        if psi_out is None:
            psi_out = np.empty_like(psi_in)
        elif psi_out.shape != psi_in.shape or psi_out.dtype != psi_in.dtype or not psi_out.flags.c_contiguous \
                or not psi_out.flags.writeable:
            raise ValueError("psi_out must be a writeable C-contiguous array like psi_in")
        nz, ny, nx = psi_in.shape
        dxs = tuple(float(v) for v in (dx if hasattr(dx, "__len__") else (dx,) * 3))
        r = GPRequest()
        r.grid[:] = [nx, ny, nz]
        r.dx[:] = dxs
        r.dt = float(dt)
        r.trap[:] = [float(v) for v in trap]
        r.g = float(g)
        r.mode = _mode(mode)
        r.steps = int(steps)
        r.tol = float(tol)
        r.psi_in = psi_in.ctypes.data
        r.psi_out = psi_out.ctypes.data
        r.tag = int(tag)
        r.real_state = 1 if real_state else 0
        rid = ctypes.c_uint64()
        _check(lib().gp_server_submit(self._handle, ctypes.byref(r), ctypes.byref(rid)), "gp_server_submit")
        self._held[rid.value] = (psi_in, psi_out)
        return rid.value

    def poll(self, max_results: int = 256, wait: float = 0.0) -> list:
        """Finished results (dicts), waiting up to `wait` seconds for the first."""
        out = (GPResult * max_results)()
        n = ctypes.c_int()
        _check(lib().gp_server_poll(self._handle, out, max_results, float(wait), ctypes.byref(n)), "gp_server_poll")
        res = []
        for r in out[:n.value]:
            held = self._held.pop(r.id, (None, None))
            res.append({"id": r.id, "tag": r.tag, "status": r.status, "converged": bool(r.converged),
                        "steps": r.steps, "obs": r.obs.as_dict(), "t_submit": r.t_submit, "t_admit": r.t_admit,
                        "t_done": r.t_done, "psi": held[1]})
        return res

    def drain(self, wait: float = 600.0) -> bool:
        """Wait until nothing is queued or resident; True if reached."""
        idle = ctypes.c_int()
        _check(lib().gp_server_drain(self._handle, float(wait), ctypes.byref(idle)), "gp_server_drain")
        return bool(idle.value)

    def stats(self) -> dict:
        c = GPServerCounters()
        _check(lib().gp_server_stats(self._handle, ctypes.byref(c)), "gp_server_stats")
        return {name: getattr(c, name) for name, _ in GPServerCounters._fields_}

    def close(self) -> None:
        if getattr(self, "_handle", None) and self._handle.value:
            lib().gp_server_destroy(self._handle)
            self._handle = ctypes.c_void_p()
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
