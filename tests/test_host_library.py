"""Host-side checks of libgpssc that need no GPU: the exported C ABI, argument
validation before any device call, the launch-shape policy, and the chunked
constant-coefficient scheme the sweep kernels run, replayed in numpy with
the library's own coefficients and compared with a dense solve."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1206_1361_amd as gp
from paper_1206_1361_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "gpssc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = gp.lib()
    declared = header_functions()
    assert declared, "no declarations found"
    assert sorted(_binding.EXPORTS) == declared
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings_and_last_error():
    L = gp.lib()
    for code in range(6):
        assert L.gp_status_string(code)
    assert L.gp_status_string(99) == b"unknown status"
    out = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(0, 4, 4)
    d = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    assert L.gp_plan_create(n, d, 0.01, 1.0, 1.0, 1.0, 1.0, 0, 0, None, ctypes.byref(out)) == 1
    assert b"grid" in L.gp_last_error()
    assert out.value is None


BAD_CREATE = [
    dict(grid=(0, 4, 4)), dict(grid=(4, -1, 4)), dict(dx=(0.1, 0.0, 0.1)), dict(dx=(0.1, float("nan"), 0.1)),
    dict(dt=0.0), dict(dt=-1.0), dict(dt=float("inf")), dict(gamma=-1.0), dict(lam=float("nan")),
    dict(g=float("inf")), dict(mode=7), dict(dtype=7),
    dict(dtype=3, mode=1), dict(dtype=4, mode=1),     # real storage is imaginary time only
]


@pytest.mark.parametrize("bad", BAD_CREATE)
def test_plan_create_rejects_bad_arguments_before_any_device_call(bad):
    args = dict(grid=(8, 8, 8), dx=(0.1, 0.1, 0.1), dt=0.01, gamma=1.0, nu=1.0, lam=1.0, g=1.0, mode=0, dtype=0)
    args.update(bad)
    L = gp.lib()
    out = ctypes.c_void_p(1234)
    n = (ctypes.c_int64 * 3)(*args["grid"])
    d = (ctypes.c_double * 3)(*args["dx"])
    st = L.gp_plan_create(n, d, args["dt"], args["gamma"], args["nu"], args["lam"], args["g"],
                          args["mode"], args["dtype"], None, ctypes.byref(out))
    assert st == _binding.ERR_INVALID
    assert out.value is None


def test_plan_create_rejects_unsupported_lengths():
    L = gp.lib()
    out = ctypes.c_void_p()
    d = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    for grid in ((1025, 8, 8), (8, 1025, 8), (8, 8, 4096)):
        n = (ctypes.c_int64 * 3)(*grid)
        assert L.gp_plan_create(n, d, 0.01, 1.0, 1.0, 1.0, 1.0, 0, 0, None, ctypes.byref(out)) == \
            _binding.ERR_UNSUPPORTED


def test_null_plan_arguments():
    L = gp.lib()
    assert L.gp_plan_destroy(None) == 0
    assert L.gp_set_g(None, 1.0) == _binding.ERR_INVALID
    assert L.gp_step(None, None, 0, 1) == _binding.ERR_INVALID
    assert L.gp_sync(None) == _binding.ERR_INVALID
    assert L.gp_observables(None, None, 0, None) == _binding.ERR_INVALID
    assert L.gp_plan_create(None, None, 0.1, 1, 1, 1, 1, 0, 0, None, None) == _binding.ERR_INVALID


def test_footprint():
    assert gp.footprint_bytes((0, 8, 8)) == 0
    small = gp.footprint_bytes((32, 32, 32))
    large = gp.footprint_bytes((512, 512, 384))
    assert 0 < small < large < 8 << 20        # tables + scratch only (O(Nx Ny)), not psi
    assert gp.footprint_bytes((512, 512, 384), "c64") < large


@pytest.mark.parametrize("n", [1, 2, 31, 63, 64, 65, 200, 240, 384, 511, 512, 1000, 1024])
def test_sweep_shapes(n):
    cx, lx = gp.sweep_shape(n, 0)
    assert lx == 64 and cx * 64 >= n and (cx == 1 or (cx - 1) * 64 < n or cx in (10, 12, 14, 16))
    for axis in (1, 2):
        c, l = gp.sweep_shape(n, axis)
        assert c * l >= n and l <= 64 and (l - 1) * c < n
    with pytest.raises(gp.GPError):
        gp.sweep_shape(2048, 1)
    # short lines take few, long chunks: at most 8 up to 128 points, 16 up
    # to 256, the same for every storage; real float32 storage cuts longer
    # lines into at most 32 chunks of at most 16 points, the 16-byte values
    # (complex128, complex64 column pairs) into chunks of at most 8 points up
    # to 384 points
    for dt in ("c128", "c64", "r32", "r64"):
        if n <= 512:
            c, l = gp.sweep_shape(n, 1, dt)
            assert c * l >= n and (l - 1) * c < n and c <= 16
            assert l <= (8 if n <= 128 else 16 if n <= 256 else 32 if dt == "r32" else 64)
            if dt != "r32" and 256 < n <= 384:
                assert c <= 8
            assert (c, l) == gp.sweep_shape(n, 2, dt)


def dense_cn_rhs_solve(n, tab, psi):
    kap = tab["kappa"]
    A = (1 + kap) * np.eye(n) - kap / 2 * (np.eye(n, k=1) + np.eye(n, k=-1))
    B = (1 - kap) * np.eye(n) + kap / 2 * (np.eye(n, k=1) + np.eye(n, k=-1))
    return np.linalg.solve(A, B @ psi)


def chunked_solve(tab, n, chunk, lanes, psi, stages=None):
    """The sweep kernels' scheme, replayed with the library's coefficients:
    per-chunk recurrences with a zero carry, Kogge-Stone over the chunks,
    rerun from the carry, padding cleared, then the boundary correction."""
    npad = chunk * lanes
    u = np.zeros(npad, complex)
    u[:n] = psi
    left = np.concatenate([[0], u[:-1]])
    right = np.concatenate([u[1:], [0]])
    kap = tab["kappa"]
    r = u + kap * ((left + right) / 2 - u)
    mr = tab["m"] * r
    a = tab["a"]
    st = tab["stage"]
    if stages is None:
        stages = 0
        for s in range(6):
            if (1 << s) < lanes and st[s] != 0 and stages == s:
                stages = s + 1

    def run(vals, carry, k, backward):
        idx = range(k * chunk, (k + 1) * chunk)
        idx = list(reversed(idx)) if backward else list(idx)
        t = carry
        out = {}
        for i in idx:
            t = vals[i] + a * t
            out[i] = t
        return t, out

    L = [run(mr, 0, k, False)[0] for k in range(lanes)]
    F = list(L)
    for s in range(stages):
        d = 1 << s
        F = [F[k] + (st[s] * F[k - d] if k >= d else 0) for k in range(lanes)]
    w = np.zeros(npad, complex)
    for k in range(lanes):
        for i, v in run(mr, F[k - 1] if k > 0 else 0, k, False)[1].items():
            w[i] = v
    w[n:] = 0
    U = [run(w, 0, k, True)[0] for k in range(lanes)]
    R = list(U)
    for s in range(stages):
        d = 1 << s
        R = [R[k] + (st[s] * R[k + d] if k + d < lanes else 0) for k in range(lanes)]
    y = np.zeros(npad, complex)
    for k in range(lanes):
        for i, v in run(w, R[k + 1] if k + 1 < lanes else 0, k, True)[1].items():
            y[i] = v
    x = y[:n] + y[0] * tab["zt"]
    return x


@pytest.mark.parametrize("mode", ["imag", "real"])
@pytest.mark.parametrize("n,dx,dt", [(1, 0.25, 0.006), (2, 0.25, 0.006), (7, 0.25, 0.006),
                                     (32, 0.25, 0.00625), (200, 0.1, 5e-5), (240, 0.1, 0.01),
                                     (384, 0.05, 1.25e-5), (512, 0.05, 0.25), (97, 0.1, 1.0),
                                     (130, 0.05, 0.5)])
def test_chunked_solve_with_library_coefficients_matches_dense_solve(mode, n, dx, dt):
    rng = np.random.default_rng(n)
    psi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for axis in (0, 1):
        chunk, lanes = gp.sweep_shape(n, axis)
        tab = gp.sweep_tables(n, dx, dt, mode, chunk, lanes)
        ref = dense_cn_rhs_solve(n, tab, psi)
        x = chunked_solve(tab, n, chunk, lanes, psi)
        assert np.max(np.abs(x - ref)) <= 1e-14 * np.max(np.abs(ref)), axis
        if lanes > 1:   # dropping the stages whose multiplier is zero changes nothing
            full = chunked_solve(tab, n, chunk, lanes, psi, stages=min(6, (lanes - 1).bit_length()))
            assert np.array_equal(full, x)


@pytest.mark.parametrize("mode", ["imag", "real"])
@pytest.mark.parametrize("kap", [1e-6, 0.0025, 0.05, 1.0, 100.0])
def test_constant_coefficient_factorisation(mode, kap):
    n = 9
    dx = 1.0
    dt = 2 * kap
    tab = gp.sweep_tables(n, dx, dt, mode, 1, n)
    kappa = (1j if mode == "real" else 1) * kap
    assert abs(tab["kappa"] - kappa) <= 1e-15 * kap
    assert abs(tab["c"]) < 1
    S = np.eye(n, k=-1)
    I = np.eye(n)
    A = (1 + kappa) * I - kappa / 2 * (S + S.T)
    fac = tab["beta"] * (I + tab["c"] * S) @ (I + tab["c"] * S.T)
    fac[0, 0] += tab["beta"] * tab["c"] ** 2
    assert np.max(np.abs(fac - A)) <= 1e-14 * np.max(np.abs(A))
    assert abs(tab["m"] * tab["beta"] - 1) <= 1e-15 and tab["a"] == -tab["c"]
    assert abs(tab["stage"][0] - tab["a"]) <= 1e-16 and abs(tab["stage"][1] - tab["a"] ** 2) <= 1e-15


def test_sweep_tables_reject_short_chunking():
    with pytest.raises(gp.GPError):
        gp.sweep_tables(10, 0.5, 0.1, "real", 1, 5)     # chunk * lanes < n


def test_gpu_path_and_oracle_share_no_code():
    """The library and the oracle neither import nor include each other."""
    pkg = os.path.join(ROOT, "paper_1206_1361_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "gpo." not in text and "gpo_" not in text, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1206_1361_amd" not in text and "gpssc" not in text, f


def test_batch_create_rejects_bad_arguments_before_any_device_call():
    L = gp.lib()
    i64 = ctypes.c_int64
    dbl = ctypes.c_double

    def create(n=2, grids=None, dx=0.2, dt=0.004, trap=1.0, g=1.0, mode=0, dtype=1, flags=0):
        grids = grids or [8, 8, 8] * n
        G = (i64 * len(grids))(*grids)
        D = (dbl * (3 * n))(*([dx] * (3 * n)))
        T = (dbl * n)(*([dt] * n))
        W = (dbl * (3 * n))(*([trap] * (3 * n)))
        Gs = (dbl * n)(*([g] * n))
        out = ctypes.c_void_p(99)
        st = L.gp_batch_create(n, G, D, T, W, Gs, mode, dtype, flags, None, ctypes.byref(out))
        return st, out.value

    assert create(n=0) == (_binding.ERR_INVALID, None)
    assert create(grids=[8, 8, 8, 0, 8, 8]) == (_binding.ERR_INVALID, None)
    assert create(dx=-1.0) == (_binding.ERR_INVALID, None)
    assert create(dt=float("nan")) == (_binding.ERR_INVALID, None)
    assert create(trap=-0.5) == (_binding.ERR_INVALID, None)
    assert create(g=float("inf")) == (_binding.ERR_INVALID, None)
    assert create(mode=5) == (_binding.ERR_INVALID, None)
    assert create(flags=16) == (_binding.ERR_INVALID, None)
    assert create(flags=8) == (_binding.ERR_UNSUPPORTED, None)   # GP_BATCH_ONE_LAUNCH, switched off
    assert create(grids=[8, 8, 8, 8, 2000, 8]) == (_binding.ERR_UNSUPPORTED, None)
    assert create(dtype=3, mode=1) == (_binding.ERR_INVALID, None)
    assert create(dtype=9) == (_binding.ERR_INVALID, None)
    assert L.gp_batch_destroy(None) == _binding.OK
    assert L.gp_batch_step(None, 1) == _binding.ERR_INVALID
    assert L.gp_batch_observables(None, None) == _binding.ERR_INVALID


def test_server_request_bytes():
    """Footprint used for admission: psi plus tables and reduction scratch,
    256-byte blocks; imaginary time adds the per-line norm partials."""
    psi = 40 * 32 * 24 * 8
    imag = gp.request_bytes((40, 32, 24), "c64", "imag")
    real = gp.request_bytes((40, 32, 24), "c64", "real")
    assert imag % 256 == 0 and real % 256 == 0
    assert psi < real < imag
    assert imag - real >= 40 * 32 * 8
    assert gp.request_bytes((40, 32, 24), "c128", "imag") > imag
    assert gp.request_bytes((2000, 8, 8), "c64", "imag") == 0
    r64 = gp.request_bytes((40, 32, 24), "r64", "imag")
    r32 = gp.request_bytes((40, 32, 24), "r32", "imag")
    assert 40 * 32 * 24 * 4 < r32 < r64 < gp.request_bytes((40, 32, 24), "c128", "imag")


def test_plan_create_nd_rejects_bad_shapes_before_any_device_call():
    L = gp.lib()
    d = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    for ndim, grid in ((0, (8, 1, 1)), (4, (8, 8, 8)), (2, (8, 8, 2)), (1, (8, 2, 1)), (1, (8, 1, 3))):
        n = (ctypes.c_int64 * 3)(*grid)
        out = ctypes.c_void_p(5)
        assert L.gp_plan_create_nd(ndim, n, d, 0.01, 1.0, 1.0, 1.0, 1.0, 0, 0, None, ctypes.byref(out)) == \
            _binding.ERR_INVALID, (ndim, grid)
        assert out.value is None


def test_plan_create_radial_rejects_bad_arguments_before_any_device_call():
    L = gp.lib()
    d = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    for geom, grid, nu in ((0, (8, 1, 1), 1.0), (4, (8, 1, 1), 1.0), (1, (8, 2, 1), 1.0), (3, (8, 8, 2), 1.0),
                           (2, (8, 1, 1), float("nan"))):
        n = (ctypes.c_int64 * 3)(*grid)
        out = ctypes.c_void_p(5)
        assert L.gp_plan_create_radial(geom, n, d, 0.01, 1.0, nu, 1.0, 1.0, 0, 0, None, ctypes.byref(out)) == \
            _binding.ERR_INVALID, (geom, grid)
        assert out.value is None


def test_noalloc_step_checks_arguments_before_any_device_call():
    """gp_step_noalloc validates like gp_plan_create and gp_step, and refuses
    grids beyond its static scratch (Nx * Ny <= 262144) with a clear error,
    all before touching a device."""
    L = gp.lib()
    d = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    psi = ctypes.c_void_p(4096)   # never dereferenced: every case fails first
    cases = [
        ((8, 8, 8), 0.0, 1, _binding.ERR_INVALID),          # dt
        ((0, 8, 8), 0.01, 1, _binding.ERR_INVALID),         # grid
        ((8, 8, 8), 0.01, -1, _binding.ERR_INVALID),        # nsteps
        ((8, 8, 2000), 0.01, 1, _binding.ERR_UNSUPPORTED),  # line too long
        ((513, 512, 4), 0.01, 1, _binding.ERR_UNSUPPORTED),  # beyond the scratch
    ]
    for grid, dt, nsteps, want in cases:
        n = (ctypes.c_int64 * 3)(*grid)
        elems = grid[0] * grid[1] * grid[2]
        st = L.gp_step_noalloc(n, d, dt, 1.0, 1.0, 1.0, 1.0, 0, 0, None, psi, elems, nsteps)
        assert st == want, (grid, dt, nsteps)
    assert b"262144" in L.gp_last_error()
