"""Pins of the oracle's one- and two-variable forms (ndim = 1, 2).

The reduced forms keep the present variables only: the Laplacian, the trap
and the cell volume of x (and y).  They are checked against a dense
Kronecker-product step, against the product of one-variable runs at g = 0,
the discrete and continuum oscillator energies, the Thomas-Fermi chemical
potentials of one and two dimensions, the d-dimensional virial theorem and
unitarity in real time -- each an independent statement of what the reduced
equation is.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1206_1361_amd import inputs

IMAG, REAL = oracle.IMAG, oracle.REAL


def kin1d(n, d):
    L = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    return -0.5 * L / (d * d)


def cn1d(n, d, dt, mode):
    tau = 1j * dt if mode == REAL else dt
    T = kin1d(n, d)
    I = np.eye(n)
    return np.linalg.solve(I + 0.5 * tau * T, I - 0.5 * tau * T)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def gaussian_nd(grid, dx, omega, ndim):
    """Normalised Gaussian of the present axes, shape (Nz, Ny, Nx)."""
    psi = inputs.gaussian(grid, dx, tuple(w if a < ndim else 0.0 for a, w in enumerate(omega)))
    dv = np.prod(dx[:ndim])
    return psi / math.sqrt(np.vdot(psi, psi).real * dv)


def relax(grid, dx, omega, g, dt, nsteps, ndim):
    psi = gaussian_nd(grid, dx, omega, ndim)
    oracle.step(psi, dx, dt, omega, g, IMAG, nsteps, ndim=ndim)
    return psi


@pytest.mark.parametrize("mode", [IMAG, REAL])
@pytest.mark.parametrize("ndim,grid", [(2, (7, 5, 1)), (1, (9, 1, 1))])
def test_step_matches_dense_operator(oracle_lib, mode, ndim, grid):
    dx, dt, omega, g = (0.35, 0.3, 0.5), 0.03, (1.0, 1.7, 0.6), 3.5
    psi0 = inputs.random_state(grid, dx, seed=7)
    nx, ny, _ = grid
    x = inputs.axis(nx, dx[0])
    y = inputs.axis(ny, dx[1])
    V = 0.5 * (omega[0] ** 2 * x[None, :] ** 2 + (omega[1] ** 2 * y[:, None] ** 2 if ndim == 2 else 0.0))
    v0 = psi0.reshape(-1)
    theta = V.reshape(-1) + g * np.abs(v0) ** 2
    nu = np.exp(-1j * dt * theta) if mode == REAL else np.exp(-dt * theta)
    ref = np.kron(np.eye(ny), cn1d(nx, dx[0], dt, mode)) @ (nu * v0)
    if ndim == 2:
        ref = np.kron(cn1d(ny, dx[1], dt, mode), np.eye(nx)) @ ref
    if mode == IMAG:
        ref = ref / math.sqrt(np.vdot(ref, ref).real * np.prod(dx[:ndim]))
    psi = psi0.copy()
    oracle.step(psi, dx, dt, omega, g, mode, 1, ndim=ndim)
    assert rel(psi.reshape(-1), ref) <= 1e-13


def test_two_variables_separate_at_g0(oracle_lib):
    """At g = 0 a product state stays a product of one-variable runs (with the
    y run using nu and dy), in both modes, to round-off."""
    dx, omega = (0.4, 0.35, 1.0), (1.0, 1.4, 0.0)
    fx = inputs.random_state((12, 1, 1), dx, seed=3).reshape(-1)
    fy = inputs.random_state((9, 1, 1), (dx[1],) * 3, seed=4).reshape(-1)
    for mode in (IMAG, REAL):
        prod = np.ascontiguousarray((fy[:, None] * fx[None, :])[None]).astype(np.complex128)
        oracle.step(prod, dx, 0.02, omega, 0.0, mode, 11, ndim=2)
        px = np.ascontiguousarray(fx.reshape(1, 1, -1)).copy()
        py = np.ascontiguousarray(fy.reshape(1, 1, -1)).copy()
        if mode == IMAG:   # a product normalised in 2D is a product of normalised factors
            px /= math.sqrt(np.vdot(px, px).real * dx[0])
            py /= math.sqrt(np.vdot(py, py).real * dx[1])
            prod0 = (py.reshape(-1)[:, None] * px.reshape(-1)[None, :])[None]
            assert abs(np.vdot(prod0, prod0).real * dx[0] * dx[1] - 1.0) < 1e-13
        oracle.step(px, (dx[0], 1.0, 1.0), 0.02, (omega[0], 0, 0), 0.0, mode, 11, ndim=1)
        oracle.step(py, (dx[1], 1.0, 1.0), 0.02, (omega[1], 0, 0), 0.0, mode, 11, ndim=1)
        out = (py.reshape(-1)[:, None] * px.reshape(-1)[None, :])[None]
        if mode == IMAG:
            out = out / math.sqrt(np.vdot(out, out).real * dx[0] * dx[1])
            prod = prod / math.sqrt(np.vdot(prod, prod).real * dx[0] * dx[1])
        else:
            # the real-time 2D run started from the unnormalised product
            pass
        assert rel(out, prod) <= 1e-12


@pytest.mark.parametrize("ndim,grid", [(1, (40, 1, 1)), (2, (24, 20, 1))])
def test_g0_ground_state_matches_discrete_eigenvalues(oracle_lib, ndim, grid):
    """Energy of the imaginary-time fixed point at g = 0 vs the lowest
    eigenvalue of the discrete present-axis Hamiltonian: O(dt^2) apart."""
    dx, omega = (0.4, 0.4, 0.4), (1.0, 1.4, 2.0)
    e0 = 0.0
    for a in range(ndim):
        x = inputs.axis(grid[a], dx[a])
        e0 += np.linalg.eigvalsh(kin1d(grid[a], dx[a]) + np.diag(0.5 * omega[a] ** 2 * x * x))[0]
    errs = []
    for dt in (0.016, 0.008):
        psi = relax(grid, dx, omega, 0.0, dt, int(round(16.0 / dt)), ndim)
        errs.append(oracle.observables(psi, dx, omega, 0.0, ndim=ndim)["energy"] / e0 - 1.0)
    assert 0 < errs[0] <= 1e-4
    assert 3.5 <= errs[0] / errs[1] <= 4.5


@pytest.mark.parametrize("ndim", [1, 2])
def test_g0_ground_state_continuum_limit(oracle_lib, ndim):
    """E -> sum of the present w_a / 2, rms_a -> 1/sqrt(2 w_a), O(dx^2)."""
    omega = (1.0, 1.4, 0.0)
    e_exact = sum(omega[:ndim]) / 2
    errs = []
    for d, n in ((0.5, 20), (0.25, 40)):
        grid = (n, n if ndim == 2 else 1, 1)
        dx = (d, d, 1.0)
        psi = relax(grid, dx, omega, 0.0, 0.1 * d * d, int(round(12.0 / (0.1 * d * d))), ndim)
        o = oracle.observables(psi, dx, omega, 0.0, ndim=ndim)
        errs.append((o["energy"] / e_exact - 1.0, o["rms_x"] * math.sqrt(2 * omega[0]) - 1.0))
        assert o["rms_z"] == 0.0 and (ndim == 2 or o["rms_y"] == 0.0)
    assert -0.007 <= errs[1][0] < 0 and -0.006 <= errs[1][1] < 0
    assert 3.5 <= errs[0][0] / errs[1][0] <= 4.5
    assert 3.5 <= errs[0][1] / errs[1][1] <= 5.0


def test_thomas_fermi_limits(oracle_lib):
    """mu -> the Thomas-Fermi value of the reduced equation as g grows:
    1D: 1/2 (3 gamma g / 2)^(2/3); 2D: sqrt(gamma nu g / pi)."""
    gam, nu = 1.0, 1.3
    ratios = {1: [], 2: []}
    for g in (100.0, 1000.0):
        # boxes of 1.3 Thomas-Fermi radii either side, relaxed for 10 trap times
        mu1 = 0.5 * (1.5 * gam * g) ** (2.0 / 3.0)
        d = 2.6 * math.sqrt(2 * mu1) / gam / 400
        psi = relax((400, 1, 1), (d, 1.0, 1.0), (gam, 0, 0), g, 0.1 * d * d, int(10 / (0.1 * d * d)), 1)
        ratios[1].append(oracle.observables(psi, (d, 1.0, 1.0), (gam, 0, 0), g, ndim=1)["mu"] / mu1)
        mu2 = math.sqrt(gam * nu * g / math.pi)
        d = 2.6 * math.sqrt(2 * mu2) / min(gam, nu) / 96
        psi = relax((96, 96, 1), (d, d, 1.0), (gam, nu, 0), g, 0.1 * d * d, int(10 / (0.1 * d * d)), 2)
        ratios[2].append(oracle.observables(psi, (d, d, 1.0), (gam, nu, 0), g, ndim=2)["mu"] / mu2)
    for nd in (1, 2):
        r1, r2 = ratios[nd]
        assert 1.0 < r2 < r1, (nd, ratios[nd])
        assert r2 <= 1.05, (nd, ratios[nd])


@pytest.mark.parametrize("ndim,grid", [(1, (160, 1, 1)), (2, (48, 40, 1))])
def test_virial_theorem(oracle_lib, ndim, grid):
    """Stationary states obey 2K - 2P + d I/2 = 0 in d dimensions."""
    dx, omega, g = (0.15 if ndim == 1 else 0.3, 0.3, 1.0), (1.0, 1.4, 0.0), 20.0
    psi = relax(grid, dx, omega, g, 0.1 * dx[0] ** 2, 3000 if ndim == 1 else 1500, ndim)
    o = oracle.observables(psi, dx, omega, g, ndim=ndim)
    v = 2 * o["kinetic"] - 2 * o["potential"] + 0.5 * ndim * o["interaction"]
    assert abs(v) <= 0.01 * o["energy"]
    # the 3D relation does not hold: the reduced equation is not the 3D one
    v3 = 2 * o["kinetic"] - 2 * o["potential"] + 1.5 * o["interaction"]
    assert abs(v3) > 5 * abs(v)


@pytest.mark.parametrize("ndim,grid", [(1, (50, 1, 1)), (2, (20, 16, 1))])
def test_real_time_is_unitary(oracle_lib, ndim, grid):
    dx = (0.3, 0.3, 1.0)
    psi = inputs.random_state(grid, dx, seed=9)
    n0 = oracle.norm(psi, dx, ndim=ndim)
    oracle.step(psi, dx, 0.01, (1.0, 1.5, 0.0), 30.0, REAL, 60, ndim=ndim)
    assert abs(oracle.norm(psi, dx, ndim=ndim) / n0 - 1.0) <= 1e-13


def test_reduced_forms_reject_bad_shapes(oracle_lib):
    psi = inputs.random_state((6, 5, 2), (0.3,) * 3, seed=1)
    for ndim in (0, 1, 2, 4):
        with pytest.raises(oracle.OracleError):
            oracle.step(psi.copy(), (0.3,) * 3, 0.01, (1, 1, 1), 1.0, IMAG, 1, ndim=ndim)
