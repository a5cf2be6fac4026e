"""Pins of the oracle's symmetric-trap forms (gpo_radial.c): circular (2D,
r), spherical (3D, r) and axially symmetric (3D, rho and z).

The radial discretisation is this oracle's own reading (the paper names the
programs but prints no scheme), so it is pinned against what does not
depend on it: the Cartesian oracle on the same physical problem, the
oscillator's closed-form energy and size with their O(h^2) approach, the
Thomas-Fermi chemical potentials, the virial theorem in D dimensions,
unitarity in real time and the realness of imaginary-time states.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1206_1361_amd import inputs

IMAG, REAL = oracle.IMAG, oracle.REAL


def radial_gaussian(n, h, w):
    r = (np.arange(n) + 0.5) * h
    return np.exp(-0.5 * w * r * r).astype(np.complex128).reshape(1, 1, n)


def axial_gaussian(nr, nz, hr, hz, gam, lam):
    r = (np.arange(nr) + 0.5) * hr
    z = inputs.axis(nz, hz)
    psi = np.exp(-0.5 * (gam * r[None, :] ** 2 + lam * z[:, None] ** 2))
    return psi.astype(np.complex128).reshape(1, nz, nr)


def relax_radial(geom, n, h, w, g, t_end, dz=1.0, nz=1, lam=0.0):
    dt = 0.1 * min(h, dz if geom == "axial" else h) ** 2
    psi = axial_gaussian(n, nz, h, dz, w, lam) if geom == "axial" else radial_gaussian(n, h, w)
    oracle.radial_step(psi, geom, (h, dz, 1.0), dt, (w, 0.0, lam), g, IMAG, int(round(t_end / dt)))
    return psi, oracle.radial_observables(psi, geom, (h, dz, 1.0), (w, 0.0, lam), g)


@pytest.mark.parametrize("geom,e_exact,r2_exact", [("circular", 1.0, 1.0), ("spherical", 1.5, 1.5)])
def test_oscillator_continuum_limit(oracle_lib, geom, e_exact, r2_exact):
    """g = 0, w = 1: E -> D/2 and <r^2> -> D/2 with an O(h^2) error."""
    errs = []
    for h, n in ((0.2, 40), (0.1, 80)):
        _, o = relax_radial(geom, n, h, 1.0, 0.0, 16.0)
        errs.append((o["energy"] / e_exact - 1.0, o["rms_x"] ** 2 / r2_exact - 1.0))
        assert abs(o["norm"] - 1.0) < 1e-13
    for q in range(2):
        assert abs(errs[1][q]) <= 3e-3
        assert 3.0 <= errs[0][q] / errs[1][q] <= 5.0, errs


def test_axial_oscillator_continuum_limit(oracle_lib):
    """g = 0: E -> gamma + lambda/2, <rho^2> -> 1/gamma, <z^2> -> 1/(2 lambda)."""
    gam, lam = 1.0, 2.0
    errs = []
    for h, nr, nz in ((0.25, 28, 40), (0.125, 56, 80)):
        _, o = relax_radial("axial", nr, h, gam, 0.0, 12.0, dz=h, nz=nz, lam=lam)
        errs.append((o["energy"] / (gam + lam / 2) - 1.0, o["rms_x"] ** 2 * gam - 1.0,
                     o["rms_y"] ** 2 * 2 * lam - 1.0))
    for q in range(3):
        assert abs(errs[1][q]) <= 6e-3
        assert 3.0 <= errs[0][q] / errs[1][q] <= 5.0, errs


def _cartesian_mu(ndim, grid, dx, omega, g, t_end):
    dt = 0.1 * dx[0] ** 2
    om = tuple(omega[a] if a < ndim else 0.0 for a in range(3))
    psi = inputs.gaussian(grid, dx, om)
    psi /= math.sqrt(np.vdot(psi, psi).real * np.prod(dx[:ndim]))
    oracle.step(psi, dx, dt, om, g, IMAG, int(round(t_end / dt)), ndim=ndim)
    return oracle.observables(psi, dx, om, g, ndim=ndim)["mu"]


def test_circular_agrees_with_the_cartesian_plane(oracle_lib):
    """The same isotropic 2D problem in polar and Cartesian form: mu agree to
    the Cartesian discretisation error, estimated from two spacings."""
    w, g = 1.0, 50.0
    mu_c = [_cartesian_mu(2, (n, n, 1), (d, d, 1.0), (w, w, 0), g, 12.0) for d, n in ((0.3, 50), (0.2, 76))]
    mu_inf = mu_c[1] + (mu_c[1] - mu_c[0]) * 0.2 ** 2 / (0.3 ** 2 - 0.2 ** 2)   # Richardson
    _, o = relax_radial("circular", 150, 0.05, w, g, 12.0)
    assert abs(mu_c[1] - mu_c[0]) > 1e-5                   # the extrapolation has something to do
    assert abs(o["mu"] / mu_inf - 1.0) <= 3e-4, (o["mu"], mu_c, mu_inf)


def test_spherical_agrees_with_cartesian_space(oracle_lib):
    w, g = 1.0, 30.0
    mu_c = [_cartesian_mu(3, (n, n, n), (d,) * 3, (w, w, w), g, 8.0) for d, n in ((0.4, 30), (0.3, 40))]
    mu_inf = mu_c[1] + (mu_c[1] - mu_c[0]) * 0.3 ** 2 / (0.4 ** 2 - 0.3 ** 2)
    _, o = relax_radial("spherical", 120, 0.05, w, g, 8.0)
    assert abs(o["mu"] / mu_inf - 1.0) <= 1.5e-3, (o["mu"], mu_c, mu_inf)


def test_axial_agrees_with_cartesian_space(oracle_lib):
    gam, lam, g = 1.0, 1.6, 30.0
    mu_c = []
    for d, n, nz in ((0.4, 30, 26), (0.3, 40, 34)):
        mu_c.append(_cartesian_mu(3, (n, n, nz), (d,) * 3, (gam, gam, lam), g, 8.0))
    mu_inf = mu_c[1] + (mu_c[1] - mu_c[0]) * 0.3 ** 2 / (0.4 ** 2 - 0.3 ** 2)
    _, o = relax_radial("axial", 60, 0.1, gam, g, 8.0, dz=0.1, nz=104, lam=lam)
    assert abs(o["mu"] / mu_inf - 1.0) <= 1.5e-3, (o["mu"], mu_c, mu_inf)


def test_thomas_fermi_limits(oracle_lib):
    """mu -> sqrt(g w^2 / pi) (circular), 1/2 (15 g w^3 / (4 pi))^(2/5)
    (spherical), 1/2 (15 g gamma^2 lambda / (4 pi))^(2/5) (axial)."""
    w, lam = 1.0, 1.5
    for geom, mu_tf in (("circular", lambda g: math.sqrt(g * w * w / math.pi)),
                        ("spherical", lambda g: 0.5 * (15 * g * w ** 3 / (4 * math.pi)) ** 0.4),
                        ("axial", lambda g: 0.5 * (15 * g * w * w * lam / (4 * math.pi)) ** 0.4)):
        ratios = []
        for g in (200.0, 4000.0):
            R = math.sqrt(2 * mu_tf(g)) / min(w, lam)
            if geom == "axial":
                h = 1.3 * R / 48
                _, o = relax_radial("axial", 48, h, w, g, 10.0, dz=h, nz=96, lam=lam)
            else:
                h = 1.3 * R / 200
                _, o = relax_radial(geom, 200, h, w, g, 10.0)
            ratios.append(o["mu"] / mu_tf(g))
        assert 1.0 < ratios[1] < ratios[0], (geom, ratios)
        assert ratios[1] <= 1.04, (geom, ratios)


@pytest.mark.parametrize("geom,dim", [("circular", 2), ("spherical", 3)])
def test_virial_theorem(oracle_lib, geom, dim):
    _, o = relax_radial(geom, 160, 0.05, 1.0, 40.0, 14.0)
    v = 2 * o["kinetic"] - 2 * o["potential"] + 0.5 * dim * o["interaction"]
    assert abs(v) <= 2e-3 * o["energy"]


def test_axial_virial_theorem(oracle_lib):
    _, o = relax_radial("axial", 50, 0.12, 1.0, 40.0, 10.0, dz=0.12, nz=100, lam=1.3)
    v = 2 * o["kinetic"] - 2 * o["potential"] + 1.5 * o["interaction"]
    assert abs(v) <= 5e-3 * o["energy"]


@pytest.mark.parametrize("geom", ["circular", "spherical", "axial"])
def test_real_time_is_unitary_and_imaginary_time_stays_real(oracle_lib, geom):
    rng = np.random.default_rng(4)
    shape = (1, 30, 40) if geom == "axial" else (1, 1, 60)
    psi = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex128)
    dx, om = (0.2, 0.2, 1.0), (1.0, 0.0, 1.4)
    n0 = oracle.radial_observables(psi, geom, dx, om, 0.0)["norm"]
    oracle.radial_step(psi, geom, dx, 0.01, om, 25.0, REAL, 40)
    assert abs(oracle.radial_observables(psi, geom, dx, om, 0.0)["norm"] / n0 - 1.0) <= 1e-13
    re = np.ascontiguousarray(psi.real).astype(np.complex128)
    oracle.radial_step(re, geom, dx, 0.01, om, 25.0, IMAG, 20)
    assert np.max(np.abs(re.imag)) == 0.0


def test_rejects_bad_shapes(oracle_lib):
    for geom, shape in (("circular", (1, 2, 10)), ("spherical", (2, 1, 10)), ("axial", (2, 3, 4))):
        psi = np.zeros(shape, np.complex128) + 1.0
        with pytest.raises(oracle.OracleError):
            oracle.radial_step(psi, geom, (0.1, 0.1, 0.1), 0.01, (1, 1, 1), 1.0, IMAG, 1)
