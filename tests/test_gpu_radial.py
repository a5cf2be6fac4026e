"""Symmetric traps (gp_plan_create_radial) against the oracle's radial forms
(gpo_radial.c), which are pinned in test_oracle_pins_radial.py."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1206_1361_amd as gp  # noqa: E402

# (psi, mu and energy) relative to the oracle.  Float storage on these grids
# of at most 26000 points: mu and E within 1e-6 (the per-store rounding is
# not averaged below 1e-7 on so few points; measured at most 3.0e-7).  The
# norm: 2e-7 in imaginary time (renormalised to within a float ulp), and in
# real time 2 (3n + 1) 2^-24 after n steps: the FP32 Crank-Nicolson and
# phase factors are unitary only to about 2^-24 each, and each store can
# move |psi|^2 by 2 x 2^-24 (measured at most 5.5e-7 at n = 6).
TOL = {"c128": (1e-12, 1e-12), "c64": (1e-5, 1e-6), "r64": (1e-12, 1e-12), "r32": (1e-5, 1e-6)}


def norm_tol(dtype, mode, nsteps):
    if dtype in ("c128", "r64"):
        return 1e-12
    return 2 * (3 * nsteps + 1) * 2.0 ** -24 if mode == "real" else 2e-7
TORCH = {"c128": torch.complex128, "c64": torch.complex64, "r64": torch.float64, "r32": torch.float32}
MODE_DTYPES = [("imag", d) for d in ("c128", "c64", "r64", "r32")] + [("real", d) for d in ("c128", "c64")]
CASES = [("circular", (1, 1, 1)), ("circular", (37, 1, 1)), ("circular", (200, 1, 1)), ("circular", (1024, 1, 1)),
         ("spherical", (64, 1, 1)), ("spherical", (301, 1, 1)),
         ("axial", (20, 33, 1)), ("axial", (64, 50, 1)), ("axial", (130, 96, 1))]
OMEGA = (1.0, 0.0, 1.6)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def start(geom, grid, dx, real_state, seed):
    rng = np.random.default_rng(seed)
    nr, nz = grid[0], grid[1]
    r = (np.arange(nr) + 0.5) * dx[0]
    z = (np.arange(nz) - 0.5 * (nz - 1)) * dx[1]
    env = np.exp(-0.5 * (OMEGA[0] * r[None, :] ** 2 + (OMEGA[2] * z[:, None] ** 2 if geom == "axial" else 0.0)))
    noise = rng.standard_normal((nz, nr)) + (0 if real_state else 1j * rng.standard_normal((nz, nr)))
    psi = env * (1.0 + 0.2 * noise)
    return np.ascontiguousarray(psi.reshape(1, nz, nr)).astype(np.complex128)


@pytest.mark.parametrize("mode,dtype", MODE_DTYPES)
@pytest.mark.parametrize("geom,grid", CASES)
def test_radial_step_matches_oracle(geom, grid, mode, dtype):
    dx = (6.0 / max(grid[0], 8), 0.2, 1.0)
    dt = (0.1 if mode == "imag" else 0.02) * dx[0] ** 2
    g, steps = 30.0, 5
    real_state = dtype in ("r64", "r32")
    psi0 = start(geom, grid, dx, real_state, sum(grid))
    if dtype in ("c64", "r32"):   # the oracle starts from the values the GPU holds
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    ref = psi0.copy()
    oracle.radial_step(ref, geom, dx, dt, OMEGA, g, oracle.IMAG if mode == "imag" else oracle.REAL, steps)
    robs = oracle.radial_observables(ref, geom, dx, OMEGA, g)
    t = torch.from_numpy(psi0.real.copy() if real_state else psi0).to(TORCH[dtype]).cuda()
    with gp.Plan(grid, dx, dt, *OMEGA, g, mode=mode, dtype=dtype, geometry=geom) as p:
        p.step(t, steps)
        obs = p.observables(t)
        assert geom in p.describe()
    got = t.cpu().numpy().astype(np.complex128)
    tpsi, tobs = TOL[dtype]
    assert rel(got, ref) <= tpsi
    assert abs(obs["norm"] - robs["norm"]) <= norm_tol(dtype, mode, steps) * robs["norm"]
    for k in ("mu", "energy", "rms_x", "rms_r"):
        assert abs(obs[k] - robs[k]) <= tobs * abs(robs[k]), k
    if geom == "axial":
        assert abs(obs["rms_y"] - robs["rms_y"]) <= tobs * robs["rms_y"]


@pytest.mark.parametrize("geom,grid,dx", [("spherical", (240, 1, 1), (0.04, 1.0, 1.0)),
                                          ("circular", (300, 1, 1), (0.04, 1.0, 1.0)),
                                          ("axial", (64, 96, 1), (0.12, 0.12, 1.0))])
def test_radial_ground_state_matches_oracle(geom, grid, dx):
    g, dt, steps = 200.0, 0.1 * dx[0] ** 2, 1500
    psi0 = start(geom, grid, dx, True, 3)
    ref = psi0.copy()
    oracle.radial_step(ref, geom, dx, dt, OMEGA, g, oracle.IMAG, steps)
    robs = oracle.radial_observables(ref, geom, dx, OMEGA, g)
    t = torch.from_numpy(psi0).cuda()
    with gp.Plan(grid, dx, dt, *OMEGA, g, mode="imag", dtype="c128", geometry=geom) as p:
        p.step(t, steps)
        obs = p.observables(t)
    assert rel(t.cpu().numpy(), ref) <= 1e-12
    for k in ("norm", "mu", "energy", "rms_x", "rms_r"):
        assert abs(obs[k] - robs[k]) <= 1e-12 * abs(robs[k]), k
    assert abs(obs["norm"] - 1.0) <= 1e-13


def test_radial_real_time_conserves_the_weighted_norm():
    grid, dx = (200, 1, 1), (0.04, 1.0, 1.0)
    t = torch.from_numpy(start("spherical", grid, dx, False, 8)).cuda()
    with gp.Plan(grid, dx, 1e-4, *OMEGA, 50.0, mode="real", dtype="c128", geometry="spherical") as p:
        n0 = p.observables(t)["norm"]
        p.step(t, 400)
        n1 = p.observables(t)["norm"]
    assert abs(n1 / n0 - 1.0) <= 1e-12


def test_radial_rejects_bad_shapes():
    for geom, grid in (("circular", (10, 2, 1)), ("spherical", (10, 1, 3)), ("axial", (10, 10, 2))):
        with pytest.raises(gp.GPInvalid):
            gp.Plan(grid, (0.1, 0.1, 0.1), 0.01, 1, 1, 1, 1.0, geometry=geom)
