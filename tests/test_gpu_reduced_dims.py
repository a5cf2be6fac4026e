"""The equation in one and two space variables (gp_plan_create_nd) against
the oracle's reduced forms, which are pinned in test_oracle_pins_nd.py."""
import numpy as np
import pytest

import oracle
from paper_1206_1361_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1206_1361_amd as gp  # noqa: E402

MODES = {"imag": oracle.IMAG, "real": oracle.REAL}
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
CASES = [(1, (1, 1, 1)), (1, (64, 1, 1)), (1, (200, 1, 1)), (1, (1024, 1, 1)),
         (2, (24, 20, 1)), (2, (33, 65, 1)), (2, (200, 130, 1)), (2, (7, 300, 1))]


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def start(grid, dx, ndim, real_state):
    psi = inputs.smooth_random_state(grid, dx, (1.0, 1.3, 0.0), seed=sum(grid) + ndim)
    if real_state:
        psi = psi.real.astype(np.complex128)
    return psi / np.sqrt(np.vdot(psi, psi).real * np.prod(dx[:ndim]))


# real storage holds imaginary-time states only
MODE_DTYPES = [("imag", d) for d in ("c128", "c64", "r64", "r32")] + [("real", d) for d in ("c128", "c64")]


@pytest.mark.parametrize("mode,dtype", MODE_DTYPES)
@pytest.mark.parametrize("ndim,grid", CASES)
def test_reduced_step_matches_oracle(ndim, grid, mode, dtype):
    dx = (0.3, 0.25, 1.0)
    dt = (0.1 if mode == "imag" else 0.02) * dx[0] ** 2
    omega, g, steps = (1.0, 1.3, 5.0), 40.0, 6
    psi0 = start(grid, dx, ndim, dtype in ("r64", "r32"))
    if dtype in ("c64", "r32"):   # the oracle starts from the values the GPU holds
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    ref = psi0.copy()
    oracle.step(ref, dx, dt, omega, g, MODES[mode], steps, ndim=ndim)
    robs = oracle.observables(ref, dx, omega, g, ndim=ndim)
    t = torch.from_numpy(psi0.real.copy() if dtype in ("r64", "r32") else psi0).to(TORCH[dtype]).cuda()
    with gp.Plan(grid, dx, dt, *omega, g, mode=mode, dtype=dtype, ndim=ndim) as p:
        p.step(t, steps)
        obs = p.observables(t)
        assert f"{ndim}D" in p.describe()
    got = t.cpu().numpy().astype(np.complex128)
    tpsi, tobs = TOL[dtype]
    assert rel(got, ref) <= tpsi
    assert abs(obs["norm"] - robs["norm"]) <= norm_tol(dtype, mode, steps) * robs["norm"]
    for k in ("mu", "energy"):
        assert abs(obs[k] - robs[k]) <= tobs * abs(robs[k]), k
    assert obs["rms_z"] == 0.0 and robs["rms_z"] == 0.0


@pytest.mark.parametrize("ndim,grid,dx", [(1, (400, 1, 1), (0.08, 1.0, 1.0)), (2, (96, 80, 1), (0.25, 0.25, 1.0))])
def test_reduced_ground_state_matches_oracle(ndim, grid, dx):
    """A long imaginary-time relaxation (every step renormalised from the
    norm partials of the last sweep present)."""
    omega, g, dt, steps = (1.0, 1.3, 0.0), 200.0, 0.1 * dx[0] ** 2, 800
    psi0 = start(grid, dx, ndim, False)
    ref = psi0.copy()
    oracle.step(ref, dx, dt, omega, g, oracle.IMAG, steps, ndim=ndim)
    robs = oracle.observables(ref, dx, omega, g, ndim=ndim)
    t = torch.from_numpy(psi0).cuda()
    with gp.Plan(grid, dx, dt, *omega, g, mode="imag", dtype="c128", ndim=ndim) as p:
        p.step(t, steps)
        obs = p.observables(t)
    assert rel(t.cpu().numpy(), ref) <= 1e-12
    for k in ("norm", "mu", "energy", "rms_x", "rms_r"):
        assert abs(obs[k] - robs[k]) <= 1e-12 * abs(robs[k]), k
    assert abs(obs["norm"] - 1.0) <= 1e-13


def test_absent_axis_trap_is_ignored():
    dx = (0.3, 0.3, 1.0)
    psi0 = start((24, 20, 1), dx, 2, False)
    a = torch.from_numpy(psi0).cuda()
    b = a.clone()
    with gp.Plan((24, 20, 1), dx, 0.01, 1.0, 1.3, 0.0, 10.0, ndim=2) as p, \
            gp.Plan((24, 20, 1), dx, 0.01, 1.0, 1.3, 7.0, 10.0, ndim=2) as q:
        p.step(a, 5)
        q.step(b, 5)
    assert torch.equal(a, b)
