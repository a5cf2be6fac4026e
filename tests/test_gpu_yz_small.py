"""Small grids: calcluy and calcluz in one launch.

On grids whose y and z lines hold at most 64 points (at most 2^18 points in
all) a plan's default strategy solves the y lines and then the z lines of a
few x columns in one block, instead of launching the two sweeps apart.  Each
line is solved by the same code with the same chunking, so the state, the
norm partials and every observable must be bitwise those of the separate
launches (GP_SWEEP_CHUNKED); the separate launches are themselves held to the
oracle by the parity tests.  Grids just past the limits keep the separate
launches.
"""
import numpy as np
import pytest

from paper_1206_1361_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1206_1361_amd as gp  # noqa: E402

FUSED = "y and z in one launch"
GRIDS = [(32, 32, 32), (16, 20, 24), (9, 17, 33), (5, 3, 7), (3, 4, 1), (1, 6, 5), (64, 64, 64), (200, 40, 30)]
TORCH = {"c128": torch.complex128, "c64": torch.complex64, "c64_f64": torch.complex64,
         "r64": torch.float64, "r32": torch.float32}


def run(grid, dtype, mode, strategy, nsteps=5):
    dx, omega, g = (0.3, 0.25, 0.35), (1.0, 1.4, 2.0), 15.0
    dt = 0.02 if mode == "imag" else 0.01
    psi0 = inputs.smooth_random_state(grid, dx, omega, seed=sum(grid))
    if dtype in ("r64", "r32"):
        psi0 = np.ascontiguousarray(psi0.real)
    psi = torch.from_numpy(psi0).to(TORCH[dtype]).cuda().contiguous()
    with gp.Plan(grid, dx, dt, *omega, g, mode=mode, dtype=dtype) as plan:
        if strategy != "auto":
            plan.set_sweep(strategy)
        d = plan.describe()
        plan.step(psi, 2)
        plan.step(psi, nsteps - 2)
        obs = plan.observables(psi)
    return psi.cpu(), obs, d


CASES = [(d, m) for d in ("c128", "c64", "c64_f64", "r64", "r32") for m in ("imag", "real")
         if not (d in ("r64", "r32") and m == "real")]


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: "x".join(map(str, g)))
@pytest.mark.parametrize("dtype,mode", CASES)
def test_one_launch_equals_separate_launches(grid, dtype, mode):
    fused, ofused, dfused = run(grid, dtype, mode, "auto")
    apart, oapart, dapart = run(grid, dtype, mode, "chunked")
    assert FUSED in dfused, dfused
    assert FUSED not in dapart, dapart
    assert torch.equal(fused, apart)
    for k in ("norm", "mu", "energy", "rms_x", "rms_y", "rms_z"):
        assert ofused[k] == oapart[k], k


@pytest.mark.parametrize("grid", [(65, 64, 64), (8, 65, 8), (8, 8, 65)], ids=lambda g: "x".join(map(str, g)))
def test_larger_grids_keep_separate_launches(grid):
    with gp.Plan(grid, (0.3,) * 3, 0.01, 1.0, 1.0, 1.0, 1.0, mode="imag") as plan:
        assert FUSED not in plan.describe()


def test_stream_strategy_turns_it_off_and_auto_back_on():
    with gp.Plan((32, 32, 32), (0.3,) * 3, 0.01, 1.0, 1.0, 1.0, 1.0, mode="imag") as plan:
        assert FUSED in plan.describe()
        plan.set_sweep("stream")
        assert FUSED not in plan.describe()
        plan.set_sweep("auto")
        assert FUSED in plan.describe()
