"""Batches (gp_batch_*): many solves advanced together.

A solve inside a batch runs the same per-line arithmetic as a single plan
(the same device functions, launch shapes that do not enter the rounding,
norm partials per line), so its result must be bitwise the single plan's --
alone or in any mix, with or without graph replay and autotuning.  The
single plans are themselves checked against the oracle in
test_gpu_parity.py; a few cases here go straight to the oracle too.
"""
import numpy as np
import pytest

import oracle
from paper_1206_1361_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1206_1361_amd as gp  # noqa: E402

MODES = {"imag": oracle.IMAG, "real": oracle.REAL}


def specs_mixed(seed=0, n=7):
    """Uneven grids (three shapes, one repeated), per-solve traps and g."""
    rng = np.random.default_rng(seed)
    shapes = [(24, 20, 16), (33, 17, 9), (24, 20, 16), (48, 40, 32), (33, 17, 9), (24, 20, 16), (48, 40, 32)]
    out = []
    for i in range(n):
        trap = tuple(rng.uniform(0.5, 3.0, 3))
        out.append(dict(grid=shapes[i % len(shapes)], dx=0.3, dt=0.01, trap=trap,
                        g=float(np.exp(rng.uniform(0, np.log(1000.0))))))
    return out


def initial(sp, seed, dtype):
    psi = inputs.smooth_random_state(sp["grid"], (sp["dx"],) * 3, sp["trap"], seed=seed)
    t = torch.from_numpy(psi)
    return t.to(torch.complex128 if dtype == "c128" else torch.complex64).cuda()


def run_single(sp, psi0, mode, dtype, nsteps, calls=1):
    psi = psi0.clone()
    with gp.Plan(sp["grid"], (sp["dx"],) * 3, sp["dt"], *sp["trap"], sp["g"], mode=mode, dtype=dtype) as p:
        for c in range(calls):
            p.step(psi, nsteps)
        obs = p.observables(psi)
    return psi, obs


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mode", ["imag", "real"])
def test_batch_matches_single_plans_bitwise(mode, dtype, graph):
    specs = specs_mixed(1)
    psi0 = [initial(sp, 10 + i, dtype) for i, sp in enumerate(specs)]
    psis = [t.clone() for t in psi0]
    with gp.Batch(specs, mode=mode, dtype=dtype, graph=graph) as b:
        b.bind(psis)
        b.step(4)
        b.step(3)
        obs = b.observables()
    for i, sp in enumerate(specs):
        ref = psi0[i].clone()
        with gp.Plan(sp["grid"], (sp["dx"],) * 3, sp["dt"], *sp["trap"], sp["g"], mode=mode, dtype=dtype) as p:
            p.step(ref, 4)
            p.step(ref, 3)
            robs = p.observables(ref)
        assert torch.equal(psis[i], ref), i
        for k in ("mu", "energy", "norm", "rms_r"):
            assert obs[i][k] == robs[k], (i, k)


@pytest.mark.parametrize("mode", ["real", "imag"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_interleaved_x_lines_across_solves(dtype, mode):
    """Three solves of 6111 x lines each: the batch's x launch interleaves 4
    lines per wavefront, with groups that straddle two solves and a ragged
    last group; a single plan of 6111 lines solves one line per wavefront.
    The lines' arithmetic does not depend on that: bitwise equal."""
    specs = [dict(sp, grid=(40, 63, 97)) for sp in specs_mixed(7, 3)]
    psi0 = [initial(sp, 50 + i, dtype) for i, sp in enumerate(specs)]
    psis = [t.clone() for t in psi0]
    with gp.Batch(specs, mode=mode, dtype=dtype, graph=False) as b:
        b.bind(psis)
        b.step(3)
    for i, sp in enumerate(specs):
        ref, _ = run_single(sp, psi0[i], mode, dtype, 3)
        assert torch.equal(psis[i], ref), i


@pytest.mark.parametrize("tune", [False, True])
def test_complex64_column_pairs_and_their_fallback(tune):
    """complex64 classes with an even nx take column pairs in y and z; a class
    with a member whose psi is only 8-byte aligned falls back to one column
    per thread.  Neither enters the rounding: bitwise the single plans."""
    # z lines of 272 points take pairs by default; y lines of 20 do not
    grids = [(24, 20, 272), (18, 16, 272), (24, 20, 272), (18, 16, 272), (33, 17, 9)]
    specs = [dict(sp, grid=g) for sp, g in zip(specs_mixed(5, len(grids)), grids)]
    psi0 = [initial(sp, 30 + i, "c64") for i, sp in enumerate(specs)]
    psis = [t.clone() for t in psi0]
    # member 3 (18x16x272) in an 8-byte-aligned view
    n3 = psis[3].numel()
    store = torch.zeros(n3 + 1, dtype=torch.complex64, device="cuda")
    psis[3] = store[1:].view(psis[3].shape)
    psis[3].copy_(psi0[3])
    with gp.Batch(specs, mode="imag", dtype="c64", graph=True, tune=tune) as b:
        before = b.describe()
        b.bind(psis)
        after = b.describe()
        b.step(6)
        obs = b.observables()
    if not tune:   # the tuner may prefer one column per thread
        assert "in pairs" in before.split("24x20x272")[1].split("|")[0]
        assert "in pairs" in after.split("24x20x272")[1].split("|")[0]
    assert "in pairs" not in after.split("18x16x272")[1].split("|")[0]
    for i, sp in enumerate(specs):
        ref, robs = run_single(sp, psi0[i], "imag", "c64", 6)
        assert torch.equal(psis[i], ref), i
        assert obs[i]["mu"] == robs["mu"], i


def test_batch_matches_oracle():
    specs = specs_mixed(2, n=4)
    psi0 = [initial(sp, 20 + i, "c128") for i, sp in enumerate(specs)]
    psis = [t.clone() for t in psi0]
    with gp.Batch(specs, mode="imag", dtype="c128") as b:
        b.bind(psis)
        b.step(5)
        obs = b.observables()
    for i, sp in enumerate(specs):
        ref = psi0[i].cpu().numpy().copy()
        oracle.step(ref, (sp["dx"],) * 3, sp["dt"], sp["trap"], sp["g"], oracle.IMAG, 5)
        got = psis[i].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        robs = oracle.observables(ref, (sp["dx"],) * 3, sp["trap"], sp["g"])
        assert abs(obs[i]["mu"] - robs["mu"]) <= 1e-12 * abs(robs["mu"])


def test_alone_and_in_the_mix_are_bitwise_equal():
    """A solve gives the same bits in a batch of one and inside a larger,
    autotuned batch."""
    specs = specs_mixed(3)
    target = 3
    psi0 = [initial(sp, 30 + i, "c64") for i, sp in enumerate(specs)]
    mix = [t.clone() for t in psi0]
    with gp.Batch(specs, mode="imag", dtype="c64", tune=True) as b:
        b.bind(mix)
        b.step(6)
    alone = [psi0[target].clone()]
    with gp.Batch([specs[target]], mode="imag", dtype="c64") as b:
        b.bind(alone)
        b.step(6)
    assert torch.equal(mix[target], alone[0])


def test_inactive_solves_are_untouched():
    specs = specs_mixed(4, n=5)
    psi0 = [initial(sp, 40 + i, "c128") for i, sp in enumerate(specs)]
    psis = [t.clone() for t in psi0]
    mask = [True, False, True, False, True]
    with gp.Batch(specs, mode="real", dtype="c128") as b:
        b.bind(psis)
        b.set_active(mask)
        b.step(3)
        obs = b.observables()
    for i, sp in enumerate(specs):
        if mask[i]:
            ref, _ = run_single(sp, psi0[i], "real", "c128", 3)
            assert torch.equal(psis[i], ref)
        else:
            assert torch.equal(psis[i], psi0[i])


def test_graph_replays_match_eager_across_calls():
    """Replays of the captured step, with the program's own eager work and
    synchronisations between them, equal eager launches every time."""
    specs = specs_mixed(5)
    psi0 = [initial(sp, 50 + i, "c128") for i, sp in enumerate(specs)]
    a = [t.clone() for t in psi0]
    e = [t.clone() for t in psi0]
    with gp.Batch(specs, mode="imag", dtype="c128", graph=True) as bg, \
            gp.Batch(specs, mode="imag", dtype="c128", graph=False) as be:
        bg.bind(a)
        be.bind(e)
        for call in range(4):
            bg.step(2)
            be.step(2)
            scratch = torch.ones(1000, device="cuda").sum()   # unrelated eager work
            torch.cuda.synchronize()
            assert float(scratch) == 1000.0
            for i in range(len(specs)):
                assert torch.equal(a[i], e[i]), (call, i)


def test_solve_imag_stops_each_solve_on_its_own():
    specs = specs_mixed(6, n=5)
    for sp in specs:
        sp["dt"] = 0.02
    psis = [initial(sp, 60 + i, "c128") for i, sp in enumerate(specs)]
    with gp.Batch(specs, mode="imag", dtype="c128") as b:
        b.bind(psis)
        obs, steps, conv = b.solve_imag(tol=1e-6, check_every=10, max_steps=3000)
        assert all(conv), (steps, conv)
        assert len(set(steps)) > 1            # solves stopped at different times
        again = b.observables()
    for i, sp in enumerate(specs):
        # the stopped state is the single plan's state after the same calls
        assert steps[i] % 10 == 0
        ref, robs = run_single(sp, initial(sp, 60 + i, "c128"), "imag", "c128", 10, calls=steps[i] // 10)
        assert torch.equal(psis[i], ref), i
        assert again[i]["mu"] == robs["mu"]
        assert abs(obs[i]["mu"] - robs["mu"]) == 0.0


def test_batch_binding_checks():
    specs = specs_mixed(7, n=2)
    with gp.Batch(specs, mode="imag", dtype="c128") as b:
        with pytest.raises(gp.GPInvalid):
            b.step(1)                       # nothing bound yet
        with pytest.raises(ValueError):
            b.bind([initial(specs[0], 1, "c128")])
        with pytest.raises(ValueError):
            b.bind([initial(specs[0], 1, "c64"), initial(specs[1], 2, "c64")])
        assert "2 solves" in b.describe()


@pytest.mark.parametrize("dtype", ["c64", "r32"])
def test_fp32_batch_with_fp64_finish_meets_the_fp32_bounds(dtype):
    """Eight imaginary-time solves stopped at |delta mu| < 1e-8 in float
    storage with the FP64 finishing phase (GP_BATCH_FINISH_F64), against the
    oracle stepped in FP64 from the same (float-rounded) starts to each
    solve's step count: mu within 1e-7 and psi within 1e-5, the bounds for
    the FP32 form."""
    rng = np.random.default_rng(12)
    shapes = [(16, 16, 16), (20, 18, 16), (14, 20, 18), (18, 14, 20)]
    specs = [dict(grid=shapes[i % 4], dx=0.6, dt=0.1 * 0.36, trap=tuple(rng.uniform(1.0, 3.0, 3)),
                  g=float(np.exp(rng.uniform(0.0, np.log(100.0))))) for i in range(8)]
    real = dtype == "r32"
    tdt = torch.float32 if real else torch.complex64
    starts = []
    for sp in specs:
        psi = inputs.gaussian(sp["grid"], (sp["dx"],) * 3, sp["trap"])
        psi = psi.real.astype(np.float32) if real else psi.astype(np.complex64)
        starts.append(psi)
    psis = [torch.from_numpy(p.copy()).to(tdt).cuda() for p in starts]
    with gp.Batch(specs, mode="imag", dtype=dtype, finish_f64=True) as b:
        b.bind(psis)
        obs, steps, conv = b.solve_imag(tol=1e-8, check_every=10, max_steps=20000)
    assert all(conv), (steps, conv)
    for i, sp in enumerate(specs):
        dx3 = (sp["dx"],) * 3
        ref = starts[i].astype(np.complex128)
        oracle.step(ref, dx3, sp["dt"], sp["trap"], sp["g"], oracle.IMAG, steps[i])
        robs = oracle.observables(ref, dx3, sp["trap"], sp["g"])
        got = psis[i].cpu().numpy().astype(np.complex128)
        print(f"solve {i} {sp['grid']}: {steps[i]} steps, mu {obs[i]['mu']:.9f} oracle {robs['mu']:.9f}")
        assert abs(obs[i]["mu"] - robs["mu"]) <= 1e-7 * abs(robs["mu"]), i
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref)), i


def specs_wide(seed=5):
    """Classes that differ in every launch parameter: x chunks of 1, 2, 3
    and 5 points (so 4, 2 and 1 lines per wavefront), y/z chunks of 2 to 16
    points over 8 to 48 chunks, and lines over 256 points (complex64
    pairs)."""
    rng = np.random.default_rng(seed)
    shapes = [(24, 20, 16), (96, 40, 300), (130, 66, 48), (300, 24, 20), (48, 130, 96), (24, 20, 16)]
    return [dict(grid=shp, dx=0.25, dt=0.01, trap=tuple(rng.uniform(0.5, 3.0, 3)),
                 g=float(np.exp(rng.uniform(0, np.log(500.0))))) for shp in shapes]


def initial_any(sp, seed, dtype):
    psi = inputs.smooth_random_state(sp["grid"], (sp["dx"],) * 3, sp["trap"], seed=seed)
    if dtype == "r32":
        return torch.from_numpy(np.ascontiguousarray(psi.real).astype(np.float32)).cuda()
    return torch.from_numpy(psi).to(torch.complex128 if dtype == "c128" else torch.complex64).cuda()


@pytest.mark.skip(reason="GP_BATCH_ONE_LAUNCH is switched off: the complex64 case of its first GPU run ended in a device fault (SIGABRT in observables) whose cause is not found; a CPU emulation of its kernels under AddressSanitizer shows every access in bounds")
@pytest.mark.parametrize("tune", [False, True])
@pytest.mark.parametrize("dtype,mode", [("c128", "imag"), ("c128", "real"), ("c64", "imag"), ("c64", "real"),
                                        ("r32", "imag")])
def test_one_launch_matches_per_class_launches_bitwise(dtype, mode, tune):
    """GP_BATCH_ONE_LAUNCH (each sweep one launch over every class) against
    the per-class launches: bitwise the same states and observables, with
    graph replay, after the active set changes, and eagerly."""
    specs = specs_wide()
    psi0 = [initial_any(sp, 30 + i, dtype) for i, sp in enumerate(specs)]
    mask = [1, 0, 1, 1, 0, 1]
    out = {}
    for one in (False, True):
        psis = [t.clone() for t in psi0]
        with gp.Batch(specs, mode=mode, dtype=dtype, graph=True, tune=tune, one_launch=one) as b:
            b.bind(psis)
            b.step(3)
            b.set_active(mask)
            b.step(2)
            b.set_active(None)
            b.step(1)
            obs = b.observables()
        out[one] = (psis, obs)
    for i in range(len(specs)):
        assert torch.equal(out[False][0][i], out[True][0][i]), i
        for k in ("mu", "energy", "norm", "rms_r"):
            assert out[False][1][i][k] == out[True][1][i][k], (i, k)


@pytest.mark.skip(reason="GP_BATCH_ONE_LAUNCH is switched off: the complex64 case of its first GPU run ended in a device fault (SIGABRT in observables) whose cause is not found; a CPU emulation of its kernels under AddressSanitizer shows every access in bounds")
def test_one_launch_solve_imag_and_eager_steps():
    """Solves dropping out of the one-launch batch as they converge, and the
    eager (graph-less) path: the same steps and bits as the per-class
    batch."""
    specs = specs_mixed(3, n=6)
    psi0 = [initial(sp, 50 + i, "c64") for i, sp in enumerate(specs)]
    res = {}
    for one in (False, True):
        psis = [t.clone() for t in psi0]
        with gp.Batch(specs, mode="imag", dtype="c64", graph=not one, one_launch=one) as b:
            b.bind(psis)
            obs, steps, conv = b.solve_imag(tol=1e-6, check_every=10, max_steps=400)
        res[one] = (psis, [o["mu"] for o in obs], list(steps), list(conv))
    assert res[False][2] == res[True][2]
    assert res[False][3] == res[True][3]
    assert res[False][1] == res[True][1]
    for i in range(len(specs)):
        assert torch.equal(res[False][0][i], res[True][0][i]), i
