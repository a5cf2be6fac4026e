"""Error paths of the C ABI on the GPU: every failure comes back as a status
code (or a Python exception from the binding), nothing aborts."""
import ctypes

import numpy as np
import pytest

from paper_1206_1361_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1206_1361_amd as gp  # noqa: E402
from paper_1206_1361_amd import _binding as B  # noqa: E402

GRID, DX = (16, 12, 10), (0.3, 0.3, 0.3)


def plan(mode="imag", dtype="c128"):
    return gp.Plan(GRID, DX, 0.01, 1.0, 1.2, 1.5, 5.0, mode=mode, dtype=dtype)


def state(dtype=torch.complex128):
    return torch.from_numpy(inputs.random_state(GRID, DX, seed=3)).to(dtype).cuda()


def test_size_mismatch_and_null_psi_are_invalid():
    with plan() as p:
        psi = state()
        L = B.lib()
        assert L.gp_step(p._handle, ctypes.c_void_p(psi.data_ptr()), psi.numel() - 1, 1) == B.ERR_INVALID
        assert L.gp_step(p._handle, None, psi.numel(), 1) == B.ERR_INVALID
        assert L.gp_step(p._handle, ctypes.c_void_p(psi.data_ptr()), psi.numel(), -1) == B.ERR_INVALID
        assert b"elements" in L.gp_last_error() or b"nsteps" in L.gp_last_error()


def test_host_pointer_is_rejected():
    with plan() as p:
        host = np.zeros(GRID[0] * GRID[1] * GRID[2], dtype=np.complex128)
        L = B.lib()
        st = L.gp_step(p._handle, ctypes.c_void_p(host.ctypes.data), host.size, 1)
        assert st == B.ERR_INVALID
        assert b"device" in L.gp_last_error()


def test_binding_checks_dtype_shape_and_device():
    with plan() as p:
        with pytest.raises(TypeError):
            p.step(state(torch.complex64), 1)
        with pytest.raises(ValueError):
            p.step(state().reshape(GRID[2], -1), 1)
        with pytest.raises(ValueError):
            p.step(state().cpu(), 1)
        with pytest.raises(ValueError):
            p.step(state().transpose(0, 2), 1)


def test_nonfinite_norm_is_reported_by_sync_and_observables():
    with plan() as p:
        psi = state()
        psi[3, 4, 5] = float("nan")
        p.step(psi, 2)
        with pytest.raises(gp.GPNonFinite):
            p.sync()
        p.sync()    # the flag is cleared once reported
        with pytest.raises(gp.GPNonFinite):
            p.observables(psi)


def test_zero_state_observables_are_nonfinite():
    with plan(mode="real") as p:
        psi = torch.zeros(GRID[::-1], dtype=torch.complex128, device="cuda")
        with pytest.raises(gp.GPNonFinite):
            p.observables(psi)


def test_bad_schedule_values_queue_nothing():
    with plan(mode="real") as p:
        psi = state()
        before = psi.clone()
        with pytest.raises(gp.GPInvalid):
            p.step_schedule(psi, g_steps=[1.0, float("nan")])
        with pytest.raises(gp.GPInvalid):
            p.step_schedule(psi, trap_steps=[[1.0, 1.0, 1.0], [1.0, -1.0, 1.0]])
        with pytest.raises(gp.GPInvalid):
            p.set_trap(1.0, float("inf"), 1.0)
        with pytest.raises(gp.GPInvalid):
            p.set_g(float("nan"))
        torch.cuda.synchronize()
        assert torch.equal(psi, before)


def test_plans_are_independent_and_destroy_is_idempotent():
    a, b = plan(mode="real"), plan(mode="imag")
    psi_a, psi_b = state(), state()
    a.step(psi_a, 3)
    b.step(psi_b, 3)
    oa, ob = a.observables(psi_a), b.observables(psi_b)
    assert abs(ob["norm"] - 1.0) < 1e-12 and abs(oa["norm"] - 1.0) < 1e-12
    a.close()
    a.close()
    b.close()
    assert B.lib().gp_plan_destroy(None) == B.OK


def test_describe_and_footprint():
    with plan() as p:
        d = p.describe()
        assert "16x12x10" in d and "imag" in d
    assert gp.footprint_bytes(GRID) > 0
