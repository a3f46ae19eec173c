"""Error behaviour of the C ABI on a device (codes as documented in
include/sllbm.h), called through ctypes directly so that the binding's own
checks do not intercept them.  The argument and state errors are rejected on
the host before any launch; the non-finite case runs the totals kernels on a
state holding a NaN and reports it."""
import ctypes
import math

import pytest
import torch

from gpu_common import Q, require_gpu

pytestmark = pytest.mark.gpu

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONFINITE = range(6)


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _ctx(precision=0):
    from paper_2012_05537_amd.sllbm import SLLBM
    return SLLBM((2, 2, 2), 2, 0.1, 0.01, precision=precision)


def test_calls_before_a_state_report_estate():
    ctx = _ctx()
    lib, h = ctx._lib, ctx._h
    buf = torch.empty((2, Q, ctx.nodes), dtype=torch.float64, device=ctx.device)
    assert lib.sllbm_step(h, 1) == ESTATE
    assert lib.sllbm_get_state(h, ctypes.c_void_p(buf.data_ptr())) == ESTATE
    tot = (ctypes.c_double * 5)()
    assert lib.sllbm_totals(h, ctypes.addressof(tot)) == ESTATE
    d3 = (ctypes.c_double * 3)()
    assert lib.sllbm_diagnostics(h, None, ctypes.addressof(d3)) == ESTATE
    assert "state" in lib.sllbm_last_error(h).decode()
    ctx.close()


def test_argument_errors_report_einval():
    ctx = _ctx()
    lib, h = ctx._lib, ctx._h
    x = torch.ones((2, Q, ctx.nodes), dtype=torch.float64, device=ctx.device)
    y = torch.empty_like(x)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    ctx.set_state(x)
    assert lib.sllbm_step(h, -1) == EINVAL
    assert lib.sllbm_step(h, 0) == OK
    assert lib.sllbm_stream(h, p(x), p(x), 0) == EINVAL              # in place
    assert lib.sllbm_set_viscosity(h, ctypes.c_double(-1.0)) == EINVAL
    assert lib.sllbm_set_viscosity(h, ctypes.c_double(math.nan)) == EINVAL
    rec = torch.empty((2, 2, Q, ctx.nodes), dtype=torch.float64, device=ctx.device)
    assert lib.sllbm_step_record(h, 2, p(rec), ctypes.c_int64(ctx.state_bytes - 8)) == EINVAL
    assert lib.sllbm_adjoint_step(h, p(x), p(y), p(y), None) == EINVAL  # lam_out aliases lam_next
    assert lib.sllbm_set_mesh(h, None, None, None) == EINVAL
    assert lib.sllbm_loss_grad(h, p(x), p(x)) == EINVAL
    ctx.close()


def test_non_finite_state_is_reported():
    ctx = _ctx()
    x = torch.ones((2, Q, ctx.nodes), dtype=torch.float64, device=ctx.device)
    x[0, 3, 5] = float("nan")
    ctx.set_state(x)
    tot = (ctypes.c_double * 5)()
    assert ctx._lib.sllbm_totals(ctx._h, ctypes.addressof(tot)) == ENONFINITE
    ctx.close()


def test_state_round_trip_and_zero_steps_fp32():
    ctx = _ctx(precision=1)
    gen = torch.Generator(device=ctx.device).manual_seed(9)
    x = torch.rand((2, Q, ctx.nodes), generator=gen, device=ctx.device, dtype=torch.float32) + 0.5
    ctx.set_state(x)
    ctx.step(0)
    assert torch.equal(ctx.get_state(), x)
    ctx.close()
