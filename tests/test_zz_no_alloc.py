"""The allocation-free entry point sllbm_totals_noalloc (static device
scratch) against sllbm_totals, through the C ABI.

CPU: sizes beyond the static scratch and NULL arguments are refused before
any device call.  GPU: two calls in a row, the second on a smaller grid (the
scratch keeps the first call's contents), give the bits of sllbm_totals of
a context holding the same state, in FP64 and FP32 storage and for both
lattices."""
import math

import numpy as np
import pytest
import torch

from paper_2012_05537_amd import inputs
from paper_2012_05537_amd.sllbm import (D2Q19, EINVAL, FP32_MIXED, FP64, CONSTANT, SLLBM, Config, SllbmError,
                                        load_library, totals_noalloc)


def _config(n_el, order, velocity_set=45, precision=FP64, length=2 * math.pi):
    c = Config()
    c.n_el[:] = list(n_el)
    c.order = order
    c.velocity_set = velocity_set
    c.viscosity_law = 0
    c.precision = precision
    c.device = 0
    c.length[:] = [length] * 3
    c.dt = 0.1
    c.gamma = 1.4
    c.prandtl = 0.71
    c.mu_inf = 0.01
    return c


def test_noalloc_refuses_oversize_grids_and_null_pointers():
    import ctypes
    lib = load_library()
    big = _config((4000, 2000, 200), 4)          # N_x + N_y + N_z = 24800 > 24576
    rc = lib.sllbm_totals_noalloc(ctypes.byref(big), ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert rc == EINVAL
    assert b"24576" in lib.sllbm_last_error(None)
    ok = _config((4, 4, 4), 2)
    assert lib.sllbm_totals_noalloc(ctypes.byref(ok), None, ctypes.c_void_p(16), None) == EINVAL
    assert lib.sllbm_totals_noalloc(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == EINVAL
    bad = _config((4, 4, 4), 9)
    assert lib.sllbm_totals_noalloc(ctypes.byref(bad), ctypes.c_void_p(16), ctypes.c_void_p(16), None) == EINVAL


def _tgv_context(n_el, p, precision):
    w = inputs.workload("c1")
    ctx = SLLBM(n_el, p, w["dt"], w["mu_inf"], precision=precision)
    xs, ys, zs = (c.numpy() for c in ctx.node_coords())
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.8, 1.4)
    dev = ctx.device
    ctx.init_equilibrium(torch.from_numpy(rho).to(dev), torch.from_numpy(u).to(dev), torch.from_numpy(T).to(dev))
    ctx.step(2)
    return ctx


def _riemann_context(n_el, p, precision):
    ctx = SLLBM(n_el, p, 1e-3, 2e-3, length=(1.0, 1.0), viscosity_law=CONSTANT, precision=precision,
                velocity_set=D2Q19)
    xs, ys = (c.numpy() for c in ctx.node_coords())
    rho, u, T = inputs.riemann_fields(xs, ys)
    dev = ctx.device
    ctx.init_equilibrium(torch.from_numpy(rho).to(dev), torch.from_numpy(u).to(dev), torch.from_numpy(T).to(dev))
    ctx.step(1)
    return ctx


@pytest.mark.gpu
@pytest.mark.parametrize("make,grids,precision", [
    (_tgv_context, [((9, 7, 6), 4), ((3, 2, 2), 3)], FP64),
    (_tgv_context, [((8, 8, 8), 4), ((2, 3, 1), 2)], FP32_MIXED),
    (_riemann_context, [((40, 24), 4), ((5, 3), 3)], FP64),
])
def test_noalloc_totals_equal_sllbm_totals(make, grids, precision):
    for n_el, p in grids:                         # the second call is on a smaller grid
        ctx = make(n_el, p, precision)
        print(f"noalloc totals: grid {n_el} p={p} precision={precision} lattice={ctx.q}", flush=True)
        ref = np.array(ctx.totals())
        state = ctx.get_state()
        out = torch.full((5,), float("nan"), dtype=torch.float64, device=ctx.device)
        totals_noalloc(ctx.cfg, state, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ctx.close()
        assert np.array_equal(got, ref), (got, ref)
