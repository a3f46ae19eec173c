"""FP32-mixed storage against FP64 (GPU) and against the FP64 oracle.

Bar (mixed mode): max |a - b| / max |b| <= 1e-5 for rho, for u (all three
components relative to max |u|) and for T.  The TGV at Ma 1.25, Re 1600 is
compared over its early steps; the floor of what any two arithmetic orders
can agree on is measured beside it (an FP64 run whose initial state differs by
one unit in the last place at every node).
"""
import sys

import numpy as np
import pytest
import torch

from gpu_common import workload_pair, require_gpu
from paper_2012_05537_amd import inputs

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _field_errs(a, b):
    ra, ua, Ta = a
    rb, ub, Tb = b
    e = lambda x, y: float((x - y).abs().max() / y.abs().max())
    return e(ra, rb), e(ua, ub), e(Ta, Tb)


def _init(ctx, w, xs, ys, zs):
    rho, u, T = inputs.tgv_fields(xs, ys, zs, w["Ma"], w["gamma"])
    dev = ctx.device
    ctx.init_equilibrium(torch.from_numpy(rho).to(dev), torch.from_numpy(u).to(dev), torch.from_numpy(T).to(dev))


def test_mixed_vs_fp64_128cubed(oracle):
    """c3 grid (32^3 cells, p = 4, 128^3 nodes, CFL 5): FP32-mixed vs FP64 on
    the GPU after 1, 2, 5, 10 and 20 steps, with the 1-ulp FP64 floor."""
    w, c64, cfg = workload_pair(oracle, "c3", precision=0)
    _, c32, _ = workload_pair(oracle, "c3", precision=1)
    _, c64b, _ = workload_pair(oracle, "c3", precision=0)
    xs, ys, zs = (t.numpy() for t in c64.node_coords())
    for c in (c64, c32, c64b):
        _init(c, w, xs, ys, zs)
    st = c64b.get_state()
    st.copy_(torch.nextafter(st, torch.full_like(st, 2.0)))   # one ulp up everywhere
    c64b.set_state(st)
    done = 0
    hist = {}
    for n in (1, 2, 5, 10, 20):
        for c in (c64, c32, c64b):
            c.step(n - done)
        done = n
        ref = c64.moments()
        err = _field_errs(c32.moments(), ref)
        floor = _field_errs(c64b.moments(), ref)
        hist[n] = (max(err), max(floor))
        _say(f"step {n}: mixed vs fp64 rho {err[0]:.2e} u {err[1]:.2e} T {err[2]:.2e}; "
             f"1-ulp fp64 floor rho {floor[0]:.2e} u {floor[1]:.2e} T {floor[2]:.2e}")
        if n <= 10:
            assert max(err) <= TOL_MIXED, (n, err)
    # Beyond t ~ 1 this flow amplifies any perturbation (it later blows up in
    # FP64 as well): the mixed-precision difference may then exceed the bar,
    # but it must grow no faster than a one-ulp FP64 perturbation does.
    growth_mixed = hist[20][0] / hist[10][0]
    growth_floor = hist[20][1] / hist[10][1]
    assert growth_mixed <= 2.0 * growth_floor, (growth_mixed, growth_floor)
    for c in (c64, c32, c64b):
        c.close()


def test_mixed_vs_fp64_stable_flow(oracle):
    """c4 grid (8^3 cells, p = 3), Ma 0.5, Re 400, CFL 2: FP32-mixed stays
    within the bar of FP64 over the whole 50-step run."""
    w, c64, cfg = workload_pair(oracle, "c4", precision=0)
    _, c32, _ = workload_pair(oracle, "c4", precision=1)
    xs, ys, zs = (t.numpy() for t in c64.node_coords())
    for c in (c64, c32):
        _init(c, w, xs, ys, zs)
    for n in range(5):
        for c in (c64, c32):
            c.step(w["steps"] // 5)
        err = _field_errs(c32.moments(), c64.moments())
        _say(f"step {(n + 1) * w['steps'] // 5}: mixed vs fp64 rho {err[0]:.2e} u {err[1]:.2e} T {err[2]:.2e}")
        assert max(err) <= TOL_MIXED, err


def test_mixed_vs_oracle_64cubed(oracle):
    """c2 grid (16^3 cells, p = 4, 64^3 nodes) at CFL 5 in FP32-mixed storage
    against two FP64 oracle steps."""
    w, ctx, cfg = workload_pair(oracle, "c2", precision=1, cfl=5.0)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, w["Ma"], w["gamma"])
    _init(ctx, w, xs, ys, zs)
    ctx.step(2)
    got = [x.cpu() for x in ctx.moments()]
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    f, g = oracle.step(cfg, f, g, 2)
    ref = [torch.from_numpy(np.asarray(x)) for x in oracle.moments(cfg, f, g)]
    err = _field_errs(got, ref)
    _say(f"mixed vs oracle after 2 steps: rho {err[0]:.2e} u {err[1]:.2e} T {err[2]:.2e}")
    assert max(err) <= TOL_MIXED, err
    ctx.close()
