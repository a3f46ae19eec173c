"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (FP64): max-abs error relative to the max magnitude of the oracle's
array, <= 1e-12, for populations, moments and totals.  FP32-mixed runs are
checked against the stated mixed-precision tolerance.
"""
import math
import sys

import numpy as np
import pytest
import torch

from gpu_common import Q, make_pair, workload_pair, tgv_init, to_np, to_dev, rel_err, require_gpu
from paper_2012_05537_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def test_node_coords_match(oracle):
    ctx, cfg = make_pair(oracle, (3, 2, 5), 4, 0.1, 0.01)
    for a, b in zip(ctx.node_coords(), oracle.node_coords(cfg)):
        assert np.allclose(a.numpy(), b, rtol=0, atol=1e-14)


# (n_el, p, dt, length): ragged tiles, single-cell axes, large departure shifts
STREAM_CASES = [
    ((4, 4, 4), 2, 0.41, 2 * math.pi),
    ((5, 3, 2), 4, 0.37, 2 * math.pi),
    ((3, 3, 3), 3, 0.9, 2 * math.pi),        # shifts of several cells
    ((7, 1, 2), 4, 0.05, 2 * math.pi),       # single-cell periodic axis
    ((2, 3, 4), 1, 0.2, 2 * math.pi),        # p = 1
    ((3, 2, 2), 5, 0.3, (2.0, 3.0, 4.5)),   # p = 5, anisotropic cells
    ((2, 2, 3), 6, 0.25, 2 * math.pi),      # p = 6
]


@pytest.mark.parametrize("n_el,p,dt,length", STREAM_CASES)
def test_stream_matches_oracle(oracle, n_el, p, dt, length):
    _say(f"stream parity n_el={n_el} p={p} dt={dt}")
    ctx, cfg = make_pair(oracle, n_el, p, dt, 0.01, length=length)
    rng = np.random.default_rng(sum(n_el) * 10 + p)
    N = oracle.num_nodes(cfg)
    f = rng.normal(size=(Q, N))
    g = rng.normal(size=(Q, N))
    out = ctx.stream(to_dev(ctx, f, g))
    fo, go = oracle.stream(cfg, f, g)
    F, G = to_np(out)
    assert rel_err(F, fo) < TOL64 and rel_err(G, go) < TOL64


# the transposed streaming marches along z in chunks when there are few tiles
# ((2, 2, 8) at p = 4); one- and two-cell axes wrap inside a source-cell group
TRANSPOSE_CASES = STREAM_CASES + [
    ((2, 2, 8), 4, 0.31, 2 * math.pi),
    ((3, 2, 3), 2, 1.3, 2 * math.pi),        # shifts of several cells, three cells along z
    ((2, 3, 12), 3, 0.2, (1.0, 2.0, 6.0)),
    ((3, 2, 1), 3, 0.6, 2 * math.pi),        # one cell along z
    ((1, 1, 1), 4, 0.7, 2 * math.pi),        # a single cell
    ((9, 2, 2), 2, 2.1, 2 * math.pi),        # shifts beyond one tile along x
]


@pytest.mark.parametrize("n_el,p,dt,length", TRANSPOSE_CASES)
def test_transposed_stream_is_adjoint(oracle, n_el, p, dt, length):
    """<S x, y> = <x, S^T y> per population and velocity, with S x from the
    oracle's direct gather and S^T y from the library."""
    _say(f"transposed stream n_el={n_el} p={p} dt={dt}")
    ctx, cfg = make_pair(oracle, n_el, p, dt, 0.01, length=length)
    rng = np.random.default_rng(7)
    N = oracle.num_nodes(cfg)
    x = rng.normal(size=(2, Q, N))
    y = rng.normal(size=(2, Q, N))
    Sx = np.stack(oracle.stream(cfg, x[0], x[1]))
    STy = ctx.stream(to_dev(ctx, y[0], y[1]), transpose=True).cpu().numpy()
    lhs = np.einsum("pin,pin->pi", Sx, y)
    rhs = np.einsum("pin,pin->pi", x, STy)
    scale = np.einsum("pin,pin->pi", np.abs(Sx), np.abs(y))
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale), np.max(np.abs(lhs - rhs) / scale)


@pytest.mark.parametrize("n_el,p,dt", [((4, 4, 4), 2, 0.41), ((5, 2, 3), 4, 0.37), ((3, 2, 1), 3, 0.6)])
def test_transposed_stream_fp32(oracle, n_el, p, dt):
    """FP32 storage (16-byte window loads where rows allow): S^T y against the
    FP64 library result on the same FP32 input, within FP32 rounding."""
    _say(f"transposed stream fp32 n_el={n_el} p={p} dt={dt}")
    c64, cfg = make_pair(oracle, n_el, p, dt, 0.01)
    c32, _ = make_pair(oracle, n_el, p, dt, 0.01, precision=1)
    gen = torch.Generator(device=c64.device).manual_seed(3)
    y = torch.randn((2, Q, c64.nodes), generator=gen, device=c64.device, dtype=torch.float32)
    t32 = c32.stream(y, transpose=True).double()
    t64 = c64.stream(y.double(), transpose=True)
    assert float((t32 - t64).abs().max() / t64.abs().max()) < 1e-6


@pytest.mark.parametrize("law,pr", [(0, 0.71), (1, 1.0), (0, 2.0)])
def test_collide_matches_oracle(oracle, law, pr):
    _say(f"collide parity law={law} Pr={pr}")
    ctx, cfg = make_pair(oracle, (3, 2, 2), 2, 0.07, 0.013, prandtl=pr, law=law)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.9, 1.4)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    rng = np.random.default_rng(3)
    _, w = oracle.velocity_set()
    f = f * (1 + 0.03 * rng.normal(size=f.shape))
    g = g * (1 + 0.03 * rng.normal(size=g.shape))
    st = to_dev(ctx, f, g)
    ctx.collide(st)
    fo, go = oracle.collide(cfg, f, g)
    F, G = to_np(st)
    assert rel_err(F, fo) < TOL64 and rel_err(G, go) < TOL64


# FP32-mixed storage: the collision reads FP32 values, computes in FP64 and
# rounds each result once, so every output lies within half an FP32 ulp
# (2^-24 relative) of the oracle's FP64 collision of the same values.  Node
# counts: 96 (one partial block of the LDS-staged kernel), 1792 (whole
# blocks), 8640 (a ragged last block) and 729 (not a multiple of 4: the
# register form).
FP32_COLLIDE_CASES = [((3, 2, 2), 2), ((7, 2, 2), 4), ((9, 5, 3), 4), ((3, 3, 3), 3)]


@pytest.mark.parametrize("n_el,p", FP32_COLLIDE_CASES)
def test_collide_fp32_rounds_the_fp64_collision(oracle, n_el, p):
    _say(f"fp32 collide n_el={n_el} p={p}")
    ctx, cfg = make_pair(oracle, n_el, p, 0.07, 0.013, precision=1)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.9, 1.4)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    rng = np.random.default_rng(5)
    f = (f * (1 + 0.03 * rng.normal(size=f.shape))).astype(np.float32).astype(np.float64)
    g = (g * (1 + 0.03 * rng.normal(size=g.shape))).astype(np.float32).astype(np.float64)
    st = to_dev(ctx, f, g)
    ctx.collide(st)
    fo, go = oracle.collide(cfg, f, g)
    for got, ref in zip(to_np(st), (fo, go)):
        assert np.all(np.abs(ref) > 0)
        err = float(np.max(np.abs(got - ref) / np.abs(ref)))
        assert err <= 2.0 ** -24 * (1 + 1e-4), err


@pytest.mark.parametrize("precision", [0, 1])
def test_collide_state_at_any_word_offset(oracle, precision):
    """A caller state that starts one element past a 16-byte boundary takes
    the register form of the collision; an aligned one the LDS-staged form
    where that applies (FP32 storage; D3Q45 in FP64 always takes the register
    form).  Both give the same values bit for bit (the same FP64 arithmetic,
    one rounding to the storage type), within half an FP32 ulp of the FP64
    oracle in FP32 storage and within 1e-12 in FP64."""
    ctx, cfg = make_pair(oracle, (7, 2, 2), 4, 0.07, 0.013, precision=precision)
    xs, ys, zs = oracle.node_coords(cfg)
    f, g = oracle.init_equilibrium(cfg, *inputs.tgv_fields(xs, ys, zs, 0.9, 1.4))
    rng = np.random.default_rng(6)
    f = f * (1 + 0.03 * rng.normal(size=f.shape))
    g = g * (1 + 0.03 * rng.normal(size=g.shape))
    if precision:
        f, g = f.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
    n = 2 * Q * ctx.nodes
    flat = torch.zeros(n + 1, dtype=ctx.dtype, device=ctx.device)
    st = flat[1:].view(2, Q, ctx.nodes)
    st.copy_(to_dev(ctx, f, g))
    al = to_dev(ctx, f, g)
    ctx.collide(st)
    ctx.collide(al)
    assert float(flat[0]) == 0.0
    assert torch.equal(st, al)
    fo, go = oracle.collide(cfg, f, g)
    for got, ref in zip(to_np(al), (fo, go)):
        if precision:
            assert float(np.max(np.abs(got - ref) / np.abs(ref))) <= 2.0 ** -24 * (1 + 1e-4)
        else:
            assert rel_err(got, ref) < TOL64


def test_init_and_moments_match_oracle(oracle):
    w, ctx, cfg = workload_pair(oracle, "c1")
    f, g = tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    F, G = to_np(ctx.get_state())
    assert rel_err(F, f) < TOL64 and rel_err(G, g) < TOL64
    rho, u, T = ctx.moments()
    r0, u0, T0 = oracle.moments(cfg, f, g)
    assert rel_err(rho.cpu().numpy(), r0) < TOL64
    assert rel_err(u.cpu().numpy(), u0) < TOL64
    assert rel_err(T.cpu().numpy(), T0) < TOL64
    tot = np.array(ctx.totals())
    tref = oracle.totals(cfg, f, g)
    assert np.all(np.abs(tot - tref) <= TOL64 * np.max(np.abs(tref)))


@pytest.mark.parametrize("nsteps", [1, 2, 10])
def test_c1_steps_match_oracle(oracle, nsteps):
    """4^3 cells, p = 2, TGV Ma 0.5 Re 100 CFL 2 (the small FP64 workload)."""
    _say(f"c1 parity {nsteps} steps")
    w, ctx, cfg = workload_pair(oracle, "c1")
    f, g = tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    ctx.step(nsteps)
    fo, go = oracle.step(cfg, f, g, nsteps)
    F, G = to_np(ctx.get_state())
    assert rel_err(F, fo) < TOL64 and rel_err(G, go) < TOL64
    rho, u, T = ctx.moments()
    r0, u0, T0 = oracle.moments(cfg, fo, go)
    for a, b in ((rho, r0), (u, u0), (T, T0)):
        assert rel_err(a.cpu().numpy(), b) < TOL64


def test_step_split_equals_step_total(oracle):
    """step(3); step(4) == step(7) bitwise; get_state in between changes nothing."""
    w, ctx, cfg = workload_pair(oracle, "c1")
    tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    ctx.step(3)
    mid = ctx.get_state()
    ctx.step(4)
    a = ctx.get_state()
    ctx.set_state(mid)
    ctx.step(4)
    b = ctx.get_state()
    assert torch.equal(a, b)
    w2, ctx2, _ = workload_pair(oracle, "c1")
    tgv_init(oracle, ctx2, cfg, w["Ma"], w["gamma"])
    ctx2.step(7)
    assert torch.equal(ctx2.get_state(), a)


@pytest.mark.parametrize("precision", [0, 1])
def test_step_record_matches_get_state(oracle, precision):
    """step_record collides into the spare buffer, step in place: bitwise equal."""
    w, ctx, cfg = workload_pair(oracle, "c1", precision=precision)
    tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    rec = torch.empty((4, 2, Q, ctx.nodes), dtype=ctx.dtype, device=ctx.device)
    s0 = ctx.get_state()
    ctx.step_record(4, rec)
    ctx2 = make_pair(oracle, w["n_el"], w["p"], w["dt"], w["mu_inf"], gamma=w["gamma"], prandtl=w["Pr"],
                     precision=precision)[0]
    ctx2.set_state(s0)
    for k in range(4):
        ctx2.step(1)
        assert torch.equal(ctx2.get_state(), rec[k])


def test_uniform_flow_stays_uniform_gpu(oracle):
    ctx, cfg = make_pair(oracle, (3, 2, 4), 4, 0.2, 0.02)
    N = ctx.nodes
    dev = ctx.device
    u = torch.tensor([0.3, -0.2, 0.1], dtype=torch.float64, device=dev)[:, None].expand(3, N).contiguous()
    ctx.init_equilibrium(torch.ones(N, dtype=torch.float64, device=dev), u, torch.ones(N, dtype=torch.float64,
                                                                                          device=dev))
    s0 = ctx.get_state()
    ctx.step(5)
    assert float((ctx.get_state() - s0).abs().max()) < 1e-13


def test_c2_one_step_sampled_nodes(oracle):
    """16^3 cells, p = 4 (64^3 nodes), Ma 1.25 Re 1600, CFL 1/5/10: one step at
    full size, in the launch configuration of the benchmark, checked at
    sampled nodes that the oracle evaluates one by one."""
    for cfl in (1.0, 5.0, 10.0):
        _say(f"c2 sampled parity cfl={cfl}")
        w, ctx, cfg = workload_pair(oracle, "c2", cfl=cfl)
        f, g = tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
        ctx.step(1)
        F, G = to_np(ctx.get_state())
        rng = np.random.default_rng(int(cfl))
        nodes = np.concatenate([[0, ctx.nodes - 1], rng.integers(0, ctx.nodes, 14)])
        fs, gs = oracle.step_at_nodes(cfg, f, g, nodes)
        scale = max(np.abs(f).max(), 1.0)
        assert np.max(np.abs(F[:, nodes].T - fs)) < TOL64 * scale
        assert np.max(np.abs(G[:, nodes].T - gs)) < TOL64 * np.abs(g).max()


def test_c2_first_steps_full_grid(oracle):
    """64^3 nodes, CFL 1: three full steps against the whole-grid oracle."""
    _say("c2 full-grid parity, 3 steps")
    w, ctx, cfg = workload_pair(oracle, "c2", cfl=1.0)
    f, g = tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    ctx.step(3)
    fo, go = oracle.step(cfg, f, g, 3)
    F, G = to_np(ctx.get_state())
    assert rel_err(F, fo) < TOL64 and rel_err(G, go) < TOL64


@pytest.mark.parametrize("cfl", [5.0, 10.0])
def test_c2_full_grid_every_step_until_non_finite(oracle, cfl):
    """64^3 nodes at CFL 5 and 10 (tau - 1/2 = 0.0073 and 0.0036): the whole
    grid against the oracle after every step, until the flow itself goes
    non-finite (steps 16 and 14 here).  Every finite step agrees to 1e-12
    (the one-ulp floor of the flow stays near 1e-14 over these steps), and
    both implementations go non-finite at the same step."""
    _say(f"c2 full-grid parity every step, cfl={cfl}")
    w, ctx, cfg = workload_pair(oracle, "c2", cfl=cfl)
    f, g = tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    for n in range(1, 21):
        ctx.step(1)
        f, g = oracle.step(cfg, f, g, 1)
        F, G = to_np(ctx.get_state())
        gpu_ok = bool(np.isfinite(F).all() and np.isfinite(G).all())
        ora_ok = bool(np.isfinite(f).all() and np.isfinite(g).all())
        assert gpu_ok == ora_ok, f"step {n}: GPU finite {gpu_ok}, oracle finite {ora_ok}"
        if not gpu_ok:
            _say(f"c2 cfl={cfl}: both non-finite at step {n}")
            break
        err = max(rel_err(F, f), rel_err(G, g))
        assert err < TOL64, f"step {n}: {err:.3e}"
    assert n > 5
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_deterministic(oracle, precision):
    """Steps, totals and an adjoint step (with its dL/dmu_inf partial sums)
    repeat bit for bit: no atomics, fixed reduction orders."""
    w, ctx, cfg = workload_pair(oracle, "c1", precision=precision)
    runs = []
    for _ in range(2):
        tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
        ctx.step(5)
        x = ctx.get_state()
        dmu = torch.zeros(1, dtype=torch.float64, device=ctx.device)
        lam = ctx.adjoint_step(x, x.clone(), dmu=dmu)
        runs.append((x, ctx.totals(), lam, dmu.item()))
    (a, ta, la, da), (b, tb, lb, db) = runs
    assert torch.equal(a, b)
    assert ta == tb
    assert torch.equal(la, lb) and da == db


def test_zero_steps_is_identity(oracle):
    w, ctx, cfg = workload_pair(oracle, "c1")
    tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    s0 = ctx.get_state()
    ctx.step(0)
    assert torch.equal(s0, ctx.get_state())


def test_fp32_mixed_matches_oracle(oracle):
    """FP32 populations vs the FP64 oracle on c1: moments within 1e-5."""
    _say("fp32 mixed c1 parity")
    w, ctx, cfg = workload_pair(oracle, "c1", precision=1)
    f, g = tgv_init(oracle, ctx, cfg, w["Ma"], w["gamma"])
    ctx.step(10)
    fo, go = oracle.step(cfg, f, g, 10)
    rho, u, T = ctx.moments()
    r0, u0, T0 = oracle.moments(cfg, fo, go)
    assert rel_err(rho.cpu().numpy(), r0) < 1e-5
    assert rel_err(u.cpu().numpy(), u0) < 1e-5
    assert rel_err(T.cpu().numpy(), T0) < 1e-5
