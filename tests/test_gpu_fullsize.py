"""Parity at the full sizes of the FP32-mixed workloads (128^3 and 256^3
nodes, order 4), in the launch configuration of the benchmark, on outputs the
oracle evaluates one by one.

* Whole z-planes of one stream and one collide, in the workloads' FP32
  storage (1e-5) and in FP64 (1e-12), the benchmark's headline precision.

* Forward: the GPU's initial state (FP32 storage) is given to the oracle,
  which computes one step at sampled nodes (each sample collides its whole
  (p+1)^3 departure stencil and interpolates); the GPU steps the same state.
  Bar: the FP32-mixed tolerance 1e-5 relative to the largest population.
* Adjoint: lambda_n = J_C(X)^T S^T lambda_{n+1} at sampled nodes, with S^T of
  the library (its transpose identity is pinned on smaller grids) and J_C^T
  from complex-step collisions of the sampled nodes in the oracle (collision
  is node-local).  Bar: 1e-4 relative (FP32 storage of X and lambda).
* Transposed streaming at 256^3: <S x, y> = <x, S^T y> for random x, y,
  both sides from the library, per population and velocity.
"""
import sys

import numpy as np
import pytest
import torch

from gpu_common import Q, workload_pair, to_np, require_gpu
from paper_2012_05537_amd import inputs

pytestmark = pytest.mark.gpu

H = 1e-30


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _init_gpu(ctx, w):
    xs, ys, zs = (t.numpy() for t in ctx.node_coords())
    rho, u, T = inputs.tgv_fields(xs, ys, zs, w["Ma"], w["gamma"])
    dev = ctx.device
    ctx.init_equilibrium(*(torch.from_numpy(x).to(dev) for x in (rho, u, T)))


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_one_step_sampled_full_size(oracle, name):
    _say(f"{name}: one FP32-mixed step at full size, sampled")
    w, ctx, cfg = workload_pair(oracle, name)
    _init_gpu(ctx, w)
    X0 = ctx.get_state()
    f0, g0 = to_np(X0)                         # the exact FP32 values, as float64
    ctx.step(1)
    X1 = ctx.get_state()
    rng = np.random.default_rng(2021 if name == "c5" else 2012)
    nodes = np.concatenate([[0, ctx.nodes - 1], rng.integers(0, ctx.nodes, 30)])
    fs, gs = oracle.step_at_nodes(cfg, f0, g0, nodes)
    idx = torch.from_numpy(nodes).to(ctx.device)
    F = X1[0][:, idx].double().cpu().numpy().T
    G = X1[1][:, idx].double().cpu().numpy().T
    del f0, g0
    ef = np.max(np.abs(F - fs)) / np.abs(fs).max()
    eg = np.max(np.abs(G - gs)) / np.abs(gs).max()
    _say(f"{name}: max rel error f {ef:.2e} g {eg:.2e}")
    assert ef < 1e-5 and eg < 1e-5
    ctx.close()


@pytest.mark.parametrize("name,precision,tol", [("c3", None, 1e-5), ("c5", None, 1e-5), ("c3", 0, 1e-12),
                                                ("c5", 0, 1e-12)])
def test_whole_z_planes_stream_and_collide_full_size(oracle, name, precision, tol):
    """One sllbm_stream and one sllbm_collide of a full-size state (two steps
    into the flow; the workload's FP32 storage, and FP64 as the benchmark's
    headline runs the 256^3-node grid) against the oracle's stream and collide
    on three whole z-planes (the periodic seam, an interior plane, the last
    plane): every node and population of those planes, element by element."""
    _say(f"{name}: whole z-planes of one stream and one collide at full size, precision {precision}")
    w, ctx, cfg = workload_pair(oracle, name, precision=precision)
    _init_gpu(ctx, w)
    ctx.step(2)
    X0 = ctx.get_state()
    Nz, Ny, Nx = ctx.shape
    P = Nx * Ny
    planes = [0, Nz // 2 + 1, Nz - 1]
    Xs = ctx.stream(X0)
    Xc = X0.clone()
    ctx.collide(Xc)
    torch.cuda.synchronize()
    f0, g0 = to_np(X0)
    n_el = w["n_el"]
    plane_cfg = oracle.make_cfg((n_el, n_el // w["p"], 1), w["p"], w["dt"], w["mu_inf"], gamma=w["gamma"],
                                prandtl=w["Pr"])
    assert oracle.num_nodes(plane_cfg) == P
    for z in planes:
        nodes = z * P + np.arange(P)
        fs, gs = oracle.stream_at_nodes(cfg, f0, g0, nodes)
        F = Xs[0][:, z * P:(z + 1) * P].double().cpu().numpy().T
        G = Xs[1][:, z * P:(z + 1) * P].double().cpu().numpy().T
        es = max(np.max(np.abs(F - fs)) / np.abs(fs).max(), np.max(np.abs(G - gs)) / np.abs(gs).max())
        fc, gc = oracle.collide(plane_cfg, f0[:, z * P:(z + 1) * P].copy(), g0[:, z * P:(z + 1) * P].copy())
        F = Xc[0][:, z * P:(z + 1) * P].double().cpu().numpy()
        G = Xc[1][:, z * P:(z + 1) * P].double().cpu().numpy()
        ec = max(np.max(np.abs(F - fc)) / np.abs(fc).max(), np.max(np.abs(G - gc)) / np.abs(gc).max())
        _say(f"{name} plane z={z}: stream max rel error {es:.2e}, collide {ec:.2e}")
        assert es < tol and ec < tol
        if Xc.dtype == torch.float32:
            # FP32 storage: every collided value is the FP64 collision of the
            # stored values rounded once (half an ulp), up to FP64 rounding
            for got, ref in ((F, fc), (G, gc)):
                slack = np.abs(got - ref) - 2.0 ** -24 * np.abs(ref)
                assert np.max(slack) <= 1e-13 * np.abs(ref).max(), np.max(slack)
    del f0, g0
    ctx.close()


def _collide_vjp_at(oracle, cfg_small, f, g, yf, yg):
    """J_C^T y for a set of nodes held as a small grid (collision is node-local)."""
    n = f.shape[1]
    lf = np.zeros((Q, n))
    lg = np.zeros((Q, n))
    for pop in range(2):
        for k in range(Q):
            fc = f.astype(np.complex128)
            gc = g.astype(np.complex128)
            (gc if pop else fc)[k] += 1j * H
            cf, cg = oracle.collide(cfg_small, fc, gc)
            col = (np.sum(yf * cf.imag, axis=0) + np.sum(yg * cg.imag, axis=0)) / H
            (lg if pop else lf)[k] = col
    return lf, lg


def test_adjoint_step_sampled_256cubed(oracle):
    """c5 size (64^3 cells, p = 4, FP32 storage, CFL 10)."""
    _say("c5: adjoint step at full size, sampled")
    w, ctx, cfg = workload_pair(oracle, "c5")
    _init_gpu(ctx, w)
    ctx.step(2)
    X = ctx.get_state()
    gen = torch.Generator(device=ctx.device).manual_seed(5)
    lam_next = torch.randn(X.shape, generator=gen, device=ctx.device, dtype=torch.float32)
    y = ctx.stream(lam_next, transpose=True)
    lam = ctx.adjoint_step(X, lam_next)
    torch.cuda.synchronize()
    nodes = np.random.default_rng(3).integers(0, ctx.nodes, 64)
    idx = torch.from_numpy(nodes).to(ctx.device)
    pick = lambda t: (t[0][:, idx].double().cpu().numpy(), t[1][:, idx].double().cpu().numpy())
    f, g = pick(X)
    yf, yg = pick(y)
    LF, LG = pick(lam)
    # the 64 sampled nodes as a 4^3-node grid of the same parameters (collision ignores geometry)
    small = oracle.make_cfg((1, 1, 1), 4, w["dt"], w["mu_inf"], gamma=w["gamma"], prandtl=w["Pr"])
    ef, eg = _collide_vjp_at(oracle, small, f, g, yf, yg)
    err = max(np.max(np.abs(LF - ef)) / np.abs(ef).max(), np.max(np.abs(LG - eg)) / np.abs(eg).max())
    _say(f"c5 adjoint sampled max rel error {err:.2e}")
    assert err < 1e-4
    ctx.close()


def test_transposed_stream_identity_256cubed(oracle):
    w, ctx, cfg = workload_pair(oracle, "c5")
    gen = torch.Generator(device=ctx.device).manual_seed(11)
    shape = (2, Q, ctx.nodes)
    x = torch.randn(shape, generator=gen, device=ctx.device, dtype=torch.float32)
    yv = torch.randn(shape, generator=gen, device=ctx.device, dtype=torch.float32)
    Sx = ctx.stream(x)
    STy = ctx.stream(yv, transpose=True)
    lhs = (Sx.double() * yv.double()).sum(dim=2)
    rhs = (x.double() * STy.double()).sum(dim=2)
    scale = (Sx.double().abs() * yv.double().abs()).sum(dim=2)
    rel = float(((lhs - rhs).abs() / scale).max())
    _say(f"c5 transposed identity: max rel {rel:.2e}")
    assert rel < 1e-5
    ctx.close()


# grids whose state exceeds the Infinity Cache at orders 1-3, 5 and 6, where
# the streaming runs its large-grid form (non-temporal stores; 32 x 16-node
# tiles except at orders 5 and 6 in FP64, whose LDS keeps 8-row tiles; the
# order-4 workloads above take it at 128^3 and 256^3 nodes): ragged tiles
# along y, shifts of several cells (CFL 3)
LARGE = [((40, 36, 30), 3, 0), ((48, 40, 36), 2, 0), ((100, 90, 100), 1, 1), ((48, 44, 40), 3, 1),
         ((24, 20, 18), 5, 0), ((16, 16, 16), 6, 0), ((28, 24, 20), 5, 1)]


@pytest.mark.parametrize("n_el,p,precision", LARGE)
def test_large_grid_stream_planes(oracle, n_el, p, precision):
    """One sllbm_stream of a random state against the oracle's streaming on
    three whole z-planes, element by element (1e-12 in FP64, 1e-5 in FP32),
    and the transposed streaming's identity <S x, y> = <x, S^T y> per
    population and velocity."""
    from gpu_common import make_pair
    import math
    _say(f"large-grid stream n_el={n_el} p={p} precision={precision}")
    dt = 3.0 * (2 * math.pi / (max(n_el) * p)) / math.sqrt(15.0)
    ctx, cfg = make_pair(oracle, n_el, p, dt, 1e-3, precision=precision)
    assert 90 * ctx.nodes * (8 if precision == 0 else 4) > 256 << 20
    gen = torch.Generator(device=ctx.device).manual_seed(p)
    X = torch.randn((2, Q, ctx.nodes), generator=gen, device=ctx.device, dtype=ctx.dtype)
    Xs = ctx.stream(X)
    torch.cuda.synchronize()
    f0, g0 = to_np(X)
    Nz, Ny, Nx = ctx.shape
    P = Nx * Ny
    tol = 1e-12 if precision == 0 else 1e-5
    for z in (0, Nz // 2 + 1, Nz - 1):
        nodes = z * P + np.arange(P)
        fs, gs = oracle.stream_at_nodes(cfg, f0, g0, nodes)
        F = Xs[0][:, z * P:(z + 1) * P].double().cpu().numpy().T
        G = Xs[1][:, z * P:(z + 1) * P].double().cpu().numpy().T
        err = max(np.max(np.abs(F - fs)) / np.abs(fs).max(), np.max(np.abs(G - gs)) / np.abs(gs).max())
        _say(f"  plane z={z}: max rel error {err:.2e}")
        assert err < tol
    del f0, g0
    # the transposed z-march in its large-grid form: <S x, y> = <x, S^T y>
    yv = torch.randn((2, Q, ctx.nodes), generator=gen, device=ctx.device, dtype=ctx.dtype)
    STy = ctx.stream(yv, transpose=True)
    lhs = (Xs.double() * yv.double()).sum(dim=2)
    rhs = (X.double() * STy.double()).sum(dim=2)
    scale = (Xs.double().abs() * yv.double().abs()).sum(dim=2)
    rel = float(((lhs - rhs).abs() / scale).max())
    _say(f"  transposed identity: max rel {rel:.2e}")
    assert rel < (1e-13 if precision == 0 else 1e-5)
    ctx.close()
