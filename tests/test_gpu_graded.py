"""GPU parity on graded meshes (periodic, axis-aligned cells of unequal
width, set with sllbm_set_mesh) against the oracle, whose graded streaming
is pinned in test_oracle_graded.py.

Bar: FP64 max-abs error relative to the oracle's largest value <= 1e-12;
FP32-mixed storage <= 1e-5 (the FP32-mixed tolerance of the equal-cell
path).  The full-size case is the 64^3-node TGV workload on the cosine-graded
mesh of the benchmark, checked on sampled nodes of one step.
"""
import math
import sys

import numpy as np
import pytest
import torch

from gpu_common import Q, to_np, to_dev, rel_err, require_gpu
from paper_2012_05537_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _rand_widths(n, length, seed, amp=0.45):
    rng = np.random.default_rng(seed)
    w = 1.0 + amp * rng.uniform(-1.0, 1.0, n)
    return w * (length / w.sum())


def _graded_pair(oracle, n_el, p, dt, widths, length=2 * math.pi, precision=0, mu=0.01):
    from paper_2012_05537_amd.sllbm import SLLBM
    if np.isscalar(length):
        length = (length,) * 3
    ctx = SLLBM(n_el, p, dt, mu, length=length, precision=precision)
    ctx.set_mesh(*widths)
    cfg = oracle.make_cfg(n_el, p, dt, mu, length=length, widths=widths)
    return ctx, cfg


# (n_el, p, dt, graded axes): ragged tiles, one-cell axes, shifts of several cells
CASES = [
    ((3, 2, 4), 2, 0.41, (1, 0, 1)),
    ((5, 3, 2), 3, 0.9, (1, 1, 1)),
    ((10, 5, 9), 4, 0.3, (1, 1, 1)),
    ((2, 1, 1), 4, 1.7, (1, 0, 0)),
    ((9, 2, 3), 1, 0.2, (0, 1, 1)),
    ((3, 4, 2), 5, 0.25, (1, 1, 0)),
    ((2, 2, 3), 6, 0.35, (1, 0, 1)),
]


def _widths_for(n_el, graded, length, seed):
    return [_rand_widths(n, length, seed + a) if graded[a] else None for a, n in enumerate(n_el)]


@pytest.mark.parametrize("n_el,p,dt,graded", CASES)
def test_graded_stream_matches_oracle(oracle, n_el, p, dt, graded):
    _say(f"graded stream n_el={n_el} p={p} dt={dt} graded={graded}")
    widths = _widths_for(n_el, graded, 2 * math.pi, 10 * p)
    ctx, cfg = _graded_pair(oracle, n_el, p, dt, widths)
    rng = np.random.default_rng(sum(n_el) + p)
    N = oracle.num_nodes(cfg)
    f, g = rng.normal(size=(Q, N)), rng.normal(size=(Q, N))
    F, G = to_np(ctx.stream(to_dev(ctx, f, g)))
    fo, go = oracle.stream(cfg, f, g)
    assert rel_err(F, fo) < 1e-12 and rel_err(G, go) < 1e-12
    ctx.close()


@pytest.mark.parametrize("n_el,p,dt,graded", [CASES[1], CASES[2], CASES[3]])
def test_graded_stream_fp32(oracle, n_el, p, dt, graded):
    widths = _widths_for(n_el, graded, 2 * math.pi, 10 * p)
    ctx, cfg = _graded_pair(oracle, n_el, p, dt, widths, precision=1)
    rng = np.random.default_rng(7)
    N = oracle.num_nodes(cfg)
    f32 = rng.normal(size=(Q, N)).astype(np.float32).astype(np.float64)
    g32 = rng.normal(size=(Q, N)).astype(np.float32).astype(np.float64)
    F, G = to_np(ctx.stream(to_dev(ctx, f32, g32)))
    fo, go = oracle.stream(cfg, f32, g32)
    assert rel_err(F, fo) < 1e-5 and rel_err(G, go) < 1e-5
    ctx.close()


def test_equal_widths_graded_kernel_matches_equal_cell_kernel(oracle):
    """The graded kernel on equal widths against the equal-cell z-march."""
    from paper_2012_05537_amd.sllbm import SLLBM
    n_el, p, dt = (8, 6, 5), 4, 0.37
    L = 2 * math.pi
    a = SLLBM(n_el, p, dt, 0.01)
    b = SLLBM(n_el, p, dt, 0.01)
    b.set_mesh(*[np.full(n, L / n) for n in n_el])
    gen = torch.Generator(device=a.device).manual_seed(4)
    x = torch.randn((2, Q, a.nodes), generator=gen, device=a.device, dtype=torch.float64)
    ya, yb = a.stream(x), b.stream(x)
    assert float((ya - yb).abs().max() / ya.abs().max()) < 1e-13
    a.close()
    b.close()


def test_graded_steps_match_oracle(oracle):
    """Three collide-and-stream steps of a TGV on a randomly graded mesh."""
    n_el, p, dt = (4, 3, 5), 3, 0.12
    widths = _widths_for(n_el, (1, 1, 1), 2 * math.pi, 50)
    ctx, cfg = _graded_pair(oracle, n_el, p, dt, widths, mu=0.02)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.6, 1.4)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    ctx.set_state(to_dev(ctx, f, g))
    ctx.step(3)
    f, g = oracle.step(cfg, f, g, 3)
    F, G = to_np(ctx.get_state())
    assert rel_err(F, f) < 1e-12 and rel_err(G, g) < 1e-12
    got = np.array(ctx.totals())
    ref = np.array(oracle.totals(cfg, f, g))
    assert np.all(np.abs(got - ref) <= 1e-12 * np.abs(ref).max())
    ctx.close()


def test_graded_node_coords(oracle):
    n_el, p = (5, 3, 2), 4
    widths = _widths_for(n_el, (1, 0, 1), 2 * math.pi, 60)
    ctx, cfg = _graded_pair(oracle, n_el, p, 0.1, widths)
    for a, b in zip(ctx.node_coords(), oracle.node_coords(cfg)):
        assert np.max(np.abs(a.numpy() - b)) < 1e-14
    ctx.close()


def test_graded_full_size_sampled(oracle):
    """64^3-node TGV (16^3 cells, p = 4, Ma 1.25, CFL 1) on the cosine-graded
    mesh of the benchmark: one FP64 step, sampled nodes against the oracle."""
    w = inputs.workload(inputs.GRADED["base"])
    n = w["n_el"]
    widths = [inputs.graded_widths(n, amplitude=inputs.GRADED["amplitude"])] * 3
    ctx, cfg = _graded_pair(oracle, (n, n, n), w["p"], w["dt"], widths, mu=w["mu_inf"])
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, w["Ma"], w["gamma"])
    dev = ctx.device
    ctx.init_equilibrium(*(torch.from_numpy(x).to(dev) for x in (rho, u, T)))
    f0, g0 = to_np(ctx.get_state())
    ctx.step(1)
    X1 = ctx.get_state()
    nodes = np.concatenate([[0, ctx.nodes - 1], np.random.default_rng(16).integers(0, ctx.nodes, 30)])
    fs, gs = oracle.step_at_nodes(cfg, f0, g0, nodes)
    idx = torch.from_numpy(nodes).to(dev)
    F = X1[0][:, idx].cpu().numpy().T
    G = X1[1][:, idx].cpu().numpy().T
    err = max(np.max(np.abs(F - fs)) / np.abs(fs).max(), np.max(np.abs(G - gs)) / np.abs(gs).max())
    _say(f"graded 64^3 sampled step: max rel error {err:.2e}")
    assert err < 1e-12
    ctx.close()


@pytest.mark.parametrize("n_el,p,dt,graded", [CASES[0], CASES[1], CASES[2], CASES[3], CASES[5]])
def test_graded_transposed_stream_is_adjoint(oracle, n_el, p, dt, graded):
    """<S x, y> = <x, S^T y> per population and velocity, S x from the oracle's
    graded gather, S^T y from the library's transposed per-node tables."""
    _say(f"graded transposed stream n_el={n_el} p={p} dt={dt}")
    widths = _widths_for(n_el, graded, 2 * math.pi, 10 * p)
    ctx, cfg = _graded_pair(oracle, n_el, p, dt, widths)
    rng = np.random.default_rng(8)
    N = oracle.num_nodes(cfg)
    x = rng.normal(size=(2, Q, N))
    y = rng.normal(size=(2, Q, N))
    Sx = np.stack(oracle.stream(cfg, x[0], x[1]))
    STy = ctx.stream(to_dev(ctx, y[0], y[1]), transpose=True).cpu().numpy()
    lhs = np.einsum("pin,pin->pi", Sx, y)
    rhs = np.einsum("pin,pin->pi", x, STy)
    scale = np.einsum("pin,pin->pi", np.abs(Sx), np.abs(y))
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale), np.max(np.abs(lhs - rhs) / scale)
    ctx.close()


def test_graded_adjoint_step_dot_product(oracle):
    """<adjoint_step(X, lam), v> = <lam, d step(X)[v]> on a graded mesh, with
    d step[v] from a complex-step oracle step (collide, then graded stream)."""
    n_el, p, dt, mu = (4, 3, 5), 3, 0.3, 0.0106
    widths = _widths_for(n_el, (1, 1, 1), 2 * math.pi, 70)
    ctx, cfg = _graded_pair(oracle, n_el, p, dt, widths, mu=mu)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.5, 1.4)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    rng = np.random.default_rng(3)
    f = f * (1.0 + 0.02 * rng.normal(size=f.shape))
    g = g * (1.0 + 0.02 * rng.normal(size=g.shape))
    N = f.shape[1]
    lf, lg = rng.normal(size=(Q, N)), rng.normal(size=(Q, N))
    LF, LG = to_np(ctx.adjoint_step(to_dev(ctx, f, g), to_dev(ctx, lf, lg)))
    H = 1e-30
    for trial in range(3):
        vf, vg = rng.normal(size=(Q, N)), rng.normal(size=(Q, N))
        sf, sg = oracle.step(cfg, f + 1j * H * vf, g + 1j * H * vg, 1)
        ref = (np.sum(lf * sf.imag) + np.sum(lg * sg.imag)) / H
        got = np.sum(LF * vf) + np.sum(LG * vg)
        assert abs(got - ref) <= 1e-12 * np.sum(np.abs(LF * vf) + np.abs(LG * vg)), (trial, got, ref)
    ctx.close()


def _noisy_graded(oracle, n_el, p, widths, seed, mu=0.01, dt=0.1):
    ctx, cfg = _graded_pair(oracle, n_el, p, dt, widths, mu=mu)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.5, 1.4)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    rng = np.random.default_rng(seed)
    f = f * (1.0 + 0.02 * rng.normal(size=f.shape))
    g = g * (1.0 + 0.02 * rng.normal(size=g.shape))
    return ctx, cfg, f, g


@pytest.mark.parametrize("n_el,p", [((3, 4, 2), 2), ((2, 3, 3), 3)])
def test_graded_loss_and_diagnostics_match_oracle(oracle, n_el, p):
    widths = _widths_for(n_el, (1, 1, 1), 2 * math.pi, 40 + p)
    ctx, cfg, f, g = _noisy_graded(oracle, n_el, p, widths, seed=p)
    X = to_dev(ctx, f, g)
    assert ctx.loss(X) == pytest.approx(oracle.loss(cfg, f, g), rel=1e-12)
    got = np.array(ctx.diagnostics(X))
    ref = np.array(oracle.diagnostics(cfg, f, g))
    assert np.all(np.abs(got - ref) <= 1e-12 * np.abs(ref))
    ctx.close()


def test_graded_loss_grad_elementwise(oracle):
    """dL/df_i(n) at every population and node from complex steps of the
    oracle's loss on the graded mesh (each cell with its own width)."""
    n_el, p = (3, 2, 2), 2
    widths = _widths_for(n_el, (1, 1, 0), 2 * math.pi, 44)
    ctx, cfg, f, g = _noisy_graded(oracle, n_el, p, widths, seed=12)
    LF, LG = to_np(ctx.loss_grad(to_dev(ctx, f, g)))
    N = f.shape[1]
    H = 1e-30
    ref = np.zeros((Q, N))
    gc = g.astype(np.complex128)
    for k in range(Q):
        for n in range(N):
            fc = f.astype(np.complex128)
            fc[k, n] += 1j * H
            ref[k, n] = oracle.loss(cfg, fc, gc).imag / H
    assert rel_err(LF, ref) < 1e-12, rel_err(LF, ref)
    assert np.all(LG == 0.0)
    ctx.close()


def test_graded_rollout_gradient(oracle):
    """Gradient of an 8-step rollout on a graded mesh (4 modes and mu_inf)
    against complex-step oracle rollouts on the same mesh."""
    from paper_2012_05537_amd.adjoint import Rollout
    n_el, p, dt, mu, Ma = (4, 3, 4), 2, 0.3, 0.0106, 0.5
    widths = _widths_for(n_el, (1, 1, 1), 2 * math.pi, 60)
    ctx, cfg = _graded_pair(oracle, n_el, p, dt, widths, mu=mu)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, Ma, 1.4)
    modes = inputs.fourier_modes(2012, 4, Ma, 1.4, 0.01)
    B = inputs.mode_basis(xs, ys, zs, modes)
    amps = np.array([m[3] for m in modes])
    n = 8
    roll = Rollout(ctx, rho, u, T, B, n, checkpoint=3)
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    m_ = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
    L = roll(a, m_)
    L.backward()
    H = 1e-30

    def directional(da, dmu):
        c = oracle.make_cfg(n_el, p, dt, mu, widths=widths, mu_inf_im=H * dmu)
        uc = u + np.tensordot(amps + 1j * H * da, B, axes=(0, 0))
        fc, gc = oracle.init_equilibrium(c, rho.astype(np.complex128), uc, T.astype(np.complex128))
        fc, gc = oracle.step(c, fc, gc, n)
        Lc = oracle.loss(c, fc, gc)
        return Lc.real, Lc.imag / H

    L_ref, _ = directional(np.zeros_like(amps), 0.0)
    assert L.item() == pytest.approx(L_ref, rel=1e-12)
    rng = np.random.default_rng(5)
    da, dmu = rng.normal(size=amps.size), float(rng.normal()) * mu
    got = float(a.grad.numpy() @ da + m_.grad.item() * dmu)
    assert got == pytest.approx(directional(da, dmu)[1], rel=1e-10)
    ctx.close()


def test_graded_bad_widths_keep_the_mesh(oracle):
    from paper_2012_05537_amd.sllbm import SLLBM, SllbmError
    n_el, p, dt = (3, 2, 2), 2, 0.2
    ctx = SLLBM(n_el, p, dt, 0.01)
    gen = torch.Generator(device=ctx.device).manual_seed(1)
    x = torch.randn((2, Q, ctx.nodes), generator=gen, device=ctx.device, dtype=torch.float64)
    ref = ctx.stream(x)
    with pytest.raises(SllbmError):
        ctx.set_mesh(np.array([1.0, -1.0, 2.0]))          # non-positive width
    with pytest.raises(ValueError):
        ctx.set_mesh(np.array([1.0, 2.0]))                # wrong count
    assert torch.equal(ctx.stream(x), ref)                # the equal-cell mesh stays
    ctx.close()


def test_graded_too_strong_grading_keeps_the_previous_mesh(oracle):
    """15 cells of width 0.01 beside one of 2 pi - 0.15: the nodes of the wide
    cell are read by 32 nodes of the axis (more than the 24 taps of the
    transposed streaming), so set_mesh fails and the previous graded mesh stays."""
    from paper_2012_05537_amd.sllbm import SLLBM, SllbmError
    n_el, p, dt = (16, 3, 2), 2, 0.2
    ctx = SLLBM(n_el, p, dt, 0.01)
    ctx.set_mesh(None, _rand_widths(3, 2 * math.pi, 5))
    gen = torch.Generator(device=ctx.device).manual_seed(2)
    x = torch.randn((2, Q, ctx.nodes), generator=gen, device=ctx.device, dtype=torch.float64)
    ref, ref_t = ctx.stream(x), ctx.stream(x, transpose=True)
    coords = [c.clone() for c in ctx.node_coords()]
    w = np.full(16, 0.01)
    w[0] = 2 * math.pi - 0.15
    with pytest.raises(SllbmError):
        ctx.set_mesh(w)
    assert torch.equal(ctx.stream(x), ref) and torch.equal(ctx.stream(x, transpose=True), ref_t)
    assert all(torch.equal(a, b) for a, b in zip(ctx.node_coords(), coords))
    ctx.close()
