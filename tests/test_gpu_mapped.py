"""GPU parity on distorted meshes (sllbm_set_displacement) through the C ABI
against the FP64 oracle, whose distorted-mesh streaming is pinned in
test_oracle_mapped.py.  Bar: 1e-12 (FP64), 1e-5 (FP32-mixed), as elsewhere.
At the 64^3-node size, where the oracle's per-node Newton searches are too
slow, two properties hold at any size: zero displacement reproduces the
equal-cell path, and on a sheared mesh a field linear inside every reference
cell streams exactly to its closed-form value."""
import ctypes
import math
import sys

import numpy as np
import pytest
import torch

from gpu_common import Q, make_pair, tgv_init, to_np, to_dev, rel_err, require_gpu

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL_MIXED = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _ref(oracle, cfg):
    xs, ys, zs = oracle.node_coords(cfg)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


def _smooth_disp(X, Y, Z, s=1.0):
    return s * np.stack([0.2 * np.sin(Y + 0.5 * Z), 0.15 * np.cos(X) * np.sin(Z), 0.1 * np.sin(X + Y)])


def _pw(x, faces, vals):
    L = faces[-1]
    xw = np.mod(x, L)
    e = np.clip(np.searchsorted(faces, xw, side="right") - 1, 0, len(faces) - 2)
    t = (xw - faces[e]) / (faces[e + 1] - faces[e])
    v1 = np.append(vals, vals[0])
    return v1[e] * (1 - t) + v1[e + 1] * t


CASES = [((3, 4, 2), 2, 0.31), ((2, 3, 3), 3, 0.8), ((2, 2, 2), 4, 0.5), ((4, 2, 3), 1, 0.2), ((2, 2, 1), 5, 0.4)]


@pytest.mark.parametrize("n_el,p,dt", CASES)
def test_stream_matches_oracle(oracle, n_el, p, dt):
    _say(f"distorted stream parity n_el={n_el} p={p}")
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, 0.01)
    X, Y, Z = _ref(oracle, cfg0)
    disp = _smooth_disp(X, Y, Z)
    ctx.set_displacement(disp)
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, disp=disp)
    rng = np.random.default_rng(p)
    f, g = rng.normal(size=(Q, X.size)), rng.normal(size=(Q, X.size))
    F, G = to_np(ctx.stream(to_dev(ctx, f, g)))
    fo, go = oracle.stream(cfg, f, g)
    assert rel_err(F, fo) <= TOL64 and rel_err(G, go) <= TOL64, (rel_err(F, fo), rel_err(G, go))


# grids on which the staged kernel's source windows are in use: (6, 6, 5) cells
# at p = 4, dt = 0.8 mixes staged blocks with blocks whose window exceeds the
# LDS budget or spans an axis (global gather); (5, 6, 4) at p = 3 stages every
# block over ragged tiles (the host test pins both counts)
STAGED = [((6, 6, 5), 4, 0.8, 0, TOL64), ((5, 6, 4), 3, 0.5, 0, TOL64), ((6, 6, 5), 4, 0.8, 1, TOL_MIXED)]


@pytest.mark.parametrize("n_el,p,dt,precision,tol", STAGED)
def test_staged_stream_matches_oracle(oracle, n_el, p, dt, precision, tol):
    _say(f"distorted staged stream parity n_el={n_el} p={p} dt={dt} precision={precision}")
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, 0.01, precision=precision)
    X, Y, Z = _ref(oracle, cfg0)
    disp = _smooth_disp(X, Y, Z)
    ctx.set_displacement(disp)
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, disp=disp)
    rng = np.random.default_rng(11 + p)
    f, g = rng.normal(size=(Q, X.size)), rng.normal(size=(Q, X.size))
    if precision:
        f, g = f.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
    F, G = to_np(ctx.stream(to_dev(ctx, f, g)))
    fo, go = oracle.stream(cfg, f, g)
    assert rel_err(F, fo) <= tol and rel_err(G, go) <= tol, (rel_err(F, fo), rel_err(G, go))


def test_stream_fp32(oracle):
    n_el, p, dt = (3, 3, 2), 4, 0.5
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, 0.01, precision=1)
    X, Y, Z = _ref(oracle, cfg0)
    disp = _smooth_disp(X, Y, Z)
    ctx.set_displacement(disp)
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, disp=disp)
    rng = np.random.default_rng(5)
    f = rng.normal(size=(Q, X.size)).astype(np.float32).astype(np.float64)
    g = rng.normal(size=(Q, X.size)).astype(np.float32).astype(np.float64)
    F, G = to_np(ctx.stream(to_dev(ctx, f, g)))
    fo, go = oracle.stream(cfg, f, g)
    assert rel_err(F, fo) <= TOL_MIXED and rel_err(G, go) <= TOL_MIXED


def test_steps_and_totals_match_oracle(oracle):
    """Three TGV steps on a smoothly distorted 4^3-cell p = 3 mesh, then the
    Jacobian-weighted totals."""
    n_el, p, dt, mu = (4, 4, 4), 3, 0.1, 0.02
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, mu)
    X, Y, Z = _ref(oracle, cfg0)
    disp = _smooth_disp(X, Y, Z, 0.8)
    cfg = oracle.make_cfg(n_el, p, dt, mu, disp=disp)
    f, g = tgv_init(oracle, ctx, cfg, 0.5, 1.4)
    ctx.set_displacement(disp)
    ctx.step(3)
    fo, go = oracle.step(cfg, f, g, 3)
    F, G = to_np(ctx.get_state())
    assert rel_err(F, fo) <= TOL64 and rel_err(G, go) <= TOL64, (rel_err(F, fo), rel_err(G, go))
    tot = np.array(ctx.totals())
    to = oracle.totals(cfg, fo, go)
    assert np.allclose(tot, to, rtol=1e-12, atol=1e-12 * abs(to[0]))


def test_reset_and_zero_displacement(oracle):
    """d = NULL returns to the equal-cell kernels bit for bit; zero
    displacement gives the equal-cell result through the distorted path."""
    n_el, p, dt = (4, 4, 4), 4, 0.3
    ctx, cfg = make_pair(oracle, n_el, p, dt, 0.01)
    rng = np.random.default_rng(2)
    N = oracle.num_nodes(cfg)
    st = to_dev(ctx, rng.normal(size=(Q, N)), rng.normal(size=(Q, N)))
    base = ctx.stream(st)
    ctx.set_displacement(np.zeros((3, N)))
    zero = ctx.stream(st)
    assert rel_err(to_np(zero)[0], to_np(base)[0]) <= TOL64
    ctx.set_displacement(None)
    assert torch.equal(ctx.stream(st), base)


def test_fullsize_sheared_mesh_closed_form(oracle):
    """64^3 nodes (16^3 cells, p = 4) with a shear d_x = a s(r_y): a field
    linear inside every reference cell streams to its value at the departure
    point's reference coordinates, known in closed form (FP64)."""
    from paper_2012_05537_amd import inputs
    w = inputs.workload("c2")
    n_el = (w["n_el"],) * 3
    ctx, cfg0 = make_pair(oracle, n_el, w["p"], w["dt"], w["mu_inf"])
    X, Y, Z = _ref(oracle, cfg0)
    L = 2 * math.pi
    faces = np.arange(n_el[0] + 1) * L / n_el[0]
    rng = np.random.default_rng(64)
    svals = rng.uniform(-0.3, 0.3, n_el[1]) * (L / n_el[0])
    vals = [rng.uniform(0.5, 1.5, n) for n in n_el]
    disp = np.zeros((3, X.size))
    disp[0] = _pw(Y, faces, svals)
    ctx.set_displacement(disp)
    phi = lambda rx, ry, rz: _pw(rx, faces, vals[0]) * _pw(ry, faces, vals[1]) * _pw(rz, faces, vals[2])
    f = np.tile(phi(X, Y, Z), (Q, 1))
    F, G = to_np(ctx.stream(to_dev(ctx, f, 0.5 * f)))
    xi, _ = oracle.velocity_set()
    dt = w["dt"]
    worst = 0.0
    for i in range(Q):
        yd, zd = Y - xi[i, 1] * dt, Z - xi[i, 2] * dt
        rx = X + disp[0] - xi[i, 0] * dt - _pw(yd, faces, svals)
        ref = phi(rx, yd, zd)
        worst = max(worst, np.max(np.abs(F[i] - ref)), np.max(np.abs(G[i] - 0.5 * ref)))
    assert worst < 1e-11, worst


def test_refusals(oracle):
    n_el, p = (3, 3, 3), 2
    ctx, cfg0 = make_pair(oracle, n_el, p, 0.1, 0.01)
    X, Y, Z = _ref(oracle, cfg0)
    N = X.size
    lib, h = ctx._lib, ctx._h
    # a folded mesh is refused and the undistorted mesh stays
    folded = np.stack([2.0 * np.sin(X), np.zeros(N), np.zeros(N)])
    with pytest.raises(Exception):
        ctx.set_displacement(folded)
    rng = np.random.default_rng(1)
    st = to_dev(ctx, rng.normal(size=(Q, N)), rng.normal(size=(Q, N)))
    ctx2, _ = make_pair(oracle, n_el, p, 0.1, 0.01)
    assert torch.equal(ctx.stream(st), ctx2.stream(st))
    ctx.set_displacement(_smooth_disp(X, Y, Z))
    x = torch.ones((2, Q, N), dtype=torch.float64, device=ctx.device)
    y = torch.empty_like(x)
    ctx.set_state(x)
    pp = lambda t: ctypes.c_void_p(t.data_ptr())
    d = (ctypes.c_double * 4)()
    # the functional and the diagnostics work on distorted meshes
    assert lib.sllbm_loss(h, pp(x), ctypes.addressof(d)) == 0
    assert lib.sllbm_diagnostics(h, None, ctypes.addressof(d)) == 0
    wd = (ctypes.c_double * 3)(1, 1, 1)
    assert lib.sllbm_set_mesh(h, ctypes.addressof(wd), None, None) == 1
    assert "distorted" in lib.sllbm_last_error(h).decode()
    # and a graded context refuses a displacement
    ctx3, _ = make_pair(oracle, n_el, p, 0.1, 0.01)
    ctx3.set_mesh([1.0, 2.0, 3.0], None, None)
    zeros = np.zeros(3 * N)
    assert lib.sllbm_set_displacement(ctx3._h, ctypes.c_void_p(zeros.ctypes.data)) == 1


def test_distorted_tgv_run():
    """100 steps of the 64^3-node TGV (Ma 0.5, Re 400, CFL 1) on the
    benchmark's distorted mesh: finite, positive, mass and energy drift below
    1e-4 (Jacobian-weighted totals)."""
    from paper_2012_05537_amd import inputs
    from paper_2012_05537_amd.sllbm import SLLBM
    w = inputs.workload("c2", Ma=0.5, Re=400.0)
    ctx = SLLBM(w["n_el"], w["p"], w["dt"], w["mu_inf"])
    xs, ys, zs = (t.numpy() for t in ctx.node_coords())
    rho, u, T = inputs.tgv_fields(xs, ys, zs, w["Ma"], w["gamma"])
    ctx.init_equilibrium(*(torch.from_numpy(a).to(ctx.device) for a in (rho, u, T)))
    X, Y, Z = inputs.mesh(xs, ys, zs)
    ctx.set_displacement(inputs.distortion(X, Y, Z, 2 * math.pi / w["n_el"], inputs.DISTORTED["amplitude"]))
    t0 = np.array(ctx.totals())
    ctx.step(100)
    t1 = np.array(ctx.totals())
    r, _, T = ctx.moments()
    assert bool(torch.isfinite(r).all()) and float(r.min()) > 0 and float(T.min()) > 0
    assert abs(t1[0] - t0[0]) < 1e-4 * t0[0] and abs(t1[4] - t0[4]) < 1e-4 * t0[4], (t0, t1)


@pytest.mark.parametrize("n_el,p,dt,precision,tol", [((3, 2, 3), 4, 0.45, 0, 1e-12), ((3, 2, 3), 4, 0.45, 1, 1e-5),
                                                    ((6, 6, 5), 4, 0.8, 0, 1e-12), ((4, 2, 3), 1, 0.2, 0, 1e-12),
                                                    ((2, 2, 2), 6, 0.4, 0, 1e-12), ((3, 3, 2), 5, 0.6, 1, 1e-5)])
def test_transposed_stream_is_adjoint(oracle, n_el, p, dt, precision, tol):
    """<S x, y> = <x, S^T y> with the distorted-mesh S (itself checked against
    the oracle above), for orders 1 to 6 (one to seven support points per
    axis); S^T sums its partial sums in a fixed order, so a second
    application gives the same bits."""
    _say(f"distorted S^T adjoint identity n_el={n_el} p={p} precision={precision}")
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, 0.01, precision=precision)
    X, Y, Z = _ref(oracle, cfg0)
    ctx.set_displacement(_smooth_disp(X, Y, Z))
    rng = np.random.default_rng(11)
    N = X.size
    x = to_dev(ctx, rng.normal(size=(Q, N)), rng.normal(size=(Q, N)))
    y = to_dev(ctx, rng.normal(size=(Q, N)), rng.normal(size=(Q, N)))
    sx = ctx.stream(x)
    sty = ctx.stream(y, transpose=True)
    for k in range(2):
        lhs = float((sx[k].double() * y[k].double()).sum())
        rhs = float((x[k].double() * sty[k].double()).sum())
        assert abs(lhs - rhs) <= tol * max(abs(lhs), 1.0) * 10, (k, lhs, rhs)
    again = ctx.stream(y, transpose=True)
    assert torch.equal(again, sty)


def test_adjoint_step_against_complex_step(oracle):
    """One reverse step on a distorted mesh: <lam_out, dX> equals the
    complex-step derivative of <lam, step(X + i h dX)> in the oracle."""
    n_el, p, dt, mu = (2, 2, 2), 3, 0.3, 0.02
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, mu)
    X, Y, Z = _ref(oracle, cfg0)
    disp = _smooth_disp(X, Y, Z, 0.5)
    ctx.set_displacement(disp)
    cfg = oracle.make_cfg(n_el, p, dt, mu, disp=disp)
    f0, g0 = tgv_init(oracle, ctx, cfg, 0.5, 1.4)
    rng = np.random.default_rng(21)
    N = X.size
    f0 = f0 * (1 + 0.02 * rng.normal(size=f0.shape))
    g0 = g0 * (1 + 0.02 * rng.normal(size=g0.shape))
    lam = rng.normal(size=(2, Q, N))
    dX = rng.normal(size=(2, Q, N))
    lam_out = ctx.adjoint_step(to_dev(ctx, f0, g0), to_dev(ctx, lam[0], lam[1]))
    got = float((lam_out.double().cpu().numpy() * dX).sum())
    h = 1e-30
    fc, gc = oracle.step(cfg, f0 + 1j * h * dX[0], g0 + 1j * h * dX[1], 1)
    ref = float((np.sum(lam[0] * fc.imag) + np.sum(lam[1] * gc.imag)) / h)
    assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)


def test_uniform_state_is_fixed(oracle):
    """A uniform equilibrium stays fixed through steps on the distorted mesh."""
    n_el, p, dt = (4, 4, 4), 4, 0.3
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, 0.01)
    X, Y, Z = _ref(oracle, cfg0)
    N = X.size
    ctx.set_displacement(_smooth_disp(X, Y, Z))
    dev = ctx.device
    u = np.tile([[0.2], [-0.1], [0.05]], (1, N))
    ctx.init_equilibrium(torch.full((N,), 1.2, dtype=torch.float64, device=dev), torch.from_numpy(u).to(dev),
                         torch.full((N,), 1.1, dtype=torch.float64, device=dev))
    s0 = ctx.get_state()
    ctx.step(3)
    for k in range(2):
        assert rel_err(to_np(ctx.get_state())[k], to_np(s0)[k]) < 1e-13


@pytest.mark.parametrize("n_el,p,scale", [((3, 2, 3), 3, 1.0), ((2, 2, 2), 4, 0.7), ((2, 3, 1), 2, 1.0)])
def test_loss_diagnostics_and_loss_gradient_match_oracle(oracle, n_el, p, scale):
    """The flow functional, its state gradient and the TGV diagnostics on a
    distorted mesh (derivatives in physical coordinates through each cell's
    map, Jacobian-weighted quadrature) against the oracle, whose
    distorted-mesh loss and diagnostics are pinned by closed forms; the
    gradient along random directions against complex-step derivatives of the
    oracle's loss."""
    _say(f"distorted loss/diagnostics n_el={n_el} p={p}")
    dt, mu = 0.3, 0.02
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, mu)
    X, Y, Z = _ref(oracle, cfg0)
    disp = _smooth_disp(X, Y, Z, scale)
    ctx.set_displacement(disp)
    cfg = oracle.make_cfg(n_el, p, dt, mu, disp=disp)
    f, g = tgv_init(oracle, ctx, cfg, 0.6, 1.4)
    rng = np.random.default_rng(p)
    f = f * (1 + 0.02 * rng.normal(size=f.shape))
    g = g * (1 + 0.02 * rng.normal(size=g.shape))
    st = to_dev(ctx, f, g)
    L = ctx.loss(st)
    assert L == pytest.approx(oracle.loss(cfg, f, g), rel=TOL64)
    d = np.array(ctx.diagnostics(st))
    do = np.array(oracle.diagnostics(cfg, f, g))
    assert np.max(np.abs(d - do) / np.abs(do)) < TOL64, (d, do)
    lam = ctx.loss_grad(st).double().cpu().numpy()
    h = 1e-30
    for k in range(3):
        dX = rng.normal(size=(2, Q, X.size))
        ref = float(oracle.loss(cfg, f + 1j * h * dX[0], g + 1j * h * dX[1]).imag / h)
        got = float(np.sum(lam * dX))
        assert got == pytest.approx(ref, rel=1e-11), (k, got, ref)


def test_rollout_gradient_on_distorted_mesh(oracle):
    """A 3-step rollout on a distorted mesh, differentiated in two mode
    amplitudes and mu_inf through the library's reverse steps (the transposed
    distorted streaming, the collision VJP, the functional's gradient),
    against complex-step derivatives of the oracle rollout."""
    from paper_2012_05537_amd import inputs
    from paper_2012_05537_amd.adjoint import Rollout
    n_el, p, dt, mu = (2, 3, 2), 3, 0.25, 0.02
    ctx, cfg0 = make_pair(oracle, n_el, p, dt, mu)
    X, Y, Z = _ref(oracle, cfg0)
    disp = _smooth_disp(X, Y, Z, 0.6)
    ctx.set_displacement(disp)
    xs, ys, zs = oracle.node_coords(cfg0)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.5, 1.4)
    modes = inputs.fourier_modes(7, 2, 0.5, 1.4, scale=0.05)
    B = inputs.mode_basis(xs, ys, zs, modes)
    amps = np.array([m[3] for m in modes])
    roll = Rollout(ctx, rho, u, T, B, 3, checkpoint=2)
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    m = torch.tensor(mu, dtype=torch.float64, requires_grad=True)
    roll(a, m).backward()
    h = 1e-30

    def cs(da, dmu):
        c = oracle.make_cfg(n_el, p, dt, mu, mu_inf_im=h * dmu, disp=disp)
        uc = u + np.tensordot(amps + 1j * h * da, B, axes=(0, 0))
        fc, gc = oracle.init_equilibrium(c, rho.astype(complex), uc, T.astype(complex))
        fc, gc = oracle.step(c, fc, gc, 3)
        return oracle.loss(c, fc, gc).imag / h

    ref = np.array([cs(np.eye(2)[k], 0.0) for k in range(2)] + [cs(np.zeros(2), 1.0)])
    got = np.concatenate([a.grad.numpy(), [m.grad.item()]])
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-10, (got, ref)
