"""GPU parity of the reverse mode (adjoint step, loss, loss gradient, moment
and initialisation VJPs, checkpointed rollout gradients) against the FP64
oracle's complex-step derivatives.

Complex-step derivatives (step h = 1e-30 on the imaginary axis) carry no
truncation or cancellation error, so the reference Jacobian products are exact
to FP64 rounding; the bar for the FP64 library path is a max-abs error
relative to the largest reference entry of 1e-10 (reverse sweeps accumulate
more rounding than the forward step; 1e-12 is kept for single operators).

Node-local operators (collision, moments, equilibrium initialisation) are
checked element by element: perturbing one population index (or one field) at
every node at once gives every node's Jacobian column in one oracle call.
"""
import math
import sys

import numpy as np
import pytest
import torch

from gpu_common import Q, make_pair, to_np, to_dev, rel_err, require_gpu
from paper_2012_05537_amd import inputs

pytestmark = pytest.mark.gpu

H = 1e-30          # complex step
TOL_OP = 1e-12     # single operators
TOL_SWEEP = 1e-10  # composed reverse sweeps


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _noisy_state(oracle, cfg, Ma, gamma, seed, noise=0.02):
    """TGV equilibrium with a relative multiplicative perturbation (non-zero Qbar^neq)."""
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, Ma, gamma)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    rng = np.random.default_rng(seed)
    f = f * (1.0 + noise * rng.normal(size=f.shape))
    g = g * (1.0 + noise * rng.normal(size=g.shape))
    return f, g


def _collide_vjp_oracle(oracle, cfg, f, g, yf, yg):
    """J_C(X)^T y, node by node, from 90 complex-step collisions."""
    N = f.shape[1]
    lf = np.zeros((Q, N))
    lg = np.zeros((Q, N))
    for pop in range(2):
        for k in range(Q):
            fc = f.astype(np.complex128)
            gc = g.astype(np.complex128)
            (gc if pop else fc)[k] += 1j * H
            cf, cg = oracle.collide(cfg, fc, gc)
            col = (np.sum(yf * cf.imag, axis=0) + np.sum(yg * cg.imag, axis=0)) / H
            (lg if pop else lf)[k] = col
    return lf, lg


def _dmu_oracle(oracle, cfg_args, f, g, yf, yg):
    """d/dmu_inf of <y, C(X)> by a complex step in mu_inf."""
    n_el, p, dt, mu, kw = cfg_args
    cfgc = oracle.make_cfg(n_el, p, dt, mu, mu_inf_im=H, **kw)
    cf, cg = oracle.collide(cfgc, f.astype(np.complex128), g.astype(np.complex128))
    return float((np.sum(yf * cf.imag) + np.sum(yg * cg.imag)) / H)


ADJ_CASES = [
    # n_el, p, dt, mu_inf, Ma, law
    ((4, 4, 4), 2, 0.4, 0.0106, 0.5, 0),
    ((3, 2, 5), 3, 0.2, 0.002, 0.8, 0),
    ((2, 3, 2), 4, 0.1, 0.004, 0.5, 1),
]


@pytest.mark.parametrize("n_el,p,dt,mu,Ma,law", ADJ_CASES)
def test_adjoint_step_collision_vjp_elementwise(oracle, n_el, p, dt, mu, Ma, law):
    """adjoint_step(X, lam) = J_C(X)^T S^T lam, with S^T from the (separately
    pinned) transposed streaming and J_C^T from complex-step columns."""
    _say(f"adjoint_step n_el={n_el} p={p} law={law}")
    ctx, cfg = make_pair(oracle, n_el, p, dt, mu, law=law)
    f, g = _noisy_state(oracle, cfg, Ma, 1.4, seed=p)
    rng = np.random.default_rng(100 + p)
    N = f.shape[1]
    lam_next = to_dev(ctx, rng.normal(size=(Q, N)), rng.normal(size=(Q, N)))
    y = ctx.stream(lam_next, transpose=True)
    yf, yg = to_np(y)
    dmu = torch.zeros(1, dtype=torch.float64, device=ctx.device)
    lam = ctx.adjoint_step(to_dev(ctx, f, g), lam_next, dmu=dmu)
    torch.cuda.synchronize()
    LF, LG = to_np(lam)
    ef, eg = _collide_vjp_oracle(oracle, cfg, f, g, yf, yg)
    assert rel_err(LF, ef) < TOL_OP, rel_err(LF, ef)
    assert rel_err(LG, eg) < TOL_OP, rel_err(LG, eg)
    dmu_ref = _dmu_oracle(oracle, (n_el, p, dt, mu, dict(viscosity_law=law)), f, g, yf, yg)
    assert abs(dmu.item() - dmu_ref) <= TOL_OP * max(abs(dmu_ref), 1e-300) * 10, (dmu.item(), dmu_ref)


@pytest.mark.parametrize("n_el,p", [((5, 3, 3), 2), ((3, 3, 3), 3)])
def test_adjoint_step_fp32_matches_fp64(oracle, n_el, p):
    """FP32-mixed adjoint step against the FP64 one (itself pinned to the
    complex-step oracle above) on the same, FP32-representable inputs: 360
    nodes (the LDS-staged FP32 collision VJP with a ragged last block) and 729
    (not a multiple of 4: the register form).  The FP32 path rounds S^T lam
    and lam to FP32, so the bar is 1e-5 of the largest entry."""
    _say(f"fp32 adjoint step n_el={n_el} p={p}")
    c64, cfg = make_pair(oracle, n_el, p, 0.2, 0.004)
    c32, _ = make_pair(oracle, n_el, p, 0.2, 0.004, precision=1)
    f, g = _noisy_state(oracle, cfg, 0.8, 1.4, seed=7)
    f, g = f.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(8)
    N = f.shape[1]
    lf = rng.normal(size=(Q, N)).astype(np.float32).astype(np.float64)
    lg = rng.normal(size=(Q, N)).astype(np.float32).astype(np.float64)
    out = {}
    for ctx in (c64, c32):
        dmu = torch.zeros(1, dtype=torch.float64, device=ctx.device)
        lam = ctx.adjoint_step(to_dev(ctx, f, g), to_dev(ctx, lf, lg), dmu=dmu)
        torch.cuda.synchronize()
        out[ctx.dtype] = (to_np(lam), dmu.item())
    (F64, G64), d64 = out[torch.float64]
    (F32, G32), d32 = out[torch.float32]
    assert rel_err(F32, F64) < 1e-5 and rel_err(G32, G64) < 1e-5, (rel_err(F32, F64), rel_err(G32, G64))
    assert abs(d32 - d64) <= 1e-5 * abs(d64), (d32, d64)


def test_adjoint_step_accumulates_dmu(oracle):
    """dmu is added to, not overwritten."""
    ctx, cfg = make_pair(oracle, (2, 2, 2), 2, 0.3, 0.01)
    f, g = _noisy_state(oracle, cfg, 0.5, 1.4, seed=7)
    rng = np.random.default_rng(8)
    N = f.shape[1]
    lam_next = to_dev(ctx, rng.normal(size=(Q, N)), rng.normal(size=(Q, N)))
    X = to_dev(ctx, f, g)
    d1 = torch.zeros(1, dtype=torch.float64, device=ctx.device)
    ctx.adjoint_step(X, lam_next, dmu=d1)
    d2 = torch.full((1,), 3.0, dtype=torch.float64, device=ctx.device)
    ctx.adjoint_step(X, lam_next, dmu=d2)
    assert d2.item() == pytest.approx(d1.item() + 3.0, rel=1e-15, abs=1e-15)


def test_full_step_dot_product(oracle):
    """<adjoint_step(X, lam), v> = <lam, d step(X)[v]> for random directions v,
    with d step[v] from a complex-step oracle step (collide then stream)."""
    n_el, p, dt, mu = (4, 4, 4), 2, 0.4, 0.0106
    ctx, cfg = make_pair(oracle, n_el, p, dt, mu)
    f, g = _noisy_state(oracle, cfg, 0.5, 1.4, seed=3)
    rng = np.random.default_rng(4)
    N = f.shape[1]
    lf, lg = rng.normal(size=(Q, N)), rng.normal(size=(Q, N))
    lam = ctx.adjoint_step(to_dev(ctx, f, g), to_dev(ctx, lf, lg))
    LF, LG = to_np(lam)
    for trial in range(3):
        vf, vg = rng.normal(size=(Q, N)), rng.normal(size=(Q, N))
        sf, sg = oracle.step(cfg, f + 1j * H * vf, g + 1j * H * vg, 1)
        ref = (np.sum(lf * sf.imag) + np.sum(lg * sg.imag)) / H
        got = np.sum(LF * vf) + np.sum(LG * vg)
        assert abs(got - ref) <= TOL_OP * np.sum(np.abs(LF * vf) + np.abs(LG * vg)), (trial, got, ref)


LOSS_CASES = [((4, 4, 4), 2, 2 * math.pi), ((3, 2, 4), 3, (2.0, 3.0, 4.5)), ((1, 2, 1), 4, 2 * math.pi)]


@pytest.mark.parametrize("n_el,p,length", LOSS_CASES)
def test_loss_matches_oracle(oracle, n_el, p, length):
    ctx, cfg = make_pair(oracle, n_el, p, 0.1, 0.01, length=length)
    f, g = _noisy_state(oracle, cfg, 0.5, 1.4, seed=11)
    got = ctx.loss(to_dev(ctx, f, g))
    ref = oracle.loss(cfg, f, g)
    assert got == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("n_el,p,length", [((2, 3, 2), 2, 2 * math.pi), ((2, 1, 2), 3, (2.0, 3.0, 4.5))])
def test_loss_grad_elementwise(oracle, n_el, p, length):
    """dL/df_i(n) for every population and node by complex steps of the oracle
    loss; dL/dg is identically zero (L depends on rho and u only)."""
    ctx, cfg = make_pair(oracle, n_el, p, 0.1, 0.01, length=length)
    f, g = _noisy_state(oracle, cfg, 0.5, 1.4, seed=12)
    lam = ctx.loss_grad(to_dev(ctx, f, g))
    LF, LG = to_np(lam)
    N = f.shape[1]
    ref = np.zeros((Q, N))
    gc = g.astype(np.complex128)
    for k in range(Q):
        for n in range(N):
            fc = f.astype(np.complex128)
            fc[k, n] += 1j * H
            ref[k, n] = oracle.loss(cfg, fc, gc).imag / H
    assert rel_err(LF, ref) < TOL_OP, rel_err(LF, ref)
    assert np.all(LG == 0.0)


def test_moments_vjp_elementwise(oracle):
    ctx, cfg = make_pair(oracle, (3, 2, 2), 3, 0.1, 0.01)
    f, g = _noisy_state(oracle, cfg, 0.7, 1.4, seed=13)
    N = f.shape[1]
    rng = np.random.default_rng(14)
    drho, du, dT = rng.normal(size=N), rng.normal(size=(3, N)), rng.normal(size=N)
    ctx.set_state(to_dev(ctx, f, g))
    dev = ctx.device
    lam = ctx.moments_vjp(torch.from_numpy(drho).to(dev), torch.from_numpy(du).to(dev), torch.from_numpy(dT).to(dev))
    LF, LG = to_np(lam)
    ref = [np.zeros((Q, N)), np.zeros((Q, N))]
    for pop in range(2):
        for k in range(Q):
            fc, gc = f.astype(np.complex128), g.astype(np.complex128)
            (gc if pop else fc)[k] += 1j * H
            r, u, T = oracle.moments(cfg, fc, gc)
            ref[pop][k] = (drho * r.imag + np.sum(du * u.imag, axis=0) + dT * T.imag) / H
    assert rel_err(LF, ref[0]) < TOL_OP
    assert rel_err(LG, ref[1]) < TOL_OP
    # NULL adjoints count as zero
    lam_T = ctx.moments_vjp(dT=torch.from_numpy(dT).to(dev))
    lam_all = ctx.moments_vjp(torch.zeros(N, dtype=torch.float64, device=dev),
                              torch.zeros((3, N), dtype=torch.float64, device=dev), torch.from_numpy(dT).to(dev))
    assert torch.equal(lam_T, lam_all)


def test_init_equilibrium_vjp_elementwise(oracle):
    ctx, cfg = make_pair(oracle, (3, 2, 2), 3, 0.1, 0.01, gamma=5.0 / 3.0)
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, 0.9, 5.0 / 3.0)
    N = rho.size
    rng = np.random.default_rng(15)
    lf, lg = rng.normal(size=(Q, N)), rng.normal(size=(Q, N))
    dev = ctx.device
    drho, du, dT = ctx.init_equilibrium_vjp(*(torch.from_numpy(x).to(dev) for x in (rho, u, T)),
                                            to_dev(ctx, lf, lg))

    def probe(r, uu, t):
        fc, gc = oracle.init_equilibrium(cfg, r, uu, t)
        return (np.sum(lf * fc.imag, axis=0) + np.sum(lg * gc.imag, axis=0)) / H

    c = lambda a: a.astype(np.complex128)
    ref_r = probe(c(rho) + 1j * H, c(u), c(T))
    ref_T = probe(c(rho), c(u), c(T) + 1j * H)
    ref_u = []
    for a in range(3):
        uc = c(u)
        uc[a] += 1j * H
        ref_u.append(probe(c(rho), uc, c(T)))
    assert rel_err(drho.cpu().numpy(), ref_r) < TOL_OP
    assert rel_err(dT.cpu().numpy(), ref_T) < TOL_OP
    assert rel_err(du.cpu().numpy(), np.array(ref_u)) < TOL_OP


# ---------------------------------------------------------------------------
# rollout gradients (checkpointed adjoint)
# ---------------------------------------------------------------------------

def _rollout_setup(oracle, name, n_modes=None, precision=None, **override):
    from paper_2012_05537_amd.adjoint import Rollout
    w = inputs.workload(name, **override)
    prec = {"fp64": 0, "fp32": 1}[w["precision"]] if precision is None else precision
    ctx, cfg = make_pair(oracle, w["n_el"], w["p"], w["dt"], w["mu_inf"], gamma=w["gamma"], prandtl=w["Pr"],
                         precision=prec)
    md = w.get("modes") or dict(seed=2012, count=4, scale=0.01)
    modes = inputs.fourier_modes(md["seed"], n_modes or md["count"], w["Ma"], w["gamma"], md["scale"])
    xs, ys, zs = oracle.node_coords(cfg)
    rho, u, T = inputs.tgv_fields(xs, ys, zs, w["Ma"], w["gamma"])
    B = inputs.mode_basis(xs, ys, zs, modes)
    amps = np.array([m[3] for m in modes])
    return w, ctx, cfg, Rollout, (rho, u, T, B, amps)


def _oracle_rollout_directional(oracle, w, cfg_kw, fields, n_steps, da, dmu):
    """d/deps of L(a + eps da, mu + eps dmu) by one complex-step oracle rollout."""
    rho, u, T, B, amps = fields
    cfg = oracle.make_cfg(w["n_el"], w["p"], w["dt"], w["mu_inf"], mu_inf_im=H * dmu, **cfg_kw)
    uc = u + np.tensordot(amps + 1j * H * da, B, axes=(0, 0))
    f, g = oracle.init_equilibrium(cfg, rho.astype(np.complex128), uc, T.astype(np.complex128))
    f, g = oracle.step(cfg, f, g, n_steps)
    L = oracle.loss(cfg, f, g)
    return L.real, L.imag / H


@pytest.mark.parametrize("checkpoint", [1, 3, "sqrt", 10])
def test_rollout_gradient_small(oracle, checkpoint):
    """Gradient of a 10-step rollout on 4^3 cells of order 2 (4 modes and mu_inf)
    against per-parameter complex-step oracle rollouts."""
    _say(f"rollout gradient checkpoint={checkpoint}")
    w, ctx, cfg, Rollout, fields = _rollout_setup(oracle, "c1", n_modes=4)
    rho, u, T, B, amps = fields
    n = 10
    roll = Rollout(ctx, rho, u, T, B, n, checkpoint=checkpoint)
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(w["mu_inf"], dtype=torch.float64, requires_grad=True)
    L = roll(a, mu)
    L.backward()
    kw = dict(gamma=w["gamma"], prandtl=w["Pr"])
    L_ref, _ = _oracle_rollout_directional(oracle, w, kw, fields, n, np.zeros_like(amps), 0.0)
    assert L.item() == pytest.approx(L_ref, rel=1e-12)
    ref = []
    for m in range(len(amps)):
        e = np.zeros_like(amps)
        e[m] = 1.0
        ref.append(_oracle_rollout_directional(oracle, w, kw, fields, n, e, 0.0)[1])
    ref_mu = _oracle_rollout_directional(oracle, w, kw, fields, n, np.zeros_like(amps), 1.0)[1]
    ga = a.grad.numpy()
    assert rel_err(ga, np.array(ref)) < TOL_SWEEP, (ga, ref)
    assert mu.grad.item() == pytest.approx(ref_mu, rel=TOL_SWEEP)


def test_rollout_gradient_checkpoint_invariant(oracle):
    """Replayed segments reproduce the forward states bit for bit, so the
    gradient does not depend on the checkpoint interval."""
    w, ctx, cfg, Rollout, fields = _rollout_setup(oracle, "c1", n_modes=4)
    rho, u, T, B, amps = fields
    grads = []
    for ck in (1, 4, "sqrt", 12):
        roll = Rollout(ctx, rho, u, T, B, 12, checkpoint=ck)
        a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
        mu = torch.tensor(w["mu_inf"], dtype=torch.float64, requires_grad=True)
        roll(a, mu).backward()
        grads.append((a.grad.clone(), mu.grad.clone()))
    for ga, gm in grads[1:]:
        assert torch.equal(ga, grads[0][0]) and torch.equal(gm, grads[0][1])


def test_rollout_zero_steps(oracle):
    """n = 0: the gradient is the loss gradient pulled back through the initialisation."""
    w, ctx, cfg, Rollout, fields = _rollout_setup(oracle, "c1", n_modes=3)
    rho, u, T, B, amps = fields
    roll = Rollout(ctx, rho, u, T, B, 0)
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(w["mu_inf"], dtype=torch.float64, requires_grad=True)
    roll(a, mu).backward()
    kw = dict(gamma=w["gamma"], prandtl=w["Pr"])
    for m in range(len(amps)):
        e = np.zeros_like(amps)
        e[m] = 1.0
        ref = _oracle_rollout_directional(oracle, w, kw, fields, 0, e, 0.0)[1]
        assert a.grad[m].item() == pytest.approx(ref, rel=1e-12)
    assert mu.grad.item() == 0.0


def test_rollout_gradient_c4_directional(oracle):
    """The c4 workload (8^3 cells of order 3, 50 steps, 16 modes, checkpoint
    every 10 steps): grad . v against one complex-step oracle rollout along
    a random direction v in (a, mu_inf)."""
    _say("rollout gradient c4 (50 steps)")
    w, ctx, cfg, Rollout, fields = _rollout_setup(oracle, "c4")
    rho, u, T, B, amps = fields
    n = w["steps"]
    roll = Rollout(ctx, rho, u, T, B, n, checkpoint=w["checkpoint"])
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(w["mu_inf"], dtype=torch.float64, requires_grad=True)
    L = roll(a, mu)
    L.backward()
    rng = np.random.default_rng(2012)
    da = rng.normal(size=amps.size)
    dmu = float(rng.normal()) * w["mu_inf"]
    kw = dict(gamma=w["gamma"], prandtl=w["Pr"])
    L_ref, dref = _oracle_rollout_directional(oracle, w, kw, fields, n, da, dmu)
    got = float(a.grad.numpy() @ da + mu.grad.item() * dmu)
    assert L.item() == pytest.approx(L_ref, rel=1e-11)
    assert got == pytest.approx(dref, rel=TOL_SWEEP)


def test_rollout_gradient_fp32_mixed(oracle):
    """FP32-mixed storage: the gradient of a 10-step rollout agrees with the
    FP64 complex-step reference to the accuracy FP32 states allow (1e-4)."""
    w, ctx, cfg, Rollout, fields = _rollout_setup(oracle, "c1", n_modes=4, precision=1)
    rho, u, T, B, amps = fields
    roll = Rollout(ctx, rho, u, T, B, 10, checkpoint="sqrt")
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(w["mu_inf"], dtype=torch.float64, requires_grad=True)
    roll(a, mu).backward()
    kw = dict(gamma=w["gamma"], prandtl=w["Pr"])
    ref = []
    for m in range(len(amps)):
        e = np.zeros_like(amps)
        e[m] = 1.0
        ref.append(_oracle_rollout_directional(oracle, w, kw, fields, 10, e, 0.0)[1])
    ref_mu = _oracle_rollout_directional(oracle, w, kw, fields, 10, np.zeros_like(amps), 1.0)[1]
    assert rel_err(a.grad.numpy(), np.array(ref)) < 1e-4
    assert mu.grad.item() == pytest.approx(ref_mu, rel=1e-4)


def test_superpose_and_project_match_numpy(oracle):
    """sllbm_superpose and sllbm_project (the rollout's mode algebra) against
    numpy on a ragged grid, with more modes than one projection pass holds;
    the projection is bitwise repeatable."""
    ctx, cfg = make_pair(oracle, (3, 2, 4), 3, 0.2, 0.01)
    rng = np.random.default_rng(3)
    N, M = ctx.nodes, 11
    base = rng.normal(size=(3, N))
    basis = rng.normal(size=(M, 3, N))
    amps = rng.normal(size=M)
    v = rng.normal(size=(3, N))
    dev = dict(dtype=torch.float64, device=ctx.device)
    base_d, basis_d, v_d = (torch.tensor(x, **dev) for x in (base, basis, v))
    out = ctx.superpose(base_d, basis_d, amps).cpu().numpy()
    ref = base + np.tensordot(amps, basis, axes=(0, 0))
    assert np.max(np.abs(out - ref)) < 1e-14 * np.abs(ref).max()
    got = np.array(ctx.project(basis_d, v_d))
    ref_p = basis.reshape(M, -1) @ v.reshape(-1)
    assert np.max(np.abs(got - ref_p)) < 1e-13 * np.abs(ref_p).max()
    assert ctx.project(basis_d, v_d) == list(got)
    assert ctx.project(basis_d[:0], v_d) == []


def test_adjoint_rejects_aliasing(oracle):
    from paper_2012_05537_amd.sllbm import SllbmError
    ctx, cfg = make_pair(oracle, (2, 2, 2), 2, 0.3, 0.01)
    f, g = _noisy_state(oracle, cfg, 0.5, 1.4, seed=1)
    X = to_dev(ctx, f, g)
    lam = torch.ones_like(X)
    with pytest.raises(SllbmError):
        ctx.adjoint_step(X, lam, lam)
    with pytest.raises(SllbmError):
        ctx.adjoint_step(X, lam, X)


def test_rollout_gradient_c4_vs_central_differences(oracle):
    """c4 workload (8^3 cells of order 3, 50 steps, 16 modes, checkpoint every
    10): the gradient in all 17 parameters (16 amplitudes and mu_inf) against
    per-component central differences of the GPU forward rollout with step
    h = 1e-6 in each parameter; bar 1e-6 in max |g - g_fd| / max |g_fd|
    (truncation O(h^2); rounding of the two rollouts about 1e-16 |L| / h)."""
    w, ctx, cfg, Rollout, fields = _rollout_setup(oracle, "c4")
    rho, u, T, B, amps = fields
    n = w["steps"]
    roll = Rollout(ctx, rho, u, T, B, n, checkpoint=w["checkpoint"])
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(w["mu_inf"], dtype=torch.float64, requires_grad=True)
    roll(a, mu).backward()
    grad = np.concatenate([a.grad.numpy(), [mu.grad.item()]])
    params = np.concatenate([amps, [w["mu_inf"]]])
    h = 1e-6
    f64 = dict(dtype=torch.float64)
    fd = np.empty_like(params)
    with torch.no_grad():
        for k in range(params.size):
            e = np.zeros_like(params)
            e[k] = h
            lp = roll(torch.tensor((params + e)[:-1], **f64), torch.tensor((params + e)[-1], **f64)).item()
            lm = roll(torch.tensor((params - e)[:-1], **f64), torch.tensor((params - e)[-1], **f64)).item()
            fd[k] = (lp - lm) / (2 * h)
    err = np.abs(grad - fd).max() / np.abs(fd).max()
    _say(f"c4 gradient vs per-component central differences (h = 1e-6): max rel error {err:.2e}, "
         f"|g|max {np.abs(fd).max():.3e}")
    assert err < 1e-6


def test_fp32_adjoint_vs_fp64_subcase(oracle):
    """The 256^3-node FP32 workload's parameters (Ma 1.25, Re 1600, CFL 10,
    16 modes seed 2021, sqrt(n) checkpoints) on its 16^3-cell subcase (64^3
    nodes) for 6 steps: the FP32-mixed gradient against the FP64 gradient."""
    grads = {}
    for prec in (0, 1):
        w, ctx, cfg, Rollout, fields = _rollout_setup(oracle, "c5", precision=prec, n_el=16)
        rho, u, T, B, amps = fields
        roll = Rollout(ctx, rho, u, T, B, 6, checkpoint="sqrt")
        a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
        mu = torch.tensor(w["mu_inf"], dtype=torch.float64, requires_grad=True)
        roll(a, mu).backward()
        grads[prec] = np.concatenate([a.grad.numpy(), [mu.grad.item()]])
        ctx.close()
    err = np.max(np.abs(grads[1] - grads[0])) / np.max(np.abs(grads[0]))
    _say(f"c5 subcase: FP32-mixed vs FP64 gradient, max rel error {err:.2e}")
    assert err < 1e-3
