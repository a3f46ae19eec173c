"""Pins of the oracle on graded meshes: periodic, axis-aligned cells of
unequal width.  Departure points are traced through the neighbouring cells
(Sec. II A); with unequal cells the per-cell interpolation matrices are no
longer shared, the case the paper singles out as memory-bound (subsection
"Numerical efficiency").

* Equal widths given as a graded mesh reproduce the equal-cell oracle.
* A field that is linear inside every cell (continuous, kinks on the cell
  faces) is reproduced exactly by every cell's interpolant, so one streaming
  step must return the field at the exact departure points, whichever cell
  they fall in (shifts of several cells, across the periodic wrap).
* Integrals of such fields are exact under the per-cell Clenshaw-Curtis rule.
* On a smooth field the streaming error falls as h^(p+1) under refinement
  with the same grading.
"""
import math

import numpy as np
import pytest

Q = 45


def _graded_widths(n, length, seed, amp=0.45):
    rng = np.random.default_rng(seed)
    w = 1.0 + amp * rng.uniform(-1.0, 1.0, n)
    return w * (length / w.sum())


def _pw_linear(x, faces, vals):
    """Periodic function linear between faces, value vals[e] at faces[e]."""
    L = faces[-1]
    xw = np.mod(x, L)
    e = np.clip(np.searchsorted(faces, xw, side="right") - 1, 0, len(faces) - 2)
    t = (xw - faces[e]) / (faces[e + 1] - faces[e])
    v1 = np.append(vals, vals[0])
    return v1[e] * (1 - t) + v1[e + 1] * t


def _field_state(oracle, cfg, fun):
    xs, ys, zs = oracle.node_coords(cfg)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    phi = fun(X.reshape(-1), Y.reshape(-1), Z.reshape(-1))
    f = np.tile(phi, (Q, 1))
    return f, 0.5 * f


def test_equal_widths_match_equal_cells(oracle):
    n_el, p, dt = (3, 2, 4), 3, 0.37
    L = 2 * math.pi
    cu = oracle.make_cfg(n_el, p, dt, 0.01)
    cg = oracle.make_cfg(n_el, p, dt, 0.01, widths=[np.full(n, L / n) for n in n_el])
    rng = np.random.default_rng(3)
    N = oracle.num_nodes(cu)
    f, g = rng.normal(size=(Q, N)), rng.normal(size=(Q, N))
    fu, gu = oracle.stream(cu, f, g)
    fg, gg = oracle.stream(cg, f, g)
    assert np.max(np.abs(fg - fu)) < 1e-13 * np.abs(fu).max()
    assert np.max(np.abs(gg - gu)) < 1e-13 * np.abs(gu).max()
    assert np.allclose(oracle.totals(cg, f, g), oracle.totals(cu, f, g), rtol=1e-13, atol=0)


def test_node_coords_on_graded_cells(oracle):
    p = 4
    w = _graded_widths(5, 3.0, 1)
    cfg = oracle.make_cfg((5, 1, 1), p, 0.1, 0.01, widths=[w, None, None], length=(3.0, 1.0, 1.0))
    xs = oracle.node_coords(cfg)[0]
    faces = np.concatenate([[0.0], np.cumsum(w)])
    t = (1 - np.cos(np.pi * np.arange(p) / p)) / 2
    ref = (faces[:-1, None] + w[:, None] * t[None, :]).reshape(-1)
    assert np.max(np.abs(xs - ref)) < 1e-14


@pytest.mark.parametrize("p,dt", [(2, 0.21), (3, 0.9), (4, 1.7)])
def test_piecewise_linear_field_streams_exactly(oracle, p, dt):
    """Graded cells on all three axes, shifts of up to several cells."""
    n_el = (5, 4, 3)
    length = (2 * math.pi, 4.0, 3.0)
    ws = [_graded_widths(n, L, 10 + a) for a, (n, L) in enumerate(zip(n_el, length))]
    faces = [np.concatenate([[0.0], np.cumsum(w)]) for w in ws]
    rng = np.random.default_rng(20 + p)
    vals = [rng.uniform(0.5, 1.5, n) for n in n_el]
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, widths=ws, length=length)

    def phi(x, y, z):
        return (_pw_linear(x, faces[0], vals[0]) * _pw_linear(y, faces[1], vals[1])
                * _pw_linear(z, faces[2], vals[2]))

    f, g = _field_state(oracle, cfg, phi)
    fo, go = oracle.stream(cfg, f, g)
    xi, _ = oracle.velocity_set()
    xs, ys, zs = oracle.node_coords(cfg)
    Z, Y, X = (v.reshape(-1) for v in np.meshgrid(zs, ys, xs, indexing="ij"))
    for i in range(Q):
        ref = phi(X - xi[i, 0] * dt, Y - xi[i, 1] * dt, Z - xi[i, 2] * dt)
        assert np.max(np.abs(fo[i] - ref)) < 1e-12, i
        assert np.max(np.abs(go[i] - 0.5 * ref)) < 1e-12, i


def test_totals_of_piecewise_linear_density(oracle):
    n_el, p = (4, 3, 2), 3
    length = (2.0, 3.0, 1.5)
    ws = [_graded_widths(n, L, 30 + a) for a, (n, L) in enumerate(zip(n_el, length))]
    faces = [np.concatenate([[0.0], np.cumsum(w)]) for w in ws]
    rng = np.random.default_rng(4)
    vals = [rng.uniform(0.5, 1.5, n) for n in n_el]
    cfg = oracle.make_cfg(n_el, p, 0.1, 0.01, widths=ws, length=length)
    xs, ys, zs = oracle.node_coords(cfg)
    Z, Y, X = (v.reshape(-1) for v in np.meshgrid(zs, ys, xs, indexing="ij"))
    rho = (_pw_linear(X, faces[0], vals[0]) * _pw_linear(Y, faces[1], vals[1])
           * _pw_linear(Z, faces[2], vals[2]))
    N = rho.size
    T0 = 1.3
    f, g = oracle.init_equilibrium(cfg, rho, np.zeros((3, N)), np.full(N, T0))
    tot = oracle.totals(cfg, f, g)
    # integral of a periodic piecewise-linear function: sum of trapezoids
    integ = [np.sum(0.5 * (v + np.roll(v, -1)) * w) for v, w in zip(vals, ws)]
    mass = integ[0] * integ[1] * integ[2]
    Cv = 1.0 / 0.4
    assert tot[0] == pytest.approx(mass, rel=1e-12)
    assert np.all(np.abs(tot[1:4]) < 1e-12 * mass)
    assert tot[4] == pytest.approx(Cv * T0 * mass, rel=1e-12)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_smooth_field_error_order(oracle, p):
    """sin along a graded x axis (cell widths 0.6 : 1 : 1.4 repeated, refined
    2x): the error ratio is 2^(p+1) within 15 %."""
    dt = 0.05
    L = 2 * math.pi
    errs = []
    for n in (12, 24):
        base = np.tile([0.6, 1.0, 1.4], n // 3)
        w = base * (L / base.sum())
        cfg = oracle.make_cfg((n, 1, 1), p, dt, 0.01, widths=[w, None, None], length=(L, 1.0, 1.0))
        f, g = _field_state(oracle, cfg, lambda x, y, z: np.sin(x))
        fo, _ = oracle.stream(cfg, f, g)
        xi, _ = oracle.velocity_set()
        xs, ys, zs = oracle.node_coords(cfg)
        X = np.meshgrid(zs, ys, xs, indexing="ij")[2].reshape(-1)
        errs.append(max(np.max(np.abs(fo[i] - np.sin(X - xi[i, 0] * dt))) for i in range(Q)))
    ratio = errs[0] / errs[1]
    assert 0.85 * 2 ** (p + 1) < ratio < 1.15 * 2 ** (p + 1), (errs, ratio)


SUTH = 0.40417


def _mu(mu_inf, T):
    return mu_inf * (1 + SUTH) * T ** 1.5 / (T + SUTH)


def _pw_closed_forms(vals, w):
    """For a periodic piecewise-linear profile: integral of v^2 and of v'^2."""
    v1 = np.roll(vals, -1)
    sq = np.sum(w * (vals * vals + vals * v1 + v1 * v1) / 3.0)
    slope2 = np.sum((v1 - vals) ** 2 / w)
    return sq, slope2


@pytest.mark.parametrize("p", [2, 3])
def test_graded_shear_diagnostics(oracle, p):
    """u_x(y) linear inside every graded y-cell: curl only, each cell with its
    own slope; kinetic energy and solenoidal dissipation in closed form."""
    n_el, L, mu_inf, T0 = (2, 5, 3), (2.0, 3.0, 1.5), 0.013, 1.4
    wy = _graded_widths(5, L[1], 80)
    cfg = oracle.make_cfg(n_el, p, 0.1, mu_inf, length=L, widths=[None, wy, None])
    fy = np.concatenate([[0.0], np.cumsum(wy)])
    vals = np.random.default_rng(81).uniform(-0.1, 0.1, 5)
    xs, ys, zs = oracle.node_coords(cfg)
    Y = np.meshgrid(zs, ys, xs, indexing="ij")[1].reshape(-1)
    N = Y.size
    u = np.zeros((3, N))
    u[0] = _pw_linear(Y, fy, vals)
    f, g = oracle.init_equilibrium(cfg, np.ones(N), u, np.full(N, T0))
    ek, es, ec = oracle.diagnostics(cfg, f, g)
    sq, slope2 = _pw_closed_forms(vals, wy)
    area = L[0] * L[2]
    assert ek == pytest.approx(0.5 * sq * area, rel=1e-12)
    assert es == pytest.approx(_mu(mu_inf, T0) * slope2 * area, rel=1e-12)
    assert abs(ec) < 1e-12 * es


@pytest.mark.parametrize("p", [2, 4])
def test_graded_compression_loss_and_diagnostics(oracle, p):
    """u_x(x) linear inside every graded x-cell: divergence only; the flow
    functional and the dilatational dissipation in closed form."""
    n_el, L, mu_inf, rho0 = (6, 1, 2), (3.0, 1.0, 2.0), 0.011, 1.2
    wx = _graded_widths(6, L[0], 90)
    cfg = oracle.make_cfg(n_el, p, 0.1, mu_inf, length=L, widths=[wx, None, None],
                          viscosity_law=oracle.CONSTANT)
    fx = np.concatenate([[0.0], np.cumsum(wx)])
    vals = np.random.default_rng(91).uniform(-0.1, 0.1, 6)
    xs, ys, zs = oracle.node_coords(cfg)
    X = np.meshgrid(zs, ys, xs, indexing="ij")[2].reshape(-1)
    N = X.size
    u = np.zeros((3, N))
    u[0] = _pw_linear(X, fx, vals)
    f, g = oracle.init_equilibrium(cfg, np.full(N, rho0), u, np.full(N, 0.9))
    sq, slope2 = _pw_closed_forms(vals, wx)
    area = L[1] * L[2]
    ek, es, ec = oracle.diagnostics(cfg, f, g)
    assert ec == pytest.approx(4.0 / 3.0 * mu_inf * slope2 * area, rel=1e-12)
    assert abs(es) < 1e-12 * ec
    assert ek == pytest.approx(0.5 * rho0 * sq * area, rel=1e-12)
    assert oracle.loss(cfg, f, g) == pytest.approx((0.5 * rho0 * sq + slope2) * area, rel=1e-12)
