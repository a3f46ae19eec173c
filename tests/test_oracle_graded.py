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


def test_loss_and_diagnostics_refuse_graded(oracle):
    cfg = oracle.make_cfg((2, 1, 1), 2, 0.1, 0.01, widths=[np.array([1.0, 2.0]), None, None])
    N = oracle.num_nodes(cfg)
    f = np.ones((Q, N))
    with pytest.raises(NotImplementedError):
        oracle.loss(cfg, f, f)
    with pytest.raises(NotImplementedError):
        oracle.diagnostics(cfg, f, f)
