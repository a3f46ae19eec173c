"""Pins of the oracle's TGV diagnostics (kinetic energy, solenoidal and
dilatational dissipation of Sec. III C) against closed forms.

Fields that are polynomial of degree <= p inside every cell are represented
exactly by the cell interpolants, and the Clenshaw-Curtis rule integrates
the resulting integrands exactly when their degree is at most p; a
piecewise-linear (triangle-wave) velocity with kinks on cell faces therefore
has closed-form diagnostics.  The populations are the equilibria of the
fields, whose moments reproduce rho, u, T.
"""
import math

import numpy as np
import pytest

SUTH = 0.40417


def _mu(mu_inf, T):
    return mu_inf * (1 + SUTH) * T ** 1.5 / (T + SUTH)


def _fields(oracle, cfg, rho, u, T):
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    return oracle.diagnostics(cfg, f, g)


def _triangle(coord, h, amp):
    """Piecewise-linear periodic wave: +-amp on alternate cell faces."""
    j = np.floor(coord / h + 1e-12).astype(int)
    frac = coord / h - j
    sign = np.where(j % 2 == 0, 1.0, -1.0)
    return amp * sign * (1.0 - 2.0 * frac)


def test_uniform_flow(oracle):
    L = (2.0, 3.0, 1.5)
    cfg = oracle.make_cfg((3, 2, 2), 3, 0.1, 0.02, length=L)
    N = oracle.num_nodes(cfg)
    rho = np.full(N, 1.3)
    uv = np.array([0.2, -0.1, 0.3])
    u = np.tile(uv[:, None], (1, N))
    T = np.full(N, 1.2)
    ek, es, ec = _fields(oracle, cfg, rho, u, T)
    vol = L[0] * L[1] * L[2]
    assert ek == pytest.approx(0.5 * 1.3 * uv @ uv * vol, rel=1e-13)
    assert abs(es) < 1e-25 and abs(ec) < 1e-25


@pytest.mark.parametrize("p", [2, 3, 4])
def test_triangle_shear(oracle, p):
    """u_x(y) triangle wave: curl only, |curl u| = 2A/h_y everywhere."""
    n_el, L, A, mu_inf, T0 = (2, 4, 3), (2.0, 3.0, 1.0), 0.05, 0.013, 1.5
    cfg = oracle.make_cfg(n_el, p, 0.1, mu_inf, length=L)
    xs, ys, zs = oracle.node_coords(cfg)
    Y = np.broadcast_to(ys[None, :, None], (len(zs), len(ys), len(xs))).reshape(-1)
    N = Y.size
    hy = L[1] / n_el[1]
    u = np.zeros((3, N))
    u[0] = _triangle(Y, hy, A)
    ek, es, ec = _fields(oracle, cfg, np.ones(N), u, np.full(N, T0))
    vol = L[0] * L[1] * L[2]
    s = 2 * A / hy
    assert es == pytest.approx(_mu(mu_inf, T0) * s * s * vol, rel=1e-12)
    assert abs(ec) < 1e-12 * es
    assert ek == pytest.approx(0.5 * A * A / 3.0 * vol, rel=1e-12)


@pytest.mark.parametrize("p", [2, 4])
def test_triangle_compression(oracle, p):
    """u_x(x) triangle wave: divergence only."""
    n_el, L, A, mu_inf = (4, 1, 2), (3.0, 1.0, 2.0), 0.07, 0.011
    cfg = oracle.make_cfg(n_el, p, 0.1, mu_inf, length=L, viscosity_law=oracle.CONSTANT)
    xs, ys, zs = oracle.node_coords(cfg)
    X = np.broadcast_to(xs[None, None, :], (len(zs), len(ys), len(xs))).reshape(-1)
    N = X.size
    hx = L[0] / n_el[0]
    u = np.zeros((3, N))
    u[0] = _triangle(X, hx, A)
    ek, es, ec = _fields(oracle, cfg, np.full(N, 1.1), u, np.full(N, 0.8))
    vol = L[0] * L[1] * L[2]
    s = 2 * A / hx
    assert ec == pytest.approx(4.0 / 3.0 * mu_inf * s * s * vol, rel=1e-12)
    assert abs(es) < 1e-12 * ec
    assert ek == pytest.approx(0.5 * 1.1 * A * A / 3.0 * vol, rel=1e-12)


def test_smooth_shear_converges(oracle):
    """u_x = A sin y on [0, 2 pi]^3 with rho = T = 1: E_k = A^2 |S| / 4 and
    eps_s = mu A^2 |S| / 2; at p = 6 the interpolation error is below 1e-5."""
    A, mu_inf = 0.1, 0.02
    cfg = oracle.make_cfg((1, 6, 1), 6, 0.1, mu_inf)
    xs, ys, zs = oracle.node_coords(cfg)
    Y = np.broadcast_to(ys[None, :, None], (len(zs), len(ys), len(xs))).reshape(-1)
    N = Y.size
    u = np.zeros((3, N))
    u[0] = A * np.sin(Y)
    ek, es, ec = _fields(oracle, cfg, np.ones(N), u, np.ones(N))
    vol = (2 * math.pi) ** 3
    assert ek == pytest.approx(A * A * vol / 4, rel=1e-5)
    assert es == pytest.approx(mu_inf * A * A * vol / 2, rel=1e-5)
    assert abs(ec) < 1e-10 * es
