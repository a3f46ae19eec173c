"""Pins of the oracle's streaming step and whole-step behaviour (Eqs. (8)-(9))."""
import math

import numpy as np
import pytest

Q = 45


def _grid(oracle, cfg):
    from paper_2012_05537_amd.inputs import mesh
    return mesh(*oracle.node_coords(cfg))


@pytest.mark.parametrize("p,n_el,dt", [(2, (3, 4, 3), 0.31), (3, (3, 3, 4), 0.17), (4, (4, 3, 3), 0.23)])
def test_stream_reproduces_polynomials(oracle, p, n_el, dt):
    """The cell-local tensor Lagrange interpolant reproduces every polynomial of
    degree <= p per axis, evaluated at the departure point x - xi dt.  Only
    nodes whose departure cell does not touch the periodic seam are checked."""
    L = (2.0, 2.5, 3.0)
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, length=L)
    xi, _ = oracle.velocity_set()
    X, Y, Z = _grid(oracle, cfg)
    rng = np.random.default_rng(p)
    cx, cy, cz = rng.normal(size=(3, p + 1))

    def poly(x, y, z):
        return np.polyval(cx, x) * np.polyval(cy, y) * np.polyval(cz, z)

    f = np.tile(poly(X, Y, Z), (Q, 1))
    g = 2.0 * f
    fo, go = oracle.stream(cfg, f, g)
    checked = 0
    for i in range(Q):
        dep = [X - xi[i, 0] * dt, Y - xi[i, 1] * dt, Z - xi[i, 2] * dt]
        ok = np.ones(X.size, bool)
        for a in range(3):
            h = L[a] / n_el[a]
            cell = np.floor(dep[a] / h)
            ok &= (cell >= 0) & (cell <= n_el[a] - 2)
        ref = poly(*dep)
        assert np.allclose(fo[i, ok], ref[ok], rtol=1e-11, atol=1e-11)
        assert np.allclose(go[i, ok], 2 * ref[ok], rtol=1e-11, atol=1e-11)
        checked += ok.sum()
    assert checked > 100


def test_stream_whole_cell_shift_is_permutation(oracle):
    """If xi_i,a dt equals one cell width on every axis, streaming of population i
    is an exact shift of the node grid by p nodes per axis."""
    xi, _ = oracle.velocity_set()
    i = int(np.argmax(np.all(np.abs(xi) > 1.0, axis=1) * np.abs(xi).min(axis=1)))
    dt = 0.1
    n_el, p = (3, 4, 2), 3
    L = tuple(n_el[a] * abs(xi[i, a]) * dt for a in range(3))
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, length=L)
    Nz, Ny, Nx = oracle.grid_shape(cfg)
    rng = np.random.default_rng(11)
    f = rng.normal(size=(Q, Nz * Ny * Nx))
    g = rng.normal(size=(Q, Nz * Ny * Nx))
    fo, go = oracle.stream(cfg, f, g)
    s = [int(np.sign(xi[i, a])) * p for a in range(3)]
    ref = np.roll(f[i].reshape(Nz, Ny, Nx), shift=(s[2], s[1], s[0]), axis=(0, 1, 2)).ravel()
    assert np.allclose(fo[i], ref, atol=1e-12)
    refg = np.roll(g[i].reshape(Nz, Ny, Nx), shift=(s[2], s[1], s[0]), axis=(0, 1, 2)).ravel()
    assert np.allclose(go[i], refg, atol=1e-12)
    # the rest velocity never moves
    assert np.allclose(fo[0], f[0], rtol=0, atol=1e-13)


def test_stream_partition_of_unity(oracle):
    cfg = oracle.make_cfg((2, 3, 2), 4, 0.37, 0.01)
    N = oracle.num_nodes(cfg)
    f = np.full((Q, N), 0.7)
    fo, _ = oracle.stream(cfg, f, f)
    assert np.allclose(fo, 0.7, atol=1e-14)


def test_uniform_flow_stays_uniform(oracle):
    cfg = oracle.make_cfg((2, 2, 3), 3, 0.21, 0.02, prandtl=0.71)
    N = oracle.num_nodes(cfg)
    u = np.array([0.3, -0.2, 0.1])
    f, g = oracle.init_equilibrium(cfg, np.ones(N), np.tile(u[:, None], (1, N)), np.ones(N))
    f2, g2 = oracle.step(cfg, f, g, 3)
    assert np.abs(f2 - f).max() < 1e-13 and np.abs(g2 - g).max() < 1e-13


def test_totals_are_domain_integrals(oracle):
    """Clenshaw-Curtis node weights integrate smooth periodic fields."""
    cfg = oracle.make_cfg((4, 4, 4), 4, 0.1, 0.01)
    from paper_2012_05537_amd.inputs import mesh
    X, Y, Z = mesh(*oracle.node_coords(cfg))
    rho = 1.0 + 0.1 * np.cos(X) * np.cos(Z)
    u = np.stack([0.2 + 0.05 * np.sin(Y), np.zeros_like(X), np.zeros_like(X)])
    T = np.ones_like(X)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    tot = oracle.totals(cfg, f, g)
    V = (2 * math.pi) ** 3
    assert abs(tot[0] - V) < 1e-5 * V
    # rho u_x = 0.2 rho + 0.05 sin(y) rho -> integral 0.2 V
    assert abs(tot[1] - 0.2 * V) < 1e-5 * V
    assert abs(tot[2]) < 1e-10 and abs(tot[3]) < 1e-10
    # rho E = rho |u|^2 / 2 + C_v rho T
    Cv = 2.5
    E_exact = V * (Cv + 0.5 * (0.04 + 0.05 ** 2 / 2))
    assert abs(tot[4] - E_exact) < 1e-4 * E_exact


def test_step_at_nodes_matches_full_step(oracle):
    from paper_2012_05537_amd.inputs import tgv_fields
    cfg = oracle.make_cfg(2, 3, 0.2, 0.01, prandtl=0.71)
    rho, u, T = tgv_fields(*oracle.node_coords(cfg), Ma=0.8, gamma=1.4)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    f1, g1 = oracle.step(cfg, f, g, 1)
    nodes = np.array([0, 5, 77, oracle.num_nodes(cfg) - 1])
    fs, gs = oracle.step_at_nodes(cfg, f, g, nodes)
    assert np.allclose(fs, f1[:, nodes].T, rtol=0, atol=1e-15)
    assert np.allclose(gs, g1[:, nodes].T, rtol=0, atol=1e-15)


@pytest.mark.parametrize("graded", [False, True])
def test_stream_at_nodes_is_the_whole_grid_stream_restricted(oracle, graded):
    """stream_at_nodes (the oracle's plain gather at listed nodes) gives the
    whole-grid stream's values at every node, on a ragged grid with a shift
    of more than a cell, equal or graded cells."""
    n_el, p = (3, 2, 4), 3
    widths = None
    if graded:
        rng = np.random.default_rng(4)
        widths = [w / w.sum() * 2 * np.pi for w in (1 + 0.4 * rng.uniform(-1, 1, n) for n in n_el)]
    cfg = oracle.make_cfg(n_el, p, 1.1, 0.01, widths=widths)
    rng = np.random.default_rng(9)
    N = oracle.num_nodes(cfg)
    f = rng.normal(size=(45, N))
    g = rng.normal(size=(45, N))
    fo, go = oracle.stream(cfg, f, g)
    nodes = np.arange(N)[::-1].copy()
    fs, gs = oracle.stream_at_nodes(cfg, f, g, nodes)
    assert np.array_equal(fs, fo[:, nodes].T) and np.array_equal(gs, go[:, nodes].T)


def test_collide_then_stream_conserves_mass_to_interpolation_accuracy(oracle):
    """Collision conserves exactly; GLC streaming is not exactly conservative but
    its mass error is small for a smooth field."""
    from paper_2012_05537_amd.inputs import tgv_fields
    cfg = oracle.make_cfg(4, 4, 0.08, 0.01, prandtl=0.71)
    rho, u, T = tgv_fields(*oracle.node_coords(cfg), Ma=0.3, gamma=1.4)
    f, g = oracle.init_equilibrium(cfg, rho, u, T)
    t0 = oracle.totals(cfg, f, g)
    f2, g2 = oracle.step(cfg, f, g, 2)
    t2 = oracle.totals(cfg, f2, g2)
    assert abs(t2[0] - t0[0]) / t0[0] < 1e-6
    assert abs(t2[4] - t0[4]) / t0[4] < 1e-6
