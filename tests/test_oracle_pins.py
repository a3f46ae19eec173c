"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
Gaussian moments, Maxwellian moments, conservation laws, textbook quadrature
identities, polynomial reproduction, and special cases with a known answer.
"""
import math

import numpy as np
import pytest

Q = 45


def gauss_moment(k):
    """E[Z^k] for a standard normal Z."""
    if k % 2:
        return 0.0
    return float(math.prod(range(k - 1, 0, -2))) if k > 0 else 1.0


def shifted_gauss_moment(k, m, v):
    """E[(m + sqrt(v) Z)^k]."""
    return sum(math.comb(k, j) * m ** (k - j) * v ** (j / 2) * gauss_moment(j) for j in range(k + 1))


# --------------------------------------------------------------------------
# Velocity set (Sec. II B: degree-nine cubature for the Gaussian weight)
# --------------------------------------------------------------------------

def test_velocity_set_is_degree_nine(oracle):
    xi, w = oracle.velocity_set()
    assert xi.shape == (Q, 3)
    worst = 0.0
    for a in range(10):
        for b in range(10 - a):
            for c in range(10 - a - b):
                exact = gauss_moment(a) * gauss_moment(b) * gauss_moment(c)
                q = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                worst = max(worst, abs(q - exact) / max(1.0, abs(exact)))
    assert worst < 1e-13
    # and not degree ten: the rule is exactly degree nine
    q = np.sum(w * xi[:, 0] ** 10)
    assert abs(q - gauss_moment(10)) > 1.0


def test_velocity_set_shells(oracle):
    xi, w = oracle.velocity_set()
    r = np.linalg.norm(xi, axis=1)
    assert abs(w.sum() - 1.0) < 1e-15
    shells = {0.0: (1, 28 / 135), math.sqrt(3): (12, 25 / 432), math.sqrt(15): (12, 1 / 2160), 3.0: (20, 1 / 216)}
    for rad, (count, weight) in shells.items():
        sel = np.abs(r - rad) < 1e-12
        assert sel.sum() == count
        assert np.allclose(w[sel], weight, rtol=0, atol=1e-16)
    # central symmetry: every abscissa has its opposite in the set
    for i in range(Q):
        assert np.min(np.linalg.norm(xi + xi[i], axis=1)) < 1e-12
    assert abs(np.abs(xi).max() - 3.294556414185328) < 1e-12


# --------------------------------------------------------------------------
# Support points, Lagrange basis, node weights (Sec. II A, Eq. (8))
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_lagrange_reproduces_polynomials(oracle, p):
    t = oracle.glc_nodes(p)
    assert t[0] == 0.0 and abs(t[-1] - 1.0) < 1e-15
    assert np.allclose(t + t[::-1], 1.0, atol=1e-15)
    rng = np.random.default_rng(p)
    for s in rng.uniform(-0.3, 1.3, 7):
        ell = oracle.lagrange(p, s)
        dell = oracle.lagrange_deriv(p, s)
        for m in range(p + 1):
            assert abs(np.dot(ell, t ** m) - s ** m) < 1e-12
            assert abs(np.dot(dell, t ** m) - (m * s ** (m - 1) if m else 0.0)) < 1e-10
    # cardinal property at the support points
    for k in range(p + 1):
        assert np.allclose(oracle.lagrange(p, t[k]), np.eye(p + 1)[k], atol=1e-15)


def test_glc_points_order4_values(oracle):
    # t_k = (1 - cos(pi k / 4)) / 2
    t = oracle.glc_nodes(4)
    assert np.allclose(t, [0.0, (1 - math.sqrt(0.5)) / 2, 0.5, (1 + math.sqrt(0.5)) / 2, 1.0], atol=1e-16)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 8])
def test_clenshaw_curtis_weights(oracle, p):
    w = oracle.cc_weights(p)
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    for m in range(p + 1 + (1 - p % 2)):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 1e-13
    table = {2: np.array([1, 4, 1]) / 3, 3: np.array([1, 8, 8, 1]) / 9, 4: np.array([1, 8, 12, 8, 1]) / 15}
    if p in table:
        assert np.allclose(w, table[p], atol=1e-15)


# --------------------------------------------------------------------------
# Equilibrium (Eq. (6), App. A, App. B)
# --------------------------------------------------------------------------

def _random_macro(rng):
    return rng.uniform(0.5, 1.6), rng.normal(0, 0.6, 3), rng.uniform(0.6, 1.5)


def test_equilibrium_matches_maxwellian_moments(oracle):
    """A 4th-order Hermite equilibrium reproduces the Maxwellian's raw moments
    up to order 4 exactly, and the degree-9 rule integrates them exactly."""
    xi, _ = oracle.velocity_set()
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho, u, T = _random_macro(rng)
        feq = oracle.equilibrium(rho, u, T)
        for a in range(5):
            for b in range(5 - a):
                for c in range(5 - a - b):
                    exact = rho * shifted_gauss_moment(a, u[0], T) * shifted_gauss_moment(b, u[1], T) \
                        * shifted_gauss_moment(c, u[2], T)
                    q = np.sum(feq * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                    assert abs(q - exact) < 1e-13 * max(1.0, abs(exact))


def test_equilibrium_scalar_invariant_form(oracle):
    """The tensor contraction equals the closed form in c = xi.u, |u|^2, |xi|^2, T - 1."""
    xi, w = oracle.velocity_set()
    rng = np.random.default_rng(2)
    D = 3
    for _ in range(5):
        rho, u, T = _random_macro(rng)
        c = xi @ u
        u2 = u @ u
        x2 = np.sum(xi * xi, axis=1)
        th = T - 1.0
        bracket = (1 + c + 0.5 * (c * c - u2 + th * (x2 - D))
                   + (c ** 3 - 3 * c * u2 + 3 * th * c * (x2 - D - 2)) / 6
                   + (c ** 4 - 6 * c * c * u2 + 3 * u2 * u2 + 6 * th * (c * c * (x2 - D - 4) - u2 * (x2 - D - 2))
                      + 3 * th * th * (x2 * x2 - 2 * (D + 2) * x2 + D * (D + 2))) / 24)
        assert np.allclose(oracle.equilibrium(rho, u, T), w * rho * bracket, rtol=0, atol=1e-15)


def test_equilibrium_over_mach_number(oracle):
    """Sec. V (equilibrium over Ma_x at rho = theta = 1): the zeroth moment stays 1
    while individual values turn negative beyond Ma = 2."""
    spread = {}
    for ma in np.linspace(0.0, 4.0, 41):
        feq = oracle.equilibrium(1.0, np.array([ma, 0.0, 0.0]), 1.0)
        assert abs(feq.sum() - 1.0) < 1e-12
        spread[round(ma, 1)] = (feq.min(), np.abs(feq).max())
    assert spread[0.0][0] > 0.0 and spread[0.5][0] > 0.0
    # beyond Ma = 2 the values grow in both directions
    assert spread[3.0][0] < -0.5 and spread[4.0][0] < -2.0
    assert spread[4.0][1] > 10 * spread[1.0][1]


def test_centred_third_moment_of_equilibrium_vanishes(oracle):
    xi, _ = oracle.velocity_set()
    rng = np.random.default_rng(3)
    for _ in range(4):
        rho, u, T = _random_macro(rng)
        feq = oracle.equilibrium(rho, u, T)
        d = xi - u
        Qt = np.einsum("i,ia,ib,ic->abc", feq, d, d, d)
        assert np.abs(Qt).max() < 1e-13


def test_init_equilibrium_energy(oracle):
    """g^eq = (2 C_v - D) T f^eq makes 2 rho E = rho |u|^2 + 2 C_v rho T."""
    cfg = oracle.make_cfg(1, 1, 0.1, 0.01, gamma=1.4)
    xi, _ = oracle.velocity_set()
    rng = np.random.default_rng(4)
    rho, u, T = _random_macro(rng)
    f, g = oracle.init_equilibrium(cfg, np.array([rho]), u.reshape(3, 1), np.array([T]))
    Cv = 1 / 0.4
    twoE = np.sum(f[:, 0] * np.sum(xi * xi, axis=1)) + g[:, 0].sum()
    assert abs(twoE - (rho * u @ u + 2 * Cv * rho * T)) < 1e-13
    assert np.allclose(g[:, 0], (2 * Cv - 3) * T * f[:, 0], rtol=1e-15)
    r, uu, TT = oracle.moments(cfg, f, g)
    assert abs(r[0] - rho) < 1e-14 and np.allclose(uu[:, 0], u, atol=1e-14) and abs(TT[0] - T) < 1e-13


# --------------------------------------------------------------------------
# Collision (Eq. (5), App. D)
# --------------------------------------------------------------------------

def _noisy_node(oracle, rng, amp=0.02):
    rho, u, T = _random_macro(rng)
    cfg1 = oracle.make_cfg(1, 1, 0.1, 0.01)
    f, g = oracle.init_equilibrium(cfg1, np.array([rho]), u.reshape(3, 1), np.array([T]))
    _, w = oracle.velocity_set()
    f = f[:, 0] + amp * w * rng.normal(size=Q)
    g = g[:, 0] + amp * w * rng.normal(size=Q)
    return f, g


def _conserved(xi, f, g):
    return np.array([f.sum(), *(xi.T @ f), np.sum(f * np.sum(xi * xi, 1)) + g.sum()])


@pytest.mark.parametrize("law", [0, 1])
def test_collision_conserves_mass_momentum_energy(oracle, law):
    xi, _ = oracle.velocity_set()
    rng = np.random.default_rng(5)
    cfg = oracle.make_cfg(4, 2, 0.05, 0.02, prandtl=0.71, viscosity_law=law)
    for _ in range(6):
        f, g = _noisy_node(oracle, rng)
        fo, go = oracle.collide_node(cfg, f, g)
        assert np.allclose(_conserved(xi, fo, go), _conserved(xi, f, g), rtol=0, atol=2e-14)
        assert np.abs(fo - f).max() > 1e-6          # it did something


def test_collision_fixed_point(oracle):
    rng = np.random.default_rng(6)
    cfg = oracle.make_cfg(4, 2, 0.05, 0.02, prandtl=0.71)
    cfg1 = oracle.make_cfg(1, 1, 0.1, 0.01)
    for _ in range(4):
        rho, u, T = _random_macro(rng)
        f, g = oracle.init_equilibrium(cfg1, np.array([rho]), u.reshape(3, 1), np.array([T]))
        fo, go = oracle.collide_node(cfg, f[:, 0], g[:, 0])
        assert np.allclose(fo, f[:, 0], atol=1e-15) and np.allclose(go, g[:, 0], atol=1e-15)


def test_collision_tau_one_pr_one_gives_equilibrium(oracle):
    """tau = mu/(P dt) + 1/2 = 1 and Pr = 1: the post-collision state is h^eq."""
    rng = np.random.default_rng(7)
    f, g = _noisy_node(oracle, rng, amp=0.05)
    xi, _ = oracle.velocity_set()
    cfg1 = oracle.make_cfg(1, 1, 0.1, 0.01)
    rho, u, T = oracle.moments(cfg1, f.reshape(Q, 1), g.reshape(Q, 1))
    mu = 0.03
    dt = mu / (rho[0] * T[0] * 0.5)
    cfg = oracle.make_cfg(4, 2, dt, mu, prandtl=1.0, viscosity_law=1)
    fo, go = oracle.collide_node(cfg, f, g)
    feq, geq = oracle.init_equilibrium(cfg1, rho, u, T)
    assert np.allclose(fo, feq[:, 0], atol=1e-15) and np.allclose(go, geq[:, 0], atol=1e-15)


def test_collision_relaxation_rates(oracle):
    """Second-order non-equilibrium relaxes with tau; the centred third-order
    non-equilibrium relaxes with tau_Pr = (tau - 1/2)/Pr + 1/2 (App. D, with
    the 1/3! of the third Hermite term)."""
    xi, _ = oracle.velocity_set()
    rng = np.random.default_rng(8)
    cfg1 = oracle.make_cfg(1, 1, 0.1, 0.01)
    for law in (0, 1):
        f, g = _noisy_node(oracle, rng, amp=0.05)
        rho, u, T = oracle.moments(cfg1, f.reshape(Q, 1), g.reshape(Q, 1))
        dt, mu_inf, Pr = 0.04, 0.015, 0.71
        cfg = oracle.make_cfg(4, 2, dt, mu_inf, prandtl=Pr, viscosity_law=law)
        S = 0.40417
        Tn = T[0]
        mu = mu_inf if law == 1 else mu_inf * (1 + S) * Tn ** 1.5 / (Tn + S)
        tau = mu / (rho[0] * Tn * dt) + 0.5
        tau_pr = (tau - 0.5) / Pr + 0.5
        feq, geq = oracle.init_equilibrium(cfg1, rho, u, T)
        feq, geq = feq[:, 0], geq[:, 0]
        fo, go = oracle.collide_node(cfg, f, g)
        d = xi - u[:, 0]
        # second moment of f
        pi_in = np.einsum("i,ia,ib->ab", f - feq, xi, xi)
        pi_out = np.einsum("i,ia,ib->ab", fo - feq, xi, xi)
        assert np.allclose(pi_out, (1 - 1 / tau) * pi_in, atol=1e-14)
        # zeroth moment of g (not conserved on its own)
        assert abs((go - geq).sum() - (1 - 1 / tau) * (g - geq).sum()) < 1e-14
        # centred third moments of f and g
        for h, heq, ho in ((f, feq, fo), (g, geq, go)):
            q_in = np.einsum("i,ia,ib,ic->abc", h - heq, d, d, d)
            q_out = np.einsum("i,ia,ib,ic->abc", ho - heq, d, d, d)
            assert np.allclose(q_out, (1 - 1 / tau_pr) * q_in, atol=1e-13)


def test_sutherland_law(oracle):
    """mu = (1 + S) T^1.5 / (T + S) mu_inf with S = 0.40417 (Sec. III C):
    checked through tau on a node at T != 1."""
    rng = np.random.default_rng(9)
    cfg1 = oracle.make_cfg(1, 1, 0.1, 0.01)
    rho, T = 1.2, 1.3
    f, g = oracle.init_equilibrium(cfg1, np.array([rho]), np.zeros((3, 1)), np.array([T]))
    _, w = oracle.velocity_set()
    f = f[:, 0] + 0.01 * w * rng.normal(size=Q)
    r, u, Tm = oracle.moments(cfg1, f.reshape(Q, 1), g.reshape(Q, 1))
    mu_inf, dt = 0.02, 0.05
    cfg = oracle.make_cfg(4, 2, dt, mu_inf, prandtl=1.0, viscosity_law=0)
    feq, _ = oracle.init_equilibrium(cfg1, r, u, Tm)
    fo, _ = oracle.collide_node(cfg, f, g[:, 0])
    # with Pr = 1: fo - feq = (1 - 1/tau)(f - feq)
    k = np.argmax(np.abs(f - feq[:, 0]))
    tau = 1.0 / (1.0 - (fo[k] - feq[k, 0]) / (f[k] - feq[k, 0]))
    mu = (tau - 0.5) * r[0] * Tm[0] * dt
    S = 0.40417
    assert abs(mu - mu_inf * 1.40417 * Tm[0] ** 1.5 / (Tm[0] + S)) < 1e-12
