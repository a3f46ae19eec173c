"""Pins of the two-dimensional oracle (D2Q19, Sec. II B; Sod shock tube,
Sec. III A), each against something fixed outside the oracle:

* the velocity set integrates every monomial of degree <= 9 exactly against
  the 2-D standard normal (brute force over all monomials), and no rule of
  this size does degree 10;
* the equilibrium reproduces the Maxwellian's moments up to order four
  (Gaussian moments expanded by the binomial theorem);
* the collision conserves mass, momentum and energy, relaxes the stress with
  1 - 1/tau and the centred third moment (heat flux) with 1 - 1/tau_Pr
  (App. D), with tau from the closed-form transport law;
* streaming is exact for fields linear inside every cell and converges as
  h^(p+1) on smooth fields;
* a periodic double shock tube with the paper's coarse setting (h = 0.01,
  p = 4, dt = 5e-4, mu = 2e-4) reproduces the exact Riemann solution.
"""
import math

import numpy as np
import pytest

from riemann_exact import sample as riemann_sample


@pytest.fixture(scope="module")
def O():
    from oracle import oracle2d
    return oracle2d


def _gauss_moment(k):
    """E[Z^k] of the standard normal."""
    if k % 2:
        return 0.0
    return float(np.prod(np.arange(k - 1, 0, -2))) if k else 1.0


def test_velocity_set_is_degree_nine(O):
    xi, w = O.velocity_set()
    assert w.shape == (19,) and np.all(w > 0)
    for deg in range(10):
        for a in range(deg + 1):
            b = deg - a
            q = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b)
            assert q == pytest.approx(_gauss_moment(a) * _gauss_moment(b), abs=1e-12), (a, b)
    # degree ten is not integrated exactly by every monomial
    err10 = max(abs(np.sum(w * xi[:, 0] ** a * xi[:, 1] ** (10 - a)) - _gauss_moment(a) * _gauss_moment(10 - a))
                for a in range(11))
    assert err10 > 1e-3


def test_velocity_set_structure(O):
    xi, w = O.velocity_set()
    r2 = np.sum(xi * xi, axis=1)
    assert np.all(xi[0] == 0)
    shells = [r2[1:7], r2[7:13], r2[13:19]]
    ref = [(48 - 8 * math.sqrt(15)) / 7, 8.0, (48 + 8 * math.sqrt(15)) / 7]
    for s, v in zip(shells, ref):
        assert np.allclose(s, v, rtol=1e-14)
    assert w[0] == pytest.approx(31 / 96, rel=1e-14)
    assert 6 * w[7] == pytest.approx(3 / 64, rel=1e-14)
    # centrally symmetric; the largest speed lies on the x axis
    for i in range(19):
        assert np.min(np.sum(np.abs(xi + xi[i]), axis=1)) < 1e-12
    assert np.max(np.abs(xi[:, 0])) == pytest.approx(math.sqrt(ref[2]), rel=1e-14)
    assert np.max(np.abs(xi[:, 1])) < math.sqrt(ref[2]) * 0.9


def _maxwell_moment(rho, u, T, a, b):
    """rho E[(u_x + sqrt(T) Z_x)^a (u_y + sqrt(T) Z_y)^b]."""
    sx = sum(math.comb(a, k) * u[0] ** (a - k) * T ** (k / 2) * _gauss_moment(k) for k in range(a + 1))
    sy = sum(math.comb(b, k) * u[1] ** (b - k) * T ** (k / 2) * _gauss_moment(k) for k in range(b + 1))
    return rho * sx * sy


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments_to_fourth_order(O, seed):
    rng = np.random.default_rng(seed)
    rho, u, T = rng.uniform(0.5, 2.0), rng.uniform(-0.4, 0.4, 2), rng.uniform(0.8, 1.3)
    feq = O.equilibrium(rho, u, T)
    xi, _ = O.velocity_set()
    for deg in range(5):
        for a in range(deg + 1):
            m = np.sum(feq * xi[:, 0] ** a * xi[:, 1] ** (deg - a))
            assert m == pytest.approx(_maxwell_moment(rho, u, T, a, deg - a), rel=1e-12, abs=1e-12), (a, deg - a)


def test_init_equilibrium_round_trip(O):
    cfg = O.make_cfg((3, 2), 3, 0.01, 1e-3)
    N = O.num_nodes(cfg)
    rng = np.random.default_rng(5)
    rho, u, T = rng.uniform(0.5, 2, N), rng.uniform(-0.3, 0.3, (2, N)), rng.uniform(0.8, 1.4, N)
    f, g = O.init_equilibrium(cfg, rho, u, T)
    r2, u2, T2 = O.moments(cfg, f, g)
    assert np.allclose(r2, rho, rtol=1e-13) and np.allclose(u2, u, atol=1e-13) and np.allclose(T2, T, rtol=1e-13)
    Cv = 1 / 0.4
    assert np.allclose(g.sum(axis=0), (2 * Cv - 2) * T * rho, rtol=1e-13)


def _sutherland(mu_inf, T):
    S = 0.40417
    return mu_inf * (1 + S) * T ** 1.5 / (T + S)


@pytest.mark.parametrize("pr", [0.71, 1.0, 2.5])
def test_collision_relaxation_rates(O, pr):
    """Random non-equilibrium node: invariants kept, stress relaxes with
    1 - 1/tau, centred third moments (heat flux) with 1 - 1/tau_Pr."""
    dt, mu_inf, gamma = 0.002, 3e-3, 1.4
    cfg = O.make_cfg((1, 1), 2, dt, mu_inf, gamma=gamma, prandtl=pr)
    rng = np.random.default_rng(int(pr * 100))
    feq = O.equilibrium(1.1, np.array([0.2, -0.1]), 1.05)
    f = feq * (1 + 0.05 * rng.normal(size=19))
    g = 2.0 * 1.05 * feq * (1 + 0.05 * rng.normal(size=19))
    xi, _ = O.velocity_set()
    fo, go = O.collide_node(cfg, f, g)

    def macro(f, g):
        rho = f.sum()
        u = (f[:, None] * xi).sum(0) / rho
        twoE = np.sum(f * np.sum(xi * xi, 1) + g)
        T = (twoE / rho - u @ u) / (2 / (gamma - 1))
        return rho, u, T, twoE

    rho, u, T, twoE = macro(f, g)
    rho2, u2, T2, twoE2 = macro(fo, go)
    assert rho2 == pytest.approx(rho, rel=1e-14)
    assert np.allclose(u2, u, atol=1e-14) and twoE2 == pytest.approx(twoE, rel=1e-14)
    tau = _sutherland(mu_inf, T) / (rho * T * dt) + 0.5
    tau_pr = (tau - 0.5) / pr + 0.5
    c = xi - u
    C2 = lambda h: np.einsum("i,ia,ib->ab", h, c, c)
    C3 = lambda h: np.einsum("i,ia,ib,ic->abc", h, c, c, c)
    eq2 = rho * T * np.eye(2)
    assert np.allclose(C2(fo) - eq2, (1 - 1 / tau) * (C2(f) - eq2), atol=1e-13)
    assert np.allclose(C3(fo), (1 - 1 / tau_pr) * C3(f), atol=1e-13)
    geq_mass = (2 / (gamma - 1) - 2) * T * rho
    assert go.sum() - geq_mass == pytest.approx((1 - 1 / tau) * (g.sum() - geq_mass), abs=1e-13)
    assert np.allclose(C3(go), (1 - 1 / tau_pr) * C3(g), atol=1e-13)


def _pw_linear(x, faces, vals):
    L = faces[-1]
    xw = np.mod(x, L)
    e = np.clip(np.searchsorted(faces, xw, side="right") - 1, 0, len(faces) - 2)
    t = (xw - faces[e]) / (faces[e + 1] - faces[e])
    v1 = np.append(vals, vals[0])
    return v1[e] * (1 - t) + v1[e + 1] * t


@pytest.mark.parametrize("p,dt", [(2, 0.013), (3, 0.09), (4, 0.21)])
def test_piecewise_linear_field_streams_exactly(O, p, dt):
    """Fields linear inside every cell: every departure value is exact,
    for shifts of several cells across the periodic wrap."""
    n_el, length = (5, 4), (1.0, 0.8)
    cfg = O.make_cfg(n_el, p, dt, 1e-3, length=length)
    faces = [np.linspace(0, L, n + 1) for n, L in zip(n_el, length)]
    rng = np.random.default_rng(p)
    vals = [rng.uniform(0.5, 1.5, n) for n in n_el]
    x, y = O.node_coords(cfg)
    Y, X = (v.reshape(-1) for v in np.meshgrid(y, x, indexing="ij"))
    phi = lambda X, Y: _pw_linear(X, faces[0], vals[0]) * _pw_linear(Y, faces[1], vals[1])
    f = np.tile(phi(X, Y), (19, 1))
    fo, go = O.stream(cfg, f, 2 * f)
    xi, _ = O.velocity_set()
    for i in range(19):
        ref = phi(X - xi[i, 0] * dt, Y - xi[i, 1] * dt)
        assert np.max(np.abs(fo[i] - ref)) < 1e-12, i
        assert np.max(np.abs(go[i] - 2 * ref)) < 1e-12, i


@pytest.mark.parametrize("p", [2, 3])
def test_smooth_field_error_order(O, p):
    L = 1.0
    errs = []
    for n in (12, 24):
        dt = 0.3 * L / n                 # the same departure points in cell units on both meshes
        cfg = O.make_cfg((n, n), p, dt, 1e-3, length=L)
        x, y = O.node_coords(cfg)
        Y, X = (v.reshape(-1) for v in np.meshgrid(y, x, indexing="ij"))
        fun = lambda X, Y: np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        f = np.tile(fun(X, Y), (19, 1))
        fo, _ = O.stream(cfg, f, f)
        xi, _ = O.velocity_set()
        errs.append(max(np.max(np.abs(fo[i] - fun(X - xi[i, 0] * dt, Y - xi[i, 1] * dt))) for i in range(19)))
    ratio = errs[0] / errs[1]
    assert 0.85 * 2 ** (p + 1) < ratio < 1.15 * 2 ** (p + 1), (errs, ratio)


def test_totals_of_piecewise_linear_density(O):
    n_el, p, length = (4, 3), 3, (2.0, 1.5)
    cfg = O.make_cfg(n_el, p, 0.01, 1e-3, length=length)
    faces = [np.linspace(0, L, n + 1) for n, L in zip(n_el, length)]
    rng = np.random.default_rng(11)
    vals = [rng.uniform(0.5, 1.5, n) for n in n_el]
    x, y = O.node_coords(cfg)
    Y, X = (v.reshape(-1) for v in np.meshgrid(y, x, indexing="ij"))
    rho = _pw_linear(X, faces[0], vals[0]) * _pw_linear(Y, faces[1], vals[1])
    N = rho.size
    T0, U = 1.2, np.array([0.1, -0.2])
    f, g = O.init_equilibrium(cfg, rho, np.tile(U[:, None], (1, N)), np.full(N, T0))
    tot = O.totals(cfg, f, g)
    integ = [np.sum(0.5 * (v + np.roll(v, -1)) * (L / len(v))) for v, L in zip(vals, length)]
    mass = integ[0] * integ[1]
    assert tot[0] == pytest.approx(mass, rel=1e-12)
    assert tot[1:3] == pytest.approx(mass * U, rel=1e-12)
    assert tot[3] == pytest.approx(mass * (0.5 * U @ U + T0 / 0.4), rel=1e-12)


def test_uniform_state_is_a_fixed_point(O):
    cfg = O.make_cfg((3, 3), 3, 0.02, 2e-3)
    N = O.num_nodes(cfg)
    f, g = O.init_equilibrium(cfg, np.full(N, 1.3), np.tile([[0.3], [-0.2]], (1, N)), np.full(N, 1.1))
    f2, g2 = O.step(cfg, f, g, 3)
    assert np.max(np.abs(f2 - f)) < 1e-14 and np.max(np.abs(g2 - g)) < 1e-13


def sod_setup(O, n_cells=200, p=4, dt=5e-4, mu=2e-4, gamma=1.4):
    """Periodic double shock tube on [0, 2]: the high state (rho 8, P 10) on
    (0.5, 1.5), the low state (1, 1) outside; one cell across y.  Each
    discontinuity is the paper's tube until the waves meet (t > 0.2)."""
    L = 2.0
    h = L / n_cells
    cfg = O.make_cfg((n_cells, 1), p, dt, mu, gamma=gamma, length=(L, h), viscosity_law=O.CONSTANT)
    x, y = O.node_coords(cfg)
    X = np.tile(x, len(y))
    hi = (X > 0.5) & (X < 1.5)
    rho = np.where(hi, 8.0, 1.0)
    P = np.where(hi, 10.0, 1.0)
    f, g = O.init_equilibrium(cfg, rho, np.zeros((2, X.size)), P / rho)
    return cfg, x, f, g


def test_sod_shock_tube_matches_exact_solution(O):
    """Sec. III A, coarse setting: h = 0.01 at p = 4, dt = 5e-4, mu = 2e-4,
    t = 0.1 (200 steps).  Density within 0.5 % (L1, relative) of the exact
    inviscid solution; velocity within 0.01 mean absolute error."""
    cfg, x, f, g = sod_setup(O)
    f, g = O.step(cfg, f, g, 200)
    rho, u, T = O.moments(cfg, f, g)
    nx = len(x)
    assert np.max(np.abs(rho.reshape(-1, nx) - rho[:nx])) < 1e-11      # uniform across y
    t = 200 * 5e-4
    right = x > 1.0
    re, ue, pe = riemann_sample((8.0, 0.0, 10.0), (1.0, 0.0, 1.0), 1.4, (x[right] - 1.5) / t)
    r = rho[:nx][right]
    assert np.sum(np.abs(r - re)) / np.sum(re) < 5e-3
    assert np.mean(np.abs(u[0, :nx][right] - ue)) < 1e-2
    # the two tubes mirror each other about x = 1
    left = x < 1.0
    xl = x[left]
    rl = np.interp(2.0 - xl, x, rho[:nx])
    assert np.max(np.abs(rl - rho[:nx][left])) < 1e-6 * 8


def test_shear_wave_decay_gives_the_viscosity(O):
    """A transverse wave u_y = U sin(k x) at uniform density and temperature
    decays as exp(-nu k^2 t), nu = mu / rho (Chapman-Enskog limit of the
    relaxation time tau = mu/(P dt) + 1/2).  Measured from the amplitude of
    the resolved mode over 50 steps at tau = 1, after 10 steps in which the
    stress relaxes from the equilibrium start: within 0.5 % (measured 0.013 %)."""
    n, p, L, dt = 16, 4, 1.0, 4e-3
    rho0, T0, U, mu = 1.0, 1.0, 1e-3, 2e-3
    cfg = O.make_cfg((n, 1), p, dt, mu, length=(L, L / n), viscosity_law=O.CONSTANT)
    x, y = O.node_coords(cfg)
    X = np.tile(x, len(y))
    N = X.size
    k = 2 * np.pi / L
    u = np.zeros((2, N))
    u[1] = U * np.sin(k * X)
    f, g = O.init_equilibrium(cfg, np.full(N, rho0), u, np.full(N, T0))
    f, g = O.step(cfg, f, g, 10)
    amp = []
    steps = 50
    for s in range(2):
        if s:
            f, g = O.step(cfg, f, g, steps)
        _, uu, _ = O.moments(cfg, f, g)
        amp.append(np.mean(uu[1] * np.sin(k * X)) / np.mean(np.sin(k * X) ** 2))
    nu_measured = -np.log(amp[1] / amp[0]) / (k * k * steps * dt)
    assert nu_measured == pytest.approx(mu / rho0, rel=0.005), nu_measured


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_standing_sound_wave_gives_the_adiabatic_sound_speed(O, gamma):
    """A density wave rho = 1 + eps sin(k x) at rest and uniform T: its
    pressure mode (the entropy part of the initial state carries none)
    oscillates as cos(c k t) with the adiabatic sound speed c = sqrt(gamma T)
    (D = 2, g^eq = (2 C_v - 2) T f^eq); the first zero crossing of the
    pressure amplitude, interpolated step by step, lies at a quarter period
    within 0.5 % (the damping delays the crossing by a relative amount that
    grows linearly with mu: 0.18 % at mu = 5e-4, 0.7 % at 2e-3)."""
    n, p, L, dt, mu = 16, 4, 1.0, 2e-3, 5e-4
    cfg = O.make_cfg((n, 1), p, dt, mu, gamma=gamma, length=(L, L / n), viscosity_law=O.CONSTANT)
    x, y = O.node_coords(cfg)
    X = np.tile(x, len(y))
    N = X.size
    k = 2 * np.pi / L
    eps = 1e-4
    f, g = O.init_equilibrium(cfg, 1.0 + eps * np.sin(k * X), np.zeros((2, N)), np.ones(N))
    s = np.sin(k * X)

    def pressure_amp(f, g):
        rho, _, T = O.moments(cfg, f, g)
        return np.mean((rho * T - 1.0) * s) / np.mean(s * s)

    amp = [pressure_amp(f, g)]
    for _ in range(150):
        f, g = O.step(cfg, f, g, 1)
        amp.append(pressure_amp(f, g))
    amp = np.array(amp)
    j = int(np.argmax(amp < 0))
    assert j > 0
    t0 = dt * (j - 1 + amp[j - 1] / (amp[j - 1] - amp[j]))
    c = np.pi / (2 * k * t0)
    assert c == pytest.approx(math.sqrt(gamma), rel=5e-3), c
