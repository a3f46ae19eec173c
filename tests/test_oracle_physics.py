"""Physics pins of the oracle: transport coefficients from the Chapman-Enskog
analysis (App. C) measured on small quasi-1-D grids, and complex-step
derivatives of the whole pipeline against central finite differences.

Transport theory used (linearised compressible Navier-Stokes):
  shear wave u_y = A sin(kx):   decays as exp(-nu k^2 t), nu = mu / rho0;
  acoustic standing wave:       energy decays as exp(-2 Gamma t),
      Gamma = k^2/2 [nu (2 - 1/C_v) + (gamma - 1) nu / Pr_eff]
  (bulk viscosity mu / C_v from the stress tensor of App. C).  At Pr = 1,
  Gamma = nu k^2 for every gamma.  With the quasi-equilibrium term acting on
  the centred third moments of f and of g, the internal-energy flux carried by
  g relaxes with tau, so the conductivity is mu (D+2)/2 / Pr + mu (C_v - D/2)
  and Pr_eff = C_p / ((D+2)/(2 Pr) + C_v - D/2).
"""
import math

import numpy as np
import pytest

from paper_2012_05537_amd.inputs import mesh, tgv_fields, fourier_modes, mode_basis


def _quasi_1d(oracle, n_el, p, dt, mu, gamma=1.4, prandtl=1.0):
    cfg = oracle.make_cfg((n_el, 1, 1), p, dt, mu, gamma=gamma, prandtl=prandtl, viscosity_law=oracle.CONSTANT)
    X, Y, Z = mesh(*oracle.node_coords(cfg))
    return cfg, X


def test_shear_wave_viscosity(oracle):
    nu, n_el, p = 0.02, 8, 4
    dt = (2 * math.pi / (n_el * p)) / math.sqrt(15.0)          # CFL = 1
    cfg, X = _quasi_1d(oracle, n_el, p, dt, nu)
    N = X.size
    u = np.zeros((3, N))
    u[1] = 1e-3 * np.sin(X)
    f, g = oracle.init_equilibrium(cfg, np.ones(N), u, np.ones(N))
    nsteps = int(round(0.25 / nu / dt))

    def amp(f, g):
        _, uu, _ = oracle.moments(cfg, f, g)
        return np.sum(uu[1] * np.sin(X)) / np.sum(np.sin(X) ** 2)

    a0 = amp(f, g)
    f, g = oracle.step(cfg, f, g, nsteps)
    rate = -math.log(amp(f, g) / a0) / (nsteps * dt)
    assert abs(rate / nu - 1.0) < 0.01


def _acoustic_rate(oracle, nu, gamma, prandtl, n_el=8, p=4, steps_per_period=100, periods=2):
    c = math.sqrt(gamma)
    dt = 2 * math.pi / c / steps_per_period
    cfg, X = _quasi_1d(oracle, n_el, p, dt, nu, gamma=gamma, prandtl=prandtl)
    N = X.size
    A = 1e-4
    rho = 1 + A * np.cos(X)
    T = 1 + (gamma - 1) * A * np.cos(X)                    # isentropic perturbation
    f, g = oracle.init_equilibrium(cfg, rho, np.zeros((3, N)), T)

    def energy(f, g):
        r, uu, TT = oracle.moments(cfg, f, g)
        aP = np.sum((r * TT - 1) * np.cos(X)) / np.sum(np.cos(X) ** 2)
        au = np.sum(uu[0] * np.sin(X)) / np.sum(np.sin(X) ** 2)
        return au * au + aP * aP / (c * c)

    e0 = energy(f, g)
    n = periods * steps_per_period
    f, g = oracle.step(cfg, f, g, n)
    return -math.log(energy(f, g) / e0) / (n * dt) / 2


def _gamma_theory(nu, gamma, pr_eff):
    Cv = 1 / (gamma - 1)
    return 0.5 * (nu * (2 - 1 / Cv) + (gamma - 1) * nu / pr_eff)


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_acoustic_damping_unit_prandtl(oracle, gamma):
    nu = 0.02
    rate = _acoustic_rate(oracle, nu, gamma, 1.0)
    assert abs(rate / _gamma_theory(nu, gamma, 1.0) - 1) < 0.01
    assert abs(rate / nu - 1) < 0.01


def test_acoustic_damping_effective_prandtl(oracle):
    nu, gamma, Pr = 0.02, 1.4, 0.71
    Cv = 1 / (gamma - 1)
    pr_eff = (Cv + 1) / (2.5 / Pr + Cv - 1.5)
    rate = _acoustic_rate(oracle, nu, gamma, Pr)
    assert abs(rate / _gamma_theory(nu, gamma, pr_eff) - 1) < 0.005
    assert abs(rate / _gamma_theory(nu, gamma, Pr) - 1) > 0.015


def _pipeline(oracle, cfg, xs, ys, zs, modes, amps, nsteps, Ma=0.5, gamma=1.4):
    rho, u, T = tgv_fields(xs, ys, zs, Ma, gamma)
    B = mode_basis(xs, ys, zs, modes)
    u = u + np.tensordot(amps, B, axes=(0, 0))
    f, g = oracle.init_equilibrium(cfg, rho.astype(u.dtype), u, T.astype(u.dtype))
    f, g = oracle.step(cfg, f, g, nsteps)
    return oracle.loss(cfg, f, g)


def test_complex_step_gradient_matches_central_differences(oracle):
    """Complex-step derivatives of (init -> 3 steps -> loss) with respect to a
    mode amplitude and to mu_inf agree with central differences (h = 1e-6)."""
    dt, mu = 0.3, 0.02
    cfg = oracle.make_cfg(2, 2, dt, mu, prandtl=0.71)
    xs, ys, zs = oracle.node_coords(cfg)
    modes = fourier_modes(7, 2, 0.5, 1.4, scale=0.05)
    amps = np.array([m[3] for m in modes])
    h = 1e-6
    # d/d a_0
    ac = amps.astype(complex)
    ac[0] += 1e-30j
    d_cs = _pipeline(oracle, cfg, xs, ys, zs, modes, ac, 3).imag / 1e-30
    ap, am = amps.copy(), amps.copy()
    ap[0] += h
    am[0] -= h
    d_fd = (_pipeline(oracle, cfg, xs, ys, zs, modes, ap, 3) - _pipeline(oracle, cfg, xs, ys, zs, modes, am, 3)) / (2 * h)
    assert abs(d_cs - d_fd) < 1e-6 * abs(d_cs) + 1e-12
    # d/d mu_inf
    cfg_c = oracle.make_cfg(2, 2, dt, mu, prandtl=0.71, mu_inf_im=1e-30)
    d_cs = _pipeline(oracle, cfg_c, xs, ys, zs, modes, amps.astype(complex), 3).imag / 1e-30
    lp = _pipeline(oracle, oracle.make_cfg(2, 2, dt, mu + h, prandtl=0.71), xs, ys, zs, modes, amps, 3)
    lm = _pipeline(oracle, oracle.make_cfg(2, 2, dt, mu - h, prandtl=0.71), xs, ys, zs, modes, amps, 3)
    d_fd = (lp - lm) / (2 * h)
    assert abs(d_cs - d_fd) < 1e-6 * abs(d_cs) + 1e-12
    assert abs(d_cs) > 1e-8
