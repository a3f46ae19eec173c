"""Seeded synthetic inputs: compressible Taylor-Green-vortex fields and the
workload table.

This module holds input recipes only (closed-form initial fields, random
perturbation modes, the conversion of Mach/Reynolds/CFL numbers into the
time step and viscosity of a run).  It contains none of the method's own
arithmetic, and it is the only code shared by the GPU path and the oracle.

Units are lattice units: c_s = 1, T0 = 1, rho0 = 1, domain [0, 2 pi]^3.
Initial condition (Sec. III C, constant-temperature initial condition):
    u = U (sin x cos y cos z, -cos x sin y cos z, 0)
    P = rho0 T0 + rho0 U^2 / 16 (cos 2x + cos 2y)(cos 2z + 2),  rho = P / T0,  T = T0
with U = Ma * sqrt(gamma T0), which reproduces the paper's rho = 1 + C/16(...)
with C = gamma Ma^2 (its Re = 1600 choice; tgv_fields also takes the C = 1 of
its Re = 100 and 400 runs).  mu_inf = rho0 U L / Re with L = 1, and
dt = CFL * (mean node spacing) / (largest abscissa speed).
"""
import math

import numpy as np

# Largest speed |xi| of the 45-velocity set (outer icosahedron shell), used
# only to turn a CFL number into a time step.
MAX_SPEED = math.sqrt(15.0)

T0 = 1.0
RHO0 = 1.0

# The five workloads the implementation is measured and checked on.
WORKLOADS = {
    "c1": dict(n_el=4, p=2, Ma=0.5, Re=100.0, gamma=1.4, Pr=0.71, cfl=2.0, steps=10,
               precision="fp64", modes=None),
    "c2": dict(n_el=16, p=4, Ma=1.25, Re=1600.0, gamma=1.4, Pr=0.71, cfl=1.0, steps=200,
               precision="fp64", modes=None),
    "c3": dict(n_el=32, p=4, Ma=1.25, Re=1600.0, gamma=1.4, Pr=0.71, cfl=5.0, steps=500,
               precision="fp32", modes=None),
    "c4": dict(n_el=8, p=3, Ma=0.5, Re=400.0, gamma=1.4, Pr=0.71, cfl=2.0, steps=50,
               precision="fp64", modes=dict(seed=2012, count=16, scale=0.01), checkpoint=10),
    "c5": dict(n_el=64, p=4, Ma=1.25, Re=1600.0, gamma=1.4, Pr=0.71, cfl=10.0, steps=200,
               precision="fp32", modes=dict(seed=2021, count=16, scale=0.01), checkpoint="sqrt"),
}


# Graded-mesh variant of the 64^3-node workload: the cells of every axis are
# stretched by a cosine profile (largest / smallest width close to
# (1 + a)/(1 - a) = 1.86 at a = 0.3), finest near the domain faces,
# coarsest in the middle.
GRADED = dict(base="c2", amplitude=0.3)


def graded_widths(n, length=2 * math.pi, amplitude=0.3):
    """n cell widths w_e proportional to 1 - a cos(2 pi (e + 1/2) / n), summing to length."""
    e = np.arange(n)
    w = 1.0 - amplitude * np.cos(2 * math.pi * (e + 0.5) / n)
    return w * (length / w.sum())


# Distorted-mesh variant of the 64^3-node workload: the equal-cell GLC nodes
# displaced by a smooth periodic field of amplitude a times the cell width,
# d = a h (sin(y + z), sin(z + x), sin(x + y)); |grad d| <= sqrt(2) a h keeps
# every cell map orientation-preserving for the a used here.
DISTORTED = dict(base="c2", amplitude=0.25)


def distortion(X, Y, Z, h, amplitude=0.25):
    """(3, N) node displacements of the distorted workload at reference coordinates X, Y, Z."""
    return amplitude * h * np.stack([np.sin(Y + Z), np.sin(Z + X), np.sin(X + Y)])


def velocity_scale(Ma, gamma):
    """U = Ma * adiabatic sound speed sqrt(gamma T0)."""
    return Ma * math.sqrt(gamma * T0)


def run_parameters(n_el, p, Ma, Re, gamma, cfl, length=2 * math.pi):
    """(dt, mu_inf) of a run: dt from the CFL number, mu_inf from Re = rho0 U L / mu_inf (L = 1)."""
    U = velocity_scale(Ma, gamma)
    mu_inf = RHO0 * U * 1.0 / Re
    dx = length / (n_el * p)
    dt = cfl * dx / MAX_SPEED
    return dt, mu_inf


def workload(name, **override):
    """Workload dict with derived dt, mu_inf and U filled in."""
    w = dict(WORKLOADS[name])
    w.update(override)
    dt, mu_inf = run_parameters(w["n_el"], w["p"], w["Ma"], w["Re"], w["gamma"], w["cfl"])
    w["dt"] = dt
    w["mu_inf"] = mu_inf
    w["U"] = velocity_scale(w["Ma"], w["gamma"])
    w["name"] = name
    return w


def mesh(xs, ys, zs):
    """3-D coordinate arrays (flattened, x fastest) from the 1-D node coordinates."""
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def tgv_fields(xs, ys, zs, Ma, gamma, numerator=None):
    """rho (N,), u (3, N), T (N,) of the compressible Taylor-Green vortex.

    numerator: the paper's C in rho = 1 + C/16 (cos 2x + cos 2y)(cos 2z + 2)
    (Sec. III C); None gives C = gamma Ma^2, the closed-form TGV pressure
    rho0 U^2/16 (...) at uniform T0 (the paper's choice at Re = 1600); the
    paper uses C = 1 at Re = 100 and 400."""
    X, Y, Z = mesh(xs, ys, zs)
    U = velocity_scale(Ma, gamma)
    u = np.stack([U * np.sin(X) * np.cos(Y) * np.cos(Z),
                  -U * np.cos(X) * np.sin(Y) * np.cos(Z),
                  np.zeros_like(X)])
    shape = (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    if numerator is None:
        rho = (RHO0 * T0 + RHO0 * U * U / 16.0 * shape) / T0
    else:
        rho = RHO0 * (1.0 + float(numerator) / 16.0 * shape)
    T = np.full_like(X, T0)
    return rho, u, T


# The paper's own Taylor-Green runs (Sec. III C), in its units: velocity
# amplitude 1, wavenumber-1 length, Re = 1/nu_inf, time step dt_paper in the
# convective time L/U.  256^3 nodes (64^3 cells of p = 4), Pr = 0.7.  The
# final times of the Re = 400 and Re = 100 runs are not in the text (their
# figures are); t = 10 stands in.
PAPER_TGV = {
    "re1600_ma125": dict(Re=1600.0, Ma=1.25, dt_paper=0.009, t_end=20.0, numerator=None),
    "re1600_ma100": dict(Re=1600.0, Ma=1.0, dt_paper=0.010, t_end=20.0, numerator=None),
    "re400_ma050": dict(Re=400.0, Ma=0.5, dt_paper=0.017, t_end=10.0, numerator=1.0),
    "re400_ma100": dict(Re=400.0, Ma=1.0, dt_paper=0.033, t_end=10.0, numerator=1.0),
    "re400_ma150": dict(Re=400.0, Ma=1.5, dt_paper=0.018, t_end=10.0, numerator=1.0),
    "re400_ma200": dict(Re=400.0, Ma=2.0, dt_paper=0.012, t_end=10.0, numerator=1.0),
    "re100_ma250": dict(Re=100.0, Ma=2.5, dt_paper=0.015, t_end=10.0, numerator=1.0),
    "re100_ma300": dict(Re=100.0, Ma=3.0, dt_paper=0.030, t_end=10.0, numerator=1.0),
}
PAPER_TGV_GRID = dict(n_el=64, p=4, gamma=1.4, Pr=0.7)


def paper_tgv(case, **override):
    """Parameters of one of the paper's TGV runs in lattice units.

    The paper's time unit is L/U; with U = Ma sqrt(gamma T0) in lattice units
    (c_s = 1, T0 = 1, L = 1) its time t_paper equals U t, so
    dt = dt_paper / U, mu_inf = rho0 U / Re, and t_end / dt_paper steps."""
    w = dict(PAPER_TGV_GRID)
    w.update(PAPER_TGV[case])
    w.update(override)
    U = velocity_scale(w["Ma"], w["gamma"])
    w["U"] = U
    w["dt"] = w["dt_paper"] / U
    w["mu_inf"] = RHO0 * U / w["Re"]
    w["steps"] = int(round(w["t_end"] / w["dt_paper"]))
    w["cfl"] = MAX_SPEED * w["dt"] / (2 * math.pi / (w["n_el"] * w["p"]))
    w["name"] = case
    return w


def fourier_modes(seed, count, Ma, gamma, scale=0.01, kmax=2):
    """Seeded divergence-free perturbation modes: list of (k, e, phase, amplitude).

    k in {-kmax..kmax}^3 without 0, e a random unit vector orthogonal to k,
    phase uniform in [0, 2 pi), amplitude ~ N(0, (scale * U)^2)."""
    rng = np.random.default_rng(seed)
    U = velocity_scale(Ma, gamma)
    modes = []
    while len(modes) < count:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if not k.any():
            continue
        v = rng.normal(size=3)
        kk = k / np.linalg.norm(k)
        e = v - (v @ kk) * kk
        e /= np.linalg.norm(e)
        phase = rng.uniform(0.0, 2 * math.pi)
        amp = rng.normal(0.0, scale * U)
        modes.append((k.astype(float), e, phase, amp))
    return modes


def mode_basis(xs, ys, zs, modes):
    """B (M, 3, N): velocity field of each mode at unit amplitude, e_m sin(k_m . x + phase_m)."""
    X, Y, Z = mesh(xs, ys, zs)
    out = np.zeros((len(modes), 3, X.size))
    for m, (k, e, ph, _) in enumerate(modes):
        s = np.sin(k[0] * X + k[1] * Y + k[2] * Z + ph)
        out[m] = e[:, None] * s[None, :]
    return out


def perturbed_tgv(xs, ys, zs, Ma, gamma, modes, amplitudes=None):
    """TGV fields with the velocity modes added (amplitudes default to the
    drawn ones), one mode at a time (no (M, 3, N) basis in memory)."""
    rho, u, T = tgv_fields(xs, ys, zs, Ma, gamma)
    if modes:
        amps = np.array([m[3] for m in modes]) if amplitudes is None else np.asarray(amplitudes)
        X, Y, Z = mesh(xs, ys, zs)
        for a, (k, e, ph, _) in zip(amps, modes):
            s = a * np.sin(k[0] * X + k[1] * Y + k[2] * Z + ph)
            for c in range(3):
                u[c] += e[c] * s
    return rho, u, T


def random_populations(shape, seed, scale=1.0):
    """Seeded standard-normal array (for adjoint seeds and perturbations)."""
    return np.random.default_rng(seed).normal(0.0, scale, size=shape)


# ---------------------------------------------------------------------------
# Two-dimensional workloads (D2Q19 lattice; Sec. III A and III B).  The
# paper's tubes and Riemann problems have open boundaries; these periodic
# stand-ins keep the shapes, states and discretisations:
#  * "sod": the coarse shock-tube setting (h = 0.01, p = 4, dt = 5e-4,
#    mu = 2e-4, t = 0.1) doubled into a periodic tube of length 2 whose
#    high-pressure state fills (0.5, 1.5); each discontinuity evolves as the
#    paper's tube until t > 0.2, one cell across y;
#  * "riemann": case 12 of the 2-D Riemann problems on 128^2 cells of p = 4
#    (512^2 nodes) over [0, 1]^2 with the quadrant corner at (0.5, 0.5),
#    t_end = 0.25; dt and mu are not given in the text, the values below
#    (largest abscissa moves 0.11 cells a step, tau - 1/2 about 1) stand in.
# Constant viscosity (the viscosity law is not stated for these cases).
# ---------------------------------------------------------------------------
WORKLOADS_2D = {
    "sod": dict(n_el=(200, 1), p=4, length=(2.0, 0.01), dt=5e-4, mu_inf=2e-4, steps=200, gamma=1.4, Pr=0.71,
                precision="fp64"),
    "riemann": dict(n_el=(128, 128), p=4, length=(1.0, 1.0), dt=5e-4, mu_inf=5e-4, steps=500, gamma=1.4,
                    Pr=0.71, precision="fp64"),
}

SOD_STATES = ((8.0, 0.0, 10.0), (1.0, 0.0, 1.0))          # (rho, u, P) inside, outside
RIEMANN12 = {                                              # quadrant: (rho, u_x, u_y, P)
    "ne": (0.5313, 0.0, 0.0, 0.4),
    "nw": (1.0, 0.7276, 0.0, 1.0),
    "sw": (0.8, 0.0, 0.0, 1.0),
    "se": (1.0, 0.0, 0.7276, 1.0),
}


def mesh2d(xs, ys):
    """2-D coordinate arrays (flattened, x fastest) from the 1-D node coordinates."""
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    return X.ravel(), Y.ravel()


def sod_fields(xs, ys):
    """rho (N,), u (2, N), T (N,) of the periodic double shock tube (T = P / rho)."""
    X, _ = mesh2d(xs, ys)
    inside = (X > 0.5) & (X < 1.5)
    (ri, ui, pi), (ro, uo, po) = SOD_STATES
    rho = np.where(inside, ri, ro)
    P = np.where(inside, pi, po)
    u = np.zeros((2, X.size))
    u[0] = np.where(inside, ui, uo)
    return rho, u, P / rho


def riemann_fields(xs, ys, corner=(0.5, 0.5)):
    """rho, u (2, N), T of Riemann case 12 (x <= corner counts as west, y <= corner as south)."""
    X, Y = mesh2d(xs, ys)
    east, north = X > corner[0], Y > corner[1]
    rho, P = np.empty(X.size), np.empty(X.size)
    u = np.empty((2, X.size))
    for key, mask in (("ne", east & north), ("nw", ~east & north), ("sw", ~east & ~north),
                      ("se", east & ~north)):
        r, ux, uy, p = RIEMANN12[key]
        rho[mask], u[0, mask], u[1, mask], P[mask] = r, ux, uy, p
    return rho, u, P / rho
