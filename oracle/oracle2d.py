"""ctypes wrapper of the plain-C FP64 oracle of the two-dimensional variant
(``sllbm2d_oracle.c``: D2Q19, periodic mesh of equal cells).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path never imports it.

Populations are numpy arrays of shape (19, N) with node index gy * Nx + gx;
fields are rho (N,), u (2, N), T (N,).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle2d.so")
_SRC = os.path.join(_HERE, "sllbm2d_oracle.c")

Q = 19
SUTHERLAND = 0
CONSTANT = 1


def build(verbose=False):
    """Compile the 2-D oracle (gcc, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", _SRC, "-o", _LIB, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)


class Cfg(ctypes.Structure):
    _fields_ = [
        ("n_el", ctypes.c_int * 2),
        ("p", ctypes.c_int),
        ("length", ctypes.c_double * 2),
        ("dt", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_inf", ctypes.c_double),
        ("viscosity_law", ctypes.c_int),
    ]


_lib_handle = []


def _lib():
    if not _lib_handle:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle2d_num_nodes.restype = ctypes.c_long
        _lib_handle.append(lib)
    return _lib_handle[0]


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def make_cfg(n_el, p, dt, mu_inf, gamma=1.4, prandtl=0.71, length=1.0, viscosity_law=SUTHERLAND):
    if np.isscalar(n_el):
        n_el = (n_el, n_el)
    if np.isscalar(length):
        length = (length, length)
    c = Cfg()
    c.n_el[0], c.n_el[1] = int(n_el[0]), int(n_el[1])
    c.p = int(p)
    c.length[0], c.length[1] = float(length[0]), float(length[1])
    c.dt = float(dt)
    c.gamma = float(gamma)
    c.prandtl = float(prandtl)
    c.mu_inf = float(mu_inf)
    c.viscosity_law = int(viscosity_law)
    return c


def num_nodes(cfg):
    return cfg.n_el[0] * cfg.p * cfg.n_el[1] * cfg.p


def grid_shape(cfg):
    """(Ny, Nx) of the unique periodic node grid."""
    return (cfg.n_el[1] * cfg.p, cfg.n_el[0] * cfg.p)


def velocity_set():
    """xi (19, 2) and w (19,) of the D2Q19 rule."""
    xi = np.zeros((Q, 2))
    w = np.zeros(Q)
    n = _lib().oracle2d_velocity_set(_ptr(xi), _ptr(w))
    assert n == Q, n
    return xi, w


def node_coords(cfg):
    x = np.zeros(cfg.n_el[0] * cfg.p)
    y = np.zeros(cfg.n_el[1] * cfg.p)
    _lib().oracle2d_node_coords(ctypes.byref(cfg), _ptr(x), _ptr(y))
    return x, y


def equilibrium(rho, u, T):
    feq = np.zeros(Q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _lib().oracle2d_equilibrium(ctypes.c_double(rho), _ptr(uu), ctypes.c_double(T), _ptr(feq))
    return feq


def collide_node(cfg, f, g):
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    fo, go = np.zeros(Q), np.zeros(Q)
    _lib().oracle2d_collide_node(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    return fo, go


def init_equilibrium(cfg, rho, u, T):
    N = num_nodes(cfg)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(2, N)
    T = np.ascontiguousarray(T, dtype=np.float64)
    f, g = np.zeros((Q, N)), np.zeros((Q, N))
    _lib().oracle2d_init_equilibrium(ctypes.byref(cfg), _ptr(rho), _ptr(u), _ptr(T), _ptr(f), _ptr(g))
    return f, g


def collide(cfg, f, g):
    f = np.array(f, dtype=np.float64, order="C")
    g = np.array(g, dtype=np.float64, order="C")
    _lib().oracle2d_collide(ctypes.byref(cfg), _ptr(f), _ptr(g))
    return f, g


def stream(cfg, f, g):
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    fo, go = np.zeros_like(f), np.zeros_like(g)
    _lib().oracle2d_stream(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    return fo, go


def step(cfg, f, g, n=1):
    f = np.array(f, dtype=np.float64, order="C")
    g = np.array(g, dtype=np.float64, order="C")
    rc = _lib().oracle2d_step(ctypes.byref(cfg), _ptr(f), _ptr(g), ctypes.c_int(n))
    assert rc == 0
    return f, g


def moments(cfg, f, g):
    N = num_nodes(cfg)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    rho, u, T = np.zeros(N), np.zeros((2, N)), np.zeros(N)
    _lib().oracle2d_moments(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(rho), _ptr(u), _ptr(T))
    return rho, u, T


def totals(cfg, f, g):
    """Area integrals of rho, rho u_x, rho u_y, rho E."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros(4)
    _lib().oracle2d_totals(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(out))
    return out
