"""ctypes wrapper of the plain-C FP64 oracle (``sllbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path never imports it.

Populations are numpy arrays of shape (45, N) (x fastest node order); fields
are rho (N,), u (3, N), T (N,).  ``complex128`` inputs run the complex-step
build (``oracle_cs_*``), used for reference derivatives.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_REAL = os.path.join(_HERE, "liboracle.so")
_LIB_CPLX = os.path.join(_HERE, "liboracle_cs.so")
_SRC = os.path.join(_HERE, "sllbm_oracle.c")

Q = 45
SUTHERLAND = 0
CONSTANT = 1


def build(verbose=False):
    """Compile the real and the complex-step builds of the oracle (gcc, -O2, OpenMP)."""
    for out, extra in ((_LIB_REAL, []), (_LIB_CPLX, ["-DORACLE_COMPLEX"])):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", *extra, _SRC, "-o", out, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)


class Cfg(ctypes.Structure):
    _fields_ = [
        ("n_el", ctypes.c_int * 3),
        ("p", ctypes.c_int),
        ("length", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_inf", ctypes.c_double),
        ("mu_inf_im", ctypes.c_double),
        ("viscosity_law", ctypes.c_int),
        ("faces", ctypes.POINTER(ctypes.c_double) * 3),
        ("disp", ctypes.POINTER(ctypes.c_double)),
    ]


_libs = {}


def _lib(cplx=False):
    key = bool(cplx)
    if key not in _libs:
        path = _LIB_CPLX if key else _LIB_REAL
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        _libs[key] = ctypes.CDLL(path)
    return _libs[key]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_cfg(n_el, p, dt, mu_inf, gamma=1.4, prandtl=0.71, length=2 * np.pi,
             viscosity_law=SUTHERLAND, mu_inf_im=0.0, widths=None, disp=None):
    """widths: None (equal cells) or, per axis, None or the n_el[a] cell widths
    of a graded axis (their sum replaces length[a]).  disp: None or the (3, N)
    node displacements of a distorted mesh (equal cells only)."""
    if np.isscalar(n_el):
        n_el = (n_el, n_el, n_el)
    if np.isscalar(length):
        length = (length, length, length)
    length = list(length)
    c = Cfg()
    c._faces = [None, None, None]            # keeps the face arrays alive with the cfg
    for a in range(3):
        w = None if widths is None else widths[a]
        if w is None:
            continue
        w = np.asarray(w, dtype=np.float64)
        if w.shape != (int(n_el[a]),) or not np.all(w > 0):
            raise ValueError("widths[%d] must hold n_el[%d] positive cell widths" % (a, a))
        faces = np.concatenate([[0.0], np.cumsum(w)])
        length[a] = float(faces[-1])
        c._faces[a] = faces
        c.faces[a] = faces.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.n_el[:] = [int(v) for v in n_el]
    c.p = int(p)
    c.length[:] = [float(v) for v in length]
    c.dt = float(dt)
    c.gamma = float(gamma)
    c.prandtl = float(prandtl)
    c.mu_inf = float(mu_inf)
    c.mu_inf_im = float(mu_inf_im)
    c.viscosity_law = int(viscosity_law)
    if disp is not None:
        if widths is not None:
            raise ValueError("a distorted mesh displaces the equal-cell grid")
        d = np.ascontiguousarray(disp, dtype=np.float64).reshape(3, -1)
        if d.shape[1] != num_nodes(c):
            raise ValueError("disp must be (3, N)")
        c._disp = d
        c.disp = d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return c


def num_nodes(cfg):
    return cfg.n_el[0] * cfg.p * cfg.n_el[1] * cfg.p * cfg.n_el[2] * cfg.p


def grid_shape(cfg):
    """(Nz, Ny, Nx) of the unique periodic node grid."""
    return (cfg.n_el[2] * cfg.p, cfg.n_el[1] * cfg.p, cfg.n_el[0] * cfg.p)


def velocity_set():
    xi = np.zeros((Q, 3))
    w = np.zeros(Q)
    n = _lib().oracle_velocity_set(_ptr(xi), _ptr(w))
    assert n == Q
    return xi, w


def glc_nodes(p):
    t = np.zeros(p + 1)
    _lib().oracle_glc_nodes(ctypes.c_int(p), _ptr(t))
    return t


def lagrange(p, s):
    ell = np.zeros(p + 1)
    _lib().oracle_lagrange(ctypes.c_int(p), ctypes.c_double(s), _ptr(ell))
    return ell


def lagrange_deriv(p, s):
    d = np.zeros(p + 1)
    _lib().oracle_lagrange_deriv(ctypes.c_int(p), ctypes.c_double(s), _ptr(d))
    return d


def cc_weights(p):
    w = np.zeros(p + 1)
    _lib().oracle_cc_weights(ctypes.c_int(p), _ptr(w))
    return w


def node_coords(cfg):
    """1-D coordinate arrays (x, y, z) of the unique nodes along each axis."""
    n = [cfg.n_el[a] * cfg.p for a in range(3)]
    x, y, z = (np.zeros(v) for v in n)
    _lib().oracle_node_coords(ctypes.byref(cfg), _ptr(x), _ptr(y), _ptr(z))
    return x, y, z


def _dt(cplx):
    return np.complex128 if cplx else np.float64


def _prefix(cplx):
    return "oracle_cs_" if cplx else "oracle_"


def _is_cplx(*arrs):
    return any(np.iscomplexobj(a) for a in arrs)


def equilibrium(rho, u, T):
    cplx = _is_cplx(np.asarray(rho), np.asarray(u), np.asarray(T))
    dt = _dt(cplx)
    uu = np.ascontiguousarray(np.asarray(u, dtype=dt))
    feq = np.zeros(Q, dtype=dt)
    lib = _lib(cplx)
    fn = getattr(lib, _prefix(cplx) + "equilibrium")
    if cplx:
        r = np.array([rho], dtype=dt)
        t = np.array([T], dtype=dt)
        # by-value complex arguments are not portable through ctypes: use the
        # one-node init routine instead
        cfg = make_cfg(1, 1, 1.0, 0.0)
        f = np.zeros((Q, 1), dt)
        g = np.zeros((Q, 1), dt)
        getattr(lib, "oracle_cs_init_equilibrium")(ctypes.byref(cfg), _ptr(r), _ptr(uu.reshape(3, 1).copy()),
                                                   _ptr(t), _ptr(f), _ptr(g))
        return f[:, 0]
    fn.argtypes = [ctypes.c_double, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    fn(float(rho), _ptr(uu), float(T), _ptr(feq))
    return feq


def collide_node(cfg, f, g):
    cplx = _is_cplx(f, g) or cfg.mu_inf_im != 0.0
    dt = _dt(cplx)
    f = np.ascontiguousarray(f, dtype=dt)
    g = np.ascontiguousarray(g, dtype=dt)
    fo = np.zeros(Q, dt)
    go = np.zeros(Q, dt)
    getattr(_lib(cplx), _prefix(cplx) + "collide_node")(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    return fo, go


def init_equilibrium(cfg, rho, u, T):
    cplx = _is_cplx(rho, u, T)
    dt = _dt(cplx)
    N = num_nodes(cfg)
    rho = np.ascontiguousarray(np.reshape(rho, N), dtype=dt)
    u = np.ascontiguousarray(np.reshape(u, (3, N)), dtype=dt)
    T = np.ascontiguousarray(np.reshape(T, N), dtype=dt)
    f = np.zeros((Q, N), dt)
    g = np.zeros((Q, N), dt)
    getattr(_lib(cplx), _prefix(cplx) + "init_equilibrium")(ctypes.byref(cfg), _ptr(rho), _ptr(u), _ptr(T),
                                                            _ptr(f), _ptr(g))
    return f, g


def collide(cfg, f, g):
    cplx = _is_cplx(f, g) or cfg.mu_inf_im != 0.0
    dt = _dt(cplx)
    f = np.array(f, dtype=dt, order="C")
    g = np.array(g, dtype=dt, order="C")
    getattr(_lib(cplx), _prefix(cplx) + "collide")(ctypes.byref(cfg), _ptr(f), _ptr(g))
    return f, g


def stream(cfg, f, g):
    cplx = _is_cplx(f, g)
    dt = _dt(cplx)
    f = np.ascontiguousarray(f, dtype=dt)
    g = np.ascontiguousarray(g, dtype=dt)
    fo = np.zeros_like(f)
    go = np.zeros_like(g)
    getattr(_lib(cplx), _prefix(cplx) + "stream")(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(fo), _ptr(go))
    return fo, go


def step(cfg, f, g, n=1):
    """n steps of (collide, stream) on pre-collision populations; returns new arrays."""
    cplx = _is_cplx(f, g) or cfg.mu_inf_im != 0.0
    dt = _dt(cplx)
    f = np.array(f, dtype=dt, order="C")
    g = np.array(g, dtype=dt, order="C")
    rc = getattr(_lib(cplx), _prefix(cplx) + "step")(ctypes.byref(cfg), _ptr(f), _ptr(g), ctypes.c_int(n))
    if rc != 0:
        raise MemoryError("oracle step: allocation failed")
    return f, g


def step_at_nodes(cfg, f, g, nodes):
    """One step evaluated only at the given node indices: returns (fo, go), each (S, 45)."""
    cplx = _is_cplx(f, g)
    dt = _dt(cplx)
    f = np.ascontiguousarray(f, dtype=dt)
    g = np.ascontiguousarray(g, dtype=dt)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    S = len(nodes)
    fo = np.zeros((S, Q), dt)
    go = np.zeros((S, Q), dt)
    getattr(_lib(cplx), _prefix(cplx) + "step_at_nodes")(ctypes.byref(cfg), _ptr(f), _ptr(g), ctypes.c_int(S),
                                                         _ptr(nodes), _ptr(fo), _ptr(go))
    return fo, go


def stream_at_nodes(cfg, f, g, nodes):
    """Streaming only, evaluated at the given node indices (equal or graded
    cells): returns (fo, go), each (S, 45)."""
    if is_mapped(cfg):
        raise ValueError("stream_at_nodes: equal or graded cells only")
    cplx = _is_cplx(f, g)
    dt = _dt(cplx)
    f = np.ascontiguousarray(f, dtype=dt)
    g = np.ascontiguousarray(g, dtype=dt)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    S = len(nodes)
    fo = np.zeros((S, Q), dt)
    go = np.zeros((S, Q), dt)
    getattr(_lib(cplx), _prefix(cplx) + "stream_at_nodes")(ctypes.byref(cfg), _ptr(f), _ptr(g), ctypes.c_int(S),
                                                           _ptr(nodes), _ptr(fo), _ptr(go))
    return fo, go


def moments(cfg, f, g):
    cplx = _is_cplx(f, g)
    dt = _dt(cplx)
    N = num_nodes(cfg)
    f = np.ascontiguousarray(f, dtype=dt)
    g = np.ascontiguousarray(g, dtype=dt)
    rho = np.zeros(N, dt)
    u = np.zeros((3, N), dt)
    T = np.zeros(N, dt)
    getattr(_lib(cplx), _prefix(cplx) + "moments")(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(rho), _ptr(u), _ptr(T))
    return rho, u, T


def totals(cfg, f, g):
    cplx = _is_cplx(f, g)
    dt = _dt(cplx)
    f = np.ascontiguousarray(f, dtype=dt)
    g = np.ascontiguousarray(g, dtype=dt)
    out = np.zeros(5, dt)
    getattr(_lib(cplx), _prefix(cplx) + "totals")(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(out))
    return out


def is_graded(cfg):
    return any(getattr(cfg, "_faces", [None] * 3)[a] is not None for a in range(3))


def loss(cfg, f, g):
    cplx = _is_cplx(f, g)
    f = np.ascontiguousarray(f, dtype=_dt(cplx))
    g = np.ascontiguousarray(g, dtype=_dt(cplx))
    if cplx:
        out = np.zeros(1, np.complex128)
        _lib(True).oracle_cs_loss_out(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(out))
        return out[0]
    fn = _lib(False).oracle_loss
    fn.restype = ctypes.c_double
    return fn(ctypes.byref(cfg), _ptr(f), _ptr(g))

def diagnostics(cfg, f, g):
    """(kinetic energy, solenoidal dissipation, dilatational dissipation) as domain integrals."""
    cplx = _is_cplx(f, g) or cfg.mu_inf_im != 0.0
    dt = _dt(cplx)
    f = np.ascontiguousarray(f, dtype=dt)
    g = np.ascontiguousarray(g, dtype=dt)
    out = np.zeros(3, dt)
    getattr(_lib(cplx), _prefix(cplx) + "diagnostics")(ctypes.byref(cfg), _ptr(f), _ptr(g), _ptr(out))
    return out


def is_mapped(cfg):
    return bool(cfg.disp)


def mapped_node_coords(cfg):
    """(3, N) physical node positions of a distorted mesh (GLC grid + displacement)."""
    xs, ys, zs = node_coords(cfg)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    ref = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)])
    return ref + (cfg._disp if is_mapped(cfg) else 0.0)


def mapped_node_weights(cfg):
    """(N,) quadrature weight of every node of a distorted mesh (|det J| included)."""
    w = np.zeros(num_nodes(cfg))
    _lib().oracle_mapped_node_weights(ctypes.byref(cfg), _ptr(w))
    return w
