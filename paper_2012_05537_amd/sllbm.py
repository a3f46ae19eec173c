"""ctypes binding of ``libsllbm.so`` (C ABI in ``include/sllbm.h``).

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are torch tensors on the context's device; pointers are passed as
integers.  The library must be built (``python -m paper_2012_05537_amd.build``)
before use; loading fails loudly otherwise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsllbm.so")

Q = 45                      # velocities of the three-dimensional set
D3Q45, D2Q19 = 45, 19       # velocity_set values (the value is the velocity count)
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONFINITE = range(6)
SUTHERLAND, CONSTANT = 0, 1
FP64, FP32_MIXED = 0, 1

_ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE", ENONFINITE: "ENONFINITE"}


class SllbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("n_el", ctypes.c_int32 * 3),
        ("order", ctypes.c_int32),
        ("velocity_set", ctypes.c_int32),
        ("viscosity_law", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("length", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_inf", ctypes.c_double),
    ]


_lib = None

_VP = ctypes.c_void_p
_SIGS = {
    "sllbm_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(_VP)]),
    "sllbm_destroy": (ctypes.c_int, [_VP]),
    "sllbm_set_stream": (ctypes.c_int, [_VP, _VP]),
    "sllbm_last_error": (ctypes.c_char_p, [_VP]),
    "sllbm_num_nodes": (ctypes.c_int64, [_VP]),
    "sllbm_state_bytes": (ctypes.c_int64, [_VP]),
    "sllbm_velocity_set": (ctypes.c_int, [_VP, _VP]),
    "sllbm_lattice": (ctypes.c_int, [ctypes.c_int32, _VP, _VP]),
    "sllbm_node_coords": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "sllbm_set_viscosity": (ctypes.c_int, [_VP, ctypes.c_double]),
    "sllbm_set_mesh": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "sllbm_set_displacement": (ctypes.c_int, [_VP, _VP]),
    "sllbm_init_equilibrium": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "sllbm_set_state": (ctypes.c_int, [_VP, _VP]),
    "sllbm_get_state": (ctypes.c_int, [_VP, _VP]),
    "sllbm_step": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "sllbm_step_record": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, ctypes.c_int64]),
    "sllbm_moments": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "sllbm_totals": (ctypes.c_int, [_VP, _VP]),
    "sllbm_loss": (ctypes.c_int, [_VP, _VP, _VP]),
    "sllbm_loss_grad": (ctypes.c_int, [_VP, _VP, _VP]),
    "sllbm_adjoint_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "sllbm_diagnostics": (ctypes.c_int, [_VP, _VP, _VP]),
    "sllbm_set_kernel_timing": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "sllbm_kernel_times": (ctypes.c_int, [_VP, _VP]),
    "sllbm_moments_vjp": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "sllbm_init_equilibrium_vjp": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "sllbm_stream": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32]),
    "sllbm_collide": (ctypes.c_int, [_VP, _VP]),
    "sllbm_totals_noalloc": (ctypes.c_int, [ctypes.POINTER(Config), _VP, _VP, _VP]),
    "sllbm_superpose": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, _VP, _VP]),
    "sllbm_project": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP]),
}

EXPORTED = tuple(_SIGS)


def load_library(path=LIB_PATH):
    """Load libsllbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} not found: build it with `python -m paper_2012_05537_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def velocity_set():
    """(xi (45, 3), w (45,)) as float64 tensors on the CPU."""
    lib = load_library()
    xi = (ctypes.c_double * (3 * Q))()
    w = (ctypes.c_double * Q)()
    n = lib.sllbm_velocity_set(ctypes.addressof(xi), ctypes.addressof(w))
    assert n == Q
    return torch.tensor(list(xi), dtype=torch.float64).reshape(Q, 3), torch.tensor(list(w), dtype=torch.float64)


def lattice(velocity_set=D3Q45):
    """(xi (Q, 3), w (Q,)) of D3Q45 or D2Q19 (z = 0) as float64 CPU tensors."""
    lib = load_library()
    xi = (ctypes.c_double * (3 * Q))()
    w = (ctypes.c_double * Q)()
    n = lib.sllbm_lattice(int(velocity_set), ctypes.addressof(xi), ctypes.addressof(w))
    if n < 0:
        raise ValueError("unknown velocity set %r" % (velocity_set,))
    return (torch.tensor(list(xi)[:3 * n], dtype=torch.float64).reshape(n, 3),
            torch.tensor(list(w)[:n], dtype=torch.float64))


def totals_noalloc(cfg, state, out, stream=None):
    """sllbm_totals_noalloc: totals of a device state into the device tensor out (5 doubles).

    cfg: a Config (e.g. SLLBM(...).cfg); stream: a torch.cuda.Stream or None
    (the current stream of the state's device)."""
    lib = load_library()
    if out.dtype != torch.float64 or out.numel() < 5 or not out.is_contiguous():
        raise ValueError("out must hold 5 contiguous float64 values")
    s = stream if stream is not None else torch.cuda.current_stream(state.device)
    rc = lib.sllbm_totals_noalloc(ctypes.byref(cfg), _ptr(state), _ptr(out), s.cuda_stream)
    if rc != OK:
        raise SllbmError(rc, lib.sllbm_last_error(None).decode())
    return out


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


class SLLBM:
    """One simulation context on one GPU (a thin owner of ``sllbm_ctx*``).

    velocity_set=D2Q19 makes a two-dimensional context: n_el and length take
    (x, y) values (z is set to one cell), states are (2, 19, N), velocity
    fields (2, N)."""

    def __init__(self, n_el, order, dt, mu_inf, gamma=1.4, prandtl=0.71, length=2 * 3.141592653589793,
                 viscosity_law=SUTHERLAND, precision=FP64, device=0, velocity_set=D3Q45):
        lib = load_library()
        dim = 2 if velocity_set == D2Q19 else 3
        if isinstance(n_el, int):
            n_el = (n_el,) * dim
        if isinstance(length, (int, float)):
            length = (length,) * dim
        n_el, length = tuple(n_el), tuple(length)
        if dim == 2:
            n_el, length = n_el[:2] + (1,), length[:2] + (1.0,)
        cfg = Config()
        cfg.n_el[:] = [int(v) for v in n_el]
        cfg.order = int(order)
        cfg.velocity_set = int(velocity_set)
        cfg.viscosity_law = int(viscosity_law)
        cfg.precision = int(precision)
        cfg.device = int(device)
        cfg.length[:] = [float(v) for v in length]
        cfg.dt = float(dt)
        cfg.gamma = float(gamma)
        cfg.prandtl = float(prandtl)
        cfg.mu_inf = float(mu_inf)
        self.cfg = cfg
        self._lib = lib
        h = _VP()
        rc = lib.sllbm_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != OK:
            raise SllbmError(rc, lib.sllbm_last_error(None).decode())
        self._h = h
        self.device = torch.device("cuda", int(device))
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        self.nodes = lib.sllbm_num_nodes(h)
        self.q, self.dim = int(velocity_set), dim
        if dim == 2:
            self.shape = (cfg.n_el[1] * order, cfg.n_el[0] * order)
        else:
            self.shape = (cfg.n_el[2] * order, cfg.n_el[1] * order, cfg.n_el[0] * order)
        self.state_bytes = lib.sllbm_state_bytes(h)
        self._stream = None

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc):
        if rc != OK:
            raise SllbmError(rc, self._lib.sllbm_last_error(self._h).decode())

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            self._check(self._lib.sllbm_set_stream(self._h, s))
            self._stream = s

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sllbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_state(self):
        return torch.empty((2, self.q, self.nodes), dtype=self.dtype, device=self.device)

    def _state_arg(self, t):
        if t.dtype != self.dtype or t.device != self.device or t.numel() != 2 * self.q * self.nodes:
            raise ValueError("state must be a contiguous (2, %d, N) tensor of the storage dtype on the device"
                             % self.q)
        return _ptr(t)

    # -- C ABI, same names -------------------------------------------------
    def node_coords(self):
        """1-D node coordinates per axis: (x, y, z), or (x, y) in two dimensions."""
        n = [self.cfg.n_el[a] * self.cfg.order for a in range(3)]
        if self.dim == 2:
            n[2] = 1
        arrs = [(ctypes.c_double * v)() for v in n]
        self._check(self._lib.sllbm_node_coords(self._h, *[ctypes.addressof(a) for a in arrs]))
        return tuple(torch.tensor(list(a), dtype=torch.float64) for a in arrs[:self.dim])

    def set_viscosity(self, mu_inf):
        self._check(self._lib.sllbm_set_viscosity(self._h, float(mu_inf)))
        self.cfg.mu_inf = float(mu_inf)

    def set_mesh(self, widths_x=None, widths_y=None, widths_z=None):
        """Graded mesh: per axis None (equal cells) or the n_el[a] cell widths."""
        arrs = []
        for a, w in enumerate((widths_x, widths_y, widths_z)):
            if w is None:
                arrs.append(None)
                continue
            v = [float(x) for x in (w.tolist() if hasattr(w, "tolist") else w)]
            if len(v) != self.cfg.n_el[a]:
                raise ValueError("axis %d needs %d cell widths" % (a, self.cfg.n_el[a]))
            arrs.append((ctypes.c_double * len(v))(*v))
        self._sync_stream()
        self._check(self._lib.sllbm_set_mesh(self._h, *[None if x is None else ctypes.addressof(x) for x in arrs]))
        for a, x in enumerate(arrs):
            if x is not None:
                self.cfg.length[a] = float(sum(x))

    def set_displacement(self, d=None):
        """Distorted mesh: d (3, N) periodic node displacements (array or tensor), or None."""
        self._sync_stream()
        if d is None:
            self._check(self._lib.sllbm_set_displacement(self._h, None))
            return
        import numpy as np
        v = np.ascontiguousarray(d.cpu().numpy() if hasattr(d, "cpu") else d, dtype=np.float64)
        if v.size != 3 * self.nodes:
            raise ValueError("d must hold (3, N) displacements")
        self._check(self._lib.sllbm_set_displacement(self._h, v.ctypes.data_as(_VP)))

    def init_equilibrium(self, rho, u, T):
        self._sync_stream()
        f64 = dict(dtype=torch.float64, device=self.device)
        rho, u, T = (x.to(**f64).contiguous() for x in (rho, u, T))
        if rho.numel() != self.nodes or T.numel() != self.nodes or u.numel() != self.dim * self.nodes:
            raise ValueError("rho, T need N values and u (%d, N)" % self.dim)
        self._check(self._lib.sllbm_init_equilibrium(self._h, _ptr(rho), _ptr(u), _ptr(T)))

    def set_state(self, state):
        self._sync_stream()
        self._check(self._lib.sllbm_set_state(self._h, self._state_arg(state)))

    def get_state(self, out=None):
        self._sync_stream()
        out = self.empty_state() if out is None else out
        self._check(self._lib.sllbm_get_state(self._h, self._state_arg(out)))
        return out

    def step(self, n=1):
        self._sync_stream()
        self._check(self._lib.sllbm_step(self._h, int(n)))

    def step_record(self, n, states):
        """states: (n, 2, Q, N) tensor receiving the pre-collision state after each step."""
        self._sync_stream()
        if states.shape[0] < n or not states.is_contiguous() or states.dtype != self.dtype:
            raise ValueError("record buffer too small or wrong dtype")
        self._check(self._lib.sllbm_step_record(self._h, int(n), _ptr(states), int(self.state_bytes)))

    def set_kernel_timing(self, on=True):
        self._sync_stream()
        self._check(self._lib.sllbm_set_kernel_timing(self._h, int(bool(on))))

    def kernel_times(self):
        """{'collide': (total_ms, launches), 'stream': (total_ms, launches)}; clears the record."""
        self._sync_stream()
        out = (ctypes.c_double * 4)()
        self._check(self._lib.sllbm_kernel_times(self._h, ctypes.addressof(out)))
        return {"collide": (out[0], int(out[1])), "stream": (out[2], int(out[3]))}

    def moments(self):
        self._sync_stream()
        f64 = dict(dtype=torch.float64, device=self.device)
        rho = torch.empty(self.nodes, **f64)
        u = torch.empty((self.dim, self.nodes), **f64)
        T = torch.empty(self.nodes, **f64)
        self._check(self._lib.sllbm_moments(self._h, _ptr(rho), _ptr(u), _ptr(T)))
        return rho, u, T

    def totals(self):
        self._sync_stream()
        out = (ctypes.c_double * 5)()
        self._check(self._lib.sllbm_totals(self._h, ctypes.addressof(out)))
        return list(out)

    def diagnostics(self, state=None):
        """(kinetic energy, solenoidal dissipation, dilatational dissipation) of the state (default: current)."""
        self._sync_stream()
        out = (ctypes.c_double * 3)()
        arg = None if state is None else self._state_arg(state)
        self._check(self._lib.sllbm_diagnostics(self._h, arg, ctypes.addressof(out)))
        return tuple(out)

    def loss(self, state):
        self._sync_stream()
        out = ctypes.c_double()
        self._check(self._lib.sllbm_loss(self._h, self._state_arg(state), ctypes.addressof(out)))
        return out.value

    def loss_grad(self, state, out=None):
        self._sync_stream()
        out = self.empty_state() if out is None else out
        self._check(self._lib.sllbm_loss_grad(self._h, self._state_arg(state), self._state_arg(out)))
        return out

    def adjoint_step(self, state_n, lam_next, lam_out=None, dmu=None):
        self._sync_stream()
        lam_out = self.empty_state() if lam_out is None else lam_out
        self._check(self._lib.sllbm_adjoint_step(self._h, self._state_arg(state_n), self._state_arg(lam_next),
                                                 self._state_arg(lam_out), _ptr(dmu)))
        return lam_out

    def moments_vjp(self, drho=None, du=None, dT=None, out=None):
        self._sync_stream()
        f64 = dict(dtype=torch.float64, device=self.device)
        args = [None if x is None else x.to(**f64).contiguous() for x in (drho, du, dT)]
        out = self.empty_state() if out is None else out
        self._check(self._lib.sllbm_moments_vjp(self._h, *[_ptr(a) for a in args], self._state_arg(out)))
        return out

    def init_equilibrium_vjp(self, rho, u, T, lam0):
        self._sync_stream()
        f64 = dict(dtype=torch.float64, device=self.device)
        rho, u, T = (x.to(**f64).contiguous() for x in (rho, u, T))
        drho = torch.empty(self.nodes, **f64)
        du = torch.empty((3, self.nodes), **f64)
        dT = torch.empty(self.nodes, **f64)
        self._check(self._lib.sllbm_init_equilibrium_vjp(self._h, _ptr(rho), _ptr(u), _ptr(T),
                                                         self._state_arg(lam0), _ptr(drho), _ptr(du), _ptr(dT)))
        return drho, du, dT

    def superpose(self, base, basis, amps, out=None):
        """base + sum_j amps[j] basis[j]: base (D, N), basis (M, D, N) device float64; amps M host values."""
        self._sync_stream()
        a = [float(x) for x in (amps.tolist() if hasattr(amps, "tolist") else amps)]
        m = len(a)
        if basis.shape[0] != m or base.numel() != self.dim * self.nodes or basis.numel() != m * base.numel():
            raise ValueError("base (D, N), basis (M, D, N) and M amplitudes")
        out = torch.empty_like(base) if out is None else out
        arr = (ctypes.c_double * max(m, 1))(*a)
        self._check(self._lib.sllbm_superpose(self._h, _ptr(base), _ptr(basis), m, ctypes.addressof(arr), _ptr(out)))
        return out

    def project(self, basis, v):
        """[<basis[j], v>] over all D*N components, a list of M floats (host)."""
        self._sync_stream()
        m = basis.shape[0]
        if v.numel() != self.dim * self.nodes or basis.numel() != m * v.numel():
            raise ValueError("basis (M, D, N) and v (D, N)")
        out = (ctypes.c_double * max(m, 1))()
        self._check(self._lib.sllbm_project(self._h, _ptr(basis), m, _ptr(v), ctypes.addressof(out)))
        return list(out)[:m]

    def stream(self, state, transpose=False, out=None):
        self._sync_stream()
        out = self.empty_state() if out is None else out
        self._check(self._lib.sllbm_stream(self._h, self._state_arg(state), self._state_arg(out), int(transpose)))
        return out

    def collide(self, state):
        self._sync_stream()
        self._check(self._lib.sllbm_collide(self._h, self._state_arg(state)))
        return state
