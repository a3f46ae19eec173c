"""Host logic of the distorted-mesh tables (no GPU): a driver compiled
against the library's table builder (csrc/tables.cpp) dumps the departure
cells, local coordinates and node weights; gathering with them exactly as
the streaming kernel does must reproduce the oracle's distorted-mesh
streaming, and the weights must equal the oracle's.  A folded mesh is
refused."""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
Q = 45


@pytest.fixture(scope="module")
def driver():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    csrc = os.path.join(ROOT, "paper_2012_05537_amd", "csrc")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "mapped_dump")
    subprocess.check_call([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                           "-I", os.path.join(ROOT, "include"), "-I", csrc,
                           os.path.join(ROOT, "tests", "host", "mapped_dump.cpp"),
                           os.path.join(csrc, "tables.cpp"), "-o", exe])
    return exe


def _run(exe, p, n_el, L, dt, disp):
    head = "%d %d %d %d %.17g %.17g %.17g %.17g\n" % (p, *n_el, *L, dt)
    body = "\n".join("%.17g" % v for v in disp.reshape(-1))
    return subprocess.run([exe], input=head + body, capture_output=True, text=True)


def _gather(oracle, cfg, cell, t, f):
    """The kernel's gather: (p+1)^3 support values of the departure cell,
    tensor Lagrange weights at the local coordinates."""
    p = cfg.p
    ne = np.array(cfg.n_el[:])
    N3 = ne * p
    N = f.shape[1]
    out = np.zeros_like(f)
    ex, ey, ez = cell % ne[0], (cell // ne[0]) % ne[1], cell // (ne[0] * ne[1])
    for i in range(Q):
        wl = [np.array([oracle.lagrange(p, tv) for tv in t[a, i]]) for a in range(3)]
        acc = np.zeros(N)
        for kz in range(p + 1):
            zz = (ez[i] * p + kz) % N3[2]
            for ky in range(p + 1):
                yy = (ey[i] * p + ky) % N3[1]
                for kx in range(p + 1):
                    xx = (ex[i] * p + kx) % N3[0]
                    acc += wl[0][:, kx] * wl[1][:, ky] * wl[2][:, kz] * f[i, (zz * N3[1] + yy) * N3[0] + xx]
        out[i] = acc
    return out


@pytest.mark.parametrize("p,n_el,dt", [(2, (3, 4, 2), 0.31), (3, (2, 3, 3), 0.8), (4, (2, 2, 2), 0.5)])
def test_tables_reproduce_oracle_streaming(oracle, driver, p, n_el, dt):
    L = (2 * math.pi, 2 * math.pi, 2 * math.pi)
    cfg0 = oracle.make_cfg(n_el, p, dt, 0.01)
    xs, ys, zs = oracle.node_coords(cfg0)
    Z, Y, X = (v.reshape(-1) for v in np.meshgrid(zs, ys, xs, indexing="ij"))
    disp = np.stack([0.2 * np.sin(Y + 0.5 * Z), 0.15 * np.cos(X) * np.sin(Z), 0.1 * np.sin(X + Y)])
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, disp=disp)
    r = _run(driver, p, n_el, L, dt, disp)
    assert r.returncode == 0, r.stdout[:200] + r.stderr
    vals = r.stdout.split()
    N = X.size
    cell = np.array(vals[:Q * N], dtype=np.int64).reshape(Q, N)
    t = np.array(vals[Q * N:4 * Q * N], dtype=np.float64).reshape(3, Q, N)
    w = np.array(vals[4 * Q * N:], dtype=np.float64)
    assert np.all((t >= 0) & (t <= 1))           # 1 when a departure point rounds onto a face
    f = np.random.default_rng(p).normal(size=(Q, N))
    ref, _ = oracle.stream(cfg, f, f)
    got = _gather(oracle, cfg, cell, t, f)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.abs(ref).max()
    assert np.allclose(w, oracle.mapped_node_weights(cfg), rtol=1e-12, atol=0)


def test_folded_mesh_is_refused(oracle, driver):
    p, n_el = 2, (3, 3, 3)
    cfg0 = oracle.make_cfg(n_el, p, 0.1, 0.01)
    xs, ys, zs = oracle.node_coords(cfg0)
    Z, Y, X = (v.reshape(-1) for v in np.meshgrid(zs, ys, xs, indexing="ij"))
    disp = np.stack([2.0 * np.sin(X), np.zeros_like(X), np.zeros_like(X)])   # d(x)/dx = 1 + 2 cos x < 0 somewhere
    r = _run(driver, p, n_el, (2 * math.pi,) * 3, 0.1, disp)
    assert r.returncode == 1 and "folds over" in r.stdout
