"""Host logic of the distorted-mesh tables (no GPU): a driver compiled
against the library's table builder (csrc/tables_mapped.cpp) dumps the departure
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
                           os.path.join(csrc, "tables.cpp"), os.path.join(csrc, "tables_mapped.cpp"), "-o", exe])
    return exe


def _run(exe, p, n_el, L, dt, disp, max_nodes=3072):
    head = "%d %d %d %d %.17g %.17g %.17g %.17g %d\n" % (p, *n_el, *L, dt, max_nodes)
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
    w = np.array(vals[4 * Q * N:4 * Q * N + N], dtype=np.float64)
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


TILE = (8, 8, 4)     # node tile of the staged streaming kernel (x, y, z)


def _window_gather(oracle, cfg, cell, t, win, f):
    """The staged kernel's gather, emulated: per (velocity, tile) the window
    of f starting at the origin cell is filled with the kernel's wrapped
    indexing, every node of the tile reads its (p+1)^3 support values at the
    window position of its departure cell (bounds asserted), and blocks
    without a window gather from the whole field."""
    p = cfg.p
    ne = np.array(cfg.n_el[:])
    N3 = ne * p
    nt = (N3 + np.array(TILE) - 1) // np.array(TILE)
    ntiles = int(np.prod(nt))
    out = np.zeros_like(f)
    direct = _gather(oracle, cfg, cell, t, f)
    staged = 0
    for i in range(Q):
        wl = [np.array([oracle.lagrange(p, tv) for tv in t[a, i]]) for a in range(3)]
        for tt in range(ntiles):
            tc = (tt % nt[0], (tt // nt[0]) % nt[1], tt // (nt[0] * nt[1]))
            ocx, ocy, ocz, dims = win[i, tt]
            gx = np.arange(tc[0] * TILE[0], min(N3[0], (tc[0] + 1) * TILE[0]))
            gy = np.arange(tc[1] * TILE[1], min(N3[1], (tc[1] + 1) * TILE[1]))
            gz = np.arange(tc[2] * TILE[2], min(N3[2], (tc[2] + 1) * TILE[2]))
            nodes = ((gz[:, None, None] * N3[1] + gy[None, :, None]) * N3[0] + gx[None, None, :]).reshape(-1)
            if dims == 0:
                out[i, nodes] = direct[i, nodes]
                continue
            staged += 1
            wx, wy, wz = dims & 1023, (dims >> 10) & 1023, dims >> 20
            k = np.arange(wx * wy * wz)
            x, y, z = k % wx, (k // wx) % wy, k // (wx * wy)
            # the kernel wraps a window node with one subtraction of N per axis
            wrapped = []
            for a, (o, v) in enumerate(((ocx, x), (ocy, y), (ocz, z))):
                u = o * p + v
                assert u.max() < 2 * N3[a]
                wrapped.append(np.where(u >= N3[a], u - N3[a], u))
            src = (wrapped[2] * N3[1] + wrapped[1]) * N3[0] + wrapped[0]
            lf = f[i, src]
            c = cell[i, nodes]
            ex, ey, ez = c % ne[0], (c // ne[0]) % ne[1], c // (ne[0] * ne[1])
            bx, by, bz = (ex - ocx) % ne[0], (ey - ocy) % ne[1], (ez - ocz) % ne[2]
            acc = np.zeros(nodes.size)
            for kz in range(p + 1):
                for ky in range(p + 1):
                    base = ((bz * p + kz) * wy + by * p + ky) * wx + bx * p
                    assert base.min() >= 0 and (base + p).max() < wx * wy * wz
                    for kx in range(p + 1):
                        acc += (wl[0][nodes, kx] * wl[1][nodes, ky] * wl[2][nodes, kz]) * lf[base + kx]
            out[i, nodes] = acc
    return out, staged


@pytest.mark.parametrize("p,n_el,dt,max_nodes,amp", [(2, (3, 4, 2), 0.31, 3072, 1.0), (3, (5, 3, 2), 0.8, 3072, 1.0),
                                                      (4, (3, 4, 3), 0.5, 3072, 1.0), (4, (4, 3, 2), 2.5, 3072, 1.0),
                                                      (4, (3, 4, 3), 0.5, 800, 1.0), (6, (2, 2, 2), 0.4, 3072, 1.5)])
def test_staged_windows_reproduce_oracle_streaming(oracle, driver, p, n_el, dt, max_nodes, amp):
    """The source windows of the staged distorted-mesh streaming (node tiles
    of 8 x 8 x 4): every departure stencil of a tile lies inside its window,
    gathering through the window gives the oracle's streaming, and blocks
    whose window exceeds the budget fall back to the direct gather."""
    L = (2 * math.pi, 2 * math.pi, 2 * math.pi)
    cfg0 = oracle.make_cfg(n_el, p, dt, 0.01)
    xs, ys, zs = oracle.node_coords(cfg0)
    Z, Y, X = (v.reshape(-1) for v in np.meshgrid(zs, ys, xs, indexing="ij"))
    disp = amp * np.stack([0.2 * np.sin(Y + 0.5 * Z), 0.15 * np.cos(X) * np.sin(Z), 0.1 * np.sin(X + Y)])
    cfg = oracle.make_cfg(n_el, p, dt, 0.01, disp=disp)
    r = _run(driver, p, n_el, L, dt, disp, max_nodes)
    assert r.returncode == 0, r.stdout[:200] + r.stderr
    vals = r.stdout.split()
    N = X.size
    cell = np.array(vals[:Q * N], dtype=np.int64).reshape(Q, N)
    t = np.array(vals[Q * N:4 * Q * N], dtype=np.float64).reshape(3, Q, N)
    largest = int(vals[4 * Q * N + N])
    win = np.array(vals[4 * Q * N + N + 1:], dtype=np.int64).reshape(Q, -1, 4)
    dims = win[:, :, 3]
    sizes = (dims & 1023) * ((dims >> 10) & 1023) * (dims >> 20)
    assert largest == sizes.max() and sizes.max() <= max_nodes
    f = np.random.default_rng(p + n_el[0]).normal(size=(Q, N))
    ref, _ = oracle.stream(cfg, f, f)
    got, staged = _window_gather(oracle, cfg, cell, t, win, f)
    assert staged > 0
    if max_nodes == 800 or p == 6:
        assert (dims == 0).any()                    # some blocks take the direct gather
    assert np.max(np.abs(got - ref)) < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n_el,p,dt,max_nodes,mixed", [((6, 6, 5), 4, 0.8, 3072, True), ((6, 6, 5), 4, 0.8, 6144, True),
                                                       ((5, 6, 4), 3, 0.5, 3072, False)])
def test_window_mix_of_gpu_staged_cases(oracle, driver, n_el, p, dt, max_nodes, mixed):
    """The grids of the GPU staged-streaming parity test use the windows as
    stated there: a mixture of staged and global-gather blocks at the FP64
    (3072 nodes) and FP32 (6144 nodes) budgets, or every block staged."""
    L = (2 * math.pi,) * 3
    cfg0 = oracle.make_cfg(n_el, p, dt, 0.01)
    xs, ys, zs = oracle.node_coords(cfg0)
    Z, Y, X = (v.reshape(-1) for v in np.meshgrid(zs, ys, xs, indexing="ij"))
    disp = np.stack([0.2 * np.sin(Y + 0.5 * Z), 0.15 * np.cos(X) * np.sin(Z), 0.1 * np.sin(X + Y)])
    r = _run(driver, p, n_el, L, dt, disp, max_nodes)
    assert r.returncode == 0, r.stdout[:200] + r.stderr
    vals = r.stdout.split()
    N = X.size
    win = np.array(vals[4 * Q * N + N + 1:], dtype=np.int64).reshape(Q, -1, 4)
    staged = int((win[:, :, 3] != 0).sum())
    total = win.shape[0] * win.shape[1]
    if mixed:
        assert 0 < staged < total, (staged, total)
    else:
        assert staged == total, (staged, total)
