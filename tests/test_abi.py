"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol declared in include/sllbm.h, validates configurations before
touching a device, and returns the same velocity set as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sllbm.h")).read()
    return sorted(set(re.findall(r"\b(sllbm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2012_05537_amd import sllbm
    return sllbm.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    from paper_2012_05537_amd import sllbm
    assert sorted(sllbm.EXPORTED) == names


def test_velocity_set_matches_oracle(oracle):
    from paper_2012_05537_amd import sllbm
    xi, w = sllbm.velocity_set()
    xo, wo = oracle.velocity_set()
    assert np.allclose(xi.numpy(), xo, rtol=0, atol=1e-15)
    assert np.allclose(w.numpy(), wo, rtol=0, atol=1e-17)


def test_two_dimensional_lattice_matches_oracle():
    from oracle import oracle2d
    from paper_2012_05537_amd import sllbm
    xi, w = sllbm.lattice(sllbm.D2Q19)
    xo, wo = oracle2d.velocity_set()
    assert xi.shape == (19, 3) and np.all(xi[:, 2].numpy() == 0)
    # same values to a few ulp (the oracle evaluates cos/sin of the ring angles)
    assert np.allclose(xi[:, :2].numpy(), xo, rtol=0, atol=4e-15)
    assert np.allclose(w.numpy(), wo, rtol=1e-15, atol=0)
    x3, w3 = sllbm.lattice(sllbm.D3Q45)
    assert x3.shape == (45, 3)
    with pytest.raises(ValueError):
        sllbm.lattice(27)


def _cfg(**kw):
    from paper_2012_05537_amd.sllbm import Config
    c = Config()
    c.n_el[:] = [2, 2, 2]
    c.order = 2
    c.velocity_set = 45
    c.viscosity_law = 0
    c.precision = 0
    c.device = 0
    c.length[:] = [1.0, 1.0, 1.0]
    c.dt = 0.1
    c.gamma = 1.4
    c.prandtl = 0.71
    c.mu_inf = 0.01
    for k, v in kw.items():
        if k in ("n_el", "length"):
            getattr(c, k)[:] = v
        else:
            setattr(c, k, v)
    return c


@pytest.mark.parametrize("bad", [
    dict(order=0), dict(order=7), dict(n_el=[0, 2, 2]), dict(length=[1.0, -1.0, 1.0]), dict(dt=0.0),
    dict(dt=float("nan")), dict(gamma=1.0), dict(prandtl=0.0), dict(mu_inf=-1.0), dict(velocity_set=27),
    dict(viscosity_law=5), dict(precision=3), dict(n_el=[1 << 20, 2, 2]),
])
def test_invalid_config_is_rejected(lib, bad):
    h = ctypes.c_void_p()
    rc = lib.sllbm_create(ctypes.byref(_cfg(**bad)), ctypes.byref(h))
    assert rc == 1                       # SLLBM_EINVAL
    assert h.value is None
    assert len(lib.sllbm_last_error(None)) > 0


@pytest.mark.parametrize("bad", [dict(n_el=[4, 4, 2]), dict(n_el=[0, 4, 1]), dict(length=[1.0, 0.0, 1.0])])
def test_invalid_two_dimensional_config_is_rejected(lib, bad):
    h = ctypes.c_void_p()
    rc = lib.sllbm_create(ctypes.byref(_cfg(velocity_set=19, **bad)), ctypes.byref(h))
    assert rc == 1 and h.value is None


def test_two_dimensional_config_ignores_z_length(lib):
    """A valid 2-D configuration passes validation (no device here: EDEVICE)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    rc = lib.sllbm_create(ctypes.byref(_cfg(velocity_set=19, n_el=[4, 3, 1], length=[1.0, 0.75, 0.0])),
                          ctypes.byref(h))
    assert rc == 3 and h.value is None


def test_null_arguments(lib):
    assert lib.sllbm_create(None, None) == 1
    assert lib.sllbm_destroy(None) == 0
    assert lib.sllbm_num_nodes(None) == -1
    assert lib.sllbm_step(None, 1) == 1
    assert lib.sllbm_velocity_set(None, None) == 1
    assert lib.sllbm_lattice(19, None, None) == -1


def test_missing_library_fails_loudly(tmp_path):
    """The binding has no fallback: a missing libsllbm.so is an error."""
    import paper_2012_05537_amd.sllbm as S
    saved = S._lib
    try:
        S._lib = None
        with pytest.raises(RuntimeError):
            S.load_library(str(tmp_path / "libsllbm.so"))
    finally:
        S._lib = saved


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with a message."""
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_baseline_times_all_cores_then_one():
    """bench.py's cpu_baseline (the oracle on the host; no GPU): the all-core
    and one-core rates, the thread count it used, and the oracle's OpenMP
    thread count restored afterwards."""
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    from oracle import oracle as O
    from paper_2012_05537_amd import inputs
    before = O._lib().omp_get_max_threads()
    r = bench.cpu_baseline(inputs.workload("c1"), 0.2)
    assert r["kind"] == "oracle" and r["unit"] == "node-updates/s"
    assert r["value"] > 0 and r["value_one_core"] > 0
    assert r["cores"] == before
    assert O._lib().omp_get_max_threads() == before
