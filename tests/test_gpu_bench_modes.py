"""bench.py in each of its measurement modes (a few steps each): one JSON
line with the contract's fields, a positive finite value and a roofline
entry for the dominant kernel."""
import json
import os
import subprocess
import sys

import pytest

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("args,kernel,metric", [
    (["--mesh", "graded"], "k_stream_graded", "node-updates/s (D3V45 f+g)"),
    (["--mesh", "distorted"], "k_stream_mapped", "node-updates/s (D3V45 f+g)"),
    (["--workload", "riemann"], None, "node-updates/s (D2V19 f+g)"),
    (["--workload", "sod", "--precision", "fp32"], None, "node-updates/s (D2V19 f+g)"),
])
def test_bench_mode(args, kernel, metric):
    require_gpu()
    print("bench", args, flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args, "--steps", "3", "--warmup", "1",
                        "--reps", "1", "--no-secondary", "--no-cpu-baseline", "--adjoint-workload", "none"],
                       capture_output=True, text=True, timeout=200)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["metric"] == metric and d["value"] > 0 and d["finite"]
    assert d["roofline"]["bound"] == "hbm" and 0 < d["roofline"]["frac"] < 1
    if kernel:
        assert d["roofline"]["kernel"] == kernel


def test_bench_default_headline_and_secondary_lines():
    """The default run: the 256^3-node FP64 headline, the FP32-mixed line on
    the same grid, and FP64 lines on the 64^3- and 128^3-node grids, the
    graded and distorted meshes and the 2-D workload, each a median of
    repetitions."""
    require_gpu()
    print("bench default (256^3 nodes, fp64 + fp32 + c2)", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
                        "--reps", "3", "--no-cpu-baseline", "--adjoint-workload", "none"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert d["config"]["nodes"] == 256 ** 3 and d["dtype"] == "f64"
    assert len(d["ms_per_step_reps"]) == 3 and d["ms_per_step"] in d["ms_per_step_reps"]
    assert d["fp32_mixed"]["nodes"] == 256 ** 3 and d["fp32_mixed"]["dtype"].startswith("f32")
    assert d["c2_fp64"]["nodes"] == 64 ** 3
    assert d["c3_fp64"]["nodes"] == 128 ** 3
    assert d["c2_graded_fp64"]["roofline"]["kernel"] == "k_stream_graded"
    assert d["c2_distorted_fp64"]["roofline"]["kernel"] == "k_stream_mapped"
    assert d["riemann_fp64"]["roofline"]["kernel"] in ("k_stream_y", "k_collide")
    assert d["fp32_over_fp64"] > 1.0
    for line in (d, d["fp32_mixed"], d["c2_fp64"], d["c3_fp64"], d["c2_graded_fp64"], d["c2_distorted_fp64"],
                 d["riemann_fp64"]):
        assert 0 < line["roofline"]["frac"] < 1 and 0 < line["roofline"]["step_frac"] < 1
        assert line["roofline"]["copy_GBps"] > 0 and line["roofline"]["frac_of_copy"] > 0


@pytest.mark.parametrize("mesh", ["graded", "distorted"])
def test_bench_adjoint_on_mesh(mesh):
    """The rollout-gradient timing follows the mesh of the bench line."""
    require_gpu()
    print("bench adjoint on", mesh, flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mesh", mesh, "--steps", "2", "--warmup", "1",
                        "--reps", "1", "--no-secondary", "--no-cpu-baseline", "--adjoint-workload", "c4",
                        "--adjoint-steps", "6"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads([l for l in r.stdout.splitlines() if l.strip()][-1])
    a = d["adjoint"]
    assert a["workload"].startswith(f"c4-{mesh}:") and a["grad_finite"]
    assert a["forward_s"] > 0 and a["backward_s"] > 0
