"""Host logic of the graded-mesh tables (no GPU): compiles a small driver
against the library's table builder (csrc/tables.cpp) and checks that the
transposed per-node rows are the exact transpose of the forward rows."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_transposed_node_tables_are_exact_transposes():
    csrc = os.path.join(ROOT, "paper_2012_05537_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tables_check")
        subprocess.check_call([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                               "-I", os.path.join(ROOT, "include"), "-I", csrc,
                               os.path.join(ROOT, "tests", "host", "tables_check.cpp"),
                               os.path.join(csrc, "tables.cpp"), "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "max |S^T - T| = 0.000e+00" in out.stdout, out.stdout
