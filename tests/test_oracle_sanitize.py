"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host,
no GPU): tests/host/oracle_sanitize.c includes the oracle source and calls
every exported operation on small grids (orders 1..6, ragged and one-cell
axes, shifts of several cells, graded and distorted cells), in the real and
in the complex-step build.  Any invalid access or undefined operation aborts
the driver."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("build", ["real", "complex"])
def test_oracle_clean_under_address_and_ub_sanitizers(build):
    src = os.path.join(ROOT, "tests", "host", "oracle_sanitize.c")
    extra = ["-DORACLE_COMPLEX"] if build == "complex" else []
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitize")
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-g", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *extra,
                               src, "-o", exe, "-lm"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0, out.stdout[-3000:] + out.stderr[-3000:]
    assert "ALL OK" in out.stdout
