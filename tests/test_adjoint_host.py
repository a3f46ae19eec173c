"""Host logic of the checkpointed adjoint (no GPU): segment schedule and the
resident-memory arithmetic of the checkpoint plans."""
import math

import pytest

from paper_2012_05537_amd.adjoint import segment_bounds


@pytest.mark.parametrize("n,ck", [(50, 10), (10, 3), (10, 1), (10, 10), (7, 100), (200, "sqrt"), (1, "sqrt"),
                                  (0, 5), (17, "sqrt")])
def test_segments_cover_steps(n, ck):
    segs = segment_bounds(n, ck)
    assert all(s1 > s0 for s0, s1 in segs)
    covered = [k for s0, s1 in segs for k in range(s0, s1)]
    assert covered == list(range(n))
    if n:
        k = max(1, math.ceil(math.sqrt(n))) if ck == "sqrt" else ck
        assert all(s1 - s0 <= k for s0, s1 in segs)
        assert len(segs) == math.ceil(n / k)


def test_sqrt_plan_c5_fits_hbm():
    """256^3 nodes in FP32: ceil(sqrt(200)) = 15-step segments; checkpoints plus
    one segment's recorded states plus the working buffers stay below 288 GB."""
    n = 200
    segs = segment_bounds(n, "sqrt")
    state = 2 * 45 * 256 ** 3 * 4
    seg_max = max(s1 - s0 for s0, s1 in segs)
    resident = len(segs) * state + (seg_max - 1) * state + 4 * state
    assert len(segs) == 14 and seg_max == 15
    assert resident < 288e9


def test_bad_checkpoint():
    with pytest.raises(ValueError):
        segment_bounds(10, 0)
    with pytest.raises(ValueError):
        segment_bounds(-1, 3)
