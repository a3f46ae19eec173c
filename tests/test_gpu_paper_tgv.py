"""The paper's own Taylor-Green setting (Sec. III C: Re 1600, Ma 1.25,
dt 0.009 in its convective units, p = 4) on the GPU.

The paper reports this run as stable to t = 20 without filtering; these tests
pin that it stays finite here too, with the conserved totals drifting only at
the level of the streaming's non-conservation on GLC nodes, and that the
kinetic energy and solenoidal dissipation follow the decay the paper shows
(energy down to about a fifth at t = 20, dissipation peaking near t = 10).
The bands are this implementation's measured values widened by a margin;
the paper's curves are figures without data, so they are not a reference."""
import math

import pytest

from paper_2012_05537_amd import tgv


@pytest.mark.gpu
def test_re1600_ma125_runs_to_t20_on_32_cubed_cells():
    print("paper TGV: Re 1600 Ma 1.25 dt 0.009, 32^3 cells p=4, 2222 steps", flush=True)
    recs = tgv.run("re1600_ma125", n_el=32, every=100)
    samples = [r for r in recs if r["kind"] == "sample"]
    assert all(r["finite"] for r in samples)
    last = samples[-1]
    assert last["step"] == 2222 and abs(last["t"] - 20.0) < 0.01
    assert abs(last["drift_mass"]) < 3e-3 and abs(last["drift_energy"]) < 5e-3
    assert max(abs(m) for m in last["momentum"]) < 1e-12
    assert 0.15 < last["Ek_ratio"] < 0.26
    peak = max(samples, key=lambda r: r["eps_s"])
    assert 7.0 < peak["t"] < 14.0 and 0.007 < peak["eps_s"] < 0.014
    # the energy decays monotonically after the early compressible transient
    late = [r["Ek_ratio"] for r in samples if r["t"] > 5.0]
    assert all(b < a for a, b in zip(late, late[1:]))


@pytest.mark.gpu
def test_re1600_ma125_first_steps_on_256_cubed_nodes():
    """The paper's grid (64^3 cells, 256^3 nodes): 200 steps in FP64 with the
    FP32-mixed run and a one-ulp-perturbed FP64 run beside it."""
    print("paper TGV: Re 1600 Ma 1.25 dt 0.009, 64^3 cells p=4, 200 steps, FP64 + FP32 + 1-ulp", flush=True)
    recs = tgv.run("re1600_ma125", compare=True, steps=200, every=100)
    samples = [r for r in recs if r["kind"] == "sample"]
    assert [r["step"] for r in samples] == [0, 100, 200]
    assert all(r["finite"] for r in samples)
    for r in samples[1:]:
        assert abs(r["drift_mass"]) < 1e-4 and abs(r["drift_energy"]) < 1e-4
        floor = r["err_fp64_ulp"]
        assert max(floor.values()) < 1e-13
    e100 = samples[1]["err_fp32_mixed"]
    assert max(e100.values()) < 1e-5, e100
    assert math.isclose(samples[0]["Ek_ratio"], 1.0)
