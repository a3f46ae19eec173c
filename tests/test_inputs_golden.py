"""The 2-D workload recipes against the initial states the paper prints
(tests/golden/paper_initial_states.json: Sec. III A shock tube, Sec. III B
Riemann case 12)."""
import json
import os

import numpy as np
import pytest

from paper_2012_05537_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_initial_states.json")


@pytest.fixture(scope="module")
def golden():
    return json.load(open(GOLDEN))


def test_sod_states(golden):
    g = golden["sod"]
    (ri, ui, pi), (ro, uo, po) = inputs.SOD_STATES
    assert (ri, ui, pi) == (g["left"]["rho"], g["left"]["u"], g["left"]["P"])
    assert (ro, uo, po) == (g["right"]["rho"], g["right"]["u"], g["right"]["P"])
    w = inputs.WORKLOADS_2D["sod"]
    # the paper's coarse tube: 100 cells of order 4 on [0, 1]; the periodic stand-in doubles it
    assert w["n_el"][0] == 2 * g["cells_coarse"] and w["length"][0] == 2.0 and w["p"] == g["order_coarse"]
    assert w["dt"] == g["dt_coarse_small_step"] and w["mu_inf"] == g["mu_coarse_small_step"]
    x = np.linspace(0, 2, 41)[:-1]
    rho, u, T = inputs.sod_fields(x, np.array([0.0]))
    assert np.all(rho[(x > 0.5) & (x < 1.5)] == ri) and np.all(rho[(x < 0.5) | (x > 1.5)] == ro)
    assert np.allclose(rho * T, np.where((x > 0.5) & (x < 1.5), pi, po))


def test_riemann_case12_states(golden):
    g = golden["riemann_case12"]
    for q in ("ne", "nw", "sw", "se"):
        assert tuple(inputs.RIEMANN12[q]) == tuple(g[q]), q
    w = inputs.WORKLOADS_2D["riemann"]
    assert w["n_el"] == (g["cells"], g["cells"]) and w["p"] == g["order"] and w["gamma"] == g["gamma"]
    assert w["steps"] * w["dt"] == pytest.approx(g["t_end"])
    x = np.array([0.25, 0.75])
    rho, u, T = inputs.riemann_fields(x, x)
    # node order: y slowest; (x, y) = (0.25, 0.25) sw, (0.75, 0.25) se, (0.25, 0.75) nw, (0.75, 0.75) ne
    for k, q in enumerate(("sw", "se", "nw", "ne")):
        r, ux, uy, p = g[q]
        assert rho[k] == r and u[0, k] == ux and u[1, k] == uy and rho[k] * T[k] == pytest.approx(p)
