"""Horizon parity against the oracle's stored results (tests/golden/
horizon_*.json, written by tests/golden/make_horizon_goldens.py, which calls
only the oracle): over a whole horizon, completed trips and the
time-averaged mean road speed of the GPU run agree within 1%.

  * C2: the 32x32 jittered grid with 100,000 vehicles, 3,600 steps from t = 0
    (bench launch configuration: fused schedule, 60-step graphs);
  * C3: the 2,464,950-vehicle city, 50 steps from a seeded synthetic state at
    t = 3,600 s (the trips completed within the window are compared).
"""

import json
import os

import pytest

from paper_2406_10661_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    with open(os.path.join(HERE, "golden", f"horizon_{name}.json")) as f:
        return json.load(f)


def within(a, b, rel=0.01):
    return abs(a - b) <= rel * abs(b)


@pytest.mark.timeout(900)
def test_c2_horizon_matches_oracle():
    from paper_2406_10661_amd.tsim import Sim
    g = golden("c2")
    w = W.config2()
    assert g["workload"] == w.name and g["steps"] == w.n_steps
    sim = Sim(w.network, w.trips, w.params)
    sim.set_graph_steps(60)
    sim.step(w.n_steps)
    m = sim.metrics()
    o = g["oracle"]
    print("c2 horizon gpu", m["n_finished"], m["mean_speed_avg"], "oracle", o["finished"], o["mean_speed_avg"],
          flush=True)
    assert m["errors"] == 0 and m["step"] == w.n_steps
    assert within(m["n_finished"], o["finished"])
    assert within(m["mean_speed_avg"], o["mean_speed_avg"])


@pytest.mark.timeout(900)
def test_c3_window_matches_oracle():
    from paper_2406_10661_amd.tsim import Sim
    g = golden("c3")
    w = W.config3()
    assert g["workload"] == w.name
    st = W.synthetic_state(w.network, w.trips, g["from_step"], seed=g["state_seed"], p_active=g["p_active"])
    assert int((st["status"] == 1).sum()) == g["active_at_start"]
    sim = Sim(w.network, w.trips, w.params)
    sim.set_state(st)
    m0 = sim.metrics()
    sim.step(g["steps"])
    m = sim.metrics()
    o = g["oracle"]
    done_gpu = m["n_finished"] - m0["n_finished"]
    done_ora = o["finished"] - g["finished_at_start"]
    print("c3 window gpu", done_gpu, m["mean_speed_avg"], "oracle", done_ora, o["mean_speed_avg"], flush=True)
    assert m["errors"] == 0
    assert within(done_gpu, done_ora)
    assert within(m["mean_speed_avg"], o["mean_speed_avg"])
