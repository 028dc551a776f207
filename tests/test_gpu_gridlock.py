"""The gridlock detector (failure detection: no vehicle on the network moved
for a run of steps, reported in the metrics): a road held at red fills and
freezes, the run of stalled steps grows step by step and ends when the light
turns green; a free-flowing grid never stalls."""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import line_network, trips_for

pytestmark = pytest.mark.gpu


def test_red_road_stalls_then_releases():
    from paper_2406_10661_amd.tsim import Sim
    net = line_network(lanes=1)
    n = 60
    trips = trips_for([[0, 2]] * n, depart=np.arange(n, dtype=np.float32) * 2.0)
    g = Sim(net, trips, W.Params())
    # junction 1 held on its second phase (road 3's approach): road 0 stays red
    g.set_signal_phases([1], [1])
    g.step(600)
    m = g.metrics()
    assert m["n_active"] > 20 and m["n_waiting"] > 0 and m["n_finished"] == 0
    s1 = m["stalled_steps"]
    assert s1 > 50 and m["max_stalled_steps"] == s1
    g.step(10)
    assert g.metrics()["stalled_steps"] == s1 + 10
    g.set_signal_phases([1], [0])
    g.step(5)
    m = g.metrics()
    assert m["stalled_steps"] == 0 and m["max_stalled_steps"] >= s1 + 10


def test_free_flow_never_stalls_for_long():
    from paper_2406_10661_amd.tsim import Sim
    w = W.config1()
    g = Sim(w.network, w.trips, w.params)
    g.step(w.n_steps)
    m = g.metrics()
    # at most a red phase (30 s) with every vehicle queued at a light
    assert m["max_stalled_steps"] < 30 and m["errors"] == 0


def test_batch_instances_stall_on_their_own():
    """In a batch, the instance held at red stalls and the one on its fixed
    plan stalls at most for about a red phase."""
    from paper_2406_10661_amd.tsim import Batch
    net = line_network(lanes=1)
    n = 60
    trips = trips_for([[0, 2]] * n, depart=np.arange(n, dtype=np.float32) * 2.0)
    b = Batch([net, net], [trips, trips], [W.Params(), W.Params()])
    b.set_signal_phases(0, [1], [1])
    b.step(600)
    m0, m1 = b.metrics(0), b.metrics(1)
    assert m0["stalled_steps"] > 50
    assert m1["max_stalled_steps"] < 35
