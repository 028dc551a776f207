"""Invariants I1-I7 after every oracle step on seeded small networks, and the
closed-form fixed-time signal schedule (Section 3.2 FIXED_TIME / MANUAL /
NONE)."""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests import simcheck as S


def _grid_workload(seed, n=3, n_veh=400, horizon=200.0):
    rng = np.random.default_rng(seed)
    net = W.grid_network(n, spacing=250.0, jitter=20.0, rng=rng, random_edges=True)
    o, d = W.uniform_od(net, rng, n_veh)
    dep = rng.uniform(0, horizon, n_veh)
    trips = W._finish_trips(net, rng, o, d, dep)
    return net, trips, W.Params(seed=seed)


def _run_checked(oracle_lib, net, trips, params, steps, manual_every=0, rng=None):
    info = S.NetInfo(net, trips)
    o = oracle_lib.OracleSim(net, trips, params)
    policy = net.junc_policy.copy()
    manual = np.zeros(net.n_junctions, np.int32)
    prev = o.get_state()
    seen = dict(changes=0, transfers=0, finished=0)
    for t in range(steps):
        if manual_every and t % manual_every == 0:
            nph = np.diff(net.junc_phase_begin)
            js = np.arange(net.n_junctions)[::2]
            ph = (rng.integers(0, 1 << 30, js.size) % nph[js]).astype(np.int32)
            o.set_signal_phases(js, ph)
            policy[js] = W.POLICY_MANUAL
            manual[js] = ph
        green = S.green_set(net, t, params.dt, policy, manual)
        o.step(1)
        assert np.array_equal(o.green().astype(bool), green), f"signals differ at step {t}"
        cur = o.get_state()
        errs = S.check_state(info, cur) + S.check_transition(info, prev, cur, green)
        assert not errs, (t, errs)
        prev = cur
    m = o.metrics()
    assert m["waiting"] + m["active"] + m["finished"] == trips.n_vehicles
    return m


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_invariants_random_grids(oracle_lib, seed):
    net, trips, params = _grid_workload(seed)
    m = _run_checked(oracle_lib, net, trips, params, 300)
    assert m["lane_changes"] > 0 and m["transfers"] > 0 and m["finished"] > 0


def test_invariants_config1_with_manual_signals(oracle_lib):
    w = W.config1()
    m = _run_checked(oracle_lib, w.network, w.trips, w.params, 400, manual_every=15,
                     rng=np.random.default_rng(9))
    assert m["finished"] > 50


def test_fixed_time_schedule_closed_form():
    d = np.array([30.0, 15.0, 45.0], np.float32)
    # cycle 90 s: [0,30) -> 0, [30,45) -> 1, [45,90) -> 2
    expect = {0: 0, 29: 0, 30: 1, 44: 1, 45: 2, 89: 2, 90: 0, 120: 1, 179: 2, 180: 0}
    for t, p in expect.items():
        assert S.fixed_time_phase(d, t, 1.0) == p


def test_oracle_signals_follow_schedule(oracle_lib):
    w = W.config1()
    net = w.network
    o = oracle_lib.OracleSim(net, w.trips, w.params)
    for t in range(0, 260):
        g = S.green_set(net, t, 1.0)
        o.step(1)
        assert np.array_equal(o.green().astype(bool), g)
    # a junction set to NONE is all green
    o.set_policy([5], [W.POLICY_NONE])
    o.step(1)
    jj = net.road_to[net.road_of_lane()[net.jl_in_lane]]
    assert o.green()[jj == 5].all()
