"""Scenario pins of the oracle's step (IDM + integration + lookahead +
transfer + signals + lane groups), each against a fact fixed by the model:

  * ring road: N equal vehicles equally spaced at the IDM equilibrium speed of
    that spacing stay there exactly (uniform flow is a fixed point of the
    ballistic update when a = 0), across the lane boundary and lookahead;
  * ring road from rest with unequal spacing relaxes to the uniform
    equilibrium speed of the mean spacing;
  * a lone vehicle before a permanently red signal stops s0 before the lane
    end and never enters the junction lane (stop rule, Appendix B.3);
  * a vehicle in the lane that does not reach its next road changes into the
    lane group and completes the turn (lane-group rule, Appendix B.3);
  * free-road speed follows v' = v + a dt with the free-road IDM until v0.
"""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import (line_network, left_turn_network, trips_for, state_from, ring_state, ring_coords,
                          v_equilibrium)

P = W.Params()


def test_ring_uniform_flow_is_fixed_point(oracle_lib):
    net, trips = W.ring_road(circumference_road=275.0, n_vehicles=10, laps=40)
    C = 275.0 + 25.0
    n = 10
    spacing = C / n
    v = v_equilibrium(spacing - 5.0, float(np.float32(13.9)))
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(ring_state(net, n, np.arange(n) * spacing + 3.0, v))
    s_prev = ring_coords(net, o.get_state())
    for t in range(120):
        o.step(1)
        st = o.get_state()
        assert np.all(st["status"] == 1)
        np.testing.assert_allclose(st["v"], v, rtol=0, atol=1e-9)
        s = ring_coords(net, st)
        adv = (s - s_prev) % C
        np.testing.assert_allclose(adv, v * P.dt, atol=1e-8)
        s_prev = s
    assert o.metrics()["transfers"] > 0


def test_ring_relaxes_to_equilibrium(oracle_lib):
    net, trips = W.ring_road(circumference_road=275.0, n_vehicles=10, laps=400)
    C, n = 300.0, 10
    rng = np.random.default_rng(3)
    pos = np.sort(rng.uniform(0, C - 8 * n, n)) + np.arange(n) * 8.0
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(ring_state(net, n, pos, 0.0))
    o.step(3000)
    st = o.get_state()
    v = v_equilibrium(C / n - 5.0, float(np.float32(13.9)))
    np.testing.assert_allclose(st["v"], v, atol=1e-3)


def test_red_light_stop(oracle_lib):
    net = line_network(lanes=1)
    # road 0 (J0->J1) continues into road 2 (J1->J2)
    trips = trips_for([[0, 2]])
    o = oracle_lib.OracleSim(net, trips, P)
    j1 = 1
    ph_begin = net.junc_phase_begin
    # find the phase of J1 that does NOT green road 0's movement
    rol = net.road_of_lane()
    road0_jl = [q for q in range(net.n_jlanes) if rol[net.jl_in_lane[q]] == 0]
    other = None
    for p in range(ph_begin[j1 + 1] - ph_begin[j1]):
        g = net.phase_green_jl[net.phase_green_begin[ph_begin[j1] + p]:net.phase_green_begin[ph_begin[j1] + p + 1]]
        if not set(road0_jl) & set(g.tolist()):
            other = p
    assert other is not None
    o.set_signal_phases([j1], [other])
    o.set_state(state_from(1, [0], [0.0], [12.0]))
    L = float(net.road_length[0])
    for t in range(400):
        o.step(1)
        st = o.get_state()
        assert st["lane"][0] == 0, "entered the junction on red"
        assert st["x"][0] <= L
    assert st["x"][0] == pytest.approx(L - P.s0, abs=0.05)
    assert st["v"][0] == pytest.approx(0.0, abs=1e-3)


def test_wrong_lane_vehicle_merges_and_turns(oracle_lib):
    net = left_turn_network(lanes=2, policy=W.POLICY_NONE)
    # road 0 = J0->J1, left turn into road 2 = J1->J2 from lane 0 only
    trips = trips_for([[0, 2]])
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(state_from(1, [1], [0.0], [10.0]))
    changed = False
    for t in range(200):
        o.step(1)
        st = o.get_state()
        if st["status"][0] == 2:
            break
        if st["lane"][0] == 0:
            changed = True
    assert changed
    assert st["status"][0] == 2


def test_free_road_acceleration(oracle_lib):
    net = line_network(lanes=1, length=2000.0, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]])
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(state_from(1, [0], [0.0], [0.0]))
    v = 0.0
    for t in range(20):
        o.step(1)
        a = P.a_max * (1 - (v / float(np.float32(13.9))) ** 4)
        v = v + a * P.dt
        assert o.get_state()["v"][0] == pytest.approx(v, abs=1e-12)
