"""Hand-derived pins of the oracle's departures, merge priority, metrics and
cooperative yielding.

Each test builds a scene of a few vehicles whose outcome follows from the
rule as the paper states it (or the reading recorded beside the rule) by
arithmetic that can be checked by eye, and names the plausible mistake it
catches:

  departures (Appendix B.2, prepare stream 3 / update stream 3: due vehicles
  enter their origin road when the connection is safe)
    * the lane with the most room behind its rearmost vehicle is taken
      (mistake: the least room);
    * room exactly s0 enters, a hair less waits (mistake: > instead of >=);
    * a departure time equal to t dt departs at step t, a later one waits
      (mistake: < instead of <=);
    * one insertion per lane per step (mistake: two heads into one lane);
    * the first head that cannot enter stops its road's queue (mistake:
      skipping past it);
    * a feeder junction lane's front vehicle that can reach the entrant's
      rear blocks the departure, exactly at the boundary reach = -L it does
      not (mistake: ignoring feeders, or a strict comparison);
  merges (junction conflicts are not modelled, Appendix B table of omitted
  features; reading: static priority by junction-lane id)
    * with two feeders able to cross, the higher-id one waits at its lane
      end with v' = 0 and one feeder block is counted; when the lower-id
      front cannot cross, the higher-id one enters (mistake: reversed
      priority, or blocking on any feeder);
  metrics (Section 3.3)
    * travelling time of a trip ending in step t is (t + 1) dt - tau
      (mistake: t dt - tau);
    * network mean speed averages road-lane vehicles only, and its horizon
      average skips steps without any (mistake: counting those as 0, or
      including junction lanes);
    * lane queue length counts the vehicles waiting at the end of the lane:
      the run of stopped vehicles from the lane front (mistake: every slow
      vehicle on the lane);
  cooperative yielding (reading: a lane keeper behind a merging vehicle's
  rear takes it as its leader)
    * a keeper at rest s0 behind a stopped merger's rear stays at rest
      (mistake: keeper ignores the merger and accelerates freely);
    * a fast keeper is bounded by the merger's rear and takes its speed.
"""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import jl_between, left_turn_network, line_network, merge_network, state_from, trips_for

P = W.Params()
LIM = float(np.float32(13.9))   # every scene's speed limit as the oracle reads it


def _state(n, lanes, xs, vs, status, route_pos=None, step=0):
    st = state_from(n, lanes, xs, vs, route_pos=route_pos, step=step, status=status)
    st["lane"] = np.where(st["status"] == 1, st["lane"], -1).astype(np.int32)
    return st


def _sim(oracle_lib, net, trips, st):
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(st)
    return o


# ------------------------------------------------------------------ departures

def test_departure_takes_the_lane_with_most_room(oracle_lib):
    net = line_network(lanes=3, policy=W.POLICY_NONE)
    # three vehicles on road 0 with rear bumpers at 25, 45 and 35 m; vehicle 3
    # is due at t = 0 on the same road (all three lanes lead on to road 2)
    trips = trips_for([[0, 2]] * 4)
    st = _state(4, [0, 1, 2, -1], [30.0, 50.0, 40.0, 0.0], [0.0, 0.0, 0.0, 0.0], [1, 1, 1, 0])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    assert s["status"][3] == 1 and s["lane"][3] == 1
    assert o.metrics()["departures"] == 1


@pytest.mark.parametrize("x_rear_vehicle,departs", [(7.0, True), (7.0 - 1e-6, False)])
def test_departure_needs_room_of_s0(oracle_lib, x_rear_vehicle, departs):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2], [0, 2]])
    # vehicle 0's rear at x - L = 2 m = s0 (exactly, or just below)
    st = _state(2, [0, -1], [x_rear_vehicle, 0.0], [0.0, 0.0], [1, 0])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    assert (s["status"][1] == 1) == departs
    if departs:
        assert s["lane"][1] == 0 and s["x"][1] == 0.0 and s["v"][1] == 0.0


@pytest.mark.parametrize("tau,departs_at", [(5.0, 5), (5.25, 6)])
def test_departure_time_is_inclusive(oracle_lib, tau, departs_at):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]], depart=[tau])
    o = _sim(oracle_lib, net, trips, _state(1, [-1], [0.0], [0.0], [0], step=5))
    o.step(1)
    assert o.get_state()["status"][0] == (1 if departs_at == 5 else 0)
    o.step(1)
    assert o.get_state()["status"][0] == 1


def test_one_departure_per_lane_per_step(oracle_lib):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2], [0, 2]])
    o = _sim(oracle_lib, net, trips, _state(2, [-1, -1], [0.0, 0.0], [0.0, 0.0], [0, 0]))
    o.step(1)
    s = o.get_state()
    # FIFO by (tau, id): vehicle 0 enters, vehicle 1 waits (no overlap)
    assert list(s["status"]) == [1, 0]
    assert o.metrics()["departures"] == 1


def test_blocked_head_stops_the_queue(oracle_lib):
    # road 0 turns left into road 2 from lane 0 only (lane group {0})
    net = left_turn_network(lanes=2, policy=W.POLICY_NONE)
    # vehicle 0 sits at x = 3 on lane 0 (rear at -2 m < s0); vehicle 1 (head,
    # turning left, so lane 0 only) cannot enter; vehicle 2 ends its trip on
    # road 0 and could use the empty lane 1, but waits behind the head
    trips = trips_for([[0, 2], [0, 2], [0]])
    st = _state(3, [0, -1, -1], [3.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1, 0, 0])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    assert s["status"][1] == 0 and s["status"][2] == 0
    assert o.metrics()["departures"] == 0


@pytest.mark.parametrize("x_feeder,v_feeder,departs", [(20.0, 10.0, False), (19.0, 0.0, True),
                                                       (19.0 + 1e-6, 0.0, False), (5.0, 0.0, True)])
def test_departure_waits_for_a_feeder_that_can_reach_it(oracle_lib, x_feeder, v_feeder, departs):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    q = jl_between(net, 0, 2)               # road 0 lane 0 -> road 2 lane 2 (straight)
    lane_jl = net.n_road_lanes + q
    # vehicle 0 on the junction lane (25 m) feeding road 2; vehicle 1 due on
    # road 2.  The feeder's front reaches x + v dt + a_max dt^2 / 2 - 25 in
    # road-2 coordinates; the entrant's rear is at -L = -5: x = 19, v = 0 is
    # the boundary (reach exactly -5, still safe)
    trips = trips_for([[0, 2], [2]])
    st = _state(2, [lane_jl, -1], [x_feeder, 0.0], [v_feeder, 0.0], [1, 0])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    assert (o.get_state()["status"][1] == 1) == departs


# ---------------------------------------------------------------------- merges

@pytest.mark.parametrize("low_front_crosses", [True, False])
def test_merge_priority_goes_to_the_lower_feeder(oracle_lib, low_front_crosses):
    net = merge_network()
    q_low, q_high = jl_between(net, 0, 4), jl_between(net, 2, 4)
    assert q_low < q_high
    NRL = net.n_road_lanes
    trips = trips_for([[0, 4], [2, 4]])
    # vehicle 1 on the higher-id feeder crosses its end this step (24 m, 10
    # m/s on a 25 m lane); vehicle 0 on the lower-id feeder either can too
    # (same place) or is far back at rest (reach 5 + 0 + 1 - 25 < 0)
    x0, v0 = (24.0, 10.0) if low_front_crosses else (5.0, 0.0)
    st = _state(2, [NRL + q_low, NRL + q_high], [x0, 24.0], [v0, 10.0], [1, 1])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    m = o.metrics()
    if low_front_crosses:
        assert s["lane"][0] == 4 and s["route_pos"][0] == 1
        assert s["lane"][1] == NRL + q_high
        assert s["x"][1] == 25.0 and s["v"][1] == 0.0
        assert m["feeder_blocks"] == 1
    else:
        assert s["lane"][1] == 4 and s["route_pos"][1] == 1
        assert s["lane"][0] == NRL + q_low
        assert m["feeder_blocks"] == 0


# --------------------------------------------------------------------- metrics

def test_travel_time_counts_the_step_the_trip_ends_in(oracle_lib):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]], depart=[3.5])
    # on its last road (route position 1), 5 m from the end at 10 m/s: the
    # trip ends during step 10, i.e. at time 11 s; travelling time 11 - 3.5
    st = _state(1, [2], [295.0], [10.0], [1], route_pos=[1], step=10)
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    m = o.metrics()
    assert s["status"][0] == 2 and s["finish_step"][0] == 10
    assert m["sum_tt"] == 7.5 and m["att"] == 7.5 and m["finished"] == 1


def test_mean_speed_skips_steps_without_road_vehicles(oracle_lib):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]])
    # cruising at its desired speed on an empty line (IDM free term zero, so
    # the speed never changes): steps 0-3 start on road 0 (x = 250 + 13.9 k
    # < 300), steps 4 and 5 on the 25 m junction lane (5.6 and 19.5 m), steps
    # 6-9 on road 2.  Eight counted steps, each with mean speed v0.
    st = _state(1, [0], [250.0], [LIM], [1])
    o = _sim(oracle_lib, net, trips, st)
    on_road = 0
    for _ in range(10):
        on_road += int(o.get_state()["lane"][0] < net.n_road_lanes)
        o.step(1)
    m = o.metrics()
    assert on_road == 8
    assert m["speed_steps"] == 8
    assert m["mean_speed_avg"] == pytest.approx(LIM, abs=1e-12)


def test_network_mean_speed_is_over_road_lanes(oracle_lib):
    net = line_network(lanes=1, length=1000.0, policy=W.POLICY_NONE)
    q = jl_between(net, 3, 1)               # road 3 (J2 -> J1) into road 1 (J1 -> J0)
    f1 = float(np.float32(0.9))
    # two cruisers at their own desired speeds on roads 0 and 1 (nobody on
    # their way ahead), and a slow vehicle on the junction lane into road 1
    # (behind the second cruiser), which does not count
    trips = trips_for([[0, 2], [1], [3, 1]], v0_factor=[1.0, 0.9, 1.0])
    st = _state(3, [0, 1, net.n_road_lanes + q], [100.0, 100.0, 2.0], [LIM, f1 * LIM, 1.0], [1, 1, 1])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    m = o.metrics()
    assert m["mean_speed_last"] == pytest.approx((LIM + f1 * LIM) / 2, abs=1e-12)
    sumv, cnt = o.road_stats()
    assert list(cnt) == [1, 1, 0, 0]
    assert sumv[0] == pytest.approx(LIM, abs=1e-12) and sumv[1] == pytest.approx(f1 * LIM, abs=1e-12)


def test_queue_length_counts_only_the_queue_at_the_lane_end(oracle_lib):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]] * 3)
    # vehicle 0 drives off at 10 m/s; vehicles 1 and 2 stand s0 behind the
    # rear ahead of them (IDM at v = 0, s = s0 gives exactly 0): they stay
    # stopped, but behind a moving front vehicle, so nobody waits at the end
    st = _state(3, [0, 0, 0], [100.0, 93.0, 86.0], [10.0, 0.0, 0.0], [1, 1, 1])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    assert s["v"][1] == 0.0 and s["v"][2] == 0.0
    assert o.lane_waiting()[0] == 0


def test_queue_length_at_a_red_light(oracle_lib):
    net = line_network(lanes=1, policy=W.POLICY_FIXED_TIME)
    trips = trips_for([[0, 2]] * 4)
    rol = net.road_of_lane()
    road0_jl = {q for q in range(net.n_jlanes) if rol[net.jl_in_lane[q]] == 0}
    j1 = 1
    pb = net.junc_phase_begin
    red = [p for p in range(pb[j1 + 1] - pb[j1])
           if not road0_jl & set(net.phase_green_jl[net.phase_green_begin[pb[j1] + p]:
                                                     net.phase_green_begin[pb[j1] + p + 1]].tolist())]
    # three vehicles at rest s0 apart, the first s0 before the red stop line
    # (each has IDM acceleration 0), and a fourth approaching at 10 m/s
    st = _state(4, [0, 0, 0, 0], [298.0, 291.0, 284.0, 150.0], [0.0, 0.0, 0.0, 10.0], [1, 1, 1, 1])
    o = _sim(oracle_lib, net, trips, st)
    o.set_signal_phases([j1], [red[0]])
    o.step(1)
    s = o.get_state()
    assert list(s["v"][:3]) == [0.0, 0.0, 0.0] and s["v"][3] > 0.1
    assert o.lane_waiting()[0] == 3


# ------------------------------------------------------------------- yielding

def test_keeper_at_rest_yields_to_a_stopped_merger(oracle_lib):
    # road 0 turns left from lane 0 only: vehicle 0 on lane 1 must merge into
    # lane 0; vehicle 1 keeps lane 0 with its front s0 behind vehicle 0's rear
    net = left_turn_network(lanes=2, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2], [0, 2]])
    st = _state(2, [1, 0], [100.0, 93.0], [0.0, 0.0], [1, 1])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    # IDM toward the merger's rear: v = 0, s = s0 -> acceleration 0 (free
    # road would give a_max = 2 and v' = 2)
    assert s["lane"][1] == 0 and s["v"][1] == 0.0 and s["x"][1] == 93.0


def test_fast_keeper_is_bounded_by_the_merger_rear(oracle_lib):
    net = left_turn_network(lanes=2, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2], [0, 2]])
    # keeper 3 m behind the merger's rear at 10 m/s: IDM brakes at the floor
    # (-9), the ballistic step reaches 92 + 10 - 4.5 = 97.5 > 95, so it stops
    # at the merger's rear (95) with the merger's speed (0)
    st = _state(2, [1, 0], [100.0, 92.0], [0.0, 10.0], [1, 1])
    o = _sim(oracle_lib, net, trips, st)
    o.step(1)
    s = o.get_state()
    assert s["lane"][1] == 0 and s["x"][1] == 95.0 and s["v"][1] == 0.0


# ---------------------------------------------------------------- lane control

@pytest.mark.parametrize("limit,expect_v", [(10.0, 10.0), (None, None)])
def test_lane_max_speed_sets_the_desired_speed(oracle_lib, limit, expect_v):
    """Section 3.2 set_lane_max_speed: a lone vehicle at 10 m/s on a lane whose
    limit becomes 10 m/s (factor 1) has zero free-road acceleration and keeps
    exactly 10 m/s; under the original 13.9 m/s limit it speeds up by
    a_max (1 - (10 / 13.9)^4) in one step (mistake caught: the new limit not
    used for the desired speed)."""
    net = line_network(lanes=1, length=1000.0, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]])
    o = _sim(oracle_lib, net, trips, _state(1, [0], [100.0], [10.0], [1]))
    if limit is not None:
        o.set_lane_max_speed([0], [float(np.float32(limit))])
    o.step(1)
    v = o.get_state()["v"][0]
    if expect_v is not None:
        assert v == expect_v
    else:
        assert v == pytest.approx(10.0 + P.a_max * (1 - (10.0 / LIM) ** 4), abs=1e-12)


# ------------------------------------------------------------------- rerouting

def test_reroute_ends_the_trip_on_the_current_road(oracle_lib):
    """Section 3.2 set_vehicle_route: a vehicle 10 m before the end of road
    0, bound for road 2, is given the route [0]; its trip ends when it
    crosses the end of road 0 (mistake caught: the old route kept, the
    vehicle enters the junction lane)."""
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]])
    o = _sim(oracle_lib, net, trips, _state(1, [0], [290.0], [12.0], [1], step=7))
    o.set_vehicle_route(0, [0])
    o.step(1)
    s = o.get_state()
    assert s["status"][0] == 2 and s["finish_step"][0] == 7


def test_reroute_of_a_waiting_vehicle_changes_its_departure_lanes(oracle_lib):
    """A waiting vehicle turning left may only enter lane 0 of its origin
    road, which is blocked; rerouted to end on its origin road it may use
    lane 1 and departs there (mistake caught: the lane group of the old
    route kept for departures)."""
    net = left_turn_network(lanes=2, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2], [0, 2]])
    o = _sim(oracle_lib, net, trips, _state(2, [0, -1], [3.0, 0.0], [0.0, 0.0], [1, 0]))
    o.step(1)
    assert o.get_state()["status"][1] == 0
    o.set_vehicle_route(1, [0])
    o.step(1)
    s = o.get_state()
    assert s["status"][1] == 1 and s["lane"][1] == 1


def test_reroute_makes_a_lane_change_mandatory(oracle_lib):
    """A vehicle on lane 1 ending its trip on road 0 (every lane in its
    group) is rerouted to turn left into road 2, which only lane 0 reaches:
    outside its lane group its utility toward lane 0 is at least 1 (mistake
    caught: the lane group of the old route kept, utility -a_th)."""
    net = left_turn_network(lanes=2, policy=W.POLICY_NONE)
    trips = trips_for([[0]])
    o = _sim(oracle_lib, net, trips, _state(1, [1], [50.0], [10.0], [1]))
    o.step(1)
    assert o.diag()["mobil"][0, 0] == pytest.approx(-W.Params().a_th, abs=1e-9)
    o.set_vehicle_route(0, [0, 2])
    o.step(1)
    assert o.diag()["mobil"][0, 0] >= 1.0
    k, route = o.route(0)
    assert list(route) == [0, 2]
