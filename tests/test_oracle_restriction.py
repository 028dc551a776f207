"""Pins of the oracle's lane restrictions (Section 3.2 "Lane":
set_lane_restriction; road lane plans are sets of restricted junction
lanes).

Reading: a restricted lane admits no new vehicle: no departure into it, no
lane change into it, and no entry from a road lane into a junction lane that
is restricted or leads into a restricted lane (such a junction lane is
closed, so the lane group of a route is formed from the open ones).  Vehicles
already on a restricted lane, or already on a junction lane leading into
one, carry on.

Each scene's outcome follows by inspection; the mistake each one catches is
named in its docstring.
"""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import jl_between, left_turn_network, line_network, state_from, trips_for

P = W.Params()


def _state(n, lanes, xs, vs, status, route_pos=None, step=0):
    st = state_from(n, lanes, xs, vs, route_pos=route_pos, step=step, status=status)
    st["lane"] = np.where(st["status"] == 1, st["lane"], -1).astype(np.int32)
    return st


def _sim(oracle_lib, net, trips, st, restricted=(), released=()):
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(st)
    if restricted:
        o.set_lane_restriction(list(restricted), [1] * len(restricted))
    if released:
        o.set_lane_restriction(list(released), [0] * len(released))
    return o


def _departure_scene():
    # three vehicles on road 0 with rear bumpers at 25, 45 and 35 m; vehicle 3
    # is due at t = 0 on the same road (every lane leads on to road 2)
    net = line_network(lanes=3, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]] * 4)
    st = _state(4, [0, 1, 2, -1], [30.0, 50.0, 40.0, 0.0], [0.0] * 4, [1, 1, 1, 0])
    return net, trips, st


@pytest.mark.parametrize("restricted,released,lane", [((), (), 1), ((1,), (), 2), ((1, 2), (), 0),
                                                      ((1,), (1,), 1)])
def test_departure_skips_restricted_lanes(oracle_lib, restricted, released, lane):
    """Most room is lane 1, then lane 2, then lane 0; restricting lane 1
    sends the entrant to lane 2, restricting both to lane 0, and releasing
    lane 1 again restores it (mistakes: restriction ignored, or sticky)."""
    net, trips, st = _departure_scene()
    o = _sim(oracle_lib, net, trips, st, restricted, released)
    o.step(1)
    s = o.get_state()
    assert s["status"][3] == 1 and s["lane"][3] == lane


def test_every_lane_restricted_keeps_the_vehicle_waiting(oracle_lib):
    """All three lanes restricted: the head waits (mistake: a restricted lane
    used when nothing else is left)."""
    net, trips, st = _departure_scene()
    o = _sim(oracle_lib, net, trips, st, (0, 1, 2))
    o.step(3)
    assert o.get_state()["status"][3] == 0 and o.metrics()["departures"] == 0


def _lanes_over(o, steps):
    out = []
    for _ in range(steps):
        o.step(1)
        out.append(int(o.get_state()["lane"][0]))
    return out


def test_no_lane_change_into_a_restricted_lane(oracle_lib):
    """Road 0 turns left into road 2 from lane 0 only.  A vehicle on lane 1
    (outside its lane group) changes to lane 0 within a few steps when lane
    0 is open (mandatory change: utility at least 1, p_LC = p_max); with lane
    0 restricted it never does and comes to rest at its lane end (mistake:
    MOBIL ignoring the restriction)."""
    net = left_turn_network(lanes=2, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]])
    st = _state(1, [1], [100.0], [8.0], [1])
    free = _lanes_over(_sim(oracle_lib, net, trips, st), 20)
    assert 0 in free
    held = _sim(oracle_lib, net, trips, st, (0,))
    lanes = _lanes_over(held, 60)
    assert set(lanes) == {1}
    s = held.get_state()
    assert s["x"][0] <= float(net.road_length[0]) and s["v"][0] < 0.1


def test_closed_junction_lane_stops_the_vehicle(oracle_lib):
    """One lane straight on from road 0 to road 2.  Open: the vehicle near
    the end of road 0 crosses onto the junction lane; with that junction lane
    restricted it stops at its lane end and stays on road 0 (mistake: a
    closed junction lane still taken, or still seen as the lookahead
    leader's lane)."""
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    g = net.n_road_lanes + jl_between(net, 0, 2)
    trips = trips_for([[0, 2]])
    st = _state(1, [0], [250.0], [10.0], [1])
    o = _sim(oracle_lib, net, trips, st)
    o.step(8)
    assert o.get_state()["lane"][0] != 0
    o = _sim(oracle_lib, net, trips, st, (g,))
    o.step(40)
    s = o.get_state()
    assert s["lane"][0] == 0 and s["x"][0] <= float(net.road_length[0]) and s["v"][0] < 0.1


def test_restricted_out_lane_closes_its_feeders_but_not_for_vehicles_on_them(oracle_lib):
    """Road 2's lane restricted: vehicle 1 on road 0 stops at its lane end
    (the junction lane into road 2 is closed), while vehicle 0, already on
    that junction lane, drives on into road 2 (mistakes: the junction lane
    left open, or vehicles on it stopped)."""
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    q = jl_between(net, 0, 2)
    g = net.n_road_lanes + q
    out = int(net.road_lane_begin[2])
    trips = trips_for([[0, 2], [0, 2]])
    st = _state(2, [g, 0], [15.0, 230.0], [10.0, 10.0], [1, 1], route_pos=[0, 0])
    o = _sim(oracle_lib, net, trips, st, (out,))
    o.step(3)
    assert o.get_state()["lane"][0] == out
    o.step(37)
    s = o.get_state()
    assert s["lane"][1] == 0 and s["v"][1] < 0.1


def test_closed_junction_lane_moves_the_lane_group(oracle_lib):
    """Two lanes straight on from road 0 to road 2 (lane 0 -> 4, lane 1 -> 5).
    A vehicle on lane 1 with nothing around keeps its lane while both
    junction lanes are open; closing lane 1's junction lane takes lane 1 out
    of the lane group, so the vehicle changes to lane 0 (mistake: lane group
    formed from every junction lane, open or not)."""
    net = line_network(lanes=2, policy=W.POLICY_NONE)
    g1 = net.n_road_lanes + jl_between(net, 1, 5)
    trips = trips_for([[0, 2]])
    st = _state(1, [1], [50.0], [10.0], [1])
    assert set(_lanes_over(_sim(oracle_lib, net, trips, st), 10)) == {1}
    assert 0 in _lanes_over(_sim(oracle_lib, net, trips, st, (g1,)), 10)
