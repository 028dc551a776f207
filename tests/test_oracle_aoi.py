"""Pins of the oracle's areas of interest (Appendix B.1: an AOI is an area
joined to the road network by connections at positions along roads, where
trips start and end; Appendix B.2: the AOI puts a due vehicle into the lane
at its connection and takes in the vehicles whose trips end there).

Reading: a trip that starts in AOI a enters at a's first listed connection
on the first road of its route, one that ends in AOI b ends at b's first
listed connection on the last road of its route; an AOI without a connection
on that road is an error.  Counts: waiting[a] = vehicles of origin a not yet
departed, arrived[b] = vehicles whose trip ended in b.

Line network, one lane, no signals; dt = 1 s, a_max = 2 m/s^2, lane limit
13.9 m/s, vehicles 5 m long.  A vehicle entering at rest on a free road ends
its first step at p + a_max dt^2 / 2 = p + 1 m with v = 2 m/s; with the IDM
free-road term a_max (1 - (v / v0)^4) it then reaches about p + 4, p + 9 and
p + 16 m after the next three steps.
"""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import line_network, trips_for

P = W.Params()
# AOI 0: a connection on road 2 listed first (never a first road here), then
# road 0 at 50 m; AOI 1: road 0 at 60 m; AOI 2: road 2 at 120 m
CB = [0, 2, 3, 4]
CR = [2, 0, 0, 2]
CS = [100.0, 50.0, 60.0, 120.0]


def _sim(oracle_lib, routes, depart=None):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    return oracle_lib.OracleSim(net, trips_for(routes, depart=depart), P)


def test_start_and_end_at_the_connections_on_the_route_s_roads(oracle_lib):
    """Vehicle 0 (route [0]) from AOI 0 to AOI 1: starts at 50 m (AOI 0's
    connection on road 0, not its first listed one on road 2) and ends at
    60 m; vehicle 1 (route [0, 2]) from AOI 0 to AOI 2 ends at 120 m on
    road 2 (mistakes: the AOI's first connection taken whatever its road,
    origin and destination swapped)."""
    o = _sim(oracle_lib, [[0], [0, 2]])
    starts, ends = o.set_aois(CB, CR, CS, [0, 0], [1, 2])
    assert starts.tolist() == [50.0, 50.0]
    assert ends.tolist() == [60.0, 120.0]


def test_enters_at_its_origin_and_finishes_at_its_destination(oracle_lib):
    """Vehicle 0 enters at 50 m in step 0 (x = 51 m, v = 2 m/s after it) and
    its front passes 60 m in step 3 (about 59 m after step 2, 66 m in step
    3): waiting[0] 1 -> 0 after the first step, arrived[1] 0 -> 1 after the
    fourth (mistakes: the start ignored, entry at 0 m, which finishes near
    step 7; the end ignored; counts by the wrong AOI)."""
    o = _sim(oracle_lib, [[0]])
    o.set_aois(CB, CR, CS, [0], [1])
    w, a = o.aoi_counts()
    assert w.tolist() == [1, 0, 0] and a.tolist() == [0, 0, 0]
    o.step(1)
    s = o.get_state()
    assert s["status"][0] == 1 and s["x"][0] == 51.0 and s["v"][0] == 2.0
    w, a = o.aoi_counts()
    assert w.tolist() == [0, 0, 0] and a.tolist() == [0, 0, 0]
    o.step(2)
    s = o.get_state()
    assert s["status"][0] == 1 and 58.5 < s["x"][0] < 60.0
    o.step(1)
    s = o.get_state()
    assert s["status"][0] == 2 and s["finish_step"][0] == 3
    w, a = o.aoi_counts()
    assert w.tolist() == [0, 0, 0] and a.tolist() == [0, 1, 0]


def test_waiting_counts_follow_departure_times(oracle_lib):
    """Two trips from AOI 0 to AOI 1 due at 0 s and 10 s: two waiting, then
    one after step 0, none after step 10; both arrived four steps after
    their departures (mistake: a due vehicle counted as still waiting, or
    the departure time taken as one step later)."""
    o = _sim(oracle_lib, [[0], [0]], depart=[0.0, 10.0])
    o.set_aois(CB, CR, CS, [0, 0], [1, 1])
    assert o.aoi_counts()[0].tolist() == [2, 0, 0]
    o.step(1)
    assert o.aoi_counts()[0].tolist() == [1, 0, 0]
    o.step(9)
    assert o.aoi_counts()[0].tolist() == [1, 0, 0]
    o.step(1)
    assert o.aoi_counts()[0].tolist() == [0, 0, 0]
    o.step(3)
    assert o.aoi_counts()[1].tolist() == [0, 2, 0]


def test_refuses_an_aoi_without_a_connection_on_the_road(oracle_lib):
    """AOI 2 has no connection on road 0, the first road of the route."""
    o = _sim(oracle_lib, [[0]])
    with pytest.raises(ValueError):
        o.set_aois(CB, CR, CS, [2], None)


def test_refuses_a_vehicle_that_has_departed(oracle_lib):
    o = _sim(oracle_lib, [[0]])
    o.step(1)
    with pytest.raises(ValueError):
        o.set_aois(CB, CR, CS, [0], [1])
