"""Pins of the oracle's trip end positions (Section 3.2 set_vehicle_route:
the trip's end position on the last road; an AOI's connection as a trip's
end, Appendix B.1).

Reading: a trip ends in the step in which the vehicle's front passes its end
position on the last road of its route (strictly beyond it, as at a road
end); the default is the end of that road.  A vehicle at rest on a free road
accelerates at a_max, so in one step of 1 s its front moves exactly 1 m.
"""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import line_network, state_from, trips_for

P = W.Params()


def _sim(oracle_lib, routes, end_s, lanes, xs, vs, route_pos=None):
    net = line_network(lanes=1, policy=W.POLICY_NONE)
    trips = trips_for(routes)
    if end_s is not None:
        trips.end_s = np.asarray(end_s, np.float32)
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(state_from(len(routes), lanes, xs, vs, route_pos=route_pos))
    return o


@pytest.mark.parametrize("end_s,finished", [(None, False), (100.0, False), (99.99, True), (50.0, True)])
def test_trip_ends_when_the_front_passes_its_end_position(oracle_lib, end_s, finished):
    """Front from 99 m to exactly 100 m: it ends only for an end position
    below 100 m (mistakes: the end position ignored, or >= instead of >)."""
    o = _sim(oracle_lib, [[0]], None if end_s is None else [end_s], [0], [99.0], [0.0])
    o.step(1)
    s = o.get_state()
    assert abs(s["x"][0] - 100.0) < 1e-12 or finished
    assert (s["status"][0] == 2) == finished
    if finished:
        assert s["finish_step"][0] == 0
        m = o.metrics()
        assert m["finished"] == 1 and abs(m["att"] - 1.0) < 1e-12   # (0 + 1) dt - tau, tau = 0


def test_end_position_only_on_the_last_road(oracle_lib):
    """Route [0, 2] with an end position of 99.6 m: passing 99.6 m on road 0
    (not the last road) neither ends the trip nor moves the vehicle on: it
    stays on road 0 at 100 m (mistake: the end position applied on every
    road of the route, as a lane end)."""
    o = _sim(oracle_lib, [[0, 2]], [99.6], [0], [99.0], [0.0])
    o.step(1)
    s = o.get_state()
    assert s["status"][0] == 1 and s["lane"][0] == 0 and abs(s["x"][0] - 100.0) < 1e-12


def test_reroute_sets_the_end_position(oracle_lib):
    """A vehicle at 99 m at rest is given the route [0] ending at 99.5 m: it
    ends in the next step (mistake: the rerouted trip keeps the road end)."""
    o = _sim(oracle_lib, [[0, 2]], None, [0], [99.0], [0.0])
    o.set_vehicle_route(0, [0], end_s=99.5)
    o.step(1)
    assert o.get_state()["status"][0] == 2
