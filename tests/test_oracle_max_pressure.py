"""Pins of the oracle's MAX_PRESSURE signal policy (Section 3.2; the
maximum-pressure algorithm the paper cites; Appendix B.2) on a four-way
junction with hand-computed pressures.

Junction J4 of ``plus_network``: phase p makes the three movements of one
approach green (phase 0 from road 0 into roads 3, 5, 7; phase 1 from road 2
into 1, 5, 7; phase 2 from road 4 into 1, 3, 7; phase 3 from road 6 into 1,
3, 5).  With n(r) vehicles on road r, a phase's pressure is the sum over its
movements of n(in) - n(out).  Plausible mistakes caught: counting only the
incoming lanes, the opposite sign, ties not going to the lowest phase, and
deciding at every step instead of every phase-0 duration.
"""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import plus_network, trips_for

P = W.Params()
J4 = 4
OUT_OF = {0: 3, 2: 1, 4: 7, 6: 5}     # an out road straight across from each in road


def scene(counts, step=0):
    """counts: {road: vehicles}, placed at rest 20 m apart from x = 20 on the
    road's single lane; vehicles on an incoming road drive straight across,
    vehicles on an outgoing road end their trip there."""
    net = plus_network(policy=W.POLICY_FIXED_TIME)
    routes, lanes, xs = [], [], []
    for r, k in counts.items():
        for c in range(k):
            routes.append([r, OUT_OF[r]] if r in OUT_OF else [r])
            lanes.append(int(net.road_lane_begin[r]))
            xs.append(20.0 * (c + 1))
    n = len(routes)
    trips = trips_for(routes if n else [[0]], depart=None if n else [1e9])
    if not n:
        n = 1
        st = dict(status=np.zeros(1, np.int32), lane=np.full(1, -1, np.int32), x=np.zeros(1), v=np.zeros(1),
                  route_pos=np.zeros(1, np.int32), finish_step=np.full(1, -1, np.int32), step=step)
    else:
        st = dict(status=np.ones(n, np.int32), lane=np.asarray(lanes, np.int32), x=np.asarray(xs, np.float64),
                  v=np.zeros(n), route_pos=np.zeros(n, np.int32), finish_step=np.full(n, -1, np.int32), step=step)
    return net, trips, st


def phase_in_force(oracle_lib, net, trips, st, held=0):
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(st)
    pol = np.array(net.junc_policy, np.int32)
    pol[J4] = 3
    ph = np.zeros(net.n_junctions, np.int32)
    ph[J4] = held
    o.set_junctions(pol, ph)
    o.step(1)
    return o, int(o.junctions()[1][J4])


def green_roads(net, o):
    g = o.green()
    rol = net.road_of_lane()
    q = [k for k in range(net.n_jlanes) if g[k] and net.jl_in_lane[k] in net.road_lane_begin[[0, 2, 4, 6]]]
    return sorted({int(rol[net.jl_in_lane[k]]) for k in q})


def test_largest_pressure_wins(oracle_lib):
    # pressures: phase 0: 3*5 - (0 + 4 + 0) = 11; phase 1: 3*1 - (0 + 4 + 0) = -1;
    # phase 2: 3*4 - (0 + 0 + 0) = 12; phase 3: 3*1 - (0 + 0 + 4) = -1.
    # Incoming counts alone would pick phase 0 (15), the opposite sign phase 1.
    net, trips, st = scene({0: 5, 2: 1, 4: 4, 6: 1, 5: 4})
    o, ph = phase_in_force(oracle_lib, net, trips, st)
    assert ph == 2
    assert green_roads(net, o) == [4]


def test_ties_go_to_the_lowest_phase(oracle_lib):
    # empty junction: every pressure 0 -> phase 0
    net, trips, st = scene({})
    assert phase_in_force(oracle_lib, net, trips, st, held=3)[1] == 0
    # phases 1 and 3 tie at 3*2 - 0 = 6 above phases 0 and 2 (their in roads
    # are empty; phase 0's out roads hold nobody either) -> phase 1
    net, trips, st = scene({2: 2, 6: 2})
    assert phase_in_force(oracle_lib, net, trips, st)[1] == 1


@pytest.mark.parametrize("step,decides", [(0, True), (29, False), (30, True), (31, False), (60, True)])
def test_decisions_every_first_phase_duration(oracle_lib, step, decides):
    # road 0 alone holds vehicles: pressure favours phase 0; the junction
    # enters the step holding phase 2 (30 s phases, dt = 1 s)
    net, trips, st = scene({0: 5}, step=step)
    o, ph = phase_in_force(oracle_lib, net, trips, st, held=2)
    assert ph == (0 if decides else 2)
    assert green_roads(net, o) == ([0] if decides else [4])
