"""Tiny hand-built networks and scenes for the oracle pins and the GPU
edge-case parity tests."""

import math

import numpy as np

from paper_2406_10661_amd import workloads as W


def line_network(lanes=1, length=300.0, limit=13.9, policy=W.POLICY_FIXED_TIME):
    """J0 -- J1 -- J2 on a straight line: roads 0 (J0->J1), 1 (J1->J0),
    2 (J1->J2), 3 (J2->J1).  Road 0 continues straight into road 2."""
    xy = np.array([[0.0, 0.0], [length + 50, 0.0], [2 * length + 100, 0.0]])
    net = W._build_network(xy, np.array([[0, 1], [1, 2]]), [length, length], [lanes, lanes],
                           [limit, limit], policy=policy)
    return net


def left_turn_network(lanes=2, length=300.0, limit=13.9, policy=W.POLICY_NONE):
    """J0 (0,0) -> J1 (L,0) -> J2 (L,L): road 0 turns left into road 2, so only
    lane 0 of road 0 connects (lane group {0})."""
    xy = np.array([[0.0, 0.0], [length, 0.0], [length, length]])
    return W._build_network(xy, np.array([[0, 1], [1, 2]]), [length, length], [lanes, lanes],
                            [limit, limit], policy=policy)


def trips_for(routes, depart=None, v0_factor=None, length=5.0):
    n = len(routes)
    rb = np.zeros(n + 1, np.int32)
    rb[1:] = np.cumsum([len(r) for r in routes])
    return W.Trips(
        depart_time=np.zeros(n, np.float32) if depart is None else np.asarray(depart, np.float32),
        route_begin=rb,
        route_roads=np.concatenate([np.asarray(r, np.int32) for r in routes]),
        v0_factor=np.ones(n, np.float32) if v0_factor is None else np.asarray(v0_factor, np.float32),
        length=np.full(n, length, np.float32),
    )


def state_from(n, lanes, xs, vs, route_pos=None, step=0, status=None):
    st = dict(status=np.full(n, 1, np.int32) if status is None else np.asarray(status, np.int32),
              lane=np.asarray(lanes, np.int32), x=np.asarray(xs, np.float64), v=np.asarray(vs, np.float64),
              route_pos=np.zeros(n, np.int32) if route_pos is None else np.asarray(route_pos, np.int32),
              finish_step=np.full(n, -1, np.int32), step=step)
    return st


def v_equilibrium(gap, v0, P=W.Params()):
    """Speed at which the IDM acceleration vanishes behind a leader of equal
    speed at the given gap (s0 + v T = gap sqrt(1 - (v / v0)^4)), by
    bisection."""
    lo, hi = 0.0, v0 * (1 - 1e-12)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s_e = (P.s0 + mid * P.T) / math.sqrt(1 - (mid / v0) ** 4)
        if s_e < gap:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def ring_state(net, n, gaps_front, v):
    """Place n vehicles on the ring (road 0 then junction lane 0) with front
    bumpers at the given ring coordinates."""
    road_len = float(net.road_length[0])
    lanes, xs, k = [], [], []
    for s in gaps_front:
        s = s % (road_len + float(net.jl_length[0]))
        if s < road_len:
            lanes.append(0); xs.append(s)
        else:
            lanes.append(1); xs.append(s - road_len)
        k.append(0)
    return state_from(n, lanes, xs, [v] * n, route_pos=k)


def ring_coords(net, st):
    road_len = float(net.road_length[0])
    return np.where(st["lane"] == 0, st["x"], st["x"] + road_len)


def merge_network(length=200.0, limit=13.9, policy=W.POLICY_NONE):
    """Two one-lane roads merging: J0 (0, 100) -> J2 (100, 0) is road 0 and
    J1 (0, -100) -> J2 is road 2; both continue straight (within 45 degrees)
    into road 4, J2 -> J3 (400, 0), so two junction lanes feed road 4's lane."""
    xy = np.array([[0.0, 100.0], [0.0, -100.0], [100.0, 0.0], [400.0, 0.0]])
    return W._build_network(xy, np.array([[0, 2], [1, 2], [2, 3]]), [length] * 3, [1, 1, 1],
                            [limit] * 3, policy=policy)


def jl_between(net, lane_in, lane_out):
    """Junction-lane index from road lane lane_in to road lane lane_out."""
    q = np.nonzero((net.jl_in_lane == lane_in) & (net.jl_out_lane == lane_out))[0]
    assert q.size == 1
    return int(q[0])


def plus_network(length=200.0, limit=13.9, policy=W.POLICY_FIXED_TIME):
    """A four-way junction J4 at (200, 200) with arms to J0 (west), J1 (east),
    J2 (south) and J3 (north), one lane each way.  Roads 0, 2, 4, 6 enter J4
    (from J0, J1, J2, J3); roads 1, 3, 5, 7 leave it (to J0, J1, J2, J3).
    J4 has one phase per approach in in-road order: phase 0 = road 0, 1 =
    road 2, 2 = road 4, 3 = road 6, each with its three movements (left,
    straight, right; no U-turn)."""
    xy = np.array([[0.0, 200.0], [400.0, 200.0], [200.0, 0.0], [200.0, 400.0], [200.0, 200.0]])
    return W._build_network(xy, np.array([[0, 4], [1, 4], [2, 4], [3, 4]]), [length] * 4, [1] * 4,
                            [limit] * 4, policy=policy)


def diamond_network():
    """Two ways from road 0 (O->S) to road 5 (T->Z): over A (roads 1 S->A,
    3 A->T) or over B (roads 2 S->B, 4 B->T).  Road lanes: road 0 lanes 0-1,
    road 1 lane 2, road 2 lanes 3-4, road 3 lane 5, road 4 lane 6, road 5
    lane 7; junction lanes 8-15 (q0-q7): q0 0->2 and q1 1->2 (two ways into
    road 1; q1 is 200 m long), q2 1->3, q3 2->5, q4 3->6, q5 4->6, q6 5->7,
    q7 6->7.  Every limit is 8 m/s and every other junction lane 8 m long,
    so a junction lane takes 1 s (q1 25 s) and roads 0-5 take 10, 20, 10,
    20, 20 and 10 s."""
    xy = np.array([[-100.0, 0.0], [0.0, 0.0], [100.0, 100.0], [100.0, -100.0], [200.0, 0.0], [300.0, 0.0]])
    return W.Network(
        junction_xy=xy,
        road_from=np.array([0, 1, 1, 2, 3, 4], np.int32),
        road_to=np.array([1, 2, 3, 4, 4, 5], np.int32),
        road_lane_begin=np.array([0, 2, 3, 5, 6, 7, 8], np.int32),
        road_length=np.array([80, 160, 80, 160, 160, 80], np.float32),
        road_limit=np.full(6, 8.0, np.float32),
        jl_in_lane=np.array([0, 1, 1, 2, 3, 4, 5, 6], np.int32),
        jl_out_lane=np.array([2, 2, 3, 5, 6, 6, 7, 7], np.int32),
        jl_length=np.array([8, 200, 8, 8, 8, 8, 8, 8], np.float32),
        jl_limit=np.full(8, 8.0, np.float32),
        junc_phase_begin=np.zeros(7, np.int32),
        phase_duration=np.zeros(0, np.float32),
        phase_green_begin=np.zeros(1, np.int32),
        phase_green_jl=np.zeros(0, np.int32),
        junc_policy=np.full(6, W.POLICY_NONE, np.int32),
    )


def empty_trips():
    """A trip table with no vehicles (for queries of the network alone)."""
    z = np.zeros(0, np.float32)
    return W.Trips(depart_time=z, route_begin=np.zeros(1, np.int32), route_roads=np.zeros(0, np.int32),
                   v0_factor=z, length=z)
