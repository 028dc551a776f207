"""Seeded synthetic mid-simulation states for one-step parity at any size.

A state places a fraction of the vehicles somewhere along their own route
(road lanes, including lanes outside the lane group, and junction lanes
toward the next road), with no two vehicles of a lane overlapping, random
speeds up to the desired speed, and the remaining vehicles waiting (some
already due to depart) or finished.  Nothing here evaluates the model.
"""

import numpy as np


def synthetic_state(net, trips, step, seed, p_active=0.5, p_finished=0.1, p_junction=0.08, min_gap=0.3):
    rng = np.random.default_rng(seed)
    N = trips.n_vehicles
    NRL = net.n_road_lanes
    rol = net.road_of_lane()
    rb, rr = trips.route_begin, trips.route_roads
    # junction lanes by (in road, out road)
    conn = {}
    for q in range(net.n_jlanes):
        conn.setdefault((int(rol[net.jl_in_lane[q]]), int(rol[net.jl_out_lane[q]])), []).append(q)
    lane_len = np.concatenate([np.repeat(net.road_length, np.diff(net.road_lane_begin)), net.jl_length]).astype(np.float64)
    u = rng.random(N)
    status = np.zeros(N, np.int32)
    status[u < p_active] = 1
    status[(u >= p_active) & (u < p_active + p_finished)] = 2
    lane = np.full(N, -1, np.int32)
    route_pos = np.zeros(N, np.int32)
    x = np.zeros(N, np.float32)
    v = np.zeros(N, np.float32)
    finish = np.full(N, -1, np.int32)
    for i in np.nonzero(status == 1)[0]:
        rl = rb[i + 1] - rb[i]
        k = int(rng.integers(0, rl))
        r = int(rr[rb[i] + k])
        if k + 1 < rl and rng.random() < p_junction:
            q = int(rng.choice(conn[(r, int(rr[rb[i] + k + 1]))]))
            lane[i] = NRL + q
        else:
            lb, le = net.road_lane_begin[r], net.road_lane_begin[r + 1]
            lane[i] = int(rng.integers(lb, le))
        route_pos[i] = k
        x[i] = np.float32(rng.uniform(0.0, lane_len[lane[i]]))
    # per lane: keep order by position, push vehicles back to remove overlaps
    act = np.nonzero(status == 1)[0]
    order = np.lexsort((act, -x[act].astype(np.float64), lane[act]))
    a = act[order]
    prev_lane, prev_rear = -1, 0.0
    for i in a:
        if lane[i] != prev_lane:
            prev_lane = lane[i]
            prev_rear = np.inf
        xi = min(float(x[i]), prev_rear - min_gap * (1.0 + rng.random()))
        if xi < 0.0:
            status[i] = 0
            lane[i] = -1
            route_pos[i] = 0
            x[i] = 0.0
            continue
        x[i] = np.float32(xi)
        if float(x[i]) > prev_rear:
            x[i] = np.nextafter(np.float32(prev_rear), np.float32(-1))
        prev_rear = float(x[i]) - float(trips.length[i])
    lim = np.concatenate([np.repeat(net.road_limit, np.diff(net.road_lane_begin)), net.jl_limit]).astype(np.float64)
    act = status == 1
    v0 = trips.v0_factor[act] * lim[lane[act]]
    v[act] = (rng.random(int(act.sum())) * v0).astype(np.float32)
    # some of the standing vehicles
    stand = act & (rng.random(N) < 0.15)
    v[stand] = 0.0
    fin = np.nonzero(status == 2)[0]
    finish[fin] = rng.integers(0, max(step, 1), fin.size)
    route_pos[fin] = (rb[fin + 1] - rb[fin] - 1)
    return dict(step=int(step), status=status, lane=lane, route_pos=route_pos, x=x, v=v, finish_step=finish)
