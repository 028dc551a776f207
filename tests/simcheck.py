"""Independent checks of simulator states (numpy, written from the model
definition, sharing nothing with the oracle or the HIP library).

Used by the oracle pin tests and the GPU parity tests alike:
  * closed-form fixed-time signal schedule (Section 3.2 FIXED_TIME);
  * lane groups (lanes of a road connected to the route's next road);
  * per-step invariants between two consecutive states:
      I1 no overlap between consecutive vehicles of a lane
      I2 v >= 0 and 0 <= x <= lane length
      I3 waiting + active + finished = N
      I4 a vehicle entering a junction lane in step t had it green at t
      I5 a vehicle in its lane group never leaves the group by a lane change
      I6 vehicles that keep their lane never overtake and never move back
      I7 no lane change on junction lanes
"""

from __future__ import annotations

import numpy as np

WAITING, ACTIVE, FINISHED = 0, 1, 2


class NetInfo:
    def __init__(self, net, trips):
        self.net, self.trips = net, trips
        self.NRL = net.n_road_lanes
        self.NL = net.n_lanes
        self.rol = net.road_of_lane()
        self.lane_len = np.concatenate([np.repeat(net.road_length, np.diff(net.road_lane_begin)),
                                        net.jl_length]).astype(np.float64)
        # junction lane of (road lane, next road)
        self.conn = {}
        for q in range(net.n_jlanes):
            self.conn[(int(net.jl_in_lane[q]), int(self.rol[net.jl_out_lane[q]]))] = self.NRL + q
        self.jl_junction = net.road_to[self.rol[net.jl_in_lane]]

    def next_road(self, i, k):
        b, e = self.trips.route_begin[i], self.trips.route_begin[i + 1]
        return int(self.trips.route_roads[b + k + 1]) if b + k + 1 < e else -1

    def in_group(self, i, k, lane):
        nr = self.next_road(i, k)
        return nr < 0 or (int(lane), nr) in self.conn


def fixed_time_phase(durations, t, dt):
    """Phase index active during step t: phases in order, phase 0 from t = 0."""
    cyc = float(np.sum(durations))
    s = (t * dt) % cyc
    acc = 0.0
    for p, d in enumerate(durations):
        acc += float(d)
        if s < acc:
            return p
    return len(durations) - 1


def green_set(net, t, dt, policy=None, manual=None):
    """Boolean [n_jlanes]: junction lanes green during step t."""
    policy = net.junc_policy if policy is None else policy
    g = np.zeros(net.n_jlanes, bool)
    for j in range(net.n_junctions):
        b, e = net.junc_phase_begin[j], net.junc_phase_begin[j + 1]
        if policy[j] == 0 or e == b:
            continue
        if policy[j] == 2:
            ph = int(manual[j])
        else:
            ph = fixed_time_phase(net.phase_duration[b:e], t, dt)
        p = b + ph
        g[net.phase_green_jl[net.phase_green_begin[p]:net.phase_green_begin[p + 1]]] = True
    jj = net.road_to[net.road_of_lane()[net.jl_in_lane]]
    nophase = np.diff(net.junc_phase_begin)[jj] == 0
    g |= (policy[jj] == 0) | nophase
    return g


def check_state(info: NetInfo, st, tol=1e-6):
    """I1, I2 and I3 on one state (x, v as floats)."""
    errs = []
    N = info.trips.n_vehicles
    s = st["status"]
    if not ((s >= 0) & (s <= 2)).all():
        errs.append("bad status")
    if int((s == WAITING).sum() + (s == ACTIVE).sum() + (s == FINISHED).sum()) != N:
        errs.append("I3 conservation")
    act = np.nonzero(s == ACTIVE)[0]
    lane, x, v = st["lane"][act], np.asarray(st["x"], np.float64)[act], np.asarray(st["v"], np.float64)[act]
    L = info.trips.length[act].astype(np.float64)
    if (v < 0).any():
        errs.append(f"I2 negative speed {v.min()}")
    ln = info.lane_len[lane]
    if (x < -tol).any() or (x > ln + tol).any():
        errs.append("I2 position outside lane")
    order = np.lexsort((act, -x, lane))
    lane_o, x_o, L_o = lane[order], x[order], L[order]
    same = lane_o[1:] == lane_o[:-1]
    gap = (x_o[:-1] - L_o[:-1]) - x_o[1:]
    bad = same & (gap < -tol)
    if bad.any():
        k = np.nonzero(bad)[0][0]
        errs.append(f"I1 overlap on lane {lane_o[k]} gap {gap[k]}")
    return errs


def check_transition(info: NetInfo, prev, cur, green_prev_step, tol=1e-6):
    """I4-I7 between the state before and after one step."""
    errs = []
    net = info.net
    was = np.nonzero((prev["status"] == ACTIVE) & (cur["status"] == ACTIVE))[0]
    l0, l1 = prev["lane"][was], cur["lane"][was]
    x0 = np.asarray(prev["x"], np.float64)[was]
    x1 = np.asarray(cur["x"], np.float64)[was]
    k0 = prev["route_pos"][was]
    # I7: on a junction lane a vehicle stays or moves to the out lane
    jl = l0 >= info.NRL
    if jl.any():
        ok = (l1[jl] == l0[jl]) | (l1[jl] == net.jl_out_lane[l0[jl] - info.NRL])
        if not ok.all():
            errs.append("I7 lane change on a junction lane")
    # I4: entry into a junction lane only when green
    entered = (~jl) & (l1 >= info.NRL)
    if entered.any():
        q = l1[entered] - info.NRL
        if not green_prev_step[q].all():
            errs.append("I4 entry on red")
    # I5: lane change within a road keeps the group
    rd = (~jl) & (l1 < info.NRL)
    same_road = rd.copy()
    same_road[rd] = info.rol[l0[rd]] == info.rol[l1[rd]]
    changed = same_road & (l0 != l1)
    for idx in np.nonzero(changed)[0]:
        i = int(was[idx])
        if info.in_group(i, int(k0[idx]), int(l0[idx])) and not info.in_group(i, int(k0[idx]), int(l1[idx])):
            errs.append(f"I5 vehicle {i} left its lane group")
            break
    # I6: lane keepers never move back and keep their order
    keep = l0 == l1
    if (x1[keep] < x0[keep] - tol).any():
        errs.append("I6 moved backwards")
    kv = was[keep]
    if kv.size > 1:
        lk = l0[keep]
        o0 = np.lexsort((kv, -x0[keep], lk))
        o1 = np.lexsort((kv, -x1[keep], lk))
        if not np.array_equal(kv[o0], kv[o1]):
            errs.append("I6 overtaking within a lane")
    return errs
