"""One-step GPU-vs-oracle comparison used by the parity tests.

Both sides start from the same state (positions and speeds as float32), take
one step, and are compared vehicle by vehicle:
  * decisions (status, lane, route position, departure) must be identical,
    except where the oracle reports a near-threshold margin for that vehicle
    (|Delta a - a_th|, |a~_new + b_safe|, gap margins, |r - boundary|,
    |x' - bound| or |x' - lane end|, departure room) -- such cases are counted
    and returned;
  * where the decision matches, x' and v' agree within
    |d| <= 1e-5 * max(|ref|, scale), scale = lane length for x and the
    desired speed for v;
  * per-lane vehicle order (the sensing index) identical on lanes without a
    near-threshold vehicle;
  * lane waiting counts and road mean speeds identical / within tolerance
    away from near cases.
"""

import numpy as np

REL = 1e-5
EPS_ACC = 1e-4       # m/s^2
EPS_POS_ABS = 1e-4   # m


def pos_eps(lane_len):
    # float32 positions carry about 8e-8 relative error per operation
    return np.maximum(EPS_POS_ABS, 2e-6 * lane_len)


def oracle_one_step(O, net, trips, params, st):
    o = O.OracleSim(net, trips, params)
    s64 = dict(st)
    s64["x"] = np.asarray(st["x"], np.float32).astype(np.float64)
    s64["v"] = np.asarray(st["v"], np.float32).astype(np.float64)
    o.set_state(s64)
    if "junc_policy" in st:
        o.set_junctions(st["junc_policy"], st["junc_phase"])
    if "lane_limits" in st:
        ids, lim = st["lane_limits"]
        o.set_lane_max_speed(ids, np.asarray(lim, np.float32).astype(np.float64))
    if "restrictions" in st:
        o.set_lane_restriction(*st["restrictions"])
    for vid, roads, *end in st.get("routes", ()):
        o.set_vehicle_route(vid, roads, *end)
    if "shortest" in st:
        oracle_reroute_shortest(o, net, trips, *st["shortest"])
    o.step(1)
    return o


def oracle_reroute_shortest(o, net, trips, vids, price=None, road_time=None):
    """The oracle's side of a reroute to least-cost routes: from the
    oracle's own state, each listed vehicle that has not finished takes the
    least-cost route from where it is (its origin road while it waits, the
    road of its lane, or, on a junction lane, the road that lane enters,
    kept after the road it left) to the last road of its route in force;
    unreachable destinations leave the route as it was.  Returns the number
    of vehicles that kept their route."""
    s = o.get_state()
    rol = net.road_of_lane()
    NRL = net.n_road_lanes
    end_s = getattr(trips, "end_s", None)
    jobs, starts, dests = [], [], []
    kept = 0
    for i in vids:
        i = int(i)
        if s["status"][i] == 2:
            kept += 1
            continue
        k, roads = o.route(i)
        prefix, start = [], int(roads[0])
        if s["status"][i] == 1:
            lane = int(s["lane"][i])
            if lane >= NRL:
                prefix, start = [int(roads[k])], int(rol[net.jl_out_lane[lane - NRL]])
            else:
                start = int(rol[lane])
        jobs.append((i, prefix))
        starts.append(start)
        dests.append(int(roads[-1]))
    begin, rr, _ = o.shortest_routes(starts, dests, price, road_time)
    for c, (i, prefix) in enumerate(jobs):
        if begin[c + 1] == begin[c]:
            kept += 1
            continue
        e = None if end_s is None or end_s[i] < 0 else float(end_s[i])
        o.set_vehicle_route(i, prefix + rr[begin[c]:begin[c + 1]].tolist(), e)
    return kept


def compare_one_step(O, sim_cls, net, trips, params, st, sim=None, stepped=False):
    """Returns a report dict; raises AssertionError on a parity failure.
    With stepped=True, `sim` (an instance view of a batch) already took the
    step from st."""
    o = oracle_one_step(O, net, trips, params, st)
    ost = o.get_state()
    od = o.diag()
    om = o.metrics()
    g = sim if sim is not None else sim_cls(net, trips, params)
    if not stepped:
        g.set_state(st)
        if "lane_limits" in st:
            g.set_lane_max_speed(*st["lane_limits"])
        if "restrictions" in st:
            g.set_lane_restriction(*st["restrictions"])
        for vid, roads, *end in st.get("routes", ()):
            g.set_vehicle_route(vid, roads, *end)
        if "shortest" in st:
            g.reroute_shortest(*st["shortest"])
        g.step(1)
    gst = g.get_state()
    gm = g.metrics()
    N = trips.n_vehicles
    lane_len = np.concatenate([np.repeat(net.road_length, np.diff(net.road_lane_begin)),
                               net.jl_length]).astype(np.float64)
    lim = np.concatenate([np.repeat(net.road_limit, np.diff(net.road_lane_begin)), net.jl_limit]).astype(np.float64)
    m = od["margin"]
    st_lane = np.asarray(st["lane"])
    ref_len = np.where(st_lane >= 0, lane_len[np.maximum(st_lane, 0)], 1.0)
    pe = pos_eps(ref_len)
    # near-threshold categories (the oracle's margins): the MOBIL threshold
    # |u_d|, a gap margin, the new follower's |a~ + b_safe|, the draw's
    # distance to a decision boundary, |x' - bound| or |x' - lane end|, and a
    # departure's room margin
    cats = {"mobil_threshold": m[:, 0] < EPS_ACC, "gap": m[:, 1] < pe, "b_safe": m[:, 2] < EPS_ACC,
            "draw": m[:, 3] < 1e-4 * (params.p_max - params.p_min), "bound_or_lane_end": m[:, 4] < pe,
            "departure_room": m[:, 5] < pe}
    near = np.zeros(len(m), bool)
    for c in cats.values():
        near |= c
    # departures cascade into their lane: a near departure marks its lane's road
    same = ((gst["status"] == ost["status"]) & (gst["lane"] == ost["lane"]) & (gst["route_pos"] == ost["route_pos"]))
    bad = ~same & ~near
    rep = dict(n=N, active=int((ost["status"] == 1).sum()), mismatched=int((~same).sum()),
               near=int(near.sum()), near_mismatch=int((~same & near).sum()),
               near_by=({k: int(c.sum()) for k, c in cats.items()}),
               near_mismatch_by=({k: int((c & ~same).sum()) for k, c in cats.items()}),
               changes=int(om["lane_changes"]), transfers=int(om["transfers"]),
               departures=int(om["departures"]))
    if bad.any():
        idx = np.nonzero(bad)[0][:10]
        detail = [(int(i), int(st["status"][i]), int(st_lane[i]), float(st["x"][i]), float(st["v"][i]),
                   "gpu", int(gst["status"][i]), int(gst["lane"][i]), float(gst["x"][i]),
                   "ora", int(ost["status"][i]), int(ost["lane"][i]), float(ost["x"][i]),
                   "dec", int(od["decision"][i]), int(od["event"][i]), m[i].tolist()) for i in idx]
        raise AssertionError(f"decision mismatch on {int(bad.sum())} vehicles: {detail}")
    ok = same & (ost["status"] == 1)
    xl = lane_len[np.maximum(ost["lane"], 0)]
    vscale = trips.v0_factor.astype(np.float64) * lim[np.maximum(ost["lane"], 0)]
    dx = np.abs(gst["x"].astype(np.float64) - ost["x"])
    dv = np.abs(gst["v"].astype(np.float64) - ost["v"])
    tx = REL * np.maximum(np.abs(ost["x"]), xl)
    tv = REL * np.maximum(np.abs(ost["v"]), vscale)
    badx = ok & (dx > tx)
    badv = ok & (dv > tv)
    if badx.any() or badv.any():
        i = int(np.nonzero(badx | badv)[0][0])
        raise AssertionError(f"value mismatch: {int(badx.sum())} x, {int(badv.sum())} v; e.g. vehicle {i} "
                             f"x {gst['x'][i]} vs {ost['x'][i]}, v {gst['v'][i]} vs {ost['v'][i]}, "
                             f"start lane {st_lane[i]} x {st['x'][i]} v {st['v'][i]}")
    rep["max_rel_dx"] = float(np.max(dx[ok] / np.maximum(np.abs(ost["x"][ok]), xl[ok]), initial=0.0))
    rep["max_rel_dv"] = float(np.max(dv[ok] / np.maximum(np.abs(ost["v"][ok]), vscale[ok]), initial=0.0))
    # sensing index: per-lane order
    off, ids = g.lane_order()
    act = np.nonzero(ost["status"] == 1)[0]
    order = act[np.lexsort((act, -ost["x"][act], ost["lane"][act]))]
    o_lane = ost["lane"][order]
    NL = net.n_lanes
    o_off = np.searchsorted(o_lane, np.arange(NL + 1))
    tainted = np.zeros(NL, bool)
    nm = np.nonzero(~same | near)[0]
    for i in nm:
        for l in (st_lane[i], ost["lane"][i], gst["lane"][i]):
            if l >= 0:
                tainted[l] = True
    g_cnt = np.diff(off)
    o_cnt = np.diff(o_off)
    clean = ~tainted
    assert np.array_equal(g_cnt[clean], o_cnt[clean]), "lane occupancy differs"
    g_lane_of = np.repeat(np.arange(NL), g_cnt)
    o_lane_of = np.repeat(np.arange(NL), o_cnt)
    ga = ids[clean[g_lane_of]]
    ob = order[clean[o_lane_of]]
    assert np.array_equal(ga, ob), f"lane order differs on {int((ga != ob).sum())} positions"
    # metrics
    gw = g.lane_waiting_counts()
    ow = o.lane_waiting()
    vnear = np.zeros(NL, bool)
    vv = np.abs(ost["v"] - 0.1) < 1e-4
    for i in np.nonzero(vv)[0]:
        vnear[st_lane[i]] = True
    wl = ~tainted & ~vnear
    assert np.array_equal(gw[wl], ow[wl]), "lane waiting counts differ"
    rs = g.road_mean_speed()
    osv, oc = o.road_stats()
    road_t = np.zeros(net.n_roads, bool)
    rol = net.road_of_lane()
    for l in np.nonzero(tainted[:net.n_road_lanes])[0]:
        road_t[rol[l]] = True
    has = (oc > 0) & ~road_t
    ors = np.where(oc > 0, osv / np.maximum(oc, 1), -1.0)
    assert np.all((rs[oc == 0] == -1.0)), "empty roads must report -1"
    np.testing.assert_allclose(rs[has], ors[has], rtol=1e-5, atol=1e-5 * 20)
    if rep["near_mismatch"] == 0:
        for k in ("lane_changes", "transfers", "departures", "feeder_blocks"):
            assert int(gm[k]) == int(om[k]), (k, gm[k], om[k])
        assert int(gm["n_finished"]) == int(om["finished"])
        assert abs(gm["mean_speed_last"] - om["mean_speed_last"]) <= 1e-5 * max(1.0, om["mean_speed_last"])
    assert gm["errors"] == 0
    # signal state after the step: policies, and the phase every MANUAL or
    # MAX_PRESSURE junction holds (decided from the step-start lane counts,
    # which no decision of this step changes)
    if "junc_policy" in st:
        opol, oph = o.junctions()
        assert np.array_equal(gst["junc_policy"], opol), "junction policies differ"
        held = (opol == 2) | (opol == 3)
        assert np.array_equal(gst["junc_phase"][held], oph[held]), "held junction phases differ"
        rep["max_pressure_junctions"] = int((opol == 3).sum())
    rep["gpu_metrics"] = gm
    rep["oracle_metrics"] = om
    return rep
