"""MOBIL pins (Appendix B.3 randomized MOBIL) on tiny scenes.

``bf_utility`` is an independent configuration-based implementation: it
builds the lane configuration before and after the prospective change,
finds every leader by scanning all vehicles, evaluates the IDM accelerations
of the ego, its new follower and its old follower in both configurations, and
forms u = (a~_ego - a_ego) + p ((a~_new - a_new) + (a~_old - a_old)) - a_th
with the feasibility conditions of the model (gap ahead, new follower's reach
and safe deceleration, same-gap yield, lane group).  The oracle's own
neighbour search uses sorted lanes and leader substitution; only the IDM
function (pinned separately by closed forms) is shared in spirit.

Also pinned: mirror symmetry u_L <-> u_R on two-lane scenes, and the decision
rule (one draw splits [0, p_LC) left-first in proportion u_L+ : u_R+) by the
empirical change frequency over many Philox draws.
"""

import math

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import line_network, trips_for, state_from

P = W.Params()
LIMIT = float(np.float32(13.9))


def idm(v, v0, s, dv):
    """IDM from the equations, floored at -a_emerg; s = inf is the free road."""
    free = 1 - (v / v0) ** P.delta
    if math.isinf(s):
        a = P.a_max * free
    elif s <= 0:
        a = -math.inf
    else:
        ss = P.s0 + max(0.0, v * P.T + v * dv / (2 * math.sqrt(P.a_max * P.b_comf)))
        a = P.a_max * (free - (ss / s) ** 2)
    return max(a, -P.a_emerg)


def bf_utility(veh, i, d, n_lanes, group, road_len, feeders=None):
    """veh: list of dicts (id, lane, x, v, L, f) on one road whose successor
    lanes are empty and green; group: set of lanes connected to the next road;
    feeders: {lane: [(x, v, length of the feeder lane)]} front vehicles of the
    junction lanes entering each lane.  Returns u (or -inf when infeasible)."""
    me = veh[i]
    lane0 = me["lane"]
    k = lane0 + d
    if not 0 <= k < n_lanes:
        return -math.inf
    def dist(l):
        return min(abs(l - g) for g in group)
    if lane0 in group:
        if k not in group:
            return -math.inf
    elif not dist(k) < dist(lane0):
        return -math.inf

    def ahead(a, b):
        return a["x"] > b["x"] or (a["x"] == b["x"] and a["id"] < b["id"])

    def leader(conf, j):
        best = None
        for o in conf:
            if o is j or o["lane"] != j["lane"] or not ahead(o, j):
                continue
            if best is None or ahead(best, o):
                best = o
        return best

    def follower(conf, j):
        best = None
        for o in conf:
            if o is j or o["lane"] != j["lane"] or ahead(o, j):
                continue
            if best is None or ahead(o, best):
                best = o
        return best

    def acc(conf, j, wrong_lane_stop=True):
        ld = leader(conf, j)
        v0 = j["f"] * LIMIT
        a = idm(j["v"], v0, math.inf, 0.0) if ld is None else idm(j["v"], v0, ld["x"] - ld["L"] - j["x"], j["v"] - ld["v"])
        if wrong_lane_stop and j["lane"] not in group:
            a = min(a, idm(j["v"], v0, road_len - j["x"], j["v"]))
        return a

    before = [dict(o) for o in veh]
    after = [dict(o) for o in veh]
    after[i]["lane"] = k
    ego_b, ego_a = before[i], after[i]
    nf_a = follower(after, ego_a)
    of_b = follower(before, ego_b)
    nl_a = leader(after, ego_a)
    # gap ahead
    if nl_a is not None and not (nl_a["x"] - nl_a["L"] - ego_a["x"] > 0):
        return -math.inf
    merging = lane0 not in group
    nf_b = None if nf_a is None else before[nf_a["id_idx"]]
    yields = nf_a is not None and merging and ego_a["x"] - ego_a["L"] > nf_a["x"]
    if nf_a is not None and not yields:
        if not (ego_a["x"] - ego_a["L"] - nf_a["x"] >= nf_a["v"] * P.dt + 0.5 * P.a_max * P.dt ** 2):
            return -math.inf
    if nf_a is not None and not yields and acc(after, nf_a) < -P.b_safe:
        return -math.inf
    # no new follower: no vehicle leaving a feeder junction lane may reach the rear
    if nf_a is None:
        for (xh, vh, lf) in (feeders or {}).get(k, []):
            if not ((ego_a["x"] - ego_a["L"]) - (xh + vh * P.dt + 0.5 * P.a_max * P.dt ** 2 - lf) >= 0):
                return -math.inf
    # same gap, rightward only: a vehicle of lane k+1 between the same k-neighbours
    if d > 0 and k + 1 < n_lanes:
        def gap_of(conf, j):
            lk = [o for o in conf if o["lane"] == k and o is not j]
            up = [o for o in lk if ahead(o, j)]
            dn = [o for o in lk if not ahead(o, j)]
            tl = min(up, key=lambda o: (o["x"], -o["id"])) if up else None
            tf = max(dn, key=lambda o: (o["x"], -o["id"])) if dn else None
            return (None if tl is None else tl["id"], None if tf is None else tf["id"])
        g_me = gap_of(before, ego_b)
        for o in before:
            if o["lane"] == k + 1 and gap_of(before, o) == g_me:
                return -math.inf
    a_e = acc(before, ego_b)
    ta_e = acc(after, ego_a, wrong_lane_stop=False)
    d_new = 0.0 if nf_a is None else acc(after, nf_a) - acc(before, nf_b)
    d_old = 0.0 if of_b is None else acc(after, after[of_b["id_idx"]]) - acc(before, of_b)
    u = (ta_e - a_e) + P.politeness * (d_new + d_old) - P.a_th
    if merging:
        u = max(u, 1.0)
    return u


def random_scene(rng, n_lanes, n_veh, road_len):
    while True:
        lanes = rng.integers(0, n_lanes, n_veh)
        xs = rng.uniform(road_len * 0.3, road_len * 0.7, n_veh)
        ok = True
        for l in range(n_lanes):
            xl = np.sort(xs[lanes == l])
            if np.any(np.diff(xl) < 5.5):
                ok = False
        if ok:
            break
    vs = rng.uniform(0.0, 14.0, n_veh)
    fs = rng.uniform(0.8, 1.2, n_veh).astype(np.float32).astype(np.float64)
    return lanes, xs, vs, fs


def run_scene(oracle_lib, n_lanes, lanes, xs, vs, fs, group_all=True):
    net = line_network(lanes=n_lanes, policy=W.POLICY_NONE)
    n = len(lanes)
    trips = trips_for([[0, 2]] * n, v0_factor=fs)
    o = oracle_lib.OracleSim(net, trips, P)
    st = state_from(n, lanes, xs, vs)
    o.set_state(st)
    o.step(1)
    return net, o.diag()


@pytest.mark.parametrize("seed", range(60))
def test_mobil_matches_bruteforce(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n_lanes = 3 if seed % 2 else 2
    n_veh = int(rng.integers(2, 7))
    L = 300.0
    lanes, xs, vs, fs = random_scene(rng, n_lanes, n_veh, L)
    net, d = run_scene(oracle_lib, n_lanes, lanes, xs, vs, fs)
    veh = [dict(id=j, id_idx=j, lane=int(lanes[j]), x=float(xs[j]), v=float(vs[j]), L=5.0, f=float(fs[j]))
           for j in range(n_veh)]
    group = set(range(n_lanes))  # straight on: every lane connects
    for i in range(n_veh):
        uL = bf_utility(veh, i, -1, n_lanes, group, L)
        uR = bf_utility(veh, i, +1, n_lanes, group, L)
        for got, want in ((d["mobil"][i, 0], uL), (d["mobil"][i, 1], uR)):
            if math.isinf(want):
                assert math.isinf(got) and got < 0, (seed, i, got, want)
            else:
                assert got == pytest.approx(want, abs=1e-9), (seed, i)


def test_mobil_mirror_symmetry(oracle_lib):
    rng = np.random.default_rng(123)
    checked = 0
    for trial in range(40):
        lanes, xs, vs, fs = random_scene(rng, 2, 4, 300.0)
        _, d1 = run_scene(oracle_lib, 2, lanes, xs, vs, fs)
        _, d2 = run_scene(oracle_lib, 2, 1 - lanes, xs, vs, fs)
        # two lanes: the same-gap rule never applies, so mirroring swaps sides
        np.testing.assert_allclose(d1["mobil"][:, 0], d2["mobil"][:, 1], atol=1e-12)
        np.testing.assert_allclose(d1["mobil"][:, 1], d2["mobil"][:, 0], atol=1e-12)
        checked += int(np.isfinite(d1["mobil"][:, :2]).sum())
    assert checked > 20


def test_decision_frequencies(oracle_lib):
    """Vehicle 0 on the middle lane of three, with slow leaders straight ahead
    and open side lanes: u_L, u_R > 0.  Over many steps (fresh Philox counters)
    the left/right frequencies match p_LC u_L+/u_T and p_LC u_R+/u_T within a
    99.9% binomial interval."""
    net = line_network(lanes=3, length=2000.0, policy=W.POLICY_NONE)
    lanes = [1, 1, 0, 2]
    xs = [100.0, 125.0, 40.0, 45.0]
    vs = [10.0, 3.0, 0.0, 0.0]
    fs = [1.0, 1.0, 1.0, 1.0]
    trips = trips_for([[0, 2]] * 4, v0_factor=fs)
    params = W.Params(politeness=0.0, p_max=0.9)
    o = oracle_lib.OracleSim(net, trips, params)
    st = state_from(4, lanes, xs, vs)
    n = 20000
    cl = cr = 0
    uL = uR = pLC = None
    for t in range(n):
        st["step"] = t
        o.set_state(st)
        o.step(1)
        d = o.diag()
        if uL is None:
            uL, uR, uT, pLC = d["mobil"][0]
        cl += d["decision"][0] == 1
        cr += d["decision"][0] == 2
    assert uL > 0 and uR > 0
    uT = uL + uR
    pl = pLC * uL / uT
    pr = pLC * uR / uT
    # p_LC from the piecewise rule with the continuous middle ramp
    if uT >= 1:
        assert pLC == pytest.approx(params.p_max)
    else:
        assert pLC == pytest.approx(params.p_min + (params.p_max - params.p_min) * uT)
    for c, p in ((cl, pl), (cr, pr)):
        sd = math.sqrt(p * (1 - p) / n)
        assert abs(c / n - p) < 3.3 * sd + 1e-9, (c / n, p)


@pytest.mark.parametrize("seed", range(40))
def test_mobil_bruteforce_lane_group(oracle_lib, seed):
    """Left turn at the road end: only lane 0 connects (lane group {0}), so
    vehicles on other lanes face the wrong-lane end obstacle, merge with a
    utility floor of 1, and followers behind a merging vehicle's rear yield."""
    from tests.scenes import left_turn_network
    rng = np.random.default_rng(1000 + seed)
    n_lanes = 3
    n_veh = int(rng.integers(2, 7))
    L = 300.0
    lanes, xs, vs, fs = random_scene(rng, n_lanes, n_veh, L)
    net = left_turn_network(lanes=n_lanes, length=L, policy=W.POLICY_NONE)
    trips = trips_for([[0, 2]] * n_veh, v0_factor=fs)
    o = oracle_lib.OracleSim(net, trips, P)
    o.set_state(state_from(n_veh, lanes, xs, vs))
    o.step(1)
    d = o.diag()
    veh = [dict(id=j, id_idx=j, lane=int(lanes[j]), x=float(xs[j]), v=float(vs[j]), L=5.0, f=float(fs[j]))
           for j in range(n_veh)]
    for i in range(n_veh):
        for col, dd in ((0, -1), (1, +1)):
            want = bf_utility(veh, i, dd, n_lanes, {0}, float(net.road_length[0]))
            got = d["mobil"][i, col]
            if math.isinf(want):
                assert math.isinf(got) and got < 0, (seed, i, dd, got)
            else:
                assert got == pytest.approx(want, abs=1e-9), (seed, i, dd)


@pytest.mark.parametrize("seed", range(40))
def test_mobil_bruteforce_with_feeder(oracle_lib, seed):
    """Two-lane road whose lane 0 is also entered from a junction lane (the
    U-turn at the dead end): a vehicle there can veto a change into lane 0
    that would leave nobody behind the changer."""
    rng = np.random.default_rng(5000 + seed)
    L = 300.0
    n_road = int(rng.integers(1, 5))
    lanes, xs, vs, fs = random_scene(rng, 2, n_road, L)
    xs = xs * 0.2  # near the lane start, where feeder entrants land
    merging = seed % 2 == 1
    if merging:
        # a merging vehicle on lane 1 close to the start, a follower on lane 0
        # behind its rear (that follower yields), and maybe one more ahead
        xi = float(rng.uniform(8.0, 18.0))
        lanes = np.array([1, 0] + ([0] if seed % 4 == 3 else []))
        xs = np.array([xi, float(rng.uniform(0.0, xi - 5.5))] + ([xi + float(rng.uniform(2.0, 30.0))] if seed % 4 == 3 else []))
        n_road = len(lanes)
        vs = rng.uniform(0.0, 14.0, n_road)
        fs = rng.uniform(0.8, 1.2, n_road).astype(np.float32).astype(np.float64)
    if merging:
        # left turn at the end: lane group {0}, vehicles on lane 1 must merge
        from tests.scenes import left_turn_network
        net = left_turn_network(lanes=2, length=L, policy=W.POLICY_NONE)
    else:
        net = line_network(lanes=2, policy=W.POLICY_NONE)
    NRL = net.n_road_lanes
    fq = [q for q in range(net.n_jlanes) if net.jl_out_lane[q] == 0][0]
    xf = float(rng.uniform(15.0, 24.9))
    vf = float(rng.uniform(0.0, 14.0))
    routes = [[0, 2]] * n_road + [[1, 0, 2]]
    assert net.road_from[1] == net.road_to[0] and net.road_to[1] == net.road_from[0]
    trips = trips_for(routes, v0_factor=list(fs) + [1.0])
    o = oracle_lib.OracleSim(net, trips, P)
    st = state_from(n_road + 1, list(lanes) + [NRL + fq], list(xs) + [xf], list(vs) + [vf],
                    route_pos=[0] * (n_road + 1))
    o.set_state(st)
    o.step(1)
    d = o.diag()
    veh = [dict(id=j, id_idx=j, lane=int(lanes[j]), x=float(xs[j]), v=float(vs[j]), L=5.0, f=float(fs[j]))
           for j in range(n_road)]
    feeders = {0: [(xf, vf, float(net.jl_length[fq]))]}
    group = {0} if merging else {0, 1}
    for i in range(n_road):
        for col, dd in ((0, -1), (1, +1)):
            want = bf_utility(veh, i, dd, 2, group, float(net.road_length[0]), feeders)
            got = d["mobil"][i, col]
            if math.isinf(want):
                assert math.isinf(got) and got < 0, (seed, i, dd, got)
            else:
                assert got == pytest.approx(want, abs=1e-9), (seed, i, dd)
