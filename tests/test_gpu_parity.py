"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

One-step parity from identical states at several sizes (decisions identical
except near-threshold cases, which are counted; x', v' within 1e-5 relative
with scale; per-lane order identical), multi-step horizon statistics within
1%, determinism, and signal control through the ABI.
"""

import json
import os

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.parity import compare_one_step
from paper_2406_10661_amd.workloads import synthetic_state
from tests import simcheck as S

pytestmark = pytest.mark.gpu

# one JSON line per parity case (counts, largest deviations); directory from
# TSIM_PARITY_REPORT_DIR, else reports/ at the repository root
REPORT = os.environ.get("TSIM_PARITY_REPORT_DIR",
                        os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "reports"))


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build()
    return O


@pytest.fixture(scope="module")
def Sim():
    from paper_2406_10661_amd.tsim import Sim
    return Sim


def _log(name, rep):
    os.makedirs(REPORT, exist_ok=True)
    keep = {k: v for k, v in rep.items() if not isinstance(v, dict)}
    with open(os.path.join(REPORT, "parity_report.jsonl"), "a") as f:
        f.write(json.dumps({"case": name, **keep}) + "\n")
    print(name, keep, flush=True)


@pytest.mark.parametrize("seed,step,p_active", [(1, 60, 0.2), (2, 200, 0.5), (3, 400, 0.7), (4, 31, 0.9)])
def test_c1_synthetic_one_step(O, Sim, seed, step, p_active):
    w = W.config1()
    st = synthetic_state(w.network, w.trips, step, seed=seed, p_active=p_active)
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log(f"c1_synth_s{seed}_t{step}", rep)
    assert rep["active"] > 100


@pytest.mark.parametrize("t", [40, 150, 300, 450])
def test_c1_oracle_trajectory_one_step(O, Sim, t):
    """States reached by the oracle's own dynamics (queues, merges, signals)."""
    w = W.config1()
    o = O.OracleSim(w.network, w.trips, w.params)
    o.step(t)
    st = o.get_state()
    st["x"] = st["x"].astype(np.float32)
    st["v"] = st["v"].astype(np.float32)
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log(f"c1_oracle_t{t}", rep)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_grid_heavy_one_step(O, Sim, seed):
    rng = np.random.default_rng(seed)
    net = W.grid_network(3, spacing=250.0, jitter=20.0, rng=rng, random_edges=True)
    o, d = W.uniform_od(net, rng, 1500)
    trips = W._finish_trips(net, rng, o, d, rng.uniform(0, 100, 1500))
    params = W.Params(seed=seed)
    for step in (50, 120):
        st = synthetic_state(net, trips, step, seed=seed * 10 + step, p_active=0.6)
        rep = compare_one_step(O, Sim, net, trips, params, st)
        _log(f"grid3_s{seed}_t{step}", rep)


@pytest.mark.parametrize("seed", [0, 1])
def test_big_tiles_one_step(O, Sim, seed):
    """Dense long roads (1.5 km, 3 lanes): tiles of several hundred vehicles
    take the kernel's global-memory path instead of the LDS-staged one."""
    rng = np.random.default_rng(100 + seed)
    net = W.grid_network(3, spacing=1500.0, length=1500.0, lanes=3)
    o, d = W.uniform_od(net, rng, 6000)
    trips = W._finish_trips(net, rng, o, d, rng.uniform(0, 50, 6000))
    params = W.Params(seed=seed)
    st = synthetic_state(net, trips, 60, seed=seed, p_active=0.95, min_gap=0.2)
    lanes = st["lane"][st["status"] == 1]
    rol = net.road_of_lane()
    per_road = np.bincount(rol[lanes[lanes < net.n_road_lanes]], minlength=net.n_roads)
    assert per_road.max() > 150
    rep = compare_one_step(O, Sim, net, trips, params, st)
    rep["max_tile"] = int(per_road.max())
    _log(f"big_tiles_s{seed}", rep)


def test_huge_tiles_global_scratch_one_step(O, Sim):
    """4 km, 3-lane roads packed with vehicles: tiles above the LDS capacity
    of the huge pass (512) run on the global per-slot scratch."""
    rng = np.random.default_rng(300)
    net = W.grid_network(3, spacing=4000.0, length=4000.0, lanes=3)
    o, d = W.uniform_od(net, rng, 20000)
    trips = W._finish_trips(net, rng, o, d, rng.uniform(0, 30, 20000))
    params = W.Params(seed=1)
    st = synthetic_state(net, trips, 40, seed=3, p_active=0.97, min_gap=0.2)
    lanes = st["lane"][st["status"] == 1]
    rol = net.road_of_lane()
    per_road = np.bincount(rol[lanes[lanes < net.n_road_lanes]], minlength=net.n_roads)
    assert (per_road > 512).sum() >= 5
    rep = compare_one_step(O, Sim, net, trips, params, st)
    rep["max_tile"] = int(per_road.max())
    _log("huge_tiles", rep)


def test_manual_signals_one_step(O, Sim):
    w = W.config1()
    st = synthetic_state(w.network, w.trips, 77, seed=5, p_active=0.5)
    rng = np.random.default_rng(1)
    nph = np.diff(w.network.junc_phase_begin)
    st["junc_policy"] = np.where(rng.random(w.network.n_junctions) < 0.5, 2, 1).astype(np.int32)
    st["junc_policy"][3] = 0
    st["junc_phase"] = (rng.integers(0, 1000, w.network.n_junctions) % nph).astype(np.int32)
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log("c1_manual_signals", rep)


@pytest.mark.parametrize("step", [90, 91])
def test_max_pressure_one_step(O, Sim, step):
    """Half the junctions of a loaded 4x4 grid under MAX_PRESSURE (the rest
    fixed-time or manual), each entering the step with a random held phase:
    at t = 90 (a multiple of the 30 s first phase: every max-pressure junction
    decides from the lane counts) and t = 91 (they hold).  Vehicles and the
    phases held after the step are compared with the oracle."""
    w = W.config1()
    st = synthetic_state(w.network, w.trips, step, seed=8, p_active=0.8)
    rng = np.random.default_rng(step)
    nph = np.diff(w.network.junc_phase_begin)
    st["junc_policy"] = np.where(rng.random(w.network.n_junctions) < 0.5, 3,
                                 rng.integers(1, 3, w.network.n_junctions)).astype(np.int32)
    st["junc_phase"] = (rng.integers(0, 1000, w.network.n_junctions) % nph).astype(np.int32)
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log(f"c1_max_pressure_t{step}", rep)
    assert rep["max_pressure_junctions"] >= 5


def test_max_pressure_horizon_statistics(O, Sim):
    """Every junction of the 4x4 grid under MAX_PRESSURE (set through the
    ABI at t = 0) for the 600-step horizon: completed trips and time-averaged
    mean road speed within 1% of the oracle's."""
    w = W.config1()
    nj = w.network.n_junctions
    o = O.OracleSim(w.network, w.trips, w.params)
    o.set_junctions(np.full(nj, 3, np.int32), np.zeros(nj, np.int32))
    o.step(w.n_steps)
    om = o.metrics()
    g = Sim(w.network, w.trips, w.params)
    g.set_signal_policy(np.arange(nj), np.full(nj, 3))
    g.step(w.n_steps)
    gm = g.metrics()
    gst = g.get_state()
    rep = dict(oracle_finished=om["finished"], gpu_finished=gm["n_finished"],
               oracle_speed=om["mean_speed_avg"], gpu_speed=gm["mean_speed_avg"])
    _log("c1_max_pressure_horizon", rep)
    assert np.all(gst["junc_policy"] == 3)
    assert gm["errors"] == 0
    assert abs(gm["n_finished"] - om["finished"]) <= 0.01 * om["finished"]
    assert abs(gm["mean_speed_avg"] - om["mean_speed_avg"]) <= 0.01 * om["mean_speed_avg"]


def test_lane_max_speed_one_step(O, Sim):
    """Section 3.2 set_lane_max_speed: 30% of the lanes of a loaded 4x4 grid
    (road and junction lanes) get limits U(5, 13.9) m/s; one step from the
    same state on both sides."""
    w = W.config1()
    st = synthetic_state(w.network, w.trips, 150, seed=9, p_active=0.7)
    rng = np.random.default_rng(4)
    ids = np.nonzero(rng.random(w.network.n_lanes) < 0.3)[0].astype(np.int32)
    st["lane_limits"] = (ids, rng.uniform(5.0, 13.9, ids.size).astype(np.float32))
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log("c1_lane_max_speed", rep)
    assert rep["active"] > 300


def test_lane_max_speed_horizon_statistics(O, Sim):
    """Every road lane of half the roads of the 4x4 grid limited to 8 m/s
    from t = 0 (through the ABI on the GPU): completed trips and mean road
    speed over the 600-step horizon within 1% of the oracle's."""
    w = W.config1()
    rl = w.network.road_of_lane()
    ids = np.nonzero(rl % 2 == 0)[0].astype(np.int32)
    lim = np.full(ids.size, 8.0, np.float32)
    o = O.OracleSim(w.network, w.trips, w.params)
    o.set_lane_max_speed(ids, lim.astype(np.float64))
    o.step(w.n_steps)
    om = o.metrics()
    g = Sim(w.network, w.trips, w.params)
    g.set_lane_max_speed(ids, lim)
    g.step(w.n_steps)
    gm = g.metrics()
    _log("c1_lane_max_speed_horizon", dict(oracle_finished=om["finished"], gpu_finished=gm["n_finished"],
                                           oracle_speed=om["mean_speed_avg"], gpu_speed=gm["mean_speed_avg"]))
    assert gm["errors"] == 0
    assert abs(gm["n_finished"] - om["finished"]) <= 0.01 * om["finished"]
    assert abs(gm["mean_speed_avg"] - om["mean_speed_avg"]) <= 0.01 * om["mean_speed_avg"]


def _restrictions(net, rng, p_road=0.2, p_jl=0.2):
    """Random lane restrictions: a share of the road lanes of multi-lane
    roads and one junction lane of a share of the movements (road to road)
    served by several, such that every movement keeps a junction lane that is
    open (neither it nor its out lane restricted) from an unrestricted lane,
    so that no route is cut off."""
    NRL = net.n_road_lanes
    rl = np.diff(net.road_lane_begin)
    rol = net.road_of_lane()
    restricted = np.zeros(net.n_lanes, bool)
    restricted[:NRL] = (rl[rol[:NRL]] > 1) & (rng.random(NRL) < p_road)
    mov = {}
    for q in range(net.n_jlanes):
        mov.setdefault((int(rol[net.jl_in_lane[q]]), int(rol[net.jl_out_lane[q]])), []).append(q)
    for qs in mov.values():
        if len(qs) > 1 and rng.random() < p_jl:
            restricted[NRL + int(rng.choice(qs))] = True
    for qs in mov.values():
        usable = [q for q in qs if not (restricted[NRL + q] or restricted[net.jl_out_lane[q]]
                                        or restricted[net.jl_in_lane[q]])]
        if not usable:
            q = qs[0]
            restricted[[NRL + q, net.jl_out_lane[q], net.jl_in_lane[q]]] = False
    ids = np.nonzero(restricted)[0].astype(np.int32)
    return ids, np.ones(ids.size, np.int32)


def test_lane_restriction_one_step(O, Sim):
    """Section 3.2 set_lane_restriction: about half of the road lanes of
    multi-lane roads and one junction lane of most movements with several
    restricted on a loaded 4x4 grid (every route keeps an open way; vehicles
    already on restricted lanes stay); one step from the same state on both
    sides."""
    w = W.config1()
    st = synthetic_state(w.network, w.trips, 150, seed=21, p_active=0.7)
    st["restrictions"] = _restrictions(w.network, np.random.default_rng(5), 0.5, 0.7)
    assert st["restrictions"][0].size > 10
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log("c1_lane_restriction", rep)
    assert rep["active"] > 300


def test_lane_restriction_released_one_step(O, Sim):
    """Restricted, then released again before the step: the same step as
    with no restriction at all (the release reaches the lane records, the
    connection table and the departure lanes)."""
    w = W.config1()
    st = synthetic_state(w.network, w.trips, 150, seed=22, p_active=0.7)
    ids, flags = _restrictions(w.network, np.random.default_rng(6), 0.5, 0.5)
    g = Sim(w.network, w.trips, w.params)
    g.set_lane_restriction(ids, flags)
    g.set_lane_restriction(ids, np.zeros_like(flags))
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st, sim=g)
    _log("c1_lane_restriction_released", rep)


def test_lane_restriction_horizon_statistics(O, Sim):
    """Restrictions set from t = 0 (through the ABI on the GPU) and changed
    at t = 300, as a lane plan changes: completed trips and mean road speed
    over the 600-step horizon within 1% of the oracle's."""
    w = W.config1()
    a_ids, a_fl = _restrictions(w.network, np.random.default_rng(7), 0.3, 0.5)
    b_ids, b_fl = _restrictions(w.network, np.random.default_rng(8), 0.3, 0.5)
    o = O.OracleSim(w.network, w.trips, w.params)
    g = Sim(w.network, w.trips, w.params)
    for s in (o, g):
        s.set_lane_restriction(a_ids, a_fl)
        s.step(300)
        s.set_lane_restriction(a_ids, np.zeros_like(a_fl))
        s.set_lane_restriction(b_ids, b_fl)
        s.step(w.n_steps - 300)
    om, gm = o.metrics(), g.metrics()
    _log("c1_lane_restriction_horizon", dict(oracle_finished=om["finished"], gpu_finished=gm["n_finished"],
                                             oracle_speed=om["mean_speed_avg"], gpu_speed=gm["mean_speed_avg"]))
    assert gm["errors"] == 0
    assert abs(gm["n_finished"] - om["finished"]) <= 0.01 * om["finished"]
    assert abs(gm["mean_speed_avg"] - om["mean_speed_avg"]) <= 0.01 * om["mean_speed_avg"]


def test_lane_restriction_in_a_batch_matches_alone(Sim):
    """Restrictions on one instance of a batch (through the batch ABI) leave
    the other untouched: each instance's state after 100 steps equals that
    of a separate handle with the same restrictions (bit for bit)."""
    from paper_2406_10661_amd.tsim import Batch
    w = W.config1()
    ids, flags = _restrictions(w.network, np.random.default_rng(9), 0.3, 0.5)
    b = Batch([w.network, w.network], [w.trips, w.trips], [w.params, w.params])
    b.set_lane_restriction(1, ids, flags)
    b.step(100)
    for k, restrict in ((0, False), (1, True)):
        g = Sim(w.network, w.trips, w.params)
        if restrict:
            g.set_lane_restriction(ids, flags)
        g.step(100)
        a, e = b.get_state(k), g.get_state()
        for f in ("status", "lane", "route_pos", "x", "v"):
            assert np.array_equal(a[f], e[f]), (k, f)


def _with_trip_ends(net, trips, rng, lo=0.2):
    """The same trips with end positions U(lo, 1) of their last road's
    length (float32, as both sides read them)."""
    import dataclasses
    last = trips.route_roads[trips.route_begin[1:] - 1]
    e = (rng.uniform(lo, 1.0, trips.n_vehicles) * net.road_length[last]).astype(np.float32)
    return dataclasses.replace(trips, end_s=e)


def test_trip_end_positions_one_step(O, Sim):
    """Trips ending at positions along their last road (Section 3.2
    set_vehicle_route end position; an AOI's connection as the trip's end):
    one step from a loaded 4x4-grid state, vehicles already past their end
    position finishing in it."""
    w = W.config1()
    trips = _with_trip_ends(w.network, w.trips, np.random.default_rng(11))
    st = synthetic_state(w.network, trips, 300, seed=23, p_active=0.7)
    rep = compare_one_step(O, Sim, w.network, trips, w.params, st)
    _log("c1_trip_end_positions", rep)
    assert rep["active"] > 300


def test_trip_end_positions_horizon_statistics(O, Sim):
    """The 4x4 grid's 600-step horizon with trip end positions: completed
    trips and mean road speed within 1% of the oracle's, more trips ending
    than with trips to the road ends."""
    w = W.config1()
    trips = _with_trip_ends(w.network, w.trips, np.random.default_rng(12))
    o = O.OracleSim(w.network, trips, w.params)
    o.step(w.n_steps)
    om = o.metrics()
    g = Sim(w.network, trips, w.params)
    g.step(w.n_steps)
    gm = g.metrics()
    _log("c1_trip_end_horizon", dict(oracle_finished=om["finished"], gpu_finished=gm["n_finished"],
                                     oracle_speed=om["mean_speed_avg"], gpu_speed=gm["mean_speed_avg"]))
    assert gm["errors"] == 0
    assert abs(gm["n_finished"] - om["finished"]) <= 0.01 * om["finished"]
    assert abs(gm["mean_speed_avg"] - om["mean_speed_avg"]) <= 0.01 * om["mean_speed_avg"]


def test_reroute_with_end_positions_one_step(O, Sim):
    """Rerouted vehicles given end positions on their new last road (half of
    the road's length): one step from the same state on both sides."""
    w = W.config1()
    st = synthetic_state(w.network, w.trips, 150, seed=24, p_active=0.7)
    routes = _reroutes(w.network, w.trips, st, np.random.default_rng(13), 150)
    st["routes"] = [(v, r, float(np.float32(0.5 * w.network.road_length[r[-1]]))) for v, r in routes]
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log("c1_reroute_end_positions", rep)


def _reroutes(net, trips, st, rng, n):
    """Valid new routes for n vehicles of state st: a waiting vehicle ends
    its trip on its origin road; an active one on a road lane turns onto a
    random road its road leads to; one on a junction lane keeps the road that
    lane enters and stops there."""
    rol = net.road_of_lane()
    NRL = net.n_road_lanes
    nexts = {}
    for q in range(net.n_jlanes):
        nexts.setdefault(int(rol[net.jl_in_lane[q]]), set()).add(int(rol[net.jl_out_lane[q]]))
    out = []
    cand = np.nonzero(st["status"] != 2)[0]
    for i in rng.choice(cand, size=min(n, cand.size), replace=False):
        rb = trips.route_begin[i]
        if st["status"][i] == 0:
            out.append((int(i), [int(trips.route_roads[rb])]))
            continue
        lane = int(st["lane"][i])
        cur = int(trips.route_roads[rb + st["route_pos"][i]])
        if lane >= NRL:
            out.append((int(i), [cur, int(rol[net.jl_out_lane[lane - NRL]])]))
        else:
            out.append((int(i), [cur, int(rng.choice(sorted(nexts[cur])))]))
    return out


def test_reroute_one_step(O, Sim):
    """Section 3.2 set_vehicle_route: 150 vehicles of a loaded 4x4 grid
    (waiting, on road lanes and on junction lanes) get new routes; one step
    from the same state on both sides."""
    w = W.config1()
    st = synthetic_state(w.network, w.trips, 120, seed=13, p_active=0.6)
    st["routes"] = _reroutes(w.network, w.trips, st, np.random.default_rng(3), 150)
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log("c1_reroute", rep)
    assert rep["active"] > 200


def test_reroute_horizon_statistics(O, Sim):
    """200 vehicles rerouted before they depart (t = 0: every one waits, so
    the new routes are valid on both sides whatever happens later): each
    turns onto a random road its origin leads to and ends there.  Completed
    trips and mean road speed over the 600-step run within 1% of the
    oracle's."""
    w = W.config1()
    o = O.OracleSim(w.network, w.trips, w.params)
    st0 = o.get_state()
    rol = w.network.road_of_lane()
    nexts = {}
    for q in range(w.network.n_jlanes):
        nexts.setdefault(int(rol[w.network.jl_in_lane[q]]), set()).add(int(rol[w.network.jl_out_lane[q]]))
    rng = np.random.default_rng(5)
    routes = []
    for i in rng.choice(np.nonzero(st0["status"] == 0)[0], size=200, replace=False):
        org = int(w.trips.route_roads[w.trips.route_begin[i]])
        routes.append((int(i), [org, int(rng.choice(sorted(nexts[org])))]))
    g = Sim(w.network, w.trips, w.params)
    for vid, roads in routes:
        o.set_vehicle_route(vid, roads)
        g.set_vehicle_route(vid, roads)
    o.step(w.n_steps)
    g.step(w.n_steps)
    om, gm = o.metrics(), g.metrics()
    _log("c1_reroute_horizon", dict(oracle_finished=om["finished"], gpu_finished=gm["n_finished"],
                                    oracle_speed=om["mean_speed_avg"], gpu_speed=gm["mean_speed_avg"]))
    assert gm["errors"] == 0
    assert abs(gm["n_finished"] - om["finished"]) <= 0.01 * om["finished"]
    assert abs(gm["mean_speed_avg"] - om["mean_speed_avg"]) <= 0.01 * om["mean_speed_avg"]


def test_c1_horizon_statistics(O, Sim):
    """Full 600-step run from t = 0 on both sides: completed trips and the
    time-averaged mean road speed agree within 1%."""
    w = W.config1()
    o = O.OracleSim(w.network, w.trips, w.params)
    o.step(w.n_steps)
    om = o.metrics()
    g = Sim(w.network, w.trips, w.params)
    g.step(w.n_steps)
    gm = g.metrics()
    rep = dict(oracle_finished=om["finished"], gpu_finished=gm["n_finished"],
               oracle_speed=om["mean_speed_avg"], gpu_speed=gm["mean_speed_avg"],
               oracle_att=om["att"], gpu_att=gm["att"])
    _log("c1_horizon", rep)
    assert gm["errors"] == 0
    assert abs(gm["n_finished"] - om["finished"]) <= 0.01 * om["finished"]
    assert abs(gm["mean_speed_avg"] - om["mean_speed_avg"]) <= 0.01 * om["mean_speed_avg"]


def test_determinism_and_invariants(Sim):
    w = W.config1()
    a = Sim(w.network, w.trips, w.params)
    b = Sim(w.network, w.trips, w.params)
    info = S.NetInfo(w.network, w.trips)
    prev = a.get_state()
    for t in range(250):
        green = S.green_set(w.network, t, 1.0)
        a.step(1)
        b.step(1)
        cur = a.get_state()
        errs = S.check_state(info, cur) + S.check_transition(info, prev, cur, green)
        assert not errs, (t, errs)
        prev = cur
    sb = b.get_state()
    for k in ("status", "lane", "route_pos", "x", "v", "finish_step"):
        assert np.array_equal(prev[k], sb[k]), k


@pytest.fixture(scope="module")
def city():
    return W.config3()


@pytest.mark.timeout(900)
def test_c2_full_size_one_step(O, Sim):
    w = W.config2()
    st = W.synthetic_state(w.network, w.trips, 1200, seed=21, p_active=0.6)
    rep = compare_one_step(O, Sim, w.network, w.trips, w.params, st)
    _log("c2_full_synth_t1200", rep)
    assert rep["active"] > 30000


@pytest.mark.timeout(900)
def test_c3_full_size_one_step(O, Sim, city):
    """The paper-scale city (2,464,950 vehicles) in the bench's launch
    configuration: one step from a synthetic state with ~1M active vehicles."""
    st = W.synthetic_state(city.network, city.trips, 3600, seed=31, p_active=0.5)
    rep = compare_one_step(O, Sim, city.network, city.trips, city.params, st)
    _log("c3_full_synth_t3600", rep)
    assert rep["active"] > 500000


@pytest.mark.timeout(900)
def test_c3_dense_state_one_step(O, Sim, city):
    """The city at t = 4,500 as densely loaded as the benchmark's window
    (a synthetic state with 95% of the due vehicles on the network, half of
    them standing, generated on the host), one step on both sides."""
    st = W.synthetic_state(city.network, city.trips, 4500, seed=33, p_active=0.95, p_finished=0.0,
                           p_standing=0.5, min_gap=0.05)
    rep = compare_one_step(O, Sim, city.network, city.trips, city.params, st)
    _log("c3_dense_synth_t4500", rep)
    assert rep["active"] > 1000000


@pytest.mark.timeout(900)
def test_c3_invariants_over_steps(Sim, city):
    """Properties at full size: I1-I7 after each of 20 GPU steps from a
    synthetic mid-horizon state."""
    st = W.synthetic_state(city.network, city.trips, 3600, seed=32, p_active=0.5)
    g = Sim(city.network, city.trips, city.params)
    g.set_state(st)
    info = S.NetInfo(city.network, city.trips)
    prev = g.get_state()
    for t in range(3600, 3620):
        green = S.green_set(city.network, t, 1.0)
        g.step(1)
        cur = g.get_state()
        errs = S.check_state(info, cur) + S.check_transition(info, prev, cur, green)
        assert not errs, (t, errs)
        prev = cur
    assert g.metrics()["errors"] == 0


@pytest.mark.timeout(900)
def test_batch_instances_oracle_one_step(O):
    """Synthetic states of different local steps loaded into five instances
    of one batch (tsim_batch_set_state; one instance of 114,725 vehicles),
    one step of the whole batch, then every instance compared with the oracle
    vehicle by vehicle, with its lane order, queue lengths, road speeds,
    metrics and held phases."""
    from paper_2406_10661_amd.tsim import Batch
    ws = [W.config1(), W.config4_instance(7), W.config4_instance(0), W.config4_instance(20),
          W.config4_instance(13)]
    assert max(w.trips.n_vehicles for w in ws) > 100000
    b = Batch([w.network for w in ws], [w.trips for w in ws], [w.params for w in ws])
    b.step(3)     # the batch is running: the instances join at global step 3 with their own steps
    sts = []
    for k, w in enumerate(ws):
        st = W.synthetic_state(w.network, w.trips, 60 + 97 * k, seed=40 + k, p_active=0.6)
        rng = np.random.default_rng(k)
        nph = np.diff(w.network.junc_phase_begin)
        st["junc_policy"] = rng.integers(1, 4, w.network.n_junctions).astype(np.int32)
        st["junc_phase"] = (rng.integers(0, 1000, w.network.n_junctions) % np.maximum(nph, 1)).astype(np.int32)
        b.set_state(k, st)
        sts.append(st)
    b.step(1)
    for k, w in enumerate(ws):
        rep = compare_one_step(O, None, w.network, w.trips, w.params, sts[k], sim=b.instance(k), stepped=True)
        _log(f"batch_oracle_inst{k}", rep)
        assert rep["active"] > 0
        assert b.metrics(k)["step"] == sts[k]["step"] + 1


def test_batch_frozen_instance_state_is_its_last(Sim):
    """An instance frozen at an odd local step while the batch goes on
    reports, bit for bit, the state of the same instance run alone to that
    step (its lanes are read from the buffer of its last step)."""
    from paper_2406_10661_amd.tsim import Batch
    ws = [W.config1(), W.config4_instance(7)]
    b = Batch([w.network for w in ws], [w.trips for w in ws], [w.params for w in ws])
    b.set_horizon(1, 77)
    b.step(120)
    alone = Sim(ws[1].network, ws[1].trips, ws[1].params)
    alone.step(77)
    a, f = alone.get_state(), b.get_state(1)
    assert f["step"] == 77
    for key in ("status", "lane", "route_pos", "x", "v", "finish_step"):
        assert np.array_equal(a[key], f[key]), key
    assert b.metrics(0)["step"] == 120


def test_batch_instances_match_alone(Sim):
    """A batch of uneven instances (different networks, sizes and seeds),
    stepped through captured graphs, gives each instance the same trajectory,
    bit for bit, as running it alone with direct launches; phases are set
    every 15 steps through both batch phase calls."""
    from paper_2406_10661_amd.tsim import Batch
    ws = [W.config4_instance(i, steps=200) for i in (3, 7, 11)]
    ws = [w if w.trips.n_vehicles <= 40000 else None for w in ws]
    ws = [w for w in ws if w is not None] + [W.config1()]
    b = Batch([w.network for w in ws], [w.trips for w in ws], [w.params for w in ws])
    alone = [Sim(w.network, w.trips, w.params) for w in ws]
    scheds = [W.random_phase_schedule(w.network, 77 + k, 20) for k, w in enumerate(ws)]
    b.set_graph_steps(15)          # the batch replays captured 15-step graphs
    for c in range(10):
        phs = [scheds[k][c] for k in range(len(ws))]
        if c % 2:
            # one batch-wide update; instance 1 left unchanged this time
            allp = [ph if k != 1 else np.full_like(ph, -1) for k, ph in enumerate(phs)]
            b.set_all_phases(np.concatenate(allp))
        for k, w in enumerate(ws):
            js = np.arange(w.network.n_junctions)
            if c % 2 == 0:
                b.set_signal_phases(k, js, phs[k])
            if c % 2 == 0 or k != 1:
                alone[k].set_signal_phases(js, phs[k])
        b.step(15)
        for a in alone:
            for _ in range(15):
                a.step(1)
    for k, w in enumerate(ws):
        sb = b.get_state(k)
        sa = alone[k].get_state()
        for key in ("status", "lane", "route_pos", "x", "v", "finish_step", "junc_policy", "junc_phase"):
            assert np.array_equal(sb[key], sa[key]), (k, key)
        mb, ma = b.metrics(k), alone[k].metrics()
        for key in ("n_finished", "vehicle_steps", "lane_changes", "transfers", "departures", "step"):
            assert mb[key] == ma[key], (k, key, mb[key], ma[key])
        assert mb["mean_speed_avg"] == ma["mean_speed_avg"]
        _log(f"batch_alone_inst{k}", {"vehicles": w.trips.n_vehicles, "active": int(ma["n_active"]),
                                      "finished": int(ma["n_finished"])})


def _dense_big_tile_case(seed=0):
    rng = np.random.default_rng(100 + seed)
    net = W.grid_network(3, spacing=1500.0, length=1500.0, lanes=3)
    o, d = W.uniform_od(net, rng, 6000)
    trips = W._finish_trips(net, rng, o, d, rng.uniform(0, 50, 6000))
    params = W.Params(seed=seed)
    st = synthetic_state(net, trips, 60, seed=seed, p_active=0.95, min_gap=0.2)
    return net, trips, params, st


def _merge_heavy_huge_case():
    """1 km, 4-lane roads holding 217-280 vehicles each, placed on random
    lanes so that many must merge towards their route's lanes: every road
    tile is worked on by a whole workgroup of several wavefronts (the huge
    pass of every schedule), where the merger buckets one wavefront fills
    are read by the others."""
    rng = np.random.default_rng(7)
    net = W.grid_network(3, spacing=1000.0, length=1000.0, lanes=4)
    o, d = W.uniform_od(net, rng, 12000)
    trips = W._finish_trips(net, rng, o, d, rng.uniform(0, 50, 12000))
    st = synthetic_state(net, trips, 60, seed=7, p_active=0.95, min_gap=0.2)
    return net, trips, W.Params(seed=7), st


def test_merge_heavy_huge_tiles_one_step(O, Sim):
    net, trips, params, st = _merge_heavy_huge_case()
    lanes = st["lane"][st["status"] == 1]
    per_road = np.bincount(net.road_of_lane()[lanes[lanes < net.n_road_lanes]], minlength=net.n_roads)
    assert per_road.min() > 176 and per_road.max() <= 448
    rep = compare_one_step(O, Sim, net, trips, params, st)
    _log("merge_heavy_huge", rep)


@pytest.mark.parametrize("case", ["c1", "grid3", "big", "merge"])
def test_schedules_bit_identical(Sim, case):
    """Every update schedule (tiles per wavefront, LDS capacity, overflow to
    the wide pass) gives the same trajectory bit for bit."""
    if case == "c1":
        w = W.config1()
        net, trips, params = w.network, w.trips, w.params
        st = synthetic_state(net, trips, 200, seed=9, p_active=0.7)
    elif case == "grid3":
        rng = np.random.default_rng(5)
        net = W.grid_network(3, spacing=250.0, jitter=20.0, rng=rng, random_edges=True)
        o, d = W.uniform_od(net, rng, 1500)
        trips = W._finish_trips(net, rng, o, d, rng.uniform(0, 100, 1500))
        params = W.Params(seed=5)
        st = synthetic_state(net, trips, 60, seed=55, p_active=0.6)
    elif case == "big":
        net, trips, params, st = _dense_big_tile_case(1)
    else:
        net, trips, params, st = _merge_heavy_huge_case()
    steps = 120 if case == "merge" else 40
    from paper_2406_10661_amd.tsim import SCHEDULES
    ref = None
    for sc in sorted(SCHEDULES):
        g = Sim(net, trips, params)
        g.set_schedule(sc)
        assert g.schedule() == sc
        g.set_state(st)
        g.step(steps)
        s, m = g.get_state(), g.metrics()
        assert m["errors"] == 0
        if ref is None:
            ref = (s, m)
            continue
        for key in ("status", "lane", "route_pos", "x", "v", "finish_step"):
            assert np.array_equal(s[key], ref[0][key]), (sc, key)
        for key in ("vehicle_steps", "lane_changes", "transfers", "departures", "feeder_blocks", "clamps",
                    "n_finished", "mean_speed_avg"):
            assert m[key] == ref[1][key], (sc, key, m[key], ref[1][key])
    _log(f"schedules_{case}", {"active": int((ref[0]["status"] == 1).sum()), "changes": int(ref[1]["lane_changes"])})


@pytest.mark.parametrize("sched", [0, 4])
def test_big_tiles_one_step_other_schedules(O, Sim, sched):
    """Oracle parity of the wide-only and 8-lane schedules on tiles far above
    every group capacity (all of them overflow to the wide pass)."""
    net, trips, params, st = _dense_big_tile_case(0)

    class S(Sim):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.set_schedule(sched)
    rep = compare_one_step(O, S, net, trips, params, st)
    _log(f"big_tiles_sched{sched}", rep)


@pytest.mark.parametrize("case,graph", [("c1", 0), ("c1", 7), ("big", 7)])
def test_concurrent_passes_bit_identical(Sim, case, graph):
    """Update passes on side streams (eager and captured) give the same
    trajectory as the serial launch order, under the schedules that use three
    and four passes."""
    if case == "c1":
        w = W.config1()
        net, trips, params = w.network, w.trips, w.params
        st = synthetic_state(net, trips, 200, seed=9, p_active=0.7)
    else:
        net, trips, params, st = _dense_big_tile_case(1)
    for sc in (1, 6):
        runs = []
        for conc in (0, 1):
            g = Sim(net, trips, params)
            g.set_schedule(sc)
            g.set_concurrency(bool(conc))
            g.set_graph_steps(graph)
            g.set_state(st)
            g.step(33)
            runs.append((g.get_state(), g.metrics()))
            g.close()
        (s0, m0), (s1, m1) = runs
        assert m0["errors"] == 0
        for key in ("status", "lane", "route_pos", "x", "v", "finish_step"):
            assert np.array_equal(s0[key], s1[key]), (sc, key)
        for key in ("step", "vehicle_steps", "lane_changes", "transfers", "departures", "n_finished",
                    "mean_speed_avg", "mean_speed_last"):
            assert m0[key] == m1[key], (sc, key, m0[key], m1[key])
    _log(f"concurrent_{case}_graph{graph}", {"changes": int(m0["lane_changes"])})


@pytest.mark.parametrize("sched", [7, 1])
def test_metrics_read_between_steps_change_nothing(Sim, sched):
    """A step's metric sums are folded by the next step's prepare kernel, or
    on demand when the host reads metrics first: reading the metrics after
    every few steps (eager and captured) gives the same final metrics as one
    read at the end, for a single instance and for the same network twice in
    a batch."""
    from paper_2406_10661_amd.tsim import Batch
    w = W.config1()
    reads = []
    for every, graph in ((None, 0), (7, 0), (7, 7), (1, 0)):
        a = Sim(w.network, w.trips, w.params)
        a.set_schedule(sched)
        a.set_graph_steps(graph)
        done = 0
        while done < 140:
            k = 140 - done if every is None else min(every, 140 - done)
            a.step(k)
            done += k
            if every is not None:
                m = a.metrics()
                assert m["step"] == done
        reads.append(a.metrics())
        a.close()
    for m in reads[1:]:
        for key in ("step", "vehicle_steps", "lane_changes", "transfers", "departures", "n_finished", "errors",
                    "sum_travel_time", "mean_speed_avg", "mean_speed_last"):
            assert m[key] == reads[0][key], (key, m[key], reads[0][key])
    b = Batch([w.network, w.network], [w.trips, w.trips], [w.params, w.params])
    b.set_schedule(sched)
    for _ in range(20):
        b.step(7)
        b.metrics(1)
    for k in range(2):
        m = b.metrics(k)
        for key in ("step", "vehicle_steps", "lane_changes", "n_finished", "mean_speed_avg", "mean_speed_last"):
            assert m[key] == reads[0][key], (k, key, m[key], reads[0][key])
    b.close()
    _log(f"metrics_reads_sched{sched}", {"vehicle_steps": int(reads[0]["vehicle_steps"])})


def test_autotune_launch_steps_like_plain(Sim):
    """The schedule-and-concurrency autotuner also runs real steps (twice as
    many as the schedule autotuner) and leaves the chosen pair set."""
    from paper_2406_10661_amd.tsim import SCHEDULES
    w = W.config1()
    a = Sim(w.network, w.trips, w.params)
    b = Sim(w.network, w.trips, w.params)
    a.step(80)
    b.step(80)
    sc, conc, us = a.autotune_launch(steps=4, rounds=1)
    b.step(4 * 2 * len(SCHEDULES))
    assert sc in SCHEDULES and a.schedule() == sc and isinstance(conc, bool)
    assert us.shape == (2, len(SCHEDULES)) and np.all(us > 0)
    a.step(25)
    b.step(25)
    sa, sb = a.get_state(), b.get_state()
    for key in ("status", "lane", "route_pos", "x", "v", "finish_step"):
        assert np.array_equal(sa[key], sb[key]), key
    assert a.metrics()["vehicle_steps"] == b.metrics()["vehicle_steps"]
    _log("autotune_launch_c1", {"chosen": sc, "concurrent": conc})


def test_autotune_steps_like_plain(Sim):
    """The autotuner's trial steps are real steps: afterwards the state equals
    a plain run of the same length, and the chosen schedule is reported."""
    from paper_2406_10661_amd.tsim import SCHEDULES
    w = W.config1()
    a = Sim(w.network, w.trips, w.params)
    b = Sim(w.network, w.trips, w.params)
    a.step(100)
    b.step(100)
    sc, us = a.autotune(steps=5, rounds=2)
    b.step(5 * 2 * len(SCHEDULES))
    assert sc in SCHEDULES and a.schedule() == sc
    assert np.all(us > 0)
    sa, sb = a.get_state(), b.get_state()
    for key in ("status", "lane", "route_pos", "x", "v", "finish_step"):
        assert np.array_equal(sa[key], sb[key]), key
    assert a.metrics()["vehicle_steps"] == b.metrics()["vehicle_steps"]
    _log("autotune_c1", {"chosen": sc, "us_per_step": [float(x) for x in us]})
