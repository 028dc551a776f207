"""GPU parity of departures from an AOI's connection partway along a lane
(Appendix B.1: a trip may start at a position in a lane; Appendix B.2: an
AOI puts a due vehicle into the lane when the connection is safe) against
the oracle: the pinned scenes step for step, one step from loaded states,
a whole horizon statistically, and a batch against its instances alone."""

import dataclasses

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from paper_2406_10661_amd.workloads import synthetic_state
from tests.parity import compare_one_step
from tests.scenes import jl_between, line_network, state_from, trips_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as O
    O.build()
    return O


@pytest.fixture(scope="module")
def Sim():
    from paper_2406_10661_amd.tsim import Sim
    return Sim


def _scene(lanes, routes, starts, vlanes, xs, vs, status):
    net = line_network(lanes=lanes, policy=W.POLICY_NONE)
    trips = trips_for(routes)
    trips.start_s = np.asarray(starts, np.float32)
    st = state_from(len(routes), vlanes, xs, vs, status=status)
    st["lane"] = np.where(st["status"] == 1, st["lane"], -1).astype(np.int32)
    return net, trips, st


def _jl(lanes):
    net = line_network(lanes=lanes, policy=W.POLICY_NONE)
    return net.n_road_lanes + jl_between(net, 0, 2)


SCENES = {
    "empty_lane": (1, [[0, 2]], [150.0], [-1], [0.0], [0.0], [0]),
    "room_s0": (1, [[0, 2]] * 3, [0.0, 150.0, 0.0], [0, -1, 0], [157.0, 0.0, 40.0], [0.0, 0.0, 0.0], [1, 0, 1]),
    "room_short": (1, [[0, 2]] * 3, [0.0, 150.0, 0.0], [0, -1, 0], [156.9, 0.0, 40.0], [0.0, 0.0, 0.0], [1, 0, 1]),
    "behind_reach_ok": (1, [[0, 2]] * 2, [0.0, 150.0], [0, -1], [140.0, 0.0], [4.0, 0.0], [1, 0]),
    "behind_reach_bad": (1, [[0, 2]] * 2, [0.0, 150.0], [0, -1], [140.5, 0.0], [4.0, 0.0], [1, 0]),
    "most_room_ahead": (2, [[0, 2]] * 4, [0.0, 0.0, 0.0, 150.0], [0, 1, 1, -1], [165.0, 175.0, 100.0, 0.0],
                        [0.0] * 4, [1, 1, 1, 0]),
    "feeder_ok": (1, [[0, 2], [2]], [0.0, 8.0], ["jl", -1], [24.0, 0.0], [3.0, 0.0], [1, 0]),
    "feeder_bad": (1, [[0, 2], [2]], [0.0, 8.0], ["jl", -1], [24.0, 0.0], [3.5, 0.0], [1, 0]),
    "vehicle_before_feeder": (1, [[2], [0, 2], [2]], [0.0, 0.0, 8.0], [2, "jl", -1], [2.0, 24.0, 0.0],
                              [0.0, 10.0, 0.0], [1, 1, 0]),
    "nearest_behind": (1, [[0, 2]] * 3, [0.0, 0.0, 150.0], [0, 0, -1], [140.0, 20.0, 0.0], [4.5, 0.0, 0.0],
                       [1, 1, 0]),
    "two_due": (1, [[0, 2]] * 2, [100.0, 200.0], [-1, -1], [0.0, 0.0], [0.0, 0.0], [0, 0]),
}


@pytest.mark.parametrize("name", sorted(SCENES))
def test_scene_matches_oracle_for_three_steps(O, Sim, name):
    lanes, routes, starts, vl, xs, vs, status = SCENES[name]
    vl = [_jl(lanes) if l == "jl" else l for l in vl]
    net, trips, st = _scene(lanes, routes, starts, vl, xs, vs, status)
    params = W.Params()
    o = O.OracleSim(net, trips, params)
    o.set_state({**st, "x": np.asarray(st["x"], np.float64), "v": np.asarray(st["v"], np.float64)})
    g = Sim(net, trips, params)
    g.set_state(st)
    for k in range(3):
        o.step(1)
        g.step(1)
        a, b = o.get_state(), g.get_state()
        for f in ("status", "lane", "route_pos"):
            assert np.array_equal(a[f], b[f]), (name, k, f, a[f], b[f])
        on = a["status"] == 1
        assert np.allclose(a["x"][on], b["x"][on], rtol=1e-5, atol=1e-4), (name, k)
        assert np.allclose(a["v"][on], b["v"][on], rtol=1e-5, atol=1e-4), (name, k)
    assert g.metrics()["departures"] == o.metrics()["departures"]


def _with_starts(net, trips, rng, hi=0.9):
    """The same trips starting at positions U(0, hi) of their origin road's
    length (float32, as both sides read them)."""
    org = trips.route_roads[trips.route_begin[:-1]]
    s = (rng.uniform(0.0, hi, trips.n_vehicles) * net.road_length[org]).astype(np.float32)
    return dataclasses.replace(trips, start_s=s)


@pytest.mark.parametrize("seed,step,p_active", [(1, 120, 0.4), (2, 250, 0.6)])
def test_starts_one_step(O, Sim, seed, step, p_active):
    """A loaded 4x4 grid whose trips start partway along their origin
    roads: one step from the same state on both sides, many departures
    into occupied lanes."""
    w = W.config1()
    trips = _with_starts(w.network, w.trips, np.random.default_rng(seed))
    st = synthetic_state(w.network, trips, step, seed=seed, p_active=p_active)
    rep = compare_one_step(O, Sim, w.network, trips, w.params, st)
    print("aoi_starts_one_step", {k: v for k, v in rep.items() if not isinstance(v, dict)}, flush=True)
    assert rep["departures"] > 10


def test_starts_horizon_statistics(O, Sim):
    """The 4x4 grid's 600-step horizon with every trip starting partway
    along its origin road: completed trips and mean road speed within 1% of
    the oracle's."""
    w = W.config1()
    trips = _with_starts(w.network, w.trips, np.random.default_rng(7))
    o = O.OracleSim(w.network, trips, w.params)
    o.step(w.n_steps)
    om = o.metrics()
    g = Sim(w.network, trips, w.params)
    g.step(w.n_steps)
    gm = g.metrics()
    print("aoi_starts_horizon", dict(oracle_finished=om["finished"], gpu_finished=gm["n_finished"],
                                     oracle_speed=om["mean_speed_avg"], gpu_speed=gm["mean_speed_avg"]), flush=True)
    assert gm["errors"] == 0
    assert abs(gm["n_finished"] - om["finished"]) <= 0.01 * om["finished"]
    assert abs(gm["mean_speed_avg"] - om["mean_speed_avg"]) <= 0.01 * om["mean_speed_avg"]


def test_starts_in_a_batch_match_alone(Sim):
    """A batch of an instance with start positions and one without: each
    instance's state after 200 steps equals that of a handle of its own."""
    from paper_2406_10661_amd.tsim import Batch
    w = W.config1()
    trips = _with_starts(w.network, w.trips, np.random.default_rng(8))
    b = Batch([w.network, w.network], [trips, w.trips], [w.params, w.params])
    b.step(200)
    for k, t in ((0, trips), (1, w.trips)):
        g = Sim(w.network, t, w.params)
        g.step(200)
        a, e = b.get_state(k), g.get_state()
        for f in ("status", "lane", "route_pos", "x", "v"):
            assert np.array_equal(a[f], e[f]), (k, f)
