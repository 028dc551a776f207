"""Generator checks: sizes, connectivity, lane-length floor, route validity."""

import numpy as np
import pytest
from scipy.sparse.csgraph import connected_components

from paper_2406_10661_amd import workloads as W


def _routes_valid(net, trips):
    rol = net.road_of_lane()
    pairs = set(zip(rol[net.jl_in_lane].tolist(), rol[net.jl_out_lane].tolist()))
    rb, rr = trips.route_begin, trips.route_roads
    for i in range(trips.n_vehicles):
        r = rr[rb[i]:rb[i + 1]]
        assert len(r) >= 1
        for a, b in zip(r[:-1], r[1:]):
            assert (int(a), int(b)) in pairs


def test_config1_sizes():
    w = W.config1()
    n = w.network
    assert n.n_junctions == 16 and n.n_roads == 48 and n.n_road_lanes == 96
    # movements: straight from every lane, turns from the outer lanes only
    assert n.n_jlanes == 136
    assert w.trips.n_vehicles == 1000
    assert (w.trips.depart_time >= 0).all() and (w.trips.depart_time < 300).all()
    _routes_valid(n, w.trips)
    # one phase per approach
    assert len(n.phase_duration) == n.n_roads
    assert np.all(n.phase_duration == 30.0)


def test_every_junction_lane_in_exactly_one_phase():
    w = W.config1()
    n = w.network
    counts = np.bincount(n.phase_green_jl, minlength=n.n_jlanes)
    assert np.all(counts == 1)


def test_lane_length_floor_single_hop():
    p = W.Params()
    vmax = 1.2 * 16.7
    floor = vmax * p.dt + 0.5 * p.a_max * p.dt ** 2
    for w in (W.config1(),):
        assert w.network.road_length.min() > floor
        assert w.network.jl_length.min() > floor


@pytest.mark.slow
def test_config2_connectivity_and_routes():
    w = W.config2()
    n = w.network
    assert n.n_junctions == 1024 and n.n_roads == 3968
    assert n.road_length.min() >= 150 and n.road_length.max() <= 400
    G = W.movement_graph(n)
    assert connected_components(G, directed=True, connection="strong")[0] == 1
    sub = W.Trips(w.trips.depart_time[:2000], w.trips.route_begin[:2001], w.trips.route_roads,
                  w.trips.v0_factor[:2000], w.trips.length[:2000])
    _routes_valid(n, sub)


def test_small_city_network_connected():
    rng = np.random.default_rng(5)
    n = W.city_network(400, rng)
    G = W.movement_graph(n)
    assert connected_components(G, directed=True, connection="strong")[0] == 1
    deg = 2 * n.n_roads / 2 / n.n_junctions
    assert abs(deg - 3.5) < 0.05
    assert n.road_length.min() >= 30.0


def test_generators_deterministic():
    a, b = W.config1(), W.config1()
    assert np.array_equal(a.trips.route_roads, b.trips.route_roads)
    assert np.array_equal(a.trips.v0_factor, b.trips.v0_factor)


def test_workload_file_roundtrip(tmp_path):
    """A workload saved to .npz loads back field for field (plain arrays, no
    pickles), with its parameters, name and horizon."""
    from dataclasses import fields
    w = W.config1()
    p = tmp_path / "w.npz"
    W.save_workload(w, p)
    v = W.load_workload(p)
    assert (v.name, v.n_steps, v.params) == (w.name, w.n_steps, w.params)
    for f in fields(W.Network):
        a, b = getattr(w.network, f.name), getattr(v.network, f.name)
        assert a.dtype == b.dtype and np.array_equal(a, b), f.name
    for f in fields(W.Trips):
        a, b = getattr(w.trips, f.name), getattr(v.trips, f.name)
        if a is None:   # optional field left unset
            assert b is None, f.name
            continue
        assert a.dtype == b.dtype and np.array_equal(a, b), f.name


def test_served_job_without_routes_keeps_every_other_draw():
    """config5_job(route=False) leaves the routes to the server and draws
    everything else as the routed job does; the origin and destination
    roads and the prices are kept for the router."""
    a = W.config5_job(3, max_vehicles=2000)
    b = W.config5_job(3, max_vehicles=2000, route=False)
    assert b.trips.route_begin is None and b.trips.route_roads is None
    for f in ("depart_time", "v0_factor", "length"):
        assert np.array_equal(getattr(a.trips, f), getattr(b.trips, f))
    o, d = b.extra["od"]
    rb = a.trips.route_begin
    assert np.array_equal(a.trips.route_roads[rb[:-1]], o)
    assert np.array_equal(a.trips.route_roads[rb[1:] - 1], d)
    assert (a.extra["price"] is None) == (a.extra["kind"] == "timing_plan")
