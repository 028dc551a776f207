"""Pins of the oracle's shortest routes (Section 4 "Congestion Pricing":
drivers move to routes of lower cost once roads carry prices; Appendix F:
every road may be priced; Appendix E: routes of shortest travel time).

Reading: the cost of a route is the sum, over every road after its first,
of the fastest open junction lane into it (length / limit), the road's own
travel time (length over the highest limit of its lanes, or a given time)
and its price; among routes of equal cost the one whose next road has the
smaller id is taken at every road (the lexicographically smallest road
sequence when the sums are exact).  Each pin below names the mistake it
catches.
"""

import itertools

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import diamond_network, empty_trips

P = W.Params()
VIA_A = [0, 1, 3, 5]
VIA_B = [0, 2, 4, 5]


def _routes(o, pairs, **kw):
    b, roads, bad = o.shortest_routes([p[0] for p in pairs], [p[1] for p in pairs], **kw)
    return [roads[b[c]:b[c + 1]].tolist() for c in range(len(pairs))], bad


def _price(**kv):
    p = np.zeros(6, np.float32)
    for k, v in kv.items():
        p[int(k[1:])] = v
    return p


@pytest.fixture
def diamond(oracle_lib):
    o = oracle_lib.OracleSim(diamond_network(), empty_trips(), P)
    yield o
    o.close()


def test_free_flow_takes_the_faster_way(diamond):
    """Over A: 21 + 21 + 11 = 53 s; over B: 11 + 21 + 11 = 43 s."""
    r, bad = _routes(diamond, [(0, 5)])
    assert r == [VIA_B] and bad == 0


def test_price_moves_drivers_to_the_other_way(diamond):
    """A price of 15 on road 2 makes B cost 58 against A's 53 (mistakes:
    the price left out, 43 < 53; the slowest of road 1's two junction lanes
    taken instead of the fastest, A = 77 > 58)."""
    r, _ = _routes(diamond, [(0, 5)], price=_price(r2=15))
    assert r == [VIA_A]
    r, _ = _routes(diamond, [(0, 5)], price=_price(r2=5))
    assert r == [VIA_B]


def test_equal_costs_take_the_smaller_next_road(diamond):
    """A price of 10 on road 2: both ways cost 53, so from road 0 the next
    road is 1, the smaller id (mistake: ties to the larger id)."""
    r, _ = _routes(diamond, [(0, 5)], price=_price(r2=10))
    assert r == [VIA_A]


def test_road_time_uses_its_fastest_lane(diamond):
    """Lane 4 (road 2's second lane) at 16 m/s makes road 2 take 80 / 16 =
    5 s; with a price of 14 on road 2, B costs 1 + 5 + 14 + 21 + 11 = 52
    against 53 (mistake: the first lane's limit, 10 s, gives 57)."""
    diamond.set_lane_max_speed([4], [16.0])
    r, _ = _routes(diamond, [(0, 5)], price=_price(r2=14))
    assert r == [VIA_B]


def test_junction_lane_time_follows_its_limit(diamond):
    """Junction lane q0 (lane 8) at 0.32 m/s takes 25 s like q1, so A costs
    77; with a price of 15 on road 2, B (58) wins (mistake: the creation
    limit kept for junction lanes, A = 53)."""
    diamond.set_lane_max_speed([8], [0.32])
    r, _ = _routes(diamond, [(0, 5)], price=_price(r2=15))
    assert r == [VIA_B]


@pytest.mark.parametrize("lane", [10, 3])
def test_closed_junction_lane_is_not_a_way(diamond, lane):
    """Restricting q2 (lane 10), or road 2's lane 3 it leads into, closes
    the only way into road 2: the route goes over A (mistakes: restrictions
    ignored; only the junction lane's own flag read)."""
    diamond.set_lane_restriction([lane], [1])
    r, _ = _routes(diamond, [(0, 5)])
    assert r == [VIA_A]


def test_given_road_times_replace_free_flow(diamond):
    """Road 4 given 40 s: B costs 11 + 41 + 11 = 63 > 53 (mistake: the
    given times ignored)."""
    t = np.array([10, 20, 10, 20, 40, 10], np.float32)
    r, _ = _routes(diamond, [(0, 5)], road_time=t)
    assert r == [VIA_A]


def test_unreachable_and_trivial_pairs(diamond):
    """Road 5 has no way out: 5 -> 0 is unreachable (empty, counted); a
    pair whose origin is its destination is that one road; roads 1 and 2
    are not joined (mistakes: an unreachable pair given a partial route, or
    a one-road route dropped)."""
    r, bad = _routes(diamond, [(5, 0), (3, 3), (1, 4), (2, 5)])
    assert r == [[], [3], [], [2, 4, 5]] and bad == 2


# -- brute force over every simple route, exact costs ------------------------

def _exact_grid(seed):
    """3x3 grid with lengths and limits chosen so that every cost is a small
    integer (exact in FP32): limits 8 m/s, road lengths 8..160 m, junction
    lanes 8 or 16 m."""
    rng = np.random.default_rng(seed)
    net = W.grid_network(3, lanes=2)
    R = net.n_roads
    net.road_length = (8.0 * rng.integers(1, 21, R)).astype(np.float32)
    net.road_limit = np.full(R, 8.0, np.float32)
    net.jl_length = (8.0 * rng.integers(1, 3, net.n_jlanes)).astype(np.float32)
    net.jl_limit = np.full(net.n_jlanes, 8.0, np.float32)
    return net, rng


def _movements(net, closed):
    """Road -> {next road: fastest open junction lane time}, exact."""
    rol = net.road_of_lane()
    NRL = net.n_road_lanes
    mv = {}
    for q in range(net.n_jlanes):
        if closed[NRL + q] or closed[net.jl_out_lane[q]]:
            continue
        a, b = int(rol[net.jl_in_lane[q]]), int(rol[net.jl_out_lane[q]])
        t = float(net.jl_length[q]) / float(net.jl_limit[q])
        mv.setdefault(a, {})
        mv[a][b] = min(mv[a].get(b, np.inf), t)
    return mv


def _brute(net, mv, price, o, d):
    """Least-cost simple route from o to d, ties to the lexicographically
    smallest road sequence, by enumerating every simple route."""
    T = net.road_length.astype(np.float64) / net.road_limit.astype(np.float64)
    best = None
    stack = [(o, (o,), 0.0)]
    while stack:
        r, path, c = stack.pop()
        if r == d:
            key = (c, path)
            if best is None or key < best:
                best = key
            continue
        for b, t in mv.get(r, {}).items():
            if b not in path:
                stack.append((b, path + (b,), c + t + T[b] + price[b]))
    return None if best is None else list(best[1])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_every_simple_route(oracle_lib, seed):
    """Random exact costs, integer prices (ties are common) and a tenth of
    the junction lanes closed: every pair's route is the least-cost simple
    route, ties to the smallest road sequence (mistakes: ties to the larger
    id, a movement cost without the road's time or price, the slowest
    parallel junction lane, a forward search from the origin that breaks
    ties at the destination end)."""
    net, rng = _exact_grid(seed)
    R = net.n_roads
    price = rng.integers(0, 7, R).astype(np.float32)
    closed = np.zeros(net.n_lanes, bool)
    closed[net.n_road_lanes + rng.choice(net.n_jlanes, net.n_jlanes // 10, replace=False)] = True
    o = oracle_lib.OracleSim(net, empty_trips(), P)
    ids = np.nonzero(closed)[0]
    o.set_lane_restriction(ids, np.ones(ids.size, np.int32))
    pairs = [(a, b) for a, b in itertools.product(range(R), range(R))]
    pairs = [pairs[i] for i in rng.choice(len(pairs), 60, replace=False)]
    pairs.sort(key=lambda p: p[1])
    got, bad = _routes(o, pairs, price=price)
    mv = _movements(net, closed)
    n_bad = 0
    for (a, b), g in zip(pairs, got):
        want = _brute(net, mv, price.astype(np.float64), a, b)
        n_bad += want is None
        assert g == (want or []), (a, b)
    assert bad == n_bad
    o.close()


def test_costs_match_scipy_dijkstra_on_a_grid(oracle_lib):
    """8x8 grid with its generator's lengths and limits and random prices:
    each route's cost (summed in FP64 over its movements) equals scipy's
    shortest distance within FP32 rounding, and consecutive roads are joined
    (mistakes: a wrong edge direction, a dropped movement)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    rng = np.random.default_rng(5)
    net = W.grid_network(8)
    R = net.n_roads
    price = rng.uniform(0, 60, R).astype(np.float32)
    mv = _movements(net, np.zeros(net.n_lanes, bool))
    T = net.road_length.astype(np.float64) / net.road_limit.astype(np.float64)
    rows, cols, vals = [], [], []
    for a, nb in mv.items():
        for b, t in nb.items():
            rows.append(a)
            cols.append(b)
            vals.append(t + T[b] + float(price[b]))
    G = csr_matrix((vals, (rows, cols)), shape=(R, R))
    dests = rng.choice(R, 6, replace=False)
    pairs = [(int(a), int(b)) for b in dests for a in rng.choice(R, 20, replace=False)]
    o = oracle_lib.OracleSim(net, empty_trips(), P)
    got, bad = _routes(o, pairs, price=price)
    dist = dijkstra(G.T.tocsr(), directed=True, indices=dests)   # cost to reach each destination
    assert bad == int(np.isinf([dist[list(dests).index(b), a] for a, b in pairs]).sum())
    for (a, b), g in zip(pairs, got):
        ref = dist[list(dests).index(b), a]
        if np.isinf(ref):
            assert g == []
            continue
        assert g[0] == a and g[-1] == b
        assert all(G[g[k], g[k + 1]] > 0 for k in range(len(g) - 1))
        cost = sum(G[g[k], g[k + 1]] for k in range(len(g) - 1))
        assert abs(cost - ref) <= 1e-5 * max(1.0, ref), (a, b, cost, ref)
    o.close()
