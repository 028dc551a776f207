"""Seeded synthetic road networks, trip tables and parameters.

These generators stand in for the city datasets of the paper's performance
comparison (Appendix C, Table A2: up to 93,564 roads, 26,479 junctions and
2,464,950 vehicles), which are not available.  They produce plain numpy arrays
in the layout the C ABI takes (``include/tsim.h``) and hold none of the
simulation arithmetic: no car-following, lane-changing, signal or transfer
rule lives here.  Both the CPU oracle and the HIP library consume exactly these
arrays.

Network conventions (Appendix B.1 object definitions):
  * a road is a set of parallel lanes sharing one length and speed limit;
    lane index 0 within a road is the leftmost lane (right-hand traffic);
  * road lanes are numbered road by road: road r owns the global lane ids
    ``road_lane_begin[r] .. road_lane_begin[r+1]-1``;
  * junction lanes connect one road lane to one road lane of the next road;
    in the global lane-id space they follow all road lanes;
  * each junction has candidate phases (Section 3.1 "map data ... candidate
    traffic signal phases"); a phase is the set of junction lanes it makes
    green.

Lane connections and phases follow one fixed rule set (movements classified by
turn angle; one phase per incoming approach, in in-road id order), so every
phase is conflict free at any junction degree.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra, connected_components, minimum_spanning_tree

POLICY_NONE = 0
POLICY_FIXED_TIME = 1
POLICY_MANUAL = 2
POLICY_MAX_PRESSURE = 3

JUNCTION_LANE_LENGTH = 25.0
TURN_STRAIGHT_DEG = 45.0


@dataclass
class Params:
    """Vehicle-model and run parameters (IDM, randomized MOBIL, step size)."""

    dt: float = 1.0
    T: float = 1.5          # IDM safe time headway [s]
    a_max: float = 2.0      # IDM maximum acceleration [m/s^2]
    b_comf: float = 4.5     # IDM comfortable deceleration [m/s^2]
    s0: float = 2.0         # IDM minimum gap [m]
    delta: float = 4.0      # IDM free-road exponent
    politeness: float = 0.1
    a_th: float = 0.2       # MOBIL switching threshold [m/s^2]
    b_safe: float = 4.0     # MOBIL safe deceleration of the new follower [m/s^2]
    p_max: float = 0.5      # lane-change probability cap
    p_min: float = 2e-8     # lane-change probability floor
    a_emerg: float = 9.0    # braking floor [m/s^2]
    seed: int = 0

    def as_dict(self):
        return asdict(self)


@dataclass
class Network:
    junction_xy: np.ndarray          # float64 [J, 2]   geometry only
    road_from: np.ndarray            # int32   [R]
    road_to: np.ndarray              # int32   [R]
    road_lane_begin: np.ndarray      # int32   [R+1]
    road_length: np.ndarray          # float32 [R]
    road_limit: np.ndarray           # float32 [R]
    jl_in_lane: np.ndarray           # int32   [NJ]  road-lane id
    jl_out_lane: np.ndarray          # int32   [NJ]  road-lane id
    jl_length: np.ndarray            # float32 [NJ]
    jl_limit: np.ndarray             # float32 [NJ]
    junc_phase_begin: np.ndarray     # int32   [J+1]
    phase_duration: np.ndarray       # float32 [P]
    phase_green_begin: np.ndarray    # int32   [P+1]
    phase_green_jl: np.ndarray       # int32   [G]   junction-lane index (0-based in NJ)
    junc_policy: np.ndarray          # int32   [J]

    @property
    def n_junctions(self):
        return int(self.junction_xy.shape[0])

    @property
    def n_roads(self):
        return int(self.road_from.shape[0])

    @property
    def n_road_lanes(self):
        return int(self.road_lane_begin[-1])

    @property
    def n_jlanes(self):
        return int(self.jl_in_lane.shape[0])

    @property
    def n_lanes(self):
        return self.n_road_lanes + self.n_jlanes

    def road_of_lane(self):
        return np.repeat(np.arange(self.n_roads, dtype=np.int32),
                         np.diff(self.road_lane_begin)).astype(np.int32)

    def nbytes(self):
        return sum(v.nbytes for v in self.__dict__.values() if isinstance(v, np.ndarray))


@dataclass
class Trips:
    depart_time: np.ndarray   # float32 [N]
    route_begin: np.ndarray   # int32   [N+1]
    route_roads: np.ndarray   # int32   [sum of route lengths]
    v0_factor: np.ndarray     # float32 [N]  desired speed = v0_factor * lane limit
    length: np.ndarray        # float32 [N]
    end_s: np.ndarray = None  # float32 [N]  trip end position on the last road (None: its end)
    start_s: np.ndarray = None  # float32 [N]  trip start position on the origin road (None: its start)

    @property
    def n_vehicles(self):
        return int(self.depart_time.shape[0])


@dataclass
class Workload:
    name: str
    network: Network
    trips: Trips
    params: Params
    n_steps: int
    extra: dict = field(default_factory=dict)


def save_workload(w: Workload, path):
    """Writes a generated workload (network, trips, parameters, horizon) to
    an .npz file of plain arrays, so that a later process can load it in
    seconds instead of generating it again."""
    from dataclasses import asdict, fields
    arrs = {"name": np.array(w.name), "n_steps": np.array(w.n_steps, np.int64)}
    for f in fields(Network):
        arrs["network." + f.name] = getattr(w.network, f.name)
    for f in fields(Trips):
        if getattr(w.trips, f.name) is not None:
            arrs["trips." + f.name] = getattr(w.trips, f.name)
    for k, v in asdict(w.params).items():
        arrs["params." + k] = np.array(v)
    np.savez(path, **arrs)


def load_workload(path) -> Workload:
    """Reads a workload written by save_workload (plain arrays only)."""
    from dataclasses import fields
    with np.load(path, allow_pickle=False) as z:
        net = Network(**{f.name: z["network." + f.name] for f in fields(Network)})
        trips = Trips(**{f.name: z["trips." + f.name] for f in fields(Trips) if "trips." + f.name in z.files})
        params = Params(**{f.name: type(f.default)(z["params." + f.name][()]) for f in fields(Params)})
        return Workload(str(z["name"][()]), net, trips, params, int(z["n_steps"][()]))


# --------------------------------------------------------------------------
# network construction
# --------------------------------------------------------------------------

def _build_network(xy, edges, e_len, e_lanes, e_limit, phase_seconds=30.0,
                   policy=POLICY_FIXED_TIME, phase_rng=None, phase_range=None):
    """Directed roads from undirected edges, movements, junction lanes, phases.

    edges: int array [E, 2] of undirected junction pairs (a < b not required);
    road 2e is a->b and road 2e+1 is b->a, both with the edge's attributes.
    """
    xy = np.asarray(xy, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.int64)
    E = edges.shape[0]
    J = xy.shape[0]
    rf = np.empty(2 * E, np.int64)
    rt = np.empty(2 * E, np.int64)
    rf[0::2], rt[0::2] = edges[:, 0], edges[:, 1]
    rf[1::2], rt[1::2] = edges[:, 1], edges[:, 0]
    R = 2 * E
    nl = np.repeat(np.asarray(e_lanes, np.int64), 2)
    rlen = np.repeat(np.asarray(e_len, np.float32), 2)
    rlim = np.repeat(np.asarray(e_limit, np.float32), 2)
    lane_begin = np.zeros(R + 1, np.int64)
    np.cumsum(nl, out=lane_begin[1:])

    # movements: for each in-road r (a->j) and out-road r2 (j->b)
    out_order = np.argsort(rf, kind="stable")
    out_start = np.searchsorted(rf[out_order], np.arange(J + 1))
    in_order = np.argsort(rt, kind="stable")
    in_start = np.searchsorted(rt[in_order], np.arange(J + 1))
    deg_nb = np.zeros(J, np.int64)  # number of distinct neighbours
    for j in range(J):
        deg_nb[j] = len(set(rt[out_order[out_start[j]:out_start[j + 1]]].tolist()))

    jl_in, jl_out, jl_lim = [], [], []
    jl_junc = []
    for j in range(J):
        outs = np.sort(out_order[out_start[j]:out_start[j + 1]])
        ins = np.sort(in_order[in_start[j]:in_start[j + 1]])
        for r in ins:
            a = rf[r]
            cand = [r2 for r2 in outs if rt[r2] != a]
            if not cand:
                cand = list(outs)  # dead end: U-turn allowed
            h1 = xy[j] - xy[a]
            n = nl[r]
            for r2 in cand:
                b = rt[r2]
                m = nl[r2]
                if b == a:
                    kind = "left"  # U-turn uses the leftmost lanes
                else:
                    h2 = xy[b] - xy[j]
                    ang = math.degrees(math.atan2(h1[0] * h2[1] - h1[1] * h2[0],
                                                  h1[0] * h2[0] + h1[1] * h2[1]))
                    if abs(ang) <= TURN_STRAIGHT_DEG:
                        kind = "straight"
                    elif ang > 0:
                        kind = "left"
                    else:
                        kind = "right"
                if kind == "straight":
                    pairs = [(i, min(i, m - 1)) for i in range(n)]
                elif kind == "left":
                    pairs = [(0, 0)]
                else:
                    pairs = [(n - 1, m - 1)]
                for (i, o) in pairs:
                    jl_in.append(lane_begin[r] + i)
                    jl_out.append(lane_begin[r2] + o)
                    jl_lim.append(min(rlim[r], rlim[r2]))
                    jl_junc.append(j)
    jl_in = np.asarray(jl_in, np.int64)
    jl_out = np.asarray(jl_out, np.int64)
    NJ = jl_in.shape[0]
    road_of_lane = np.repeat(np.arange(R), nl)

    # phases: one per incoming approach, in in-road id order
    ph_begin = np.zeros(J + 1, np.int64)
    ph_dur = []
    gr_begin = [0]
    gr_jl = []
    jl_in_road = road_of_lane[jl_in]
    jl_junc = np.asarray(jl_junc, np.int64)
    order = np.lexsort((np.arange(NJ), jl_in_road, jl_junc))
    ptr = 0
    for j in range(J):
        ins = np.sort(in_order[in_start[j]:in_start[j + 1]])
        cnt = 0
        for r in ins:
            members = []
            while ptr < NJ and jl_junc[order[ptr]] == j and jl_in_road[order[ptr]] == r:
                members.append(order[ptr])
                ptr += 1
            if not members:
                continue
            gr_jl.extend(sorted(members))
            gr_begin.append(len(gr_jl))
            if phase_range is not None:
                ph_dur.append(float(phase_rng.integers(phase_range[0], phase_range[1] + 1)))
            else:
                ph_dur.append(phase_seconds)
            cnt += 1
        ph_begin[j + 1] = ph_begin[j] + cnt
    assert ptr == NJ

    return Network(
        junction_xy=xy,
        road_from=rf.astype(np.int32), road_to=rt.astype(np.int32),
        road_lane_begin=lane_begin.astype(np.int32),
        road_length=rlen, road_limit=rlim,
        jl_in_lane=jl_in.astype(np.int32), jl_out_lane=jl_out.astype(np.int32),
        jl_length=np.full(NJ, JUNCTION_LANE_LENGTH, np.float32),
        jl_limit=np.asarray(jl_lim, np.float32),
        junc_phase_begin=ph_begin.astype(np.int32),
        phase_duration=np.asarray(ph_dur, np.float32),
        phase_green_begin=np.asarray(gr_begin, np.int32),
        phase_green_jl=np.asarray(gr_jl, np.int32),
        junc_policy=np.full(J, policy, np.int32),
    )


def grid_network(n, spacing=200.0, jitter=0.0, lanes=2, length=200.0, limit=13.9,
                 rng=None, random_edges=False, phase_seconds=30.0, phase_range=None):
    """n x n grid of junctions.  With random_edges, every undirected edge draws
    length U(150,400) m, lanes U{1..4} and limit from {11.1, 13.9, 16.7} m/s."""
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    xy = np.stack([ii.ravel() * spacing, jj.ravel() * spacing], 1).astype(np.float64)
    if jitter > 0:
        xy = xy + rng.uniform(-jitter, jitter, xy.shape)
    idx = (ii * n + jj)
    edges = np.concatenate([
        np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], 1),
        np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1)])
    E = edges.shape[0]
    if random_edges:
        e_len = rng.uniform(150.0, 400.0, E)
        e_lanes = rng.integers(1, 5, E)
        e_limit = rng.choice(np.array([11.1, 13.9, 16.7]), E)
    else:
        e_len = np.full(E, length)
        e_lanes = np.full(E, lanes)
        e_limit = np.full(E, limit)
    return _build_network(xy, edges, e_len, e_lanes, e_limit, phase_seconds=phase_seconds,
                          phase_rng=rng, phase_range=phase_range)


def city_network(n_junctions, rng, side=None, mean_degree=3.5):
    """Planar Delaunay-style city.  Uniform junction points, Delaunay edges,
    then a random spanning tree plus uniformly drawn further Delaunay edges
    until the mean junction degree reaches ``mean_degree`` (the ratio of the
    paper's largest road network, 93,564 roads / 26,479 junctions, Table A2).
    Road lengths follow a lognormal law (median 250 m, sigma 0.6, clipped at
    30 m) assigned in rank order of the geometric edge lengths, so longer
    edges stay longer; lanes U{1..5}; limits from {11.1, 13.9, 16.7} m/s."""
    from scipy.spatial import Delaunay
    if side is None:
        side = 250.0 * math.sqrt(n_junctions)
    xy = rng.uniform(0.0, side, (n_junctions, 2))
    tri = Delaunay(xy)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e = np.unique(np.sort(e, 1), axis=0)
    w = rng.random(e.shape[0]) + 1e-9
    A = csr_matrix((w, (e[:, 0], e[:, 1])), shape=(n_junctions, n_junctions))
    mst = minimum_spanning_tree(A).tocoo()
    tree = np.stack([np.minimum(mst.row, mst.col), np.maximum(mst.row, mst.col)], 1).astype(np.int64)
    key_all = e[:, 0] * n_junctions + e[:, 1]
    in_tree = np.isin(key_all, tree[:, 0] * n_junctions + tree[:, 1])
    rest = np.nonzero(~in_tree)[0]
    target = int(round(mean_degree * n_junctions / 2))
    extra = rng.permutation(rest)[:max(0, target - tree.shape[0])]
    edges = np.concatenate([tree, e[extra]])
    edges = edges[np.lexsort((edges[:, 1], edges[:, 0]))]
    E = edges.shape[0]
    glen = np.linalg.norm(xy[edges[:, 0]] - xy[edges[:, 1]], axis=1)
    ln = np.sort(np.maximum(30.0, 250.0 * np.exp(0.6 * rng.standard_normal(E))))
    e_len = np.empty(E)
    e_len[np.argsort(glen, kind="stable")] = ln
    e_lanes = rng.integers(1, 6, E)
    e_limit = rng.choice(np.array([11.1, 13.9, 16.7]), E)
    return _build_network(xy, edges, e_len, e_lanes, e_limit)


# --------------------------------------------------------------------------
# routing (shortest free-flow time on the movement graph)
# --------------------------------------------------------------------------

def movement_graph(net: Network, road_price=None):
    """Sparse matrix M[r, r2] = cost of entering road r2 from road r:
    junction-lane free-flow time + road r2 free-flow time (+ optional price)."""
    rol = net.road_of_lane()
    src = rol[net.jl_in_lane].astype(np.int64)
    dst = rol[net.jl_out_lane].astype(np.int64)
    cost = (net.jl_length / net.jl_limit + net.road_length[dst] / net.road_limit[dst]).astype(np.float64)
    if road_price is not None:
        cost = cost + np.asarray(road_price, np.float64)[dst]
    key = src * net.n_roads + dst
    uk, first = np.unique(key, return_index=True)
    cmin = np.full(uk.shape[0], np.inf)
    np.minimum.at(cmin, np.searchsorted(uk, key), cost)
    R = net.n_roads
    return csr_matrix((cmin, (uk // R, uk % R)), shape=(R, R))


def _routes_for_chunk(args):
    GT, ud_chunk, vs, row, origins, dests = args
    _, pred = dijkstra(GT, directed=True, indices=ud_chunk, return_predecessors=True)
    pv, pr, pk = [], [], []
    bad_v = []
    cur = origins.copy()
    alive = np.ones(vs.size, bool)
    k = 0
    while alive.any():
        ai = np.nonzero(alive)[0]
        pv.append(vs[ai])
        pr.append(cur[ai])
        pk.append(np.full(ai.size, k, np.int64))
        done = cur[ai] == dests[ai]
        nxt = pred[row[ai], cur[ai]]
        bad = (~done) & (nxt < 0)
        bad_v.append(vs[ai[bad]])
        alive[ai[done | bad]] = False
        cur[ai] = np.where(done | bad, cur[ai], nxt)
        k += 1
        if k > 100000:
            raise RuntimeError("route extraction did not terminate")
    cat = lambda x, dt: np.concatenate(x) if x else np.zeros(0, dt)
    return cat(pv, np.int64), cat(pr, np.int64), cat(pk, np.int64), cat(bad_v, np.int64)


def shortest_routes(net: Network, origins, dests, road_price=None, chunk=64, workers=None):
    """Routes (CSR of road ids, origin first, destination last) for each
    (origin, destination) road pair, by reverse Dijkstra from each distinct
    destination.  Returns (route_begin, route_roads, reachable_mask)."""
    import os
    origins = np.asarray(origins, np.int64)
    dests = np.asarray(dests, np.int64)
    N = origins.shape[0]
    G = movement_graph(net, road_price)
    GT = G.T.tocsr()
    ud, inv = np.unique(dests, return_inverse=True)
    veh_by_d = np.argsort(inv, kind="stable")
    d_start = np.searchsorted(inv[veh_by_d], np.arange(ud.shape[0] + 1))
    jobs = []
    for c0 in range(0, ud.shape[0], chunk):
        c1 = min(ud.shape[0], c0 + chunk)
        vs = veh_by_d[d_start[c0]:d_start[c1]]
        if vs.size:
            jobs.append((GT, ud[c0:c1], vs, inv[vs] - c0, origins[vs], dests[vs]))
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if (ud.shape[0] > 512 and G.shape[0] > 20000) else 1
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            outs = pool.map(_routes_for_chunk, jobs, chunksize=1)
    else:
        outs = [_routes_for_chunk(j) for j in jobs]
    v = np.concatenate([o[0] for o in outs])
    r = np.concatenate([o[1] for o in outs])
    k = np.concatenate([o[2] for o in outs])
    reach = np.ones(N, bool)
    reach[np.concatenate([o[3] for o in outs])] = False
    order = np.lexsort((k, v))
    v, r = v[order], r[order]
    counts = np.bincount(v, minlength=N)
    begin = np.zeros(N + 1, np.int64)
    np.cumsum(counts, out=begin[1:])
    return begin, r, reach


def _finish_trips(net, rng, origins, dests, depart, road_price=None, length=5.0, workers=None, route=True):
    """Trip table of the given origin-destination roads; route=False leaves
    the routes unset (None) for a router that runs elsewhere."""
    begin = roads = None
    if route:
        begin, roads, reach = shortest_routes(net, origins, dests, road_price, workers=workers)
        if not reach.all():
            # keep only reachable trips (the generators redraw before this point)
            raise RuntimeError(f"{(~reach).sum()} unreachable trips")
        begin, roads = begin.astype(np.int32), roads.astype(np.int32)
    N = origins.shape[0]
    return Trips(
        depart_time=np.asarray(depart, np.float32),
        route_begin=begin,
        route_roads=roads,
        v0_factor=rng.uniform(0.8, 1.2, N).astype(np.float32),
        length=np.full(N, length, np.float32),
    )


def uniform_od(net, rng, n):
    R = net.n_roads
    o = rng.integers(0, R, n)
    d = rng.integers(0, R - 1, n)
    d = d + (d >= o)
    return o, d


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config1(seed=0, workers=None):
    """4x4 signalised grid, 200 m roads, 2 lanes per direction, 13.9 m/s;
    1,000 vehicles, uniform O!=D roads, departures U(0,300) s; 600 steps."""
    rng = np.random.default_rng(seed)
    net = grid_network(4)
    o, d = uniform_od(net, rng, 1000)
    dep = rng.uniform(0.0, 300.0, 1000)
    trips = _finish_trips(net, rng, o, d, dep, workers=workers)
    return Workload("grid4x4_1k", net, trips, Params(seed=seed), 600)


def jittered_grid(n, rng, phase_range=None):
    return grid_network(n, spacing=300.0, jitter=20.0, rng=rng, random_edges=True,
                        phase_range=phase_range)


def config2(seed=1, workers=None):
    """32x32 jittered grid (+-20 m), lengths U(150,400) m, 1-4 lanes, limits
    {11.1,13.9,16.7}; 100,000 vehicles, departures U(0,1800) s; 3,600 steps."""
    rng = np.random.default_rng(seed)
    net = jittered_grid(32, rng)
    o, d = uniform_od(net, rng, 100_000)
    dep = rng.uniform(0.0, 1800.0, 100_000)
    trips = _finish_trips(net, rng, o, d, dep, workers=workers)
    return Workload("grid32x32_100k", net, trips, Params(seed=seed), 3600)


def city_trips(net, rng, n, pool=1024, trip_median=6000.0, trip_sigma=0.5):
    """Origins uniform over roads; destinations from a seeded pool of roads,
    the pool road nearest to origin + a random offset whose length is
    lognormal (median ``trip_median`` metres) and direction uniform."""
    from scipy.spatial import cKDTree
    R = net.n_roads
    pool_roads = rng.choice(R, size=min(pool, R), replace=False)
    mid = 0.5 * (net.junction_xy[net.road_from] + net.junction_xy[net.road_to])
    tree = cKDTree(mid[pool_roads])
    o = rng.integers(0, R, n)
    dist = trip_median * np.exp(trip_sigma * rng.standard_normal(n))
    ang = rng.uniform(0, 2 * np.pi, n)
    tgt = mid[o] + np.stack([dist * np.cos(ang), dist * np.sin(ang)], 1)
    lo, hi = net.junction_xy.min(0), net.junction_xy.max(0)
    tgt = np.clip(tgt, lo, hi)
    _, k = tree.query(tgt, k=2)
    d = pool_roads[k[:, 0]]
    same = d == o
    d[same] = pool_roads[k[same, 1]]
    return o, d


def config3(seed=2, n_junctions=50_000, n_vehicles=2_464_950, workers=None):
    """Synthetic city at the paper's largest scale: ~50,000 junctions,
    planar Delaunay-style topology, 2,464,950 vehicles, departures
    N(3600 s, 1200 s) clipped to [0, 7200); 7,200 steps."""
    rng = np.random.default_rng(seed)
    net = city_network(n_junctions, rng)
    o, d = city_trips(net, rng, n_vehicles)
    dep = np.clip(rng.normal(3600.0, 1200.0, n_vehicles), 0.0, np.nextafter(7200.0, 0))
    trips = _finish_trips(net, rng, o, d, dep, workers=workers)
    return Workload("city50k_2464950", net, trips, Params(seed=seed), 7200)


def config4_instance(i, steps=1800):
    """Instance i of the batched workload: jittered grid of side U{4..40}
    with N = round(1000 + 149000 (n^2-16)/1584) vehicles, departures
    U(0,900) s; 1,800 steps; signal phases set every 15 steps by a seeded
    random policy (see ``random_phase_schedule``)."""
    rng = np.random.default_rng(1000 + i)
    n = int(rng.integers(4, 41))
    N = int(round(1000 + 149000 * (n * n - 16) / 1584))
    net = jittered_grid(n, rng)
    o, d = uniform_od(net, rng, N)
    dep = rng.uniform(0.0, 900.0, N)
    trips = _finish_trips(net, rng, o, d, dep, workers=1)
    return Workload(f"batch_inst{i}_grid{n}_{N}", net, trips, Params(seed=1000 + i), steps,
                    extra={"policy_seed": 5000 + i, "policy_every": 15})


def _instance_worker(args):
    kind, i, kw = args
    if kind == "batch":
        return config4_instance(i, **kw)
    return config5_job(i, workers=1, **kw)


def batch_workload(n_instances=256, steps=1800, workers=None, first=0):
    """The batched workload: instances first .. first+n_instances-1 of
    ``config4_instance``, generated in parallel processes."""
    import os
    import multiprocessing as mp
    ids = list(range(first, first + n_instances))
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    jobs = [("batch", i, {"steps": steps}) for i in ids]
    if workers > 1 and n_instances > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_instance_worker, jobs, chunksize=1)
    return [_instance_worker(j) for j in jobs]


def served_jobs(n_jobs, workers=None, max_vehicles=None, route=True):
    """Jobs 0 .. n_jobs-1 of ``config5_job``, generated in parallel processes
    (route=False: routes left for the server to compute)."""
    import os
    import multiprocessing as mp
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    jobs = [("serve", j, {"max_vehicles": max_vehicles, "route": route}) for j in range(n_jobs)]
    if workers > 1 and n_jobs > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_instance_worker, jobs, chunksize=1)
    return [_instance_worker(j) for j in jobs]


def random_phase_schedule(net: Network, seed, n_updates):
    """[n_updates, J] phase indices, each uniform over the junction's phases."""
    rng = np.random.default_rng(seed)
    nph = np.diff(net.junc_phase_begin).astype(np.int64)
    u = rng.random((n_updates, net.n_junctions))
    return np.minimum((u * nph[None, :]).astype(np.int32), np.maximum(nph - 1, 0)[None, :]).astype(np.int32)


def config5_job(j, max_vehicles=None, workers=None, route=True):
    """Job j of the served workload: w.p. 1/2 a C1-style grid (n~U{4..16}),
    else a jittered grid (n~U{8..32}); N log-uniform in [10k, 500k] capped by
    the grid-size coupling; horizon U{300..3600}; w.p. 1/2 a signal-timing
    plan (phases U{15..60} s) else per-road prices U(0,120) s added to the
    routing cost.  The job's origin and destination roads and its prices are
    kept in ``extra`` ("od", "price"); route=False leaves the routes to the
    server (every other draw is the same)."""
    rng = np.random.default_rng(10000 + j)
    plan = rng.random() < 0.5
    c1_style = rng.random() < 0.5
    n = int(rng.integers(4, 17)) if c1_style else int(rng.integers(8, 33))
    cap = int(round(1000 + 149000 * (n * n - 16) / 1584))
    N = int(round(math.exp(rng.uniform(math.log(10_000), math.log(500_000)))))
    N = min(N, max(cap, 10_000))
    if max_vehicles is not None:
        N = min(N, max_vehicles)
    H = int(rng.integers(300, 3601))
    phase_range = (15, 60) if plan else None
    if c1_style:
        net = grid_network(n, rng=rng, phase_range=phase_range)
    else:
        net = jittered_grid(n, rng, phase_range=phase_range)
    price = None if plan else rng.uniform(0.0, 120.0, net.n_roads)
    o, d = uniform_od(net, rng, N)
    dep = rng.uniform(0.0, 0.5 * H, N)
    trips = _finish_trips(net, rng, o, d, dep, road_price=price, workers=workers, route=route)
    return Workload(f"job{j}", net, trips, Params(seed=10000 + j), H,
                    extra={"kind": "timing_plan" if plan else "pricing", "od": (o, d), "price": price})


def poisson_arrivals(n_jobs, rate=20.0, seed=7):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n_jobs))


def ring_road(circumference_road=300.0, n_vehicles=10, laps=50, v0_factor=1.0):
    """One single-lane road whose only movement loops back onto itself
    through one junction lane (no signal), so the route can repeat it."""
    xy = np.array([[0.0, 0.0], [100.0, 0.0]])
    net = Network(
        junction_xy=xy,
        road_from=np.array([0], np.int32), road_to=np.array([0], np.int32),
        road_lane_begin=np.array([0, 1], np.int32),
        road_length=np.array([circumference_road], np.float32),
        road_limit=np.array([13.9], np.float32),
        jl_in_lane=np.array([0], np.int32), jl_out_lane=np.array([0], np.int32),
        jl_length=np.array([JUNCTION_LANE_LENGTH], np.float32),
        jl_limit=np.array([13.9], np.float32),
        junc_phase_begin=np.array([0, 1, 1], np.int32)[:2],
        phase_duration=np.array([30.0], np.float32),
        phase_green_begin=np.array([0, 1], np.int32),
        phase_green_jl=np.array([0], np.int32),
        junc_policy=np.array([POLICY_NONE], np.int32),
    )
    net.junction_xy = xy[:1]
    N = n_vehicles
    trips = Trips(
        depart_time=np.zeros(N, np.float32),
        route_begin=(np.arange(N + 1) * laps).astype(np.int32),
        route_roads=np.zeros(N * laps, np.int32),
        v0_factor=np.full(N, v0_factor, np.float32),
        length=np.full(N, 5.0, np.float32),
    )
    return net, trips


def synthetic_state(net, trips, step, seed, p_active=0.5, p_finished=0.1, p_junction=0.08, min_gap=0.3,
                    p_standing=0.15):
    """Seeded mid-simulation state at time step*dt (dt = 1 s): among vehicles
    already due to depart, a fraction sits somewhere along its own route (a road lane of the current road, lane group or not,
    or a junction lane toward the next road) with uniformly drawn position and
    speed up to the desired speed; vehicles overlapping the one ahead on their
    lane are put back to waiting; others wait (some already due) or have
    finished.  Evaluates nothing of the vehicle model."""
    rng = np.random.default_rng(seed)
    N = trips.n_vehicles
    NRL = net.n_road_lanes
    rol = net.road_of_lane().astype(np.int64)
    rb = trips.route_begin.astype(np.int64)
    rr = trips.route_roads.astype(np.int64)
    R = net.n_roads
    lane_len = np.concatenate([np.repeat(net.road_length, np.diff(net.road_lane_begin)),
                               net.jl_length]).astype(np.float64)
    lim = np.concatenate([np.repeat(net.road_limit, np.diff(net.road_lane_begin)),
                          net.jl_limit]).astype(np.float64)
    # junction lanes grouped by (in road, out road)
    jkey = rol[net.jl_in_lane] * R + rol[net.jl_out_lane]
    jorder = np.argsort(jkey, kind="stable")
    jsorted = jkey[jorder]
    u = rng.random(N)
    status = np.zeros(N, np.int32)
    due = trips.depart_time.astype(np.float64) <= step * 1.0
    status[(u < p_active) & due] = 1
    status[(u >= p_active) & (u < p_active + p_finished) & due] = 2
    act = np.nonzero(status == 1)[0]
    rl = rb[act + 1] - rb[act]
    k = np.minimum((rng.random(act.size) * rl).astype(np.int64), rl - 1)
    r = rr[rb[act] + k]
    lane = np.full(N, -1, np.int64)
    lb = net.road_lane_begin[r].astype(np.int64)
    nl = net.road_lane_begin[r + 1].astype(np.int64) - lb
    lane_a = lb + np.minimum((rng.random(act.size) * nl).astype(np.int64), nl - 1)
    to_jl = (k + 1 < rl) & (rng.random(act.size) < p_junction)
    if to_jl.any():
        ji = np.nonzero(to_jl)[0]
        key = r[ji] * R + rr[rb[act[ji]] + k[ji] + 1]
        lo = np.searchsorted(jsorted, key, "left")
        hi = np.searchsorted(jsorted, key, "right")
        pick = lo + np.minimum((rng.random(ji.size) * (hi - lo)).astype(np.int64), hi - lo - 1)
        lane_a[ji] = NRL + jorder[pick]
    lane[act] = lane_a
    route_pos = np.zeros(N, np.int64)
    route_pos[act] = k
    x = np.zeros(N, np.float64)
    x[act] = rng.random(act.size) * lane_len[lane_a]
    gap = min_gap * (1.0 + rng.random(N))
    L = trips.length.astype(np.float64)
    # drop vehicles that overlap the vehicle ahead on their lane until none do
    alive = act.copy()
    while alive.size:
        o = alive[np.lexsort((alive, -x[alive], lane[alive]))]
        same = np.zeros(o.size, bool)
        same[1:] = lane[o[1:]] == lane[o[:-1]]
        prev_rear = np.full(o.size, np.inf)
        prev_rear[1:] = x[o[:-1]] - L[o[:-1]]
        bad = same & (x[o] > prev_rear - gap[o])
        if not bad.any():
            break
        # drop every vehicle that overlaps its current predecessor
        drop = o[bad]
        status[drop] = 0
        alive = np.setdiff1d(alive, drop)
    lane[status != 1] = -1
    route_pos[status != 1] = 0
    x[status != 1] = 0.0
    v = np.zeros(N, np.float64)
    a2 = np.nonzero(status == 1)[0]
    v[a2] = rng.random(a2.size) * trips.v0_factor[a2] * lim[lane[a2]]
    v[a2[rng.random(a2.size) < p_standing]] = 0.0
    finish = np.full(N, -1, np.int64)
    fin = np.nonzero(status == 2)[0]
    lo = np.ceil(trips.depart_time[fin].astype(np.float64)).astype(np.int64)
    finish[fin] = lo + (rng.random(fin.size) * np.maximum(step - lo, 1)).astype(np.int64)
    route_pos[fin] = rb[fin + 1] - rb[fin] - 1
    return dict(step=int(step), status=status, lane=lane.astype(np.int32), route_pos=route_pos.astype(np.int32),
                x=x.astype(np.float32), v=v.astype(np.float32), finish_step=finish.astype(np.int32))


CONFIGS = {1: config1, 2: config2, 3: config3}
