"""ctypes binding of the FP64 CPU oracle (``tsim_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It takes the
same plain generator arrays as the HIP library and nothing else.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tsim_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

WAITING, ACTIVE, FINISHED = 0, 1, 2
EV_TRANSFER, EV_FINISH, EV_FEEDER_BLOCK, EV_CLAMP, EV_DEPART = 1, 2, 4, 8, 16
NMARGIN = 6
METRIC_NAMES = ["t", "waiting", "active", "finished", "sum_tt", "att", "mean_speed_last",
                "mean_speed_avg", "vehicle_steps", "lane_changes", "transfers", "clamps",
                "feeder_blocks", "departures", "speed_steps", "_"]


def build(force=False):
    """Compile the oracle with gcc (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.osim_create.restype = C.c_void_p
        L.osim_create.argtypes = ([C.c_int, C.c_int] + [C.c_void_p] * 5 + [C.c_int] + [C.c_void_p] * 9
                                  + [C.c_int] + [C.c_void_p] * 5 + [C.c_void_p, C.c_uint64])
        L.osim_destroy.argtypes = [C.c_void_p]
        L.osim_step.argtypes = [C.c_void_p, C.c_int]
        L.osim_get_state.argtypes = [C.c_void_p] + [C.c_void_p] * 7
        L.osim_set_state.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 6
        L.osim_set_signal_phases.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.osim_set_policy.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.osim_set_junctions.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.osim_set_lane_max_speed.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.osim_set_lane_restriction.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.osim_set_vehicle_route.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_double]
        L.osim_set_trip_ends.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.osim_set_trip_starts.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.osim_get_route.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.osim_get_junctions.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.osim_get_metrics.argtypes = [C.c_void_p, C.c_void_p]
        L.osim_get_road_stats.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.osim_get_lane_waiting.argtypes = [C.c_void_p, C.c_void_p]
        L.osim_get_green.argtypes = [C.c_void_p, C.c_void_p]
        L.osim_eval_signals.argtypes = [C.c_void_p, C.c_void_p]
        L.osim_last_diag.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        L.osim_idm.restype = C.c_double
        L.osim_idm.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double]
        L.osim_philox.argtypes = [C.c_uint64, C.c_void_p, C.c_void_p]
        L.osim_shortest_routes.restype = C.c_int
        L.osim_shortest_routes.argtypes = [C.c_void_p] + [C.c_void_p] * 2 + [C.c_int] + [C.c_void_p] * 4 + [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def params_array(params):
    return np.array([params.dt, params.T, params.a_max, params.b_comf, params.s0, params.delta,
                     params.politeness, params.a_th, params.b_safe, params.p_max, params.p_min,
                     params.a_emerg], np.float64)


def idm(params, v, v0, s, dv):
    pa = params_array(params)
    return lib().osim_idm(_p(pa), float(v), float(v0), float(s), float(dv))


def philox(seed, ctr):
    c = np.ascontiguousarray(np.asarray(ctr, np.uint32))
    out = np.zeros(4, np.uint32)
    lib().osim_philox(C.c_uint64(seed), _p(c), _p(out))
    return out


class OracleSim:
    """One oracle simulation instance over a generator network and trip table."""

    def __init__(self, net, trips, params):
        L = lib()
        self.net, self.trips, self.params = net, trips, params
        i32 = lambda a: np.ascontiguousarray(a, np.int32)
        f32 = lambda a: np.ascontiguousarray(a, np.float32)
        self._keep = [i32(net.road_from), i32(net.road_to), i32(net.road_lane_begin), f32(net.road_length),
                      f32(net.road_limit), i32(net.jl_in_lane), i32(net.jl_out_lane), f32(net.jl_length),
                      f32(net.jl_limit), i32(net.junc_phase_begin), f32(net.phase_duration),
                      i32(net.phase_green_begin), i32(net.phase_green_jl), i32(net.junc_policy),
                      f32(trips.depart_time), i32(trips.route_begin), i32(trips.route_roads),
                      f32(trips.v0_factor), f32(trips.length), params_array(params)]
        k = self._keep
        self.N = trips.n_vehicles
        self.R = net.n_roads
        self.NL = net.n_lanes
        self.NJL = net.n_jlanes
        self.h = L.osim_create(net.n_junctions, net.n_roads, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]),
                               net.n_jlanes, _p(k[5]), _p(k[6]), _p(k[7]), _p(k[8]), _p(k[9]), _p(k[10]),
                               _p(k[11]), _p(k[12]), _p(k[13]),
                               self.N, _p(k[14]), _p(k[15]), _p(k[16]), _p(k[17]), _p(k[18]),
                               _p(k[19]), C.c_uint64(params.seed))
        if not self.h:
            raise MemoryError("oracle create failed")
        end_s = getattr(trips, "end_s", None)
        if end_s is not None:
            e = np.ascontiguousarray(end_s, np.float32).astype(np.float64)
            ids = np.arange(self.N, dtype=np.int32)
            L.osim_set_trip_ends(self.h, self.N, _p(ids), _p(e))
        start_s = getattr(trips, "start_s", None)
        if start_s is not None:
            b = np.ascontiguousarray(start_s, np.float32).astype(np.float64)
            ids = np.arange(self.N, dtype=np.int32)
            L.osim_set_trip_starts(self.h, self.N, _p(ids), _p(b))

    def close(self):
        if self.h:
            lib().osim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        lib().osim_step(self.h, int(n))

    def get_state(self):
        N = self.N
        t = np.zeros(1, np.int64)
        st = dict(status=np.zeros(N, np.int32), lane=np.zeros(N, np.int32), route_pos=np.zeros(N, np.int32),
                  x=np.zeros(N, np.float64), v=np.zeros(N, np.float64), finish_step=np.zeros(N, np.int32))
        lib().osim_get_state(self.h, _p(t), _p(st["status"]), _p(st["lane"]), _p(st["route_pos"]),
                             _p(st["x"]), _p(st["v"]), _p(st["finish_step"]))
        st["step"] = int(t[0])
        return st

    def set_state(self, st):
        a = {k: np.ascontiguousarray(st[k], np.int32) for k in ("status", "lane", "route_pos", "finish_step")}
        x = np.ascontiguousarray(st["x"], np.float64)
        v = np.ascontiguousarray(st["v"], np.float64)
        lib().osim_set_state(self.h, C.c_int64(int(st["step"])), _p(a["status"]), _p(a["lane"]),
                             _p(a["route_pos"]), _p(x), _p(v), _p(a["finish_step"]))

    def set_signal_phases(self, junctions, phases):
        j = np.ascontiguousarray(junctions, np.int32)
        p = np.ascontiguousarray(phases, np.int32)
        lib().osim_set_signal_phases(self.h, int(j.size), _p(j), _p(p))

    def set_policy(self, junctions, policies):
        j = np.ascontiguousarray(junctions, np.int32)
        p = np.ascontiguousarray(policies, np.int32)
        lib().osim_set_policy(self.h, int(j.size), _p(j), _p(p))

    def set_junctions(self, policy, phase):
        """Policy and phase of every junction (MANUAL phase, or the phase in
        force of a MAX_PRESSURE junction)."""
        p = np.ascontiguousarray(policy, np.int32)
        ph = np.ascontiguousarray(phase, np.int32)
        assert p.size == ph.size == self.net.n_junctions
        lib().osim_set_junctions(self.h, _p(p), _p(ph))

    def set_lane_max_speed(self, lanes, speeds):
        """Speed limits of lanes (global lane ids) from the next step on."""
        l = np.ascontiguousarray(lanes, np.int32)
        v = np.ascontiguousarray(speeds, np.float64)
        lib().osim_set_lane_max_speed(self.h, int(l.size), _p(l), _p(v))

    def set_lane_restriction(self, lanes, flags):
        """Lanes (global lane ids) restricted (flag != 0: no new vehicle
        enters) or released, from the next step on."""
        l = np.ascontiguousarray(lanes, np.int32)
        f = np.ascontiguousarray(flags, np.int32)
        lib().osim_set_lane_restriction(self.h, int(l.size), _p(l), _p(f))

    def set_vehicle_route(self, vid, route, end_s=None):
        """Vehicle vid follows `route` (road ids, beginning with the road it is
        on) from the next step on, at route position 0; its trip ends at
        end_s metres along the last road (None: that road's end)."""
        r = np.ascontiguousarray(route, np.int32)
        e = -1.0 if end_s is None else float(np.float32(end_s))
        lib().osim_set_vehicle_route(self.h, int(vid), _p(r), int(r.size), e)

    def set_aois(self, conn_begin, conn_road, conn_s, origin_aoi=None, dest_aoi=None):
        """Areas of interest (Appendix B.1: an area joined to the road network
        by connections at positions along roads, where trips start and end).
        Reading: a vehicle whose trip starts in AOI a enters at a's first
        listed connection on the first road of its route; one whose trip ends
        in AOI b ends at b's first listed connection on the last road of its
        route.  Only vehicles still waiting may be given AOIs.  Returns the
        (start, end) positions given to the vehicles (nan: unchanged).
        Plain loops over the vehicles: small cases only."""
        n_aoi = len(conn_begin) - 1
        conn = [[(int(conn_road[c]), float(np.float32(conn_s[c]))) for c in range(conn_begin[a], conn_begin[a + 1])]
                for a in range(n_aoi)]

        def place(a, road):
            for r, x in conn[a]:
                if r == road:
                    return x
            raise ValueError(f"AOI {a} has no connection on road {road}")

        st = self.get_state()["status"]
        starts = np.full(self.N, np.nan)
        ends = np.full(self.N, np.nan)
        self.aoi_origin = np.full(self.N, -1, np.int64)
        self.aoi_dest = np.full(self.N, -1, np.int64)
        for v in range(self.N):
            o = -1 if origin_aoi is None else int(origin_aoi[v])
            d = -1 if dest_aoi is None else int(dest_aoi[v])
            if o < 0 and d < 0:
                continue
            if st[v] != WAITING:
                raise ValueError(f"vehicle {v} has departed")
            _, roads = self.route(v)
            if o >= 0:
                starts[v] = place(o, int(roads[0]))
                self.aoi_origin[v] = o
            if d >= 0:
                ends[v] = place(d, int(roads[-1]))
                self.aoi_dest[v] = d
        L = lib()
        ids = np.nonzero(~np.isnan(starts))[0].astype(np.int32)
        if ids.size:
            b = np.ascontiguousarray(starts[ids], np.float64)
            L.osim_set_trip_starts(self.h, int(ids.size), _p(ids), _p(b))
        ids = np.nonzero(~np.isnan(ends))[0].astype(np.int32)
        if ids.size:
            e = np.ascontiguousarray(ends[ids], np.float64)
            L.osim_set_trip_ends(self.h, int(ids.size), _p(ids), _p(e))
        self.n_aoi = n_aoi
        return starts, ends

    def aoi_counts(self):
        """(waiting, arrived) per AOI: vehicles of each origin AOI not yet
        departed, vehicles whose trip ended in each destination AOI."""
        st = self.get_state()["status"]
        w = np.zeros(self.n_aoi, np.int64)
        a = np.zeros(self.n_aoi, np.int64)
        for v in range(self.N):
            if st[v] == WAITING and self.aoi_origin[v] >= 0:
                w[self.aoi_origin[v]] += 1
            if st[v] == FINISHED and self.aoi_dest[v] >= 0:
                a[self.aoi_dest[v]] += 1
        return w, a

    def route(self, vid, max_len=100000):
        """(route position, roads of the route in force) of vehicle vid."""
        k = np.zeros(1, np.int32)
        n = np.zeros(1, np.int32)
        out = np.zeros(max_len, np.int32)
        lib().osim_get_route(self.h, int(vid), _p(k), _p(n), _p(out), max_len)
        return int(k[0]), out[:int(n[0])].copy()

    def shortest_routes(self, origins, dests, price=None, road_time=None):
        """Routes of least cost for (origin road, destination road) pairs
        under the lane limits and restrictions in force, road prices and
        road times (None: free-flow), as (begin[n+1], roads, n_unreachable):
        route c is roads[begin[c]:begin[c+1]], empty when unreachable."""
        o = np.ascontiguousarray(origins, np.int32)
        d = np.ascontiguousarray(dests, np.int32)
        n = int(o.size)
        pr = None if price is None else np.ascontiguousarray(price, np.float32)
        rt = None if road_time is None else np.ascontiguousarray(road_time, np.float32)
        begin = np.zeros(n + 1, np.int32)
        cap = max(1, n * self.R)
        roads = np.zeros(cap, np.int32)
        bad = lib().osim_shortest_routes(self.h, None if pr is None else _p(pr), None if rt is None else _p(rt),
                                         n, _p(o), _p(d), _p(begin), _p(roads), cap)
        if bad < 0:
            raise RuntimeError("route buffer too small")
        return begin, roads[:begin[n]].copy(), int(bad)

    def junctions(self):
        p = np.zeros(self.net.n_junctions, np.int32)
        ph = np.zeros(self.net.n_junctions, np.int32)
        lib().osim_get_junctions(self.h, _p(p), _p(ph))
        return p, ph

    def metrics(self):
        out = np.zeros(16, np.float64)
        lib().osim_get_metrics(self.h, _p(out))
        return dict(zip(METRIC_NAMES, out.tolist()))

    def road_stats(self):
        sv = np.zeros(self.R, np.float64)
        c = np.zeros(self.R, np.int32)
        lib().osim_get_road_stats(self.h, _p(sv), _p(c))
        return sv, c

    def lane_waiting(self):
        out = np.zeros(self.NL, np.int32)
        lib().osim_get_lane_waiting(self.h, _p(out))
        return out

    def green(self):
        out = np.zeros(self.NJL, np.uint8)
        lib().osim_get_green(self.h, _p(out))
        return out

    def eval_signals(self):
        out = np.zeros(self.NJL, np.uint8)
        lib().osim_eval_signals(self.h, _p(out))
        return out

    def diag(self):
        N = self.N
        m = np.zeros((N, NMARGIN), np.float64)
        mob = np.zeros((N, 4), np.float64)
        dec = np.zeros(N, np.int32)
        ev = np.zeros(N, np.int32)
        lib().osim_last_diag(self.h, _p(m), _p(mob), _p(dec), _p(ev))
        return dict(margin=m, mobil=mob, decision=dec, event=ev)
