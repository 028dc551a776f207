"""Python binding of the C ABI in ``include/tsim.h`` (argument marshalling only).

Every step of the simulation runs in the HIP library ``libtsim.so``; torch only
provides the device arena (one uint8 tensor) and the HIP stream.  Importing
this module never falls back to any other implementation: when the library is
missing or no GPU is present, the calls raise.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsim.so")

TSIM_OK, TSIM_EINVAL, TSIM_ENOMEM, TSIM_EDEVICE, TSIM_ESTATE = 0, -1, -2, -3, -4
WAITING, ACTIVE, FINISHED = 0, 1, 2


class TsimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tsim error {code}: {msg}")
        self.code = code


class tsim_network(C.Structure):
    _fields_ = [("n_junctions", C.c_int32), ("n_roads", C.c_int32),
                ("road_from", C.c_void_p), ("road_to", C.c_void_p), ("road_lane_begin", C.c_void_p),
                ("road_length", C.c_void_p), ("road_limit", C.c_void_p),
                ("n_jlanes", C.c_int32),
                ("jl_in_lane", C.c_void_p), ("jl_out_lane", C.c_void_p), ("jl_length", C.c_void_p),
                ("jl_limit", C.c_void_p), ("junc_phase_begin", C.c_void_p), ("phase_duration", C.c_void_p),
                ("phase_green_begin", C.c_void_p), ("phase_green_jl", C.c_void_p), ("junc_policy", C.c_void_p)]


class tsim_trips(C.Structure):
    _fields_ = [("n_vehicles", C.c_int32), ("depart_time", C.c_void_p), ("route_begin", C.c_void_p),
                ("route_roads", C.c_void_p), ("v0_factor", C.c_void_p), ("length", C.c_void_p),
                ("end_s", C.c_void_p), ("start_s", C.c_void_p)]


class tsim_params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("dt", "T", "a_max", "b_comf", "s0", "delta", "politeness", "a_th",
                                           "b_safe", "p_max", "p_min", "a_emerg")] + [("seed", C.c_uint64)]


class tsim_metrics(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_waiting", C.c_int64), ("n_active", C.c_int64), ("n_finished", C.c_int64),
                ("sum_travel_time", C.c_double), ("att", C.c_double), ("mean_speed_last", C.c_double),
                ("mean_speed_avg", C.c_double), ("vehicle_steps", C.c_int64), ("lane_changes", C.c_int64),
                ("transfers", C.c_int64), ("clamps", C.c_int64), ("feeder_blocks", C.c_int64),
                ("departures", C.c_int64), ("speed_steps", C.c_int64), ("errors", C.c_int64),
                ("lane_steps", C.c_int64), ("road_entries", C.c_int64), ("stalled_steps", C.c_int64),
                ("max_stalled_steps", C.c_int64)]


class tsim_state_host(C.Structure):
    _fields_ = [("step", C.c_int64), ("status", C.c_void_p), ("lane", C.c_void_p), ("route_pos", C.c_void_p),
                ("x", C.c_void_p), ("v", C.c_void_p), ("finish_step", C.c_void_p), ("junc_policy", C.c_void_p),
                ("junc_phase", C.c_void_p)]


class tsim_batch_capacity(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("instances", "junctions", "roads", "road_lanes", "jlanes", "phases",
                                         "vehicles")] + [("route_entries", C.c_int64), ("slots", C.c_int64)]


CAPACITY_FIELDS = [n for n, _ in tsim_batch_capacity._fields_]

_lib = None

EXPORTS = ["tsim_footprint", "tsim_create", "tsim_step", "tsim_set_signal_phases", "tsim_get_metrics",
           "tsim_get_road_mean_speed", "tsim_get_lane_waiting_counts", "tsim_get_lane_order", "tsim_get_state",
           "tsim_set_state", "tsim_set_profiling", "tsim_get_kernel_times", "tsim_destroy", "tsim_last_error",
           "tsim_batch_footprint", "tsim_batch_create", "tsim_batch_step", "tsim_batch_set_signal_phases",
           "tsim_batch_get_metrics", "tsim_batch_get_state", "tsim_batch_destroy", "tsim_batch_set_all_phases",
           "tsim_set_graph_steps", "tsim_batch_set_graph_steps", "tsim_set_schedule", "tsim_get_schedule",
           "tsim_autotune", "tsim_batch_set_horizon", "tsim_set_concurrency", "tsim_autotune_launch",
           "tsim_set_signal_policy", "tsim_batch_set_signal_policy", "tsim_batch_set_state",
           "tsim_batch_get_road_mean_speed", "tsim_batch_get_lane_waiting_counts", "tsim_batch_get_lane_order",
           "tsim_instance_build", "tsim_instance_free", "tsim_instance_capacity", "tsim_batch_reserve_footprint",
           "tsim_batch_reserve", "tsim_batch_add", "tsim_batch_add_member", "tsim_batch_remove",
           "tsim_batch_capacity_left", "tsim_batch_num_instances", "tsim_set_signal_phases_noalloc",
           "tsim_set_lane_max_speed", "tsim_batch_set_lane_max_speed", "tsim_set_lane_restriction",
           "tsim_batch_set_lane_restriction", "tsim_set_vehicle_route",
           "tsim_batch_set_vehicle_route", "tsim_set_trajectory", "tsim_get_trajectory_count",
           "tsim_route_footprint", "tsim_shortest_routes", "tsim_reroute_footprint", "tsim_reroute_shortest",
           "tsim_batch_reroute_footprint", "tsim_batch_reroute_shortest", "tsim_aoi_footprint", "tsim_set_aois",
           "tsim_get_aoi_counts", "tsim_batch_aoi_footprint", "tsim_batch_set_aois", "tsim_batch_get_aoi_counts"]

SCHEDULES = {0: "wide", 1: "16x32", 2: "16x64", 3: "32x64", 4: "8x16", 5: "16x32+pipelined wide", 6: "8x16+16x32+pipelined wide",
             7: "8x16+16x32+wide, fused launch"}


def lib():
    """Loads libtsim.so (built by ``paper_2406_10661_amd.build``); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2406_10661_amd.build.build()")
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()   # the HIP runtime knows the GPUs before the library registers its device data
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.tsim_footprint.argtypes = [P, P, P, C.POINTER(C.c_size_t)]
        L.tsim_create.argtypes = [P, P, P, P, P, C.c_size_t, C.POINTER(C.c_void_p)]
        L.tsim_step.argtypes = [P, C.c_int32]
        L.tsim_set_signal_phases.argtypes = [P, P, P, C.c_int32]
        L.tsim_set_signal_policy.argtypes = [P, P, P, C.c_int32]
        L.tsim_set_signal_phases_noalloc.argtypes = [P, P, P, C.c_int32]
        L.tsim_set_lane_max_speed.argtypes = [P, P, P, C.c_int32]
        L.tsim_set_lane_restriction.argtypes = [P, P, P, C.c_int32]
        L.tsim_set_vehicle_route.argtypes = [P, C.c_int32, P, C.c_int32, C.c_float]
        L.tsim_set_trajectory.argtypes = [P, P, C.c_int64, C.c_int32]
        L.tsim_get_trajectory_count.argtypes = [P, P]
        L.tsim_aoi_footprint.argtypes = [P, C.c_int32, C.POINTER(C.c_size_t)]
        L.tsim_set_aois.argtypes = [P, C.c_int32, P, P, P, P, P, P, C.c_size_t]
        L.tsim_get_aoi_counts.argtypes = [P, P, P, C.c_int32]
        L.tsim_batch_aoi_footprint.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
        L.tsim_batch_set_aois.argtypes = [P, C.c_int32, C.c_int32, P, P, P, P, P, P, C.c_size_t]
        L.tsim_batch_get_aoi_counts.argtypes = [P, C.c_int32, P, P, C.c_int32]
        L.tsim_batch_set_vehicle_route.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int32, C.c_float]
        SZ = C.POINTER(C.c_size_t)
        L.tsim_route_footprint.argtypes = [P, C.c_int32, SZ, SZ]
        L.tsim_shortest_routes.argtypes = [P, P, P, P, P, C.c_int32, P, P, C.c_size_t, P, P, C.c_int64, P]
        L.tsim_reroute_footprint.argtypes = [P, C.c_int32, SZ, SZ]
        L.tsim_reroute_shortest.argtypes = [P, P, C.c_int32, P, P, P, C.c_size_t, P]
        L.tsim_batch_reroute_footprint.argtypes = [P, C.c_int32, C.c_int32, SZ, SZ]
        L.tsim_batch_reroute_shortest.argtypes = [P, C.c_int32, P, C.c_int32, P, P, P, C.c_size_t, P]
        L.tsim_batch_set_lane_max_speed.argtypes = [P, C.c_int32, P, P, C.c_int32]
        L.tsim_batch_set_lane_restriction.argtypes = [P, C.c_int32, P, P, C.c_int32]
        L.tsim_batch_set_signal_policy.argtypes = [P, C.c_int32, P, P, C.c_int32]
        L.tsim_get_metrics.argtypes = [P, P]
        L.tsim_get_road_mean_speed.argtypes = [P, P, C.c_int32]
        L.tsim_get_lane_waiting_counts.argtypes = [P, P, C.c_int32]
        L.tsim_get_lane_order.argtypes = [P, P, P, C.c_int32, C.c_int32]
        L.tsim_get_state.argtypes = [P, P]
        L.tsim_set_state.argtypes = [P, P]
        L.tsim_set_profiling.argtypes = [P, C.c_int32]
        L.tsim_set_graph_steps.argtypes = [P, C.c_int32]
        L.tsim_set_schedule.argtypes = [P, C.c_int32]
        L.tsim_set_concurrency.argtypes = [P, C.c_int32]
        L.tsim_batch_set_horizon.argtypes = [P, C.c_int32, C.c_int64]
        L.tsim_get_schedule.argtypes = [P, P]
        L.tsim_autotune.argtypes = [P, C.c_int32, C.c_int32, P, P]
        L.tsim_autotune_launch.argtypes = [P, C.c_int32, C.c_int32, P, P, P]
        L.tsim_batch_set_graph_steps.argtypes = [P, C.c_int32]
        L.tsim_get_kernel_times.argtypes = [P, P, P, C.c_int32]
        L.tsim_destroy.argtypes = [P]
        L.tsim_batch_footprint.argtypes = [P, P, P, C.c_int32, C.POINTER(C.c_size_t)]
        L.tsim_batch_create.argtypes = [P, P, P, C.c_int32, P, P, C.c_size_t, C.POINTER(C.c_void_p)]
        L.tsim_batch_step.argtypes = [P, C.c_int32]
        L.tsim_batch_set_signal_phases.argtypes = [P, C.c_int32, P, P, C.c_int32]
        L.tsim_batch_get_metrics.argtypes = [P, C.c_int32, P]
        L.tsim_batch_set_all_phases.argtypes = [P, P, C.c_int32]
        L.tsim_batch_get_state.argtypes = [P, C.c_int32, P]
        L.tsim_batch_set_state.argtypes = [P, C.c_int32, P]
        L.tsim_batch_get_road_mean_speed.argtypes = [P, C.c_int32, P, C.c_int32]
        L.tsim_batch_get_lane_waiting_counts.argtypes = [P, C.c_int32, P, C.c_int32]
        L.tsim_batch_get_lane_order.argtypes = [P, C.c_int32, P, P, C.c_int32, C.c_int32]
        L.tsim_instance_build.argtypes = [P, P, P, C.POINTER(C.c_void_p)]
        L.tsim_instance_free.argtypes = [P]
        L.tsim_instance_capacity.argtypes = [P, P]
        L.tsim_batch_reserve_footprint.argtypes = [P, C.POINTER(C.c_size_t)]
        L.tsim_batch_reserve.argtypes = [P, P, P, P, C.c_size_t, C.POINTER(C.c_void_p)]
        L.tsim_batch_add.argtypes = [P, P, P]
        L.tsim_batch_add_member.argtypes = [P, P, P]
        L.tsim_batch_remove.argtypes = [P, C.c_int32]
        L.tsim_batch_capacity_left.argtypes = [P, P]
        L.tsim_batch_num_instances.argtypes = [P, P]
        L.tsim_batch_destroy.argtypes = [P]
        L.tsim_last_error.argtypes = [P]
        L.tsim_last_error.restype = C.c_char_p
        for name in EXPORTS:
            getattr(L, name).restype = C.c_int if name != "tsim_last_error" else C.c_char_p
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class _Inputs:
    """Keeps the contiguous host arrays alive while a C structure points at them."""

    def __init__(self, net, trips, params):
        i32 = lambda a: np.ascontiguousarray(a, np.int32)
        f32 = lambda a: np.ascontiguousarray(a, np.float32)
        self.arrays = dict(
            road_from=i32(net.road_from), road_to=i32(net.road_to), road_lane_begin=i32(net.road_lane_begin),
            road_length=f32(net.road_length), road_limit=f32(net.road_limit), jl_in_lane=i32(net.jl_in_lane),
            jl_out_lane=i32(net.jl_out_lane), jl_length=f32(net.jl_length), jl_limit=f32(net.jl_limit),
            junc_phase_begin=i32(net.junc_phase_begin), phase_duration=f32(net.phase_duration),
            phase_green_begin=i32(net.phase_green_begin), phase_green_jl=i32(net.phase_green_jl),
            junc_policy=i32(net.junc_policy), depart_time=f32(trips.depart_time),
            route_begin=i32(trips.route_begin), route_roads=i32(trips.route_roads),
            v0_factor=f32(trips.v0_factor), length=f32(trips.length))
        a = self.arrays
        end_s = getattr(trips, "end_s", None)
        if end_s is not None:
            a["end_s"] = f32(end_s)
        start_s = getattr(trips, "start_s", None)
        if start_s is not None:
            a["start_s"] = f32(start_s)
        self.net = tsim_network(net.n_junctions, net.n_roads, *[_p(a[k]) for k in (
            "road_from", "road_to", "road_lane_begin", "road_length", "road_limit")], net.n_jlanes,
            *[_p(a[k]) for k in ("jl_in_lane", "jl_out_lane", "jl_length", "jl_limit", "junc_phase_begin",
                                 "phase_duration", "phase_green_begin", "phase_green_jl", "junc_policy")])
        self.trips = tsim_trips(trips.n_vehicles, *[_p(a[k]) for k in (
            "depart_time", "route_begin", "route_roads", "v0_factor", "length")],
            _p(a["end_s"]) if "end_s" in a else None, _p(a["start_s"]) if "start_s" in a else None)
        self.params = None if params is None else _Inputs.params_of(params)

    @staticmethod
    def params_of(params):
        return tsim_params(params.dt, params.T, params.a_max, params.b_comf, params.s0, params.delta,
                           params.politeness, params.a_th, params.b_safe, params.p_max, params.p_min,
                           params.a_emerg, int(params.seed))


def _check(rc, h=None):
    if rc != TSIM_OK:
        msg = lib().tsim_last_error(h)
        raise TsimError(rc, msg.decode() if msg else "")


def footprint(net, trips, params):
    ins = _Inputs(net, trips, params)
    n = C.c_size_t(0)
    _check(lib().tsim_footprint(C.byref(ins.net), C.byref(ins.trips), C.byref(ins.params), C.byref(n)))
    return int(n.value)


class _NoTrips:
    """A trip table with no vehicles (network-only calls)."""
    n_vehicles = 0
    depart_time = v0_factor = length = np.zeros(0, np.float32)
    route_begin = np.zeros(1, np.int32)
    route_roads = np.zeros(0, np.int32)
    end_s = None


_NO_TRIPS = _NoTrips()


def _opt_f32(a):
    return None if a is None else np.ascontiguousarray(a, np.float32)


def _workspace(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def route_workspace_bytes(net, n_pairs, least=False):
    """Device work space for shortest_routes over n_pairs pairs of net: the
    suggested size (few passes), or with least=True the least one."""
    ins = _Inputs(net, _NO_TRIPS, None)
    lo, hint = C.c_size_t(0), C.c_size_t(0)
    _check(lib().tsim_route_footprint(C.byref(ins.net), int(n_pairs), C.byref(lo), C.byref(hint)))
    return int(lo.value if least else hint.value)


def shortest_routes(net, origins, dests, price=None, road_time=None, device="cuda:0", stream=None,
                    workspace=None):
    """Routes of least cost for (origin road, destination road) pairs of a
    network (Section 4 congestion pricing: road prices price[R] in seconds;
    road_time[R] replaces the free-flow times), computed on the GPU.
    Returns (begin[n+1], roads, n_unreachable): route c is
    roads[begin[c]:begin[c+1]], empty when unreachable."""
    import torch
    ins = _Inputs(net, _NO_TRIPS, None)
    o = np.ascontiguousarray(origins, np.int32)
    d = np.ascontiguousarray(dests, np.int32)
    n = int(o.size)
    pr, rt = _opt_f32(price), _opt_f32(road_time)
    lo, hint = C.c_size_t(0), C.c_size_t(0)
    _check(lib().tsim_route_footprint(C.byref(ins.net), n, C.byref(lo), C.byref(hint)))
    dev = torch.device(device)
    ws = workspace if workspace is not None else _workspace(hint.value, dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    begin = np.zeros(n + 1, np.int32)
    bad = np.zeros(1, np.int32)
    cap = max(48 * n, 1)
    while True:
        roads = np.empty(cap, np.int32)
        with torch.cuda.device(dev):   # the kernels run on the current GPU
            rc = lib().tsim_shortest_routes(C.byref(ins.net), None if pr is None else _p(pr),
                                            None if rt is None else _p(rt), _p(o), _p(d), n,
                                            C.c_void_p(st.cuda_stream), C.c_void_p(ws.data_ptr()),
                                            C.c_size_t(ws.numel()), _p(begin), _p(roads), cap, _p(bad))
        if rc == TSIM_ENOMEM and int(begin[n]) > cap:
            cap = int(begin[n])
            continue
        _check(rc)
        return begin, roads[:int(begin[n])], int(bad[0])


class Sim:
    """One simulation instance resident in GPU memory."""

    def __init__(self, net, trips, params, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("tsim needs a GPU: torch.cuda.is_available() is False")
        self.net, self.trips, self.params = net, trips, params
        self.N = trips.n_vehicles
        self.R = net.n_roads
        self.NL = net.n_lanes
        self.NJ = net.n_junctions
        ins = _Inputs(net, trips, params)
        nbytes = C.c_size_t(0)
        _check(lib().tsim_footprint(C.byref(ins.net), C.byref(ins.trips), C.byref(ins.params), C.byref(nbytes)))
        self.device = torch.device(device)
        self.arena = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().tsim_create(C.byref(ins.net), C.byref(ins.trips), C.byref(ins.params),
                                 C.c_void_p(self.stream.cuda_stream), C.c_void_p(self.arena.data_ptr()),
                                 C.c_size_t(self.arena.numel()), C.byref(h)))
        self.h = h
        self.traj = None

    def close(self):
        if getattr(self, "h", None):
            lib().tsim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().tsim_step(self.h, int(n)), self.h)

    def set_signal_phases(self, junctions, phases):
        j = np.ascontiguousarray(junctions, np.int32)
        p = np.ascontiguousarray(phases, np.int32)
        _check(lib().tsim_set_signal_phases(self.h, _p(j), _p(p), int(j.size)), self.h)

    def record_trajectory(self, every, capacity):
        """Record every vehicle's (step, id, lane, x, v) at each step boundary
        whose step is a multiple of `every` into a device buffer of
        `capacity` records (every = 0 stops)."""
        import torch
        if every > 0:
            self.traj = torch.zeros((int(capacity), 24), dtype=torch.uint8, device=self.device)
            ptr = C.c_void_p(self.traj.data_ptr())
        else:
            self.traj, ptr = None, C.c_void_p()
        _check(lib().tsim_set_trajectory(self.h, ptr, int(capacity) if every > 0 else 0, int(every)), self.h)

    def trajectory(self):
        """The recorded trajectory as numpy arrays (step, vehicle, lane, x, v),
        sorted by (step, vehicle), and the number of records dropped for want
        of capacity."""
        n = np.zeros(1, np.int64)
        _check(lib().tsim_get_trajectory_count(self.h, _p(n)), self.h)
        cap = 0 if self.traj is None else self.traj.shape[0]
        k = int(min(n[0], cap))
        raw = self.traj[:k].cpu().numpy().reshape(-1)
        rec = np.frombuffer(raw.tobytes(), dtype=np.dtype([("step", "<i8"), ("vehicle", "<i4"), ("lane", "<i4"),
                                                           ("x", "<f4"), ("v", "<f4")]))
        rec = np.sort(rec, order=["step", "vehicle"])
        return {f: rec[f].copy() for f in rec.dtype.names}, int(n[0]) - k

    def set_aois(self, conn_begin, conn_road, conn_s, origin_aoi=None, dest_aoi=None):
        """Areas of interest: AOI a's connections are conn_road / conn_s
        [conn_begin[a]:conn_begin[a+1]]; each waiting vehicle named in
        origin_aoi / dest_aoi (-1: none) starts / ends at its AOI's
        connection on the first / last road of its route."""
        import torch
        cb = np.ascontiguousarray(conn_begin, np.int32)
        n_aoi = int(cb.size) - 1
        cr = np.ascontiguousarray(conn_road, np.int32)
        cs = np.ascontiguousarray(conn_s, np.float32)
        o = None if origin_aoi is None else np.ascontiguousarray(origin_aoi, np.int32)
        d = None if dest_aoi is None else np.ascontiguousarray(dest_aoi, np.int32)
        for a in (o, d):
            if a is not None and a.size != self.N:
                raise ValueError("one AOI id per vehicle")
        nb = C.c_size_t()
        _check(lib().tsim_aoi_footprint(self.h, n_aoi, C.byref(nb)), self.h)
        # written in full by the library on its stream (no fill here, which
        # would run on torch's stream)
        buf = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        _check(lib().tsim_set_aois(self.h, n_aoi, _p(cb), _p(cr), _p(cs), _p(o) if o is not None else None,
                                   _p(d) if d is not None else None, C.c_void_p(buf.data_ptr()), int(nb.value)),
               self.h)
        self.aoi_buf, self.n_aoi = buf, n_aoi

    def aoi_counts(self):
        """(waiting, arrived) per AOI at the current step boundary."""
        w = np.zeros(self.n_aoi, np.int32)
        a = np.zeros(self.n_aoi, np.int32)
        _check(lib().tsim_get_aoi_counts(self.h, _p(w), _p(a), int(self.n_aoi)), self.h)
        return w, a

    def set_vehicle_route(self, vid, roads, end_s=None):
        """Vehicle vid follows `roads` (beginning with the road it is on) from
        the next step on; its trip ends at end_s metres along the last road
        (None: that road's end)."""
        r = np.ascontiguousarray(roads, np.int32)
        e = -1.0 if end_s is None else float(end_s)
        _check(lib().tsim_set_vehicle_route(self.h, int(vid), _p(r), int(r.size), e), self.h)

    def reroute_shortest(self, vehicle_ids, price=None, road_time=None, workspace=None):
        """Vehicles take, from the next step on, the route of least cost from
        where they are to the last road of their route (road prices price[R],
        road times road_time[R] or free-flow), computed on the GPU.  Returns
        the number of vehicles that kept their route."""
        v = np.ascontiguousarray(vehicle_ids, np.int32)
        pr, rt = _opt_f32(price), _opt_f32(road_time)
        if workspace is None:
            lo, hint = C.c_size_t(0), C.c_size_t(0)
            _check(lib().tsim_reroute_footprint(self.h, int(v.size), C.byref(lo), C.byref(hint)), self.h)
            workspace = _workspace(hint.value, self.device)
        kept = np.zeros(1, np.int32)
        _check(lib().tsim_reroute_shortest(self.h, _p(v), int(v.size), None if pr is None else _p(pr),
                                           None if rt is None else _p(rt), C.c_void_p(workspace.data_ptr()),
                                           C.c_size_t(workspace.numel()), _p(kept)), self.h)
        return int(kept[0])

    def set_lane_max_speed(self, lanes, speeds):
        """Speed limits of lanes (network lane ids) from the next step on."""
        l = np.ascontiguousarray(lanes, np.int32)
        v = np.ascontiguousarray(speeds, np.float32)
        _check(lib().tsim_set_lane_max_speed(self.h, _p(l), _p(v), int(l.size)), self.h)

    def set_lane_restriction(self, lanes, flags):
        """Restrict (flag != 0) or release lanes (network lane ids) from the
        next step on: a restricted lane admits no new vehicle (departure,
        lane change, or entry through a junction lane that is restricted or
        leads into it); vehicles already on it carry on."""
        l = np.ascontiguousarray(lanes, np.int32)
        f = np.ascontiguousarray(flags, np.int32)
        _check(lib().tsim_set_lane_restriction(self.h, _p(l), _p(f), int(l.size)), self.h)

    def set_road_lane_plan(self, plans, index):
        """Put a road's lane plan in force (see lane_plan_flags)."""
        self.set_lane_restriction(*lane_plan_flags(plans, index))

    def set_signal_policy(self, junctions, policies):
        """Signal policy per junction (TSIM_POLICY_*: 0 none, 1 fixed time,
        2 manual, 3 max pressure) from the next step on."""
        j = np.ascontiguousarray(junctions, np.int32)
        p = np.ascontiguousarray(policies, np.int32)
        _check(lib().tsim_set_signal_policy(self.h, _p(j), _p(p), int(j.size)), self.h)

    def metrics(self, check=True):
        m = tsim_metrics()
        rc = lib().tsim_get_metrics(self.h, C.byref(m))
        if check:
            _check(rc, self.h)
        return {k: getattr(m, k) for k, _ in tsim_metrics._fields_}

    def road_mean_speed(self):
        out = np.zeros(self.R, np.float32)
        _check(lib().tsim_get_road_mean_speed(self.h, _p(out), self.R), self.h)
        return out

    def lane_waiting_counts(self):
        out = np.zeros(self.NL, np.int32)
        _check(lib().tsim_get_lane_waiting_counts(self.h, _p(out), self.NL), self.h)
        return out

    def lane_order(self):
        off = np.zeros(self.NL + 1, np.int32)
        ids = np.zeros(max(self.N, 1), np.int32)
        _check(lib().tsim_get_lane_order(self.h, _p(off), _p(ids), self.NL, ids.size), self.h)
        return off, ids[:off[-1]]

    def set_profiling(self, enable=True):
        _check(lib().tsim_set_profiling(self.h, 1 if enable else 0), self.h)

    def set_graph_steps(self, chunk):
        """Replay `chunk`-step HIP graphs inside step(); 0 = direct launches."""
        _check(lib().tsim_set_graph_steps(self.h, int(chunk)), self.h)

    def set_schedule(self, schedule):
        _check(lib().tsim_set_schedule(self.h, int(schedule)), self.h)

    def set_concurrency(self, enable=True):
        """Run the update passes of each step on side streams, concurrently."""
        _check(lib().tsim_set_concurrency(self.h, 1 if enable else 0), self.h)

    def schedule(self):
        out = np.zeros(1, np.int32)
        _check(lib().tsim_get_schedule(self.h, _p(out)), self.h)
        return int(out[0])

    def autotune(self, steps=10, rounds=2):
        """Tries every schedule for `rounds` x `steps` real steps (the state
        advances), keeps the fastest; returns (schedule, us_per_step array)."""
        ch = np.zeros(1, np.int32)
        us = np.zeros(len(SCHEDULES), np.float32)
        _check(lib().tsim_autotune(self.h, int(steps), int(rounds), _p(ch), _p(us)), self.h)
        return int(ch[0]), us

    def autotune_launch(self, steps=10, rounds=2):
        """As autotune over (schedule, pass concurrency) pairs (2 x the
        steps of autotune); returns (schedule, concurrent, us_per_step of
        shape (2, n_schedules): serial row, then concurrent row)."""
        sc = np.zeros(1, np.int32)
        cc = np.zeros(1, np.int32)
        us = np.zeros(2 * len(SCHEDULES), np.float32)
        _check(lib().tsim_autotune_launch(self.h, int(steps), int(rounds), _p(sc), _p(cc), _p(us)), self.h)
        return int(sc[0]), bool(cc[0]), us.reshape(2, len(SCHEDULES))

    def kernel_times(self):
        """{'update': (ms, launches), 'prepare': (ms, launches)} since profiling was enabled."""
        ms = np.zeros(2, np.float64)
        n = np.zeros(2, np.int64)
        _check(lib().tsim_get_kernel_times(self.h, _p(ms), _p(n), 2), self.h)
        return {"update": (float(ms[0]), int(n[0])), "prepare": (float(ms[1]), int(n[1]))}

    def get_state(self):
        st, s = _state_arrays(self.N, self.NJ)
        _check(lib().tsim_get_state(self.h, C.byref(s)), self.h)
        st["step"] = int(s.step)
        return st

    def set_state(self, st):
        keep, s = _state_in(st, self.net)
        _check(lib().tsim_set_state(self.h, C.byref(s)), self.h)


def lane_plan_flags(plans, index):
    """A road lane plan (Section 3.2 "Road" set_road_lane_plan) as lane
    restrictions.  plans: a road's alternative sets of junction lanes in use
    (network lane ids), e.g. a dynamic lane's left-turn or straight-on
    movement; plan `index` is put in force by restricting every junction
    lane of the plans that it does not use and releasing those it uses.
    Returns (lanes, flags) for set_lane_restriction."""
    every = sorted(set().union(*[set(int(l) for l in p) for p in plans]))
    use = set(int(l) for l in plans[index])
    return np.asarray(every, np.int32), np.asarray([0 if l in use else 1 for l in every], np.int32)


def _state_arrays(N, NJ):
    st = dict(status=np.zeros(N, np.int32), lane=np.zeros(N, np.int32), route_pos=np.zeros(N, np.int32),
              x=np.zeros(N, np.float32), v=np.zeros(N, np.float32), finish_step=np.zeros(N, np.int32),
              junc_policy=np.zeros(NJ, np.int32), junc_phase=np.zeros(NJ, np.int32))
    s = tsim_state_host(0, *[_p(st[k]) for k in ("status", "lane", "route_pos", "x", "v", "finish_step",
                                                   "junc_policy", "junc_phase")])
    return st, s


def _state_in(st, net):
    NJ = net.n_junctions
    a = dict(status=np.ascontiguousarray(st["status"], np.int32),
             lane=np.ascontiguousarray(st["lane"], np.int32),
             route_pos=np.ascontiguousarray(st["route_pos"], np.int32),
             x=np.ascontiguousarray(st["x"], np.float32), v=np.ascontiguousarray(st["v"], np.float32),
             finish_step=np.ascontiguousarray(st["finish_step"], np.int32),
             junc_policy=np.ascontiguousarray(st.get("junc_policy", net.junc_policy), np.int32),
             junc_phase=np.ascontiguousarray(st.get("junc_phase", np.zeros(NJ, np.int32)), np.int32))
    s = tsim_state_host(int(st["step"]), *[_p(a[k]) for k in ("status", "lane", "route_pos", "x", "v",
                                                               "finish_step", "junc_policy", "junc_phase")])
    return a, s


class Instance:
    """A simulation validated and laid out on the host (tsim_instance_build),
    ready to join a batch; building needs no GPU."""

    def __init__(self, net, trips, params):
        self.net, self.trips, self.params = net, trips, params
        ins = _Inputs(net, trips, params)
        h = C.c_void_p()
        _check(lib().tsim_instance_build(C.byref(ins.net), C.byref(ins.trips), C.byref(ins.params), C.byref(h)))
        self.h = h

    def capacity(self):
        c = tsim_batch_capacity()
        _check(lib().tsim_instance_capacity(self.h, C.byref(c)))
        return {k: int(getattr(c, k)) for k in CAPACITY_FIELDS}

    def close(self):
        if getattr(self, "h", None):
            lib().tsim_instance_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _capacity_struct(cap):
    return tsim_batch_capacity(*[int(cap[k]) for k in CAPACITY_FIELDS])


def reserve_footprint(cap):
    n = C.c_size_t(0)
    _check(lib().tsim_batch_reserve_footprint(C.byref(_capacity_struct(cap)), C.byref(n)))
    return int(n.value)


def add_capacity(a, b, scale=1):
    return {k: int(a.get(k, 0)) + int(scale * b[k]) for k in CAPACITY_FIELDS}


class Batch:
    """Many independent instances resident together and stepped by the same
    launches (tsim_batch_* in include/tsim.h)."""

    @classmethod
    def reserve(cls, capacity, params, device="cuda:0", stream=None):
        """An empty batch with room for the given totals (a dict of the
        tsim_batch_capacity fields); instances join with add()."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("tsim needs a GPU: torch.cuda.is_available() is False")
        self = cls.__new__(cls)
        self.n = 0
        self.nets, self.trips, self.params = [], [], []
        self._ins = []
        cs = _capacity_struct(capacity)
        nbytes = C.c_size_t(0)
        _check(lib().tsim_batch_reserve_footprint(C.byref(cs), C.byref(nbytes)))
        self.device = torch.device(device)
        self.arena = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        p = _Inputs.params_of(params)
        h = C.c_void_p()
        _check(lib().tsim_batch_reserve(C.byref(cs), C.byref(p), C.c_void_p(self.stream.cuda_stream),
                                        C.c_void_p(self.arena.data_ptr()), C.c_size_t(self.arena.numel()),
                                        C.byref(h)))
        self.h = h
        return self

    def add(self, net, trips=None, params=None):
        """Appends an instance (an Instance, or net/trips/params) at the step
        boundary, starting at its local step 0; returns its id."""
        inst = net if isinstance(net, Instance) else Instance(net, trips, params)
        k = C.c_int32(0)
        _check(lib().tsim_batch_add(self.h, inst.h, C.byref(k)), self.h)
        self._place(int(k.value), inst.net, inst.trips, inst.params)
        return int(k.value)

    def add_member(self, sim):
        """Appends a copy of a live Sim (network, trips, parameters and
        current state); returns its id."""
        k = C.c_int32(0)
        _check(lib().tsim_batch_add_member(self.h, sim.h, C.byref(k)), self.h)
        self._place(int(k.value), sim.net, sim.trips, sim.params)
        return int(k.value)

    def _place(self, k, net, trips, params):
        del self.nets[k:], self.trips[k:], self.params[k:]
        self.nets.append(net)
        self.trips.append(trips)
        self.params.append(params)
        self.n = len(self.nets)

    def remove(self, k):
        """Freezes instance k for good; trailing removed instances give their
        space (and ids) back."""
        _check(lib().tsim_batch_remove(self.h, int(k)), self.h)
        n = self.num_instances()
        del self.nets[n:], self.trips[n:], self.params[n:]
        self.n = n

    def num_instances(self):
        n = C.c_int32(0)
        _check(lib().tsim_batch_num_instances(self.h, C.byref(n)), self.h)
        return int(n.value)

    def capacity_left(self):
        c = tsim_batch_capacity()
        _check(lib().tsim_batch_capacity_left(self.h, C.byref(c)), self.h)
        return {k: int(getattr(c, k)) for k in CAPACITY_FIELDS}

    def __init__(self, nets, trips, params, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("tsim needs a GPU: torch.cuda.is_available() is False")
        n = len(nets)
        assert len(trips) == n and len(params) == n and n > 0
        self.n = n
        self.nets, self.trips, self.params = nets, trips, params
        self._ins = [_Inputs(a, b, c) for a, b, c in zip(nets, trips, params)]
        self._net_arr = (tsim_network * n)(*[i.net for i in self._ins])
        self._trip_arr = (tsim_trips * n)(*[i.trips for i in self._ins])
        self._par_arr = (tsim_params * n)(*[i.params for i in self._ins])
        nbytes = C.c_size_t(0)
        _check(lib().tsim_batch_footprint(self._net_arr, self._trip_arr, self._par_arr, n, C.byref(nbytes)))
        self.device = torch.device(device)
        self.arena = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().tsim_batch_create(self._net_arr, self._trip_arr, self._par_arr, n,
                                       C.c_void_p(self.stream.cuda_stream), C.c_void_p(self.arena.data_ptr()),
                                       C.c_size_t(self.arena.numel()), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().tsim_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().tsim_batch_step(self.h, int(n)), self.h)

    def set_graph_steps(self, chunk):
        _check(lib().tsim_batch_set_graph_steps(self.h, int(chunk)), self.h)

    def set_profiling(self, enable=True):
        _check(lib().tsim_set_profiling(self.h, 1 if enable else 0), self.h)

    def kernel_times(self):
        """{'update': (ms, launches), 'prepare': (ms, launches)} since profiling was enabled."""
        return Sim.kernel_times(self)

    def set_schedule(self, schedule):
        Sim.set_schedule(self, schedule)

    def set_concurrency(self, enable=True):
        Sim.set_concurrency(self, enable)

    def schedule(self):
        return Sim.schedule(self)

    def autotune(self, steps=10, rounds=2):
        return Sim.autotune(self, steps, rounds)

    def autotune_launch(self, steps=10, rounds=2):
        return Sim.autotune_launch(self, steps, rounds)

    def set_signal_phases(self, instance, junctions, phases):
        j = np.ascontiguousarray(junctions, np.int32)
        p = np.ascontiguousarray(phases, np.int32)
        _check(lib().tsim_batch_set_signal_phases(self.h, int(instance), _p(j), _p(p), int(j.size)), self.h)

    def set_signal_policy(self, instance, junctions, policies):
        j = np.ascontiguousarray(junctions, np.int32)
        p = np.ascontiguousarray(policies, np.int32)
        _check(lib().tsim_batch_set_signal_policy(self.h, int(instance), _p(j), _p(p), int(j.size)), self.h)

    def set_vehicle_route(self, instance, vid, roads, end_s=None):
        r = np.ascontiguousarray(roads, np.int32)
        e = -1.0 if end_s is None else float(end_s)
        _check(lib().tsim_batch_set_vehicle_route(self.h, int(instance), int(vid), _p(r), int(r.size), e), self.h)

    def set_lane_max_speed(self, instance, lanes, speeds):
        l = np.ascontiguousarray(lanes, np.int32)
        v = np.ascontiguousarray(speeds, np.float32)
        _check(lib().tsim_batch_set_lane_max_speed(self.h, int(instance), _p(l), _p(v), int(l.size)), self.h)

    def set_lane_restriction(self, instance, lanes, flags):
        l = np.ascontiguousarray(lanes, np.int32)
        f = np.ascontiguousarray(flags, np.int32)
        _check(lib().tsim_batch_set_lane_restriction(self.h, int(instance), _p(l), _p(f), int(l.size)), self.h)

    def set_road_lane_plan(self, instance, plans, index):
        self.set_lane_restriction(instance, *lane_plan_flags(plans, index))

    def reroute_shortest(self, instance, vehicle_ids, price=None, road_time=None, workspace=None):
        """As Sim.reroute_shortest, for vehicles of one instance (local ids;
        price and road_time over the instance's roads)."""
        v = np.ascontiguousarray(vehicle_ids, np.int32)
        pr, rt = _opt_f32(price), _opt_f32(road_time)
        if workspace is None:
            lo, hint = C.c_size_t(0), C.c_size_t(0)
            _check(lib().tsim_batch_reroute_footprint(self.h, int(instance), int(v.size), C.byref(lo),
                                                      C.byref(hint)), self.h)
            workspace = _workspace(hint.value, self.device)
        kept = np.zeros(1, np.int32)
        _check(lib().tsim_batch_reroute_shortest(self.h, int(instance), _p(v), int(v.size),
                                                 None if pr is None else _p(pr), None if rt is None else _p(rt),
                                                 C.c_void_p(workspace.data_ptr()), C.c_size_t(workspace.numel()),
                                                 _p(kept)), self.h)
        return int(kept[0])

    def set_horizon(self, instance, n_steps):
        """Freeze instance after n_steps local steps (the others go on)."""
        _check(lib().tsim_batch_set_horizon(self.h, int(instance), int(n_steps)), self.h)

    def set_all_phases(self, phases):
        """phases: one entry per junction of the batch, instance order; -1 = unchanged."""
        p = np.ascontiguousarray(phases, np.int32)
        _check(lib().tsim_batch_set_all_phases(self.h, _p(p), int(p.size)), self.h)

    def metrics(self, instance, check=True):
        m = tsim_metrics()
        rc = lib().tsim_batch_get_metrics(self.h, int(instance), C.byref(m))
        if check:
            _check(rc, self.h)
        return {k: getattr(m, k) for k, _ in tsim_metrics._fields_}

    def get_state(self, instance):
        st, s = _state_arrays(self.trips[instance].n_vehicles, self.nets[instance].n_junctions)
        _check(lib().tsim_batch_get_state(self.h, int(instance), C.byref(s)), self.h)
        st["step"] = int(s.step)
        return st

    def set_state(self, instance, st):
        """Replaces one instance's state at the step boundary (it continues
        from its own step st['step']; the others are untouched)."""
        keep, s = _state_in(st, self.nets[instance])
        _check(lib().tsim_batch_set_state(self.h, int(instance), C.byref(s)), self.h)

    def set_aois(self, instance, conn_begin, conn_road, conn_s, origin_aoi=None, dest_aoi=None):
        """As Sim.set_aois, for one instance (its local road and vehicle ids)."""
        import torch
        cb = np.ascontiguousarray(conn_begin, np.int32)
        n_aoi = int(cb.size) - 1
        cr = np.ascontiguousarray(conn_road, np.int32)
        cs = np.ascontiguousarray(conn_s, np.float32)
        o = None if origin_aoi is None else np.ascontiguousarray(origin_aoi, np.int32)
        d = None if dest_aoi is None else np.ascontiguousarray(dest_aoi, np.int32)
        for a in (o, d):
            if a is not None and a.size != self.trips[instance].n_vehicles:
                raise ValueError("one AOI id per vehicle of the instance")
        nb = C.c_size_t()
        _check(lib().tsim_batch_aoi_footprint(self.h, int(instance), n_aoi, C.byref(nb)), self.h)
        # written in full by the library on its stream
        buf = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        _check(lib().tsim_batch_set_aois(self.h, int(instance), n_aoi, _p(cb), _p(cr), _p(cs),
                                         _p(o) if o is not None else None, _p(d) if d is not None else None,
                                         C.c_void_p(buf.data_ptr()), int(nb.value)), self.h)
        if not hasattr(self, "aoi_bufs"):
            self.aoi_bufs = {}
        self.aoi_bufs[int(instance)] = (buf, n_aoi)

    def aoi_counts(self, instance):
        """(waiting, arrived) per AOI of one instance."""
        n_aoi = self.aoi_bufs[int(instance)][1]
        w = np.zeros(n_aoi, np.int32)
        a = np.zeros(n_aoi, np.int32)
        _check(lib().tsim_batch_get_aoi_counts(self.h, int(instance), _p(w), _p(a), n_aoi), self.h)
        return w, a

    def road_mean_speed(self, instance):
        out = np.zeros(self.nets[instance].n_roads, np.float32)
        _check(lib().tsim_batch_get_road_mean_speed(self.h, int(instance), _p(out), out.size), self.h)
        return out

    def lane_waiting_counts(self, instance):
        out = np.zeros(self.nets[instance].n_lanes, np.int32)
        _check(lib().tsim_batch_get_lane_waiting_counts(self.h, int(instance), _p(out), out.size), self.h)
        return out

    def lane_order(self, instance):
        NL = self.nets[instance].n_lanes
        off = np.zeros(NL + 1, np.int32)
        ids = np.zeros(max(self.trips[instance].n_vehicles, 1), np.int32)
        _check(lib().tsim_batch_get_lane_order(self.h, int(instance), _p(off), _p(ids), NL, ids.size), self.h)
        return off, ids[:off[-1]]

    def instance(self, k):
        """A view of instance k with the single-instance accessors (state,
        metrics, per-lane getters); step() steps the whole batch."""
        return BatchInstance(self, k)


class BatchInstance:
    """One instance of a Batch seen through the single-instance interface."""

    def __init__(self, batch, k):
        self.b, self.k = batch, int(k)

    def set_state(self, st):
        self.b.set_state(self.k, st)

    def get_state(self):
        return self.b.get_state(self.k)

    def step(self, n=1):
        self.b.step(n)

    def metrics(self, check=True):
        return self.b.metrics(self.k, check)

    def road_mean_speed(self):
        return self.b.road_mean_speed(self.k)

    def lane_waiting_counts(self):
        return self.b.lane_waiting_counts(self.k)

    def lane_order(self):
        return self.b.lane_order(self.k)
