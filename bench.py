"""Benchmark of the gfx950 stepper on the paper-scale synthetic city.

Workload: ~50,000-junction planar city with 2,464,950 vehicles (departures
N(3600 s, 1200 s)), dt = 1 s, FP32 on the GPU; one "step" is one simulation
timestep of the whole per-vehicle update (signals, departures, sensing index,
IDM, randomized MOBIL, integration, transfers, metrics).

Timed region: K steps (default 200) from the run's own loaded state at step
S (default 4,500 of the 7,200-step horizon, about 1.7M vehicles on the
network), which is reached by stepping from t = 0 outside the timed region and
snapshotted; W warm-up steps run from the snapshot, which is then restored.
The K steps replay captured HIP graphs of min(K, graph-steps) steps, bracketed
by device synchronisation and HIP events on the library's stream.  value = sum
over the K steps of active vehicles / seconds.

Also reported: simulated Hz, the achieved bandwidth of one whole step
(k_prepare plus the update) against MI355X HBM peak on algorithmic bytes (48 B
per active vehicle-step, 24 B per non-empty lane-step and 4 B per crossing
onto the next road, counted on the device over the window), the window's HBM
traffic from rocprofv3 counters when they were taken on the current kernel
source over the same window, and the CPU oracle's throughput on a bounded
sample (a synthetic state of the same city at time S).

The same line carries, under "batched" and "served", compact forms of the
two serving-style workloads timed in the same run (64 instances for 300
steps; 100 jobs of at most 100,000 vehicles), each against its plain
one-instance-at-a-time loop, and under "routing" the device shortest routes
of a served pricing job (--no-legs leaves them out).

--workload batch: 256 uneven jittered-grid instances (1k-150k vehicles each,
about 15M in total) stepped together through captured 15-step HIP graphs for
1,800 steps, with every junction's phase set from a seeded random policy every
15 steps; the same instances stepped one at a time by the plain stepper on the
same schedule are the baseline (ratio in "vs_plain_loop").

--workload route: least-cost routes under road prices (Section 4 congestion
pricing) for 150,000 trips of a 32x32 jittered grid computed on the GPU,
against the host's Dijkstra and the oracle on a bounded sample.

--workload serve: a Poisson stream (20 jobs/s) of pre-generated jobs (signal
timing plans or road prices; 10k-500k vehicles; 300-3,600 steps; each job's
trips routed on the GPU under its prices before the stream starts) run by the
continuous-batching loop of ``paper_2406_10661_amd.serve`` under an HBM
budget (default: jobs gathered into batches, each frozen at its own
horizon); reports jobs/s, p50/p99 latency and the plain one-job-at-a-time
loop, and the served capacity: the same jobs all arriving at once
("saturated").

Prints one JSON line on stdout.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of a step (what the method must move, independent of this
# layout): per active vehicle its position, speed, lane and route cursor read
# and written (2 x 16 B), its desired-speed factor and length read (8 B) and
# its place in the lane order read and written (8 B); per lane holding
# vehicles its length, limit, successor / signal word and segment bounds
# (24 B); per crossing onto the next road one route word (4 B)
BYTES_PER_ACTIVE = 48
BYTES_PER_LANE = 24
BYTES_PER_ROAD_ENTRY = 4
# the roofline's unit: one whole step as launched in the timed region
# (k_prepare, then the update: k_update_fused under the fused schedule, else
# the per-class passes k_update_block and k_update_grouped), its time taken
# from the events around the timed region


def step_label(schedule_name):
    upd = "k_update_fused" if "fused" in schedule_name else "update passes (k_update_block, k_update_grouped)"
    return f"one step: k_prepare + {upd}"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources with comments and white space removed (a
    change to either invalidates counters taken before it)."""
    import re
    h = hashlib.sha256()
    for f in ("tsim_kernels.hip", "tsim_internal.h"):
        with open(os.path.join(ROOT, "paper_2406_10661_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(name, window):
    """HBM bytes per step of the step's kernels measured by rocprofv3
    counters for this workload and window (profiles/traffic_<name>.md, lines
    'kernel_hash: ...', 'window: ...' and 'hbm_bytes_per_step: ...'), if they
    were taken on the current kernel source over the same window; else None."""
    import re
    p = os.path.join(ROOT, "profiles", f"traffic_{name}.md")
    if not os.path.exists(p):
        return None
    txt = open(p).read()
    h = re.search(r"^kernel_hash:\s*(\S+)", txt, re.M)
    wn = re.search(r"^window:\s*(.+?)\s*$", txt, re.M)
    b = re.search(r"^hbm_bytes_per_step:\s*([0-9.eE+]+)", txt, re.M)
    if not h or not b or h.group(1) != kernel_source_hash():
        return None
    if window is not None and (not wn or wn.group(1) != window):
        return None
    return float(b.group(1))


def cpu_baseline(w, step, seconds=12.0):
    """The oracle (single-threaded FP64 C) stepping a seeded synthetic state
    of the same city at the timed window's start time (vehicles due by then
    placed along their routes, 95% of them on the network), for about
    `seconds` of CPU time.  Its input is generated on the host, never taken
    from the GPU run."""
    from oracle import oracle as O
    from paper_2406_10661_amd.workloads import synthetic_state
    O.build()
    st = synthetic_state(w.network, w.trips, step, seed=99, p_active=0.95, p_finished=0.0)
    st["x"] = st["x"].astype("float64")
    st["v"] = st["v"].astype("float64")
    o = O.OracleSim(w.network, w.trips, w.params)
    o.set_state(st)
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    vs = o.metrics()["vehicle_steps"]
    return {"value": vs / el, "unit": "vehicle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{w.name}: seeded synthetic state at t={step} s with {int((st['status'] == 1).sum())} "
                      f"active vehicles, {steps} oracle steps in {el:.1f} s",
            "hz": steps / el, "host_cpus": os.cpu_count()}


METRIC = "vehicle-steps/s + sim Hz at 2.46M veh; batched jobs/s, p50/p99 job latency"


def roofline(alg_bytes, ms, steps, traffic, label):
    """Achieved bandwidth of one step: algorithmic bytes of the timed steps
    over their event-timed milliseconds."""
    achieved = alg_bytes / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": label,
            "us_per_launch": ms / max(steps, 1) * 1e3, "bytes_per_launch": alg_bytes / max(steps, 1)}


def tune(obj, steps, concurrent):
    """Autotunes the schedule of a Sim or Batch, and its pass concurrency
    unless that is fixed; returns (schedule, concurrent, us_per_step)."""
    if concurrent is None:
        return obj.autotune_launch(steps=steps, rounds=2)
    obj.set_concurrency(concurrent)
    sched, us = obj.autotune(steps=steps, rounds=2)
    return sched, concurrent, us


def concurrency_arg(args):
    """--concurrent: None (autotuned) or a fixed bool."""
    return None if args.concurrent == "auto" else args.concurrent == "1"


def run_batch(args, emit=True):
    """Batched RL-style stepping of many uneven instances versus the plain
    per-instance loop on the same phase schedule."""
    import numpy as np
    import torch
    from paper_2406_10661_amd import workloads as W
    from paper_2406_10661_amd.tsim import Batch, Sim
    every = 15
    t0 = time.time()
    ws = W.batch_workload(args.instances, steps=args.steps)
    n_chunks = args.steps // every
    scheds = [W.random_phase_schedule(w.network, w.extra["policy_seed"], n_chunks) for w in ws]
    allph = [np.concatenate([sc[c] for sc in scheds]) for c in range(n_chunks)]
    nets, trips, pars = [w.network for w in ws], [w.trips for w in ws], [w.params for w in ws]
    nveh = sum(w.trips.n_vehicles for w in ws)
    lanes = sum(w.network.n_lanes for w in ws)
    log(f"[bench] batch of {len(ws)} instances, {nveh} vehicles, {lanes} lanes, generated in "
        f"{time.time() - t0:.1f} s")

    from paper_2406_10661_amd.tsim import SCHEDULES
    # schedule: autotuned on a throw-away batch once traffic has built up
    b = Batch(nets, trips, pars)
    for c in range(min(450 // every, n_chunks)):
        b.set_all_phases(allph[c])
        b.step(every)
    sched, conc, us = tune(b, every, concurrency_arg(args))
    b.close()
    del b
    torch.cuda.synchronize()
    log(f"[bench] autotuned schedule {sched} ({SCHEDULES[sched]}), concurrent passes {conc}; us/step "
        f"{[[round(float(x), 1) for x in row] for row in us] if us.ndim == 2 else [round(float(x), 1) for x in us]}")

    def batched(profile):
        b = Batch(nets, trips, pars)
        b.set_schedule(sched)
        b.set_concurrency(conc)
        if profile:
            b.set_profiling(True)
        else:
            b.set_graph_steps(every)
            b.step(0)                      # captures the graph outside the timed region
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        for c in range(n_chunks):
            b.set_all_phases(allph[c])
            b.step(every)
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        kt = b.kernel_times() if profile else None
        ms_inst = [b.metrics(k) for k in range(len(ws))]
        log(f"[bench] batched{' (profiled)' if profile else ''}: {n_chunks * every} steps in {ms:.1f} ms")
        b.close()
        del b
        torch.cuda.synchronize()
        return ms, kt, ms_inst

    _, kt, met_p = batched(True)
    ms_b, _, met_b = batched(False)
    vs_b = sum(m["vehicle_steps"] for m in met_b)
    vs_p = sum(m["vehicle_steps"] for m in met_p)

    # plain loop: one instance at a time, direct launches, same schedule
    plain_ms = 0.0
    same = True
    for k, w in enumerate(ws):
        sim = Sim(w.network, w.trips, w.params)
        sim.set_schedule(sched)
        js = np.arange(w.network.n_junctions, dtype=np.int32)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        for c in range(n_chunks):
            sim.set_signal_phases(js, scheds[k][c])
            sim.step(every)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        plain_ms += e0.elapsed_time(e1)
        m = sim.metrics()
        same &= (m["vehicle_steps"] == met_b[k]["vehicle_steps"] and m["n_finished"] == met_b[k]["n_finished"]
                 and m["mean_speed_avg"] == met_b[k]["mean_speed_avg"])
        sim.close()
        del sim
    log(f"[bench] plain loop: {plain_ms:.1f} ms; identical per-instance results: {same}")
    upd_ms, upd_n = kt["update"]
    steps = n_chunks * every
    alg = (BYTES_PER_ACTIVE * vs_b + BYTES_PER_LANE * sum(m["lane_steps"] for m in met_b)
           + BYTES_PER_ROAD_ENTRY * sum(m["road_entries"] for m in met_b))
    out = {
        "metric": METRIC, "value": vs_b / (ms_b / 1e3), "unit": "vehicle-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": 0, "ms_per_step": ms_b / steps, "sim_hz": steps / (ms_b / 1e3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch{len(ws)}_jittered_grids", "instances": len(ws), "vehicles": nveh,
                   "lanes": lanes, "steps_per_phase_update": every, "launch": "captured 15-step HIP graphs",
                   "schedule": SCHEDULES[sched], "concurrent_passes": bool(conc)},
        "vs_plain_loop": plain_ms / ms_b,
        "plain_loop": {"value": vs_b / (plain_ms / 1e3), "ms": plain_ms, "identical_results": bool(same)},
        "roofline": roofline(alg, ms_b, steps, traffic_from_profiles(f"batch{len(ws)}", None), step_label(SCHEDULES[sched])),
        "update_passes_us_eager": upd_ms / max(upd_n, 1) * 1e3,
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def run_serve(args, emit=True):
    """Continuous batching of a Poisson job stream versus the plain loop."""
    import numpy as np
    import torch
    from paper_2406_10661_amd import workloads as W
    from paper_2406_10661_amd import serve as SV
    from paper_2406_10661_amd.tsim import Sim
    t0 = time.time()
    ws = W.served_jobs(args.jobs, max_vehicles=getattr(args, "max_vehicles", None), route=False)
    arr = W.poisson_arrivals(args.jobs, rate=args.rate)
    t_route = SV.route_jobs_on_device(ws)
    log(f"[bench] {len(ws)} jobs generated in {time.time() - t0:.1f} s, routed on the GPU in {t_route:.2f} s; "
        f"{sum(w.trips.n_vehicles for w in ws)} vehicles in total")
    jobs = [SV.Job(jid=k, arrival=float(arr[k]), network=w.network, trips=w.trips, params=w.params,
                   horizon=w.n_steps) for k, w in enumerate(ws)]
    if args.serve_mode == "batched":
        fac = SV.BatchFactory(n_streams=args.streams, graph_steps=args.tick, concurrent=args.concurrent == "1")
        loop = SV.BatchedServeLoop(fac, hbm_budget=int(args.budget_gib * 2**30), steps_per_tick=args.tick,
                                   max_batches=args.max_batches)
    else:
        fac = SV.GpuFactory(n_streams=args.streams, graph_steps=args.tick)
        loop = SV.ServeLoop(fac, hbm_budget=int(args.budget_gib * 2**30), steps_per_tick=args.tick)
    res = loop.run(jobs)
    summ = SV.summarize(res, skip=args.skip)
    log(f"[bench] served: {json.dumps(summ)}")
    # served capacity: the same jobs all arriving at once, so that the loop
    # is never short of work (the Poisson stream above is bound by its rate)
    summ_s = None
    if not args.no_saturate:
        jobs_s = [SV.Job(jid=k, arrival=0.0, network=w.network, trips=w.trips, params=w.params,
                         horizon=w.n_steps) for k, w in enumerate(ws)]
        if args.serve_mode == "batched":
            loop_s = SV.BatchedServeLoop(fac, hbm_budget=int(args.budget_gib * 2**30), steps_per_tick=args.tick,
                                         max_batches=args.max_batches)
        else:
            loop_s = SV.ServeLoop(fac, hbm_budget=int(args.budget_gib * 2**30), steps_per_tick=args.tick)
        summ_s = SV.summarize(loop_s.run(jobs_s))
        log(f"[bench] saturated: {json.dumps(summ_s)}")
    # plain loop over the measured jobs: one job at a time, direct launches
    sel = sorted(res["jobs"], key=lambda j: j.arrival)[args.skip:]
    plain_ms = 0.0
    vs = 0
    same = True
    for j in sel:
        sim = Sim(j.network, j.trips, j.params)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(j.horizon)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        plain_ms += e0.elapsed_time(e1)
        m = sim.metrics()
        vs += m["vehicle_steps"]
        same &= (m["vehicle_steps"] == j.metrics["vehicle_steps"] and m["n_finished"] == j.metrics["n_finished"])
        sim.close()
    plain = vs / (plain_ms / 1e3)
    log(f"[bench] plain loop over {len(sel)} jobs: {plain_ms:.1f} ms of steps, {plain:.3e} vehicle-steps/s, "
        f"identical results {same}")
    offered = sum(j.horizon * j.trips.n_vehicles for j in sel)
    out = {
        "metric": METRIC, "value": summ["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1,
        "steps": int(sum(j.horizon for j in sel)), "warmup": args.skip,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served_poisson", "jobs": len(jobs), "measured_after": args.skip,
                   "rate_jobs_per_s": args.rate, "hbm_budget_gib": args.budget_gib, "steps_per_tick": args.tick,
                   "streams": args.streams, "mode": args.serve_mode, "batches": res.get("batches"),
                   "routing": "GPU (tsim_shortest_routes)", "routing_s": t_route,
                   "route_entries": int(sum(len(w.trips.route_roads) for w in ws))},
        "latency_p50_s": summ["latency_p50_s"], "latency_p99_s": summ["latency_p99_s"],
        "queue_wait_p99_s": summ["queue_wait_p99_s"],
        "vehicle_steps_per_s": summ["vehicle_steps_per_s"],
        "vs_plain_loop": summ["vehicle_steps_per_s"] / plain,
        "plain_loop": {"vehicle_steps_per_s": plain, "ms": plain_ms, "identical_results": bool(same)},
        "offered_vehicle_trip_steps": offered,
    }
    if summ_s is not None:
        out["saturated"] = {"jobs": summ_s["jobs"], "jobs_per_s": summ_s["jobs_per_s"],
                            "vehicle_steps_per_s": summ_s["vehicle_steps_per_s"],
                            "vs_plain_loop": summ_s["vehicle_steps_per_s"] / plain,
                            "latency_p50_s": summ_s["latency_p50_s"], "latency_p99_s": summ_s["latency_p99_s"],
                            "wall_s": summ_s["wall_s"]}
        # share of the loop's capacity that the Poisson stream used
        out["utilisation"] = summ["vehicle_steps_per_s"] / summ_s["vehicle_steps_per_s"]
    if emit:
        print(json.dumps(out), flush=True)
    return out


def run_copy(args):
    """Plain device copy of a known size (calibrates the HBM byte counters:
    FETCH_SIZE and WRITE_SIZE of this kernel versus its 2 x bytes moved)."""
    import torch
    n = int(args.copy_mib) << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps or 10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (args.steps or 10)
    print(json.dumps({"workload": "copy", "bytes_read": n, "bytes_written": n, "ms_per_copy": ms,
                      "GBps": 2 * n / (ms / 1e3) / 1e9}), flush=True)


def run_route(args, emit=True):
    """Device shortest routes for a served pricing job at the largest served
    network size: a 32x32 jittered grid with per-road prices U(0, 120) s
    and --route-trips uniform origin-destination trips.  The whole call
    (pairs up, routes down, work space allocated beforehand) is timed over
    --steps calls after one warm-up, against the host routing the served
    jobs are generated with (scipy's Dijkstra from every destination, one
    process) and the oracle on a bounded sample of destinations."""
    import numpy as np
    import torch
    from paper_2406_10661_amd import tsim
    from paper_2406_10661_amd import workloads as W
    rng = np.random.default_rng(12)
    net = W.jittered_grid(32, rng)
    R = net.n_roads
    n = int(args.route_trips)
    price = rng.uniform(0, 120, R).astype(np.float32)
    og, dg = W.uniform_od(net, rng, n)
    ins = tsim._Inputs(net, tsim._NO_TRIPS, None)
    import ctypes as C
    lo, hint = C.c_size_t(0), C.c_size_t(0)
    tsim._check(tsim.lib().tsim_route_footprint(C.byref(ins.net), n, C.byref(lo), C.byref(hint)))
    ws = torch.empty(hint.value, dtype=torch.uint8, device="cuda")
    calls = args.steps or 5
    b, r, bad = tsim.shortest_routes(net, og, dg, price=price, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        b, r, bad = tsim.shortest_routes(net, og, dg, price=price, workspace=ws)
    dev_s = (time.perf_counter() - t0) / calls
    t0 = time.perf_counter()
    hb, hr, reach = W.shortest_routes(net, og, dg, road_price=price, workers=1)
    host_s = time.perf_counter() - t0
    # route costs (FP64 over the movement costs) of both: equal up to FP32 rounding
    G = W.movement_graph(net, price).tocsr()
    dc, hc = route_costs(G, b, r), route_costs(G, hb, hr)
    rel = np.abs(dc - hc) / np.maximum(hc, 1.0)
    step = max(1, n // 2000)
    same = np.mean([np.array_equal(r[b[c]:b[c + 1]], hr[hb[c]:hb[c + 1]]) for c in range(0, n, step)])
    out = {"workload": f"route_pricing_jittered32_{n}", "metric": "routes/s", "value": n / dev_s,
           "unit": "routes/s", "ms_per_call": dev_s * 1e3, "calls": calls, "pairs": n, "roads": R,
           "movements": int(G.nnz), "unreachable": bad, "mean_route_roads": float(b[-1]) / n,
           "host_scipy": {"value": n / host_s, "unit": "routes/s", "s": host_s, "cores": 1},
           "vs_host": host_s / dev_s, "cost_max_rel_diff_vs_host": float(rel.max(initial=0.0)),
           "identical_routes_vs_host_sampled": float(same)}
    if not args.no_cpu_baseline:
        # the oracle's FP32 Dijkstra on the trips of a bounded set of destinations
        from oracle import oracle as O
        O.build()
        z = np.zeros(0, np.float32)
        empty = W.Trips(depart_time=z, route_begin=np.zeros(1, np.int32), route_roads=np.zeros(0, np.int32),
                        v0_factor=z, length=z)
        osim = O.OracleSim(net, empty, W.Params())
        dsel = np.unique(dg)[:args.route_oracle_dests]
        idx = np.nonzero(np.isin(dg, dsel))[0]
        idx = idx[np.argsort(dg[idx], kind="stable")]
        t0 = time.perf_counter()
        osim.shortest_routes(og[idx], dg[idx], price)
        el = time.perf_counter() - t0
        osim.close()
        out["cpu_baseline"] = {"value": idx.size / el, "unit": "routes/s", "cores": 1, "kind": "oracle",
                               "sample": f"the {idx.size} trips to {dsel.size} destinations, {el:.1f} s"}
    if emit:
        print(json.dumps(out), flush=True)
    return out


def route_costs(G, begin, roads):
    """Cost of each route of a CSR (begin, roads): the sum of G[a, b] over
    its consecutive roads (a sparse movement-cost matrix)."""
    import numpy as np
    n = len(begin) - 1
    if len(roads) < 2:
        return np.zeros(n)
    k = np.arange(len(roads) - 1)
    seg = np.searchsorted(begin, k, side="right") - 1
    valid = (k + 1) < begin[seg + 1]
    w = np.asarray(G[roads[:-1][valid], roads[1:][valid]]).reshape(-1)
    return np.bincount(seg[valid], weights=w, minlength=n)


def summarize_window(path, steps, out=sys.stdout):
    """Reads a rocprofv3 CSV of a city run of this script (kernel trace, or
    counter collection of FETCH_SIZE / WRITE_SIZE) and prints, per step
    kernel, the averages over the timed window: the last 2 K dispatches of
    k_prepare and of the update are the timed pass (first K) and the
    profiling pass (last K), both from the same snapshot."""
    import csv
    from collections import defaultdict
    rows = list(csv.DictReader(open(path)))
    counters = "Counter_Name" in rows[0]
    disp = defaultdict(dict)   # kernel -> dispatch id -> [start, end, {counter: value}]
    for r in rows:
        k = r["Kernel_Name"]
        d = disp[k].setdefault(int(r["Dispatch_Id"]), [int(r["Start_Timestamp"]), int(r["End_Timestamp"]), {}])
        if counters:
            c = d[2]
            c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    step_kernels = [k for k in disp if "k_prepare" in k or "k_update_fused" in k]
    res = {}
    for k in sorted(step_kernels):
        ds = sorted(disp[k].values(), key=lambda d: d[0])
        if len(ds) < 2 * steps:
            raise SystemExit(f"{k}: {len(ds)} dispatches, fewer than 2 x {steps}")
        for name, part in (("timed", ds[-2 * steps:-steps]), ("profiling", ds[-steps:])):
            dur = sum(d[1] - d[0] for d in part) / steps / 1e3
            cs = {}
            for d in part:
                for c, v in d[2].items():
                    cs[c] = cs.get(c, 0.0) + v / steps
            res[(k, name)] = (dur, cs, part[0][0], part[-1][1])
    print("| Kernel | Pass | Dispatches | Average (us) | " + ("Counters per dispatch (KiB) |" if counters else "")
          , file=out)
    print("|---|---|---|---|" + ("---|" if counters else ""), file=out)
    for (k, name), (dur, cs, _, _) in res.items():
        cstr = ", ".join(f"{c} {v:.0f}" for c, v in sorted(cs.items()))
        print(f"| `{k}` | {name} | {steps} | {dur:.1f} |" + (f" {cstr} |" if counters else ""), file=out)
    for name in ("timed", "profiling"):
        st = [v for (k, n), v in res.items() if n == name]
        if st:
            span = (max(v[3] for v in st) - min(v[2] for v in st)) / steps / 1e3
            tot = sum(v[0] for v in st)
            print(f"\n{name} pass: kernels {tot:.1f} us per step, first start to last end {span:.1f} us per step",
                  file=out)
            if counters:
                tot_c = {}
                for v in st:
                    for c, x in v[1].items():
                        tot_c[c] = tot_c.get(c, 0.0) + x
                print(f"{name} pass counters per step (KiB, sum over the step's kernels): "
                      + ", ".join(f"{c} {x:.0f}" for c, x in sorted(tot_c.items())), file=out)
    return res


def traffic_report(pmc_dir, steps, window, copy_mib=1024, out=sys.stdout):
    """Writes the counter-traffic summary read by traffic_from_profiles from
    four rocprofv3 counter runs under pmc_dir: city_FETCH_SIZE/,
    city_WRITE_SIZE/ (city runs of this script over the window) and
    copy_FETCH_SIZE/, copy_WRITE_SIZE/ (--workload copy of copy_mib MiB,
    which calibrates KiB of each counter against bytes moved)."""
    import csv
    import glob

    def csv_of(sub):
        f = sorted(glob.glob(os.path.join(pmc_dir, sub, "*counter_collection.csv")))
        if not f:
            raise SystemExit(f"no counter CSV under {os.path.join(pmc_dir, sub)}")
        return f[0]

    n = copy_mib << 20
    factor = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        per = {}
        for r in csv.DictReader(open(csv_of(f"copy_{c}"))):
            if "copy" in r["Kernel_Name"].lower() and r["Counter_Name"] == c:
                per[int(r["Dispatch_Id"])] = per.get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
        if not per:
            raise SystemExit(f"copy_{c}: no copy kernel dispatches")
        kib = sum(per.values()) / len(per)
        factor[c] = (n, kib)
    res = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        import io
        res[c] = summarize_window(csv_of(f"city_{c}"), steps, out=io.StringIO())
    kernels = sorted({k for (k, p) in res["FETCH_SIZE"]})
    print(f"| Kernel | Dispatches | FETCH_SIZE (KiB, mean) | WRITE_SIZE (KiB, mean) |", file=out)
    print("|---|---|---|---|", file=out)
    per_step = {"FETCH_SIZE": 0.0, "WRITE_SIZE": 0.0}
    for k in kernels:
        f = res["FETCH_SIZE"][(k, "timed")][1].get("FETCH_SIZE", 0.0)
        w_ = res["WRITE_SIZE"][(k, "timed")][1].get("WRITE_SIZE", 0.0)
        print(f"| `{k}` | {steps} | {f:.0f} | {w_:.0f} |", file=out)
        per_step["FETCH_SIZE"] += f
        per_step["WRITE_SIZE"] += w_
    scale = {c: factor[c][0] / (factor[c][1] * 1024) for c in factor}
    rd = per_step["FETCH_SIZE"] * 1024 * scale["FETCH_SIZE"]
    wr = per_step["WRITE_SIZE"] * 1024 * scale["WRITE_SIZE"]
    print(f"\nCalibration (plain {copy_mib} MiB device copy): FETCH_SIZE {factor['FETCH_SIZE'][1]:.0f} KiB and "
          f"WRITE_SIZE {factor['WRITE_SIZE'][1]:.0f} KiB per copy, so bytes = FETCH_SIZE KiB x 1024 x "
          f"{scale['FETCH_SIZE']:.3f} and WRITE_SIZE KiB x 1024 x {scale['WRITE_SIZE']:.3f}.", file=out)
    print(f"\nPer step (timed pass, sum over the step's kernels): read {rd / 1e6:.1f} MB, written "
          f"{wr / 1e6:.1f} MB, {(rd + wr) / 1e6:.1f} MB in all.\n", file=out)
    print(f"kernel_hash: {kernel_source_hash()}", file=out)
    print(f"window: {window}", file=out)
    print(f"hbm_bytes_per_step: {rd + wr:.0f}", file=out)
    return rd + wr


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["city", "batch", "serve", "copy", "route"], default="city")
    ap.add_argument("--route-trips", type=int, default=150000, help="route: origin-destination pairs")
    ap.add_argument("--route-oracle-dests", type=int, default=40, help="route: destinations of the oracle sample")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--summarize", default=None, metavar="CSV",
                    help="print the timed window's per-kernel figures from a rocprofv3 CSV of a city run "
                         "(kernel trace or counter collection) made with the same --steps, then exit")
    ap.add_argument("--traffic-report", default=None, metavar="DIR",
                    help="print the counter-traffic summary from rocprofv3 counter runs under DIR "
                         "(city_FETCH_SIZE/, city_WRITE_SIZE/, copy_FETCH_SIZE/, copy_WRITE_SIZE/) made with the "
                         "same --steps and --from-step, then exit")
    ap.add_argument("--from-step", type=int, default=None,
                    help="city: first step of the timed window (default 5/8 of the horizon)")
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--gen-workers", type=int, default=None,
                    help="city: processes that generate the routes (default: up to 16; fewer keeps a "
                         "profiled run, whose children all hold the GPU, within the box's process limit)")
    ap.add_argument("--workload-file", default=None, metavar="NPZ",
                    help="city: load the generated workload from this file if it exists, else generate it "
                         "and save it there")
    ap.add_argument("--state-out", default=None, metavar="NPZ", help="city: save the state at --from-step")
    ap.add_argument("--state-in", default=None, metavar="NPZ",
                    help="city: start from a state saved by --state-out instead of stepping to --from-step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="city: skip the compact batched and served legs added to the line")
    ap.add_argument("--max-vehicles", type=int, default=None, help="serve: cap on a job's vehicles")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--jobs", type=int, default=400)
    ap.add_argument("--skip", type=int, default=50)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--no-saturate", action="store_true", help="serve: skip the all-at-once capacity run")
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--tick", type=int, default=30)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--graph-steps", type=int, default=60)
    ap.add_argument("--schedule", type=int, default=None, help="fixed update schedule (default: autotuned)")
    ap.add_argument("--concurrent", choices=["auto", "0", "1"], default="auto",
                    help="update passes of a step on side streams (1), serial (0), or autotuned with the schedule "
                         "(auto; on when the schedule is fixed; serving: off)")
    ap.add_argument("--serve-mode", choices=["batched", "streams"], default="batched")
    ap.add_argument("--max-batches", type=int, default=3)
    args = ap.parse_args()
    if args.traffic_report:
        fs = args.from_step if args.from_step is not None else 4500
        traffic_report(args.traffic_report, args.steps if args.steps is not None else 200,
                       f"from_step={fs} steps={args.steps if args.steps is not None else 200}", args.copy_mib)
        return
    if args.summarize:
        summarize_window(args.summarize, args.steps if args.steps is not None else 200)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the stepper has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        args.steps = args.steps or 1800
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "copy":
        return run_copy(args)
    if args.workload == "route":
        return run_route(args)
    return run_city(args)


def run_city(args):
    """The paper-scale city: K steps timed from the run's own loaded state."""
    from paper_2406_10661_amd import workloads as W
    from paper_2406_10661_amd.tsim import SCHEDULES
    t0 = time.time()
    if args.workload_file and os.path.exists(args.workload_file):
        w = W.load_workload(args.workload_file)
        log(f"[bench] loaded {args.workload_file}")
    else:
        w = W.CONFIGS[args.config](workers=args.gen_workers)
        if args.workload_file:
            W.save_workload(w, args.workload_file)
    log(f"[bench] workload {w.name}: {w.network.n_roads} roads, {w.network.n_lanes} lanes, "
        f"{w.trips.n_vehicles} vehicles, generated in {time.time() - t0:.1f} s")
    from_step = w.n_steps * 5 // 8 if args.from_step is None else args.from_step
    steps = args.steps if args.steps is not None else 200
    if from_step < 0 or steps < 1 or from_step + steps > w.n_steps:
        raise SystemExit(f"window [{from_step}, {from_step + steps}) outside the {w.n_steps}-step horizon")

    import numpy as np
    import torch
    from paper_2406_10661_amd.tsim import Sim
    sim = Sim(w.network, w.trips, w.params)
    stream = sim.stream   # the library's stream: every step kernel and graph launch goes there
    log(f"[bench] device arena {sim.arena.numel() / 2**30:.2f} GiB")
    # the loaded state: the run's own state at from_step, reached by stepping
    # from t = 0 outside the timed region (captured graphs unless disabled)
    if args.state_in:
        # a snapshot of the same run at from_step, written by --state-out
        # (lets counter-collection runs, which serialise every dispatch,
        # skip the thousands of steps that reach the loaded state)
        with np.load(args.state_in, allow_pickle=False) as z:
            st = {k: z[k] for k in z.files}
        st["step"] = int(st["step"])
        if st["step"] != from_step or st["status"].size != w.trips.n_vehicles:
            raise SystemExit(f"{args.state_in}: snapshot of step {st['step']} with {st['status'].size} vehicles, "
                             f"expected step {from_step} of {w.name}")
        sim.set_state(st)
        log(f"[bench] loaded the step-{from_step} snapshot {args.state_in}")
    else:
        if args.graph_steps:
            sim.set_graph_steps(args.graph_steps)
        done = 0
        while done < from_step:
            n = min(1000, from_step - done)
            sim.step(n)
            torch.cuda.synchronize()
            done += n
            log(f"[bench] reached step {done}")
        sim.set_graph_steps(0)
    snap = sim.get_state()
    if args.state_out:
        np.savez(args.state_out, **snap)
        log(f"[bench] wrote the step-{from_step} snapshot {args.state_out}")
    m_snap = sim.metrics()
    log(f"[bench] state at step {snap['step']}: {m_snap['n_active']} active, {m_snap['n_finished']} finished, "
        f"{m_snap['n_waiting']} waiting")
    # schedule and pass concurrency: autotuned on this state (the autotuner's
    # steps are real; the state is restored afterwards)
    if args.schedule is None:
        sched, conc, us = tune(sim, 10, concurrency_arg(args))
        log(f"[bench] autotuned schedule {sched} ({SCHEDULES[sched]}), concurrent passes {conc}; us/step by "
            f"schedule {[[round(float(x), 1) for x in row] for row in us] if us.ndim == 2 else [round(float(x), 1) for x in us]}")
    else:
        sched = args.schedule
        conc = concurrency_arg(args)
        conc = False if conc is None else conc
        sim.set_schedule(sched)
        sim.set_concurrency(conc)
        log(f"[bench] fixed schedule {sched} ({SCHEDULES[sched]}), concurrent passes {conc}")
    if args.warmup:
        sim.set_state(snap)
        sim.step(args.warmup)
        torch.cuda.synchronize()
    sim.set_state(snap)

    # timed pass: K steps from the snapshot, replayed from captured HIP graphs
    # of `chunk` steps (the remainder of K launched directly)
    chunk = min(args.graph_steps, steps) if args.graph_steps else 0
    if chunk:
        sim.set_graph_steps(chunk)
        sim.step(0)                     # capture outside the timed region
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    m0 = sim.metrics()
    w0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    m1 = sim.metrics()
    d = {k: m1[k] - m0[k] for k in ("vehicle_steps", "lane_steps", "road_entries", "lane_changes", "transfers",
                                     "n_finished", "departures")}
    vsteps = d["vehicle_steps"]
    secs = ms / 1e3
    log(f"[bench] steps {from_step}..{from_step + steps}: {ms:.2f} ms (wall {wall:.3f} s), vehicle-steps {vsteps} "
        f"({vsteps / steps:.0f} active per step), non-empty lane-steps {d['lane_steps']}, road entries "
        f"{d['road_entries']}, finished {d['n_finished']}, errors {m1['errors']}")

    # kernel timing pass (events around every launch) over the same window
    sim.set_graph_steps(0)
    sim.set_state(snap)
    sim.set_profiling(True)
    sim.step(steps)
    kt = sim.kernel_times()
    sim.set_profiling(False)
    upd_ms, upd_n = kt["update"]
    prep_ms, prep_n = kt["prepare"]
    alg_bytes = BYTES_PER_ACTIVE * vsteps + BYTES_PER_LANE * d["lane_steps"] + BYTES_PER_ROAD_ENTRY * d["road_entries"]
    window = f"from_step={from_step} steps={steps}"
    rl = roofline(alg_bytes, ms, steps, traffic_from_profiles(w.name, window), step_label(SCHEDULES[sched]))
    log(f"[bench] eager launches with events: update {upd_ms / max(upd_n, 1) * 1e3:.1f} us/step, prepare "
        f"{prep_ms / max(prep_n, 1) * 1e3:.1f} us/step; timed steps {ms / steps * 1e3:.1f} us, "
        f"algorithmic {alg_bytes / steps / 1e6:.1f} MB/step, achieved {rl['achieved']:.1f} GB/s")

    out = {
        "metric": METRIC,
        "value": vsteps / secs,
        "unit": "vehicle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "sim_hz": steps / secs,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "junctions": w.network.n_junctions, "roads": w.network.n_roads,
                   "lanes": w.network.n_lanes, "vehicles": w.trips.n_vehicles, "dt_s": w.params.dt,
                   "horizon_steps": w.n_steps, "timed_from_step": from_step,
                   "active_at_start": m_snap["n_active"], "mean_active_per_step": vsteps / steps,
                   "schedule": SCHEDULES[sched], "concurrent_passes": bool(conc), "graph_steps": chunk},
        "window": {"vehicle_steps": vsteps, "nonempty_lane_steps": d["lane_steps"],
                   "road_entries": d["road_entries"], "finished": d["n_finished"], "departures": d["departures"],
                   "lane_changes": d["lane_changes"], "transfers": d["transfers"],
                   "mean_road_speed": m1["mean_speed_avg"], "errors": m1["errors"],
                   "max_stalled_steps": m1["max_stalled_steps"]},
        "roofline": rl,
        "eager_us_per_step": {"update": upd_ms / max(upd_n, 1) * 1e3, "prepare": prep_ms / max(prep_n, 1) * 1e3},
        "paper_context": {"hz": 84.09, "vehicles": 2464950, "hardware": "RTX 4090 + Xeon Platinum 8462Y",
                          "note": "whole 3,600-step run of the paper's own city data; not the same workload"},
    }
    del sim
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, from_step, args.cpu_seconds)
    if not args.no_legs:
        out.update(compact_legs(args))
    print(json.dumps(out), flush=True)


def compact_legs(args):
    """The batched and served forms at a compact size, timed in the same
    run: 64 uneven jittered-grid instances (3.8M vehicles) stepped together
    for 300 steps with phases set every 15 steps, against the same instances
    stepped one by one; and 100 served jobs (at most 100,000 vehicles each,
    Poisson 20 jobs/s, statistics after the first 10) through the
    continuous-batching loop, against the one-job-at-a-time loop; and the
    device routes of a served pricing job at its largest (150,000 trips on a
    32x32 jittered grid) against the host routing."""
    import copy
    b = copy.copy(args)
    b.instances, b.steps, b.concurrent = 64, 300, "0"
    rb = run_batch(b, emit=False)
    v = copy.copy(args)
    v.jobs, v.skip, v.rate, v.budget_gib, v.tick, v.streams = 100, 10, 20.0, 16.0, 30, 3
    v.max_batches, v.serve_mode, v.no_saturate, v.max_vehicles, v.concurrent = 3, "batched", False, 100000, "0"
    rs = run_serve(v, emit=False)
    batched = {k: rb[k] for k in ("value", "unit", "steps", "ms_per_step", "vs_plain_loop", "plain_loop")}
    batched["config"] = rb["config"]
    batched["roofline_frac"] = rb["roofline"]["frac"]
    served = {k: rs[k] for k in ("value", "unit", "latency_p50_s", "latency_p99_s", "queue_wait_p99_s",
                                 "vehicle_steps_per_s", "vs_plain_loop", "plain_loop", "utilisation")
              if k in rs}
    served["config"] = rs["config"]
    if "saturated" in rs:
        served["saturated"] = rs["saturated"]
    r = copy.copy(args)
    r.steps, r.route_trips = 5, 150000
    routing = run_route(r, emit=False)
    return {"batched": batched, "served": served, "routing": routing}


if __name__ == "__main__":
    main()
