"""Served jobs on the GPU: each job's result is the same whether it runs alone
or in the continuous-batching mix (other jobs resident and stepping on the
same streams, admission bound by an HBM budget, captured-graph chunks)."""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("step", "n_finished", "n_active", "n_waiting", "vehicle_steps", "lane_changes", "transfers",
        "departures", "feeder_blocks", "clamps", "errors", "sum_travel_time", "mean_speed_avg",
        "mean_speed_last")


def test_served_jobs_match_alone():
    from paper_2406_10661_amd import serve as SV
    from paper_2406_10661_amd.tsim import Sim
    ws = W.served_jobs(8, workers=4, max_vehicles=12000)
    horizons = [min(w.n_steps, 300 + 37 * k) for k, w in enumerate(ws)]
    jobs = [SV.Job(jid=k, arrival=0.002 * k, network=w.network, trips=w.trips, params=w.params,
                   horizon=horizons[k]) for k, w in enumerate(ws)]
    fac = SV.GpuFactory(n_streams=4, graph_steps=30)
    fps = [fac.footprint(j) for j in jobs]
    budget = 3 * max(fps)                      # admission binds: at most ~3 resident at once
    res = SV.ServeLoop(fac, hbm_budget=budget, steps_per_tick=30).run(jobs)
    assert res["peak_bytes"] <= budget
    assert len(res["jobs"]) == len(jobs)
    for j in res["jobs"]:
        w = ws[j.jid]
        sim = Sim(w.network, w.trips, w.params)
        sim.step(j.horizon)
        m = sim.metrics()
        sim.close()
        for k in KEYS:
            assert m[k] == j.metrics[k], (j.jid, k, m[k], j.metrics[k])
        assert m["step"] == j.horizon
    s = SV.summarize(res)
    print("served", s, flush=True)
    assert s["latency_p99_s"] >= s["latency_p50_s"] > 0


def test_batched_serving_jobs_match_alone():
    """The continuous-batching serve loop (jobs joining resident batches
    while others run, each frozen at its own horizon and removed) gives every
    job the same metrics as running it alone."""
    from paper_2406_10661_amd import serve as SV
    from paper_2406_10661_amd.tsim import Sim
    ws = W.served_jobs(10, workers=4, max_vehicles=12000)
    horizons = [min(w.n_steps, 200 + 41 * k) for k, w in enumerate(ws)]
    jobs = [SV.Job(jid=k, arrival=0.003 * k, network=w.network, trips=w.trips, params=w.params,
                   horizon=horizons[k]) for k, w in enumerate(ws)]
    fac = SV.BatchFactory(n_streams=2, graph_steps=30)
    budget = 4 * max(fac.footprint(j) for j in jobs)
    res = SV.BatchedServeLoop(fac, hbm_budget=budget, steps_per_tick=30, max_batches=2).run(jobs)
    assert len(res["jobs"]) == len(jobs) and res["batches"] == 2
    assert sum(1 for j in res["jobs"] if j.g0 > 0) >= 3      # joined a batch that was already running
    for j in res["jobs"]:
        w = ws[j.jid]
        sim = Sim(w.network, w.trips, w.params)
        sim.step(j.horizon)
        m = sim.metrics()
        sim.close()
        for k in KEYS:
            assert m[k] == j.metrics[k], (j.jid, k, m[k], j.metrics[k])
    print("batched served", SV.summarize(res), res["batches"], flush=True)


def test_served_jobs_routed_on_the_gpu():
    """Served jobs whose trips arrive without routes are routed on the GPU
    (Section 4 congestion pricing: least cost under the job's road prices;
    free-flow time for a timing-plan job): every route joins its trip's
    origin and destination through movements, costs as little as the
    host's Dijkstra route up to FP32 rounding, and equals the oracle's route
    (bit for bit) on a sample; the routed jobs then run in the batched
    serving loop with the results they have alone."""
    from oracle import oracle as O
    from paper_2406_10661_amd import serve as SV
    from paper_2406_10661_amd.tsim import Sim
    from tests.scenes import empty_trips
    O.build()
    ids = [0, 1, 2, 3, 5, 8]
    dev = [W.config5_job(j, max_vehicles=8000, route=False) for j in ids]
    host = [W.config5_job(j, max_vehicles=8000) for j in ids]
    assert {w.extra["kind"] for w in dev} == {"pricing", "timing_plan"}
    SV.route_jobs_on_device(dev)
    rng = np.random.default_rng(2)
    for w, h in zip(dev, host):
        o, d = w.extra["od"]
        b, r = w.trips.route_begin, w.trips.route_roads
        assert np.array_equal(r[b[:-1]], o) and np.array_equal(r[b[1:] - 1], d)
        price = w.extra["price"]
        G = W.movement_graph(w.network, None if price is None else np.asarray(price, np.float32)).tocsr()
        def cost(begin, roads):
            out = np.zeros(len(begin) - 1)
            for c in range(len(begin) - 1):
                x = roads[begin[c]:begin[c + 1]]
                ws = [G[x[k], x[k + 1]] for k in range(len(x) - 1)]
                assert all(v > 0 for v in ws)
                out[c] = sum(ws)
            return out
        sel = rng.choice(len(o), 300, replace=False)
        sb = np.concatenate([[0], np.cumsum(np.diff(b)[sel])])
        sr = np.concatenate([r[b[c]:b[c + 1]] for c in sel])
        hb, hr = h.trips.route_begin, h.trips.route_roads
        hsb = np.concatenate([[0], np.cumsum(np.diff(hb)[sel])])
        hsr = np.concatenate([hr[hb[c]:hb[c + 1]] for c in sel])
        dc, hc = cost(sb, sr), cost(hsb, hsr)
        assert np.all(np.abs(dc - hc) <= 2e-5 * np.maximum(hc, 1.0)), w.name
        # the oracle's FP32 routes for the trips of two destinations
        dsel = np.unique(d)[:2]
        k = np.nonzero(np.isin(d, dsel))[0]
        k = k[np.argsort(d[k], kind="stable")]
        osim = O.OracleSim(w.network, empty_trips(), w.params)
        ob, orr, _ = osim.shortest_routes(o[k], d[k], None if price is None else np.asarray(price, np.float32))
        osim.close()
        for c, i in enumerate(k):
            assert np.array_equal(orr[ob[c]:ob[c + 1]], r[b[i]:b[i + 1]]), (w.name, int(i))
    jobs = [SV.Job(jid=c, arrival=0.0, network=w.network, trips=w.trips, params=w.params,
                   horizon=min(w.n_steps, 400)) for c, w in enumerate(dev)]
    fac = SV.BatchFactory(n_streams=2, graph_steps=30)
    res = SV.BatchedServeLoop(fac, hbm_budget=2 << 30, steps_per_tick=30, max_batches=2).run(jobs)
    for j in res["jobs"]:
        w = dev[j.jid]
        sim = Sim(w.network, w.trips, w.params)
        sim.step(j.horizon)
        m = sim.metrics()
        sim.close()
        for key in KEYS:
            assert m[key] == j.metrics[key], (j.jid, key)


def test_served_job_whole_horizon_schedules_and_batch_identical():
    """One served job (57k vehicles, routed on the GPU, roads of up to ~190
    vehicles) over its whole horizon: every update schedule, and the job as
    the only instance of a batch, give the same trajectory bit for bit.
    Long horizons are where a rare ordering difference between the passes
    of a schedule would show."""
    from paper_2406_10661_amd import serve as SV
    from paper_2406_10661_amd.tsim import SCHEDULES, Batch, Sim
    ws = [W.config5_job(3, max_vehicles=100000, route=False)]
    SV.route_jobs_on_device(ws)
    w = ws[0]
    ref = None
    for sc in sorted(SCHEDULES):
        g = Sim(w.network, w.trips, w.params)
        g.set_schedule(sc)
        g.step(w.n_steps)
        s, m = g.get_state(), g.metrics()
        g.close()
        assert m["errors"] == 0
        if ref is None:
            ref = (s, m)
            continue
        for key in ("status", "lane", "route_pos", "x", "v", "finish_step"):
            assert np.array_equal(s[key], ref[0][key]), (sc, key)
        for key in KEYS:
            assert m[key] == ref[1][key], (sc, key, m[key], ref[1][key])
    b = Batch([w.network], [w.trips], [w.params])
    b.step(w.n_steps)
    s, m = b.get_state(0), b.metrics(0)
    b.close()
    for key in ("status", "lane", "route_pos", "x", "v", "finish_step"):
        assert np.array_equal(s[key], ref[0][key]), ("batch", key)
    for key in KEYS:
        assert m[key] == ref[1][key], ("batch", key, m[key], ref[1][key])
    print("served job 3:", w.trips.n_vehicles, "vehicles,", w.n_steps, "steps, finished", ref[1]["n_finished"],
          flush=True)
