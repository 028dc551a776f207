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
