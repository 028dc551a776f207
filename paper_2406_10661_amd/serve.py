"""Continuous-batching request loop over resident simulation jobs.

Jobs (a network, a trip table, parameters and a horizon) arrive over time.
Each arriving job is admitted when its device footprint (``tsim_footprint``)
fits the free part of an HBM budget; until then it waits in FIFO order.  An
admitted job is built and uploaded once by a preparation thread (its state
stays resident in HBM until it finishes), then joins the set of running jobs
at the next tick.  Every tick enqueues the next few steps of every running job
(at most two chunks ahead of the device), each job on one stream of a pool, so
the kernels of different jobs overlap on the device.  A job leaves once its
horizon is reached on the device; its metrics are read, its memory is
released, and its latency (result delivered minus arrival) is recorded.

The loop only sees a stepper factory with ``footprint``, ``create`` (returning
an object with ``step(n)``, ``metrics()`` and ``close()``, and a stream),
``done_event`` (an object with ``query()``) and ``sync``; the default factory
uses the HIP library through ``paper_2406_10661_amd.tsim``.
"""

from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field


@dataclass
class Job:
    jid: int
    arrival: float          # seconds after the loop starts
    network: object
    trips: object
    params: object
    horizon: int            # steps to simulate
    footprint: int = 0
    # filled by the loop
    admitted: float = -1.0
    started: float = -1.0
    finished: float = -1.0
    steps_done: int = 0
    metrics: dict = field(default_factory=dict)
    sim: object = None
    stream: object = None
    inflight: object = None


class GpuFactory:
    """Resident jobs as tsim handles on a pool of default-priority streams."""

    def __init__(self, n_streams=4, device="cuda:0", graph_steps=0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.graph_steps = int(graph_steps)
        self._next = 0
        self._lock = threading.Lock()

    def footprint(self, job):
        from paper_2406_10661_amd.tsim import footprint
        return footprint(job.network, job.trips, job.params)

    def create(self, job):
        from paper_2406_10661_amd.tsim import Sim
        with self._lock:
            s = self.streams[self._next % len(self.streams)]
            self._next += 1
        with self.torch.cuda.stream(s):
            sim = Sim(job.network, job.trips, job.params, device=self.device, stream=s)
            if self.graph_steps:
                sim.set_graph_steps(self.graph_steps)
        return sim, s

    def done_event(self, stream):
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def sync(self):
        self.torch.cuda.synchronize(self.device)


class ServeLoop:
    """hbm_budget: bytes of device memory the resident jobs may hold together;
    steps_per_tick: steps enqueued per job per tick; depth: ticks a job may
    have in flight on its stream before the loop waits for it; builders:
    preparation threads (table building and upload run outside the GIL)."""

    def __init__(self, factory, hbm_budget, steps_per_tick=30, depth=2, builders=4, clock=time.perf_counter):
        self.f = factory
        self.budget = int(hbm_budget)
        self.k = int(steps_per_tick)
        self.depth = int(depth)
        self.n_builders = int(builders)
        self.clock = clock

    def run(self, jobs):
        """Runs every job to completion; returns per-job records and totals."""
        jobs = sorted(jobs, key=lambda j: j.arrival)
        for j in jobs:
            j.footprint = self.f.footprint(j)
            if j.footprint > self.budget:
                raise ValueError(f"job {j.jid} needs {j.footprint} bytes, more than the whole budget")
        t0 = self.clock()
        now = lambda: self.clock() - t0
        waiting = collections.deque(jobs)        # not yet admitted (arrived or not)
        ready = collections.deque()              # built, waiting for the next tick
        running = []
        used = 0
        peak_used = 0
        lock = threading.Lock()
        build_q = collections.deque()
        build_cv = threading.Condition(lock)
        stop = [False]
        errors = []

        def builder():
            while True:
                with build_cv:
                    while not build_q and not stop[0]:
                        build_cv.wait(0.05)
                    if stop[0] and not build_q:
                        return
                    job = build_q.popleft()
                try:
                    job.sim, job.stream = self.f.create(job)
                except Exception as e:  # surfaced by the main loop
                    errors.append(e)
                    return
                with lock:
                    ready.append(job)

        threads = [threading.Thread(target=builder, daemon=True) for _ in range(self.n_builders)]
        for th in threads:
            th.start()
        done = []
        ticks = 0
        try:
            while len(done) < len(jobs):
                if errors:
                    raise errors[0]
                tnow = now()
                # admission: FIFO, by footprint against the free budget
                with lock:
                    while waiting and waiting[0].arrival <= tnow and used + waiting[0].footprint <= self.budget:
                        job = waiting.popleft()
                        used += job.footprint
                        peak_used = max(peak_used, used)
                        job.admitted = tnow
                        build_q.append(job)
                        build_cv.notify()
                    while ready:
                        job = ready.popleft()
                        job.started = now()
                        job.inflight = collections.deque()
                        running.append(job)
                # advance every running job by its next chunk, at most `depth` chunks ahead
                enqueued = 0
                still = []
                for job in running:
                    while job.inflight and job.inflight[0].query():
                        job.inflight.popleft()
                    if job.steps_done < job.horizon and len(job.inflight) < self.depth:
                        n = min(self.k, job.horizon - job.steps_done)
                        job.sim.step(n)
                        job.steps_done += n
                        job.inflight.append(self.f.done_event(job.stream))
                        enqueued += 1
                    if job.steps_done >= job.horizon and not job.inflight:
                        # result delivered: read metrics, release the memory
                        job.metrics = job.sim.metrics()
                        job.finished = now()
                        job.sim.close()
                        job.sim = None
                        with lock:
                            used -= job.footprint
                        done.append(job)
                    else:
                        still.append(job)
                running = still
                ticks += 1
                if not enqueued:
                    time.sleep(0.0002)
        finally:
            with build_cv:
                stop[0] = True
                build_cv.notify_all()
            for th in threads:
                th.join(timeout=60)
        self.f.sync()
        wall = now()
        return {"jobs": done, "wall_s": wall, "ticks": ticks, "peak_bytes": peak_used}


class BatchFactory:
    """Jobs grouped into batches (``tsim_batch_*``: one set of launches steps
    every instance of a batch), each batch on one stream of a pool; each
    instance is frozen at its own horizon.  ``concurrent`` runs each batch's
    update passes on side streams (``tsim_set_concurrency``)."""

    def __init__(self, n_streams=3, device="cuda:0", graph_steps=30, concurrent=False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.graph_steps = int(graph_steps)
        self.concurrent = bool(concurrent)
        self._next = 0
        self._lock = threading.Lock()

    def footprint(self, job):
        from paper_2406_10661_amd.tsim import footprint
        return footprint(job.network, job.trips, job.params)

    def create_batch(self, jobs):
        from paper_2406_10661_amd.tsim import Batch
        with self._lock:
            s = self.streams[self._next % len(self.streams)]
            self._next += 1
        with self.torch.cuda.stream(s):
            b = Batch([j.network for j in jobs], [j.trips for j in jobs], [j.params for j in jobs],
                      device=self.device, stream=s)
            for k, j in enumerate(jobs):
                b.set_horizon(k, j.horizon)
            if self.concurrent:
                b.set_concurrency(True)
            if self.graph_steps:
                b.set_graph_steps(self.graph_steps)
        return b, s

    def done_event(self, stream):
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def sync(self):
        self.torch.cuda.synchronize(self.device)


class BatchedServeLoop:
    """Continuous batching over batches of jobs: admitted jobs that are not
    yet running are gathered into a new batch whenever fewer than
    ``max_batches`` batches are running or being built; each batch is stepped
    in chunks of ``steps_per_tick`` steps (at most ``depth`` chunks ahead of
    the device) until its longest job's horizon, and each job's result is
    read as soon as the device has passed that job's own horizon.  A job's
    memory stays counted against the budget until its batch is released."""

    def __init__(self, factory, hbm_budget, steps_per_tick=30, depth=2, max_batches=3, max_jobs_per_batch=64,
                 builders=2, clock=time.perf_counter):
        self.f = factory
        self.budget = int(hbm_budget)
        self.k = int(steps_per_tick)
        self.depth = int(depth)
        self.max_batches = int(max_batches)
        self.max_jobs = int(max_jobs_per_batch)
        self.n_builders = int(builders)
        self.clock = clock

    def run(self, jobs):
        jobs = sorted(jobs, key=lambda j: j.arrival)
        for j in jobs:
            j.footprint = self.f.footprint(j)
            if j.footprint > self.budget:
                raise ValueError(f"job {j.jid} needs {j.footprint} bytes, more than the whole budget")
        t0 = self.clock()
        now = lambda: self.clock() - t0
        waiting = collections.deque(jobs)
        admitted = collections.deque()
        lock = threading.Lock()
        build_q = collections.deque()
        build_cv = threading.Condition(lock)
        ready = collections.deque()
        stop = [False]
        errors = []
        state = {"used": 0, "peak": 0, "building": 0}

        def builder():
            while True:
                with build_cv:
                    while not build_q and not stop[0]:
                        build_cv.wait(0.05)
                    if stop[0] and not build_q:
                        return
                    grp = build_q.popleft()
                try:
                    b, st = self.f.create_batch(grp)
                except Exception as e:
                    errors.append(e)
                    return
                with lock:
                    ready.append({"batch": b, "stream": st, "jobs": grp, "steps": 0, "inflight": collections.deque(),
                                  "done_steps": 0, "horizon": max(j.horizon for j in grp)})

        threads = [threading.Thread(target=builder, daemon=True) for _ in range(self.n_builders)]
        for th in threads:
            th.start()
        running = []
        done = []
        n_batches = 0
        try:
            while len(done) < len(jobs):
                if errors:
                    raise errors[0]
                tnow = now()
                with lock:
                    while waiting and waiting[0].arrival <= tnow and state["used"] + waiting[0].footprint <= self.budget:
                        j = waiting.popleft()
                        state["used"] += j.footprint
                        state["peak"] = max(state["peak"], state["used"])
                        j.admitted = tnow
                        admitted.append(j)
                    if admitted and len(running) + state["building"] < self.max_batches:
                        grp = [admitted.popleft() for _ in range(min(self.max_jobs, len(admitted)))]
                        state["building"] += 1
                        build_q.append(grp)
                        build_cv.notify()
                    while ready:
                        rb = ready.popleft()
                        state["building"] -= 1
                        n_batches += 1
                        tst = now()
                        for j in rb["jobs"]:
                            j.started = tst
                        running.append(rb)
                enqueued = 0
                still = []
                for rb in running:
                    # chunks the device has finished
                    while rb["inflight"] and rb["inflight"][0][0].query():
                        rb["done_steps"] = rb["inflight"].popleft()[1]
                    for j in rb["jobs"]:
                        if j.finished < 0 and j.horizon <= rb["done_steps"]:
                            k = rb["jobs"].index(j)
                            j.metrics = rb["batch"].metrics(k)
                            j.steps_done = j.horizon
                            j.finished = now()
                            done.append(j)
                    if rb["steps"] < rb["horizon"] and len(rb["inflight"]) < self.depth:
                        n = min(self.k, rb["horizon"] - rb["steps"])
                        rb["batch"].step(n)
                        rb["steps"] += n
                        rb["inflight"].append((self.f.done_event(rb["stream"]), rb["steps"]))
                        enqueued += 1
                    if rb["done_steps"] >= rb["horizon"] and all(j.finished >= 0 for j in rb["jobs"]):
                        rb["batch"].close()
                        rb["batch"] = None
                        with lock:
                            state["used"] -= sum(j.footprint for j in rb["jobs"])
                    else:
                        still.append(rb)
                running = still
                if not enqueued:
                    time.sleep(0.0002)
        finally:
            with build_cv:
                stop[0] = True
                build_cv.notify_all()
            for th in threads:
                th.join(timeout=60)
        self.f.sync()
        return {"jobs": done, "wall_s": now(), "batches": n_batches, "peak_bytes": state["peak"]}


def summarize(result, skip=0):
    """p50/p99 latency, jobs/s and vehicle-steps/s over the jobs after the
    first `skip` (by arrival)."""
    import numpy as np
    jobs = sorted(result["jobs"], key=lambda j: j.arrival)
    sel = jobs[skip:] if len(jobs) > skip else jobs
    lat = np.array([j.finished - j.arrival for j in sel])
    queue = np.array([j.admitted - j.arrival for j in sel])
    first = min(j.arrival for j in sel)
    last = max(j.finished for j in sel)
    vsteps = sum(int(j.metrics.get("vehicle_steps", 0)) for j in sel)
    span = max(last - first, 1e-9)
    return {
        "jobs": len(sel),
        "jobs_per_s": len(sel) / span,
        "vehicle_steps_per_s": vsteps / span,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "queue_wait_p50_s": float(np.percentile(queue, 50)),
        "queue_wait_p99_s": float(np.percentile(queue, 99)),
        "wall_s": result["wall_s"],
    }
