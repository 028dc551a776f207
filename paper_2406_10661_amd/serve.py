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
    """Resident batches reserved once (``tsim_batch_reserve``), each on one
    stream of a pool; jobs are laid out on the host (``tsim_instance_build``,
    no GPU work, so builder threads can do it) and join a running batch at
    its next step boundary (``tsim_batch_add``).  ``concurrent`` runs each
    batch's update passes on side streams (``tsim_set_concurrency``)."""

    def __init__(self, n_streams=3, device="cuda:0", graph_steps=30, concurrent=False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.graph_steps = int(graph_steps)
        self.concurrent = bool(concurrent)
        self._next = 0

    def footprint(self, job):
        from paper_2406_10661_amd.tsim import footprint
        return footprint(job.network, job.trips, job.params)

    def instance(self, job):
        from paper_2406_10661_amd.tsim import Instance
        return Instance(job.network, job.trips, job.params)

    def capacity_of(self, job):
        inst = self.instance(job)
        cap = inst.capacity()
        inst.close()
        return cap

    def reserve_footprint(self, cap):
        from paper_2406_10661_amd.tsim import reserve_footprint
        return reserve_footprint(cap)

    def reserve(self, cap, params):
        from paper_2406_10661_amd.tsim import Batch
        s = self.streams[self._next % len(self.streams)]
        self._next += 1
        with self.torch.cuda.stream(s):
            b = Batch.reserve(cap, params, device=self.device, stream=s)
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


CAP_KEYS = ("instances", "junctions", "roads", "road_lanes", "jlanes", "phases", "vehicles", "route_entries", "slots")


def fits(need, left):
    return all(need[k] <= left[k] for k in CAP_KEYS)


def batch_capacity(caps, budget_bytes, reserve_footprint):
    """Totals of one batch sized to a byte budget: every dimension scaled from
    the largest per-vehicle ratio among the given job capacities, plus room
    for the largest single job, so that any of the jobs fits an empty batch."""
    ratio = {k: max(c[k] / max(c["vehicles"], 1) for c in caps) for k in CAP_KEYS}
    big = {k: max(c[k] for c in caps) for k in CAP_KEYS}

    def cap_for(v):
        return {k: int(big[k] + ratio[k] * v) + (1 if k == "instances" else 0) for k in CAP_KEYS}

    def ok(v):
        try:
            return reserve_footprint(cap_for(v)) <= budget_bytes
        except Exception:       # past the library's limits
            return False

    if not ok(0):
        raise ValueError("the HBM share of a batch cannot hold the largest job")
    lo, hi = 0, 1
    while ok(hi):
        lo, hi = hi, 2 * hi
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return cap_for(lo)


class BatchedServeLoop:
    """Continuous batching: ``max_batches`` resident batches share the HBM
    budget, each reserved once (``batch_capacity``).  An arriving job is laid
    out on the host by a builder thread; it then joins the first running
    batch with room for it (arrival order, first fit) at that batch's next
    step boundary, with its horizon set, so requests that arrive while others
    are on the GPU join them.  Each batch is stepped in chunks of
    ``steps_per_tick`` steps (at most ``depth`` chunks ahead of the device);
    when a job's horizon has passed on the device, or a waiting job fits, the
    batch stops taking new chunks until the device has caught up, then the
    finished jobs' results are read and the jobs removed
    (``tsim_batch_remove``), and waiting jobs are added."""

    def __init__(self, factory, hbm_budget, steps_per_tick=30, depth=2, max_batches=3, builders=2,
                 capacity=None, clock=time.perf_counter, max_jobs_per_batch=None):
        self.f = factory
        self.budget = int(hbm_budget)
        self.k = int(steps_per_tick)
        self.depth = int(depth)
        self.max_batches = int(max_batches)
        self.n_builders = int(builders)
        self.capacity = capacity
        self.clock = clock

    def run(self, jobs):
        jobs = sorted(jobs, key=lambda j: j.arrival)
        if not jobs:
            return {"jobs": [], "wall_s": 0.0, "batches": 0, "peak_bytes": 0}
        # batch sizing from the jobs' shapes (host work, before the clock starts)
        insts = {}
        for j in jobs:
            j.footprint = self.f.footprint(j)
        cap = self.capacity
        if cap is None:
            sample = [self.f.capacity_of(j) for j in jobs]
            cap = batch_capacity(sample, self.budget // self.max_batches, self.f.reserve_footprint)
        batches = []
        for _ in range(self.max_batches):
            b, st = self.f.reserve(cap, jobs[0].params)
            batches.append({"batch": b, "stream": st, "jobs": {}, "inflight": collections.deque(), "steps": 0,
                            "done": 0})
        reserved = sum(self.f.reserve_footprint(cap) for _ in batches)
        t0 = self.clock()
        now = lambda: self.clock() - t0
        waiting = collections.deque(jobs)     # not yet arrived
        lock = threading.Lock()
        build_q = collections.deque()
        build_cv = threading.Condition(lock)
        ready = []                            # built, waiting for room (arrival order)
        stop = [False]
        errors = []

        def builder():
            while True:
                with build_cv:
                    while not build_q and not stop[0]:
                        build_cv.wait(0.05)
                    if stop[0] and not build_q:
                        return
                    j = build_q.popleft()
                try:
                    inst = self.f.instance(j)
                    need = inst.capacity()
                except Exception as e:  # surfaced by the main loop
                    errors.append(e)
                    return
                with lock:
                    insts[j.jid] = (inst, need)
                    ready.append(j)
                    ready.sort(key=lambda x: x.arrival)

        threads = [threading.Thread(target=builder, daemon=True) for _ in range(self.n_builders)]
        for th in threads:
            th.start()
        done = []
        try:
            while len(done) < len(jobs):
                if errors:
                    raise errors[0]
                tnow = now()
                with lock:
                    while waiting and waiting[0].arrival <= tnow:
                        build_q.append(waiting.popleft())
                        build_cv.notify()
                    cand = list(ready)
                enqueued = 0
                for rb in batches:
                    b = rb["batch"]
                    while rb["inflight"] and rb["inflight"][0][0].query():
                        rb["done"] = rb["inflight"].popleft()[1]
                    fin = [(k, j) for k, j in rb["jobs"].items() if j.g0 + j.horizon <= rb["done"]]
                    left = b.capacity_left() if cand else None
                    joining = [j for j in cand if fits(insts[j.jid][1], left)] if cand else []
                    if (fin or joining) and not rb["inflight"]:
                        # step boundary on the device: deliver, remove, add
                        for k, j in sorted(fin, reverse=True):
                            j.metrics = b.metrics(k)
                            j.steps_done = j.horizon
                            j.finished = now()
                            done.append(j)
                            del rb["jobs"][k]
                            b.remove(k)
                        left = b.capacity_left()
                        for j in cand:
                            if j.jid not in insts or not fits(insts[j.jid][1], left):
                                continue
                            inst = insts[j.jid][0]
                            k = b.add(inst)
                            b.set_horizon(k, j.horizon)
                            j.k, j.g0 = k, rb["steps"]
                            j.admitted = j.started = now()
                            rb["jobs"][k] = j
                            with lock:
                                ready.remove(j)
                                del insts[j.jid]
                            inst.close()
                            left = b.capacity_left()
                        cand = [j for j in cand if j.jid in insts]
                        continue
                    if fin or joining:
                        continue   # let the device reach the step boundary first
                    active = [j.g0 + j.horizon - rb["steps"] for j in rb["jobs"].values()]
                    todo = max(active, default=0)
                    if todo > 0 and len(rb["inflight"]) < self.depth:
                        n = min(self.k, todo)
                        b.step(n)
                        rb["steps"] += n
                        rb["inflight"].append((self.f.done_event(rb["stream"]), rb["steps"]))
                        enqueued += 1
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
        for rb in batches:
            rb["batch"].close()
        return {"jobs": done, "wall_s": wall, "batches": len(batches), "peak_bytes": reserved, "capacity": cap}


def route_jobs_on_device(workloads, device="cuda:0"):
    """Routes, on the GPU, every job whose trips arrive without routes: the
    least-cost route of each trip from its origin road to its destination
    road (``extra['od']``) under the job's road prices (``extra['price']``,
    none for a timing-plan job), the congestion-pricing routing of Section 4
    done by ``tsim_shortest_routes``.  One work space serves every job.
    Returns the seconds spent."""
    import numpy as np
    import torch
    from paper_2406_10661_amd import tsim
    t0 = time.perf_counter()
    ws = None
    for w in workloads:
        if w.trips.route_roads is not None:
            continue
        o, d = w.extra["od"]
        price = w.extra.get("price")
        need = tsim.route_workspace_bytes(w.network, len(o))
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=device)
        b, r, bad = tsim.shortest_routes(w.network, o, d, price=None if price is None else np.asarray(price, np.float32),
                                         device=device, workspace=ws)
        if bad:
            raise RuntimeError(f"{w.name}: {bad} trips cannot reach their destination")
        w.trips.route_begin, w.trips.route_roads = b, r
    torch.cuda.synchronize(device)
    return time.perf_counter() - t0


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
