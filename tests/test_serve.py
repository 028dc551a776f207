"""Host logic of the continuous-batching serve loop, on the CPU.

A fake stepper factory stands in for the HIP library: each chunk of steps
"runs" for a fixed time per step after it is enqueued, and the factory records
which jobs are resident so that the HBM-budget admission can be checked at
every moment.
"""

import threading
import time

import numpy as np
import pytest

from paper_2406_10661_amd import serve as SV


class FakeEvent:
    def __init__(self, t_done):
        self.t_done = t_done

    def query(self):
        return time.perf_counter() >= self.t_done


class FakeSim:
    def __init__(self, fac, job):
        self.fac, self.job = fac, job
        self.steps = 0
        self.chunks = []
        self.busy_until = time.perf_counter()

    def step(self, n):
        self.chunks.append(n)
        self.steps += n
        self.busy_until = max(self.busy_until, time.perf_counter()) + n * self.fac.sec_per_step

    def metrics(self):
        return {"vehicle_steps": self.steps * 100, "n_finished": self.job.jid}

    def close(self):
        with self.fac.lock:
            self.fac.resident.discard(self.job.jid)
            self.fac.closed.append(self.job.jid)
            self.fac.chunks[self.job.jid] = list(self.chunks)


class FakeStream:
    def __init__(self):
        self.sim = None


class FakeFactory:
    def __init__(self, sec_per_step=2e-5):
        self.sec_per_step = sec_per_step
        self.lock = threading.Lock()
        self.resident = set()
        self.sizes = {}
        self.max_resident_bytes = 0
        self.closed = []
        self.created = []
        self.chunks = {}

    def footprint(self, job):
        return job.params["bytes"]

    def create(self, job):
        sim = FakeSim(self, job)
        st = FakeStream()
        st.sim = sim
        with self.lock:
            self.resident.add(job.jid)
            self.sizes[job.jid] = job.params["bytes"]
            self.created.append(job.jid)
            cur = sum(self.sizes[j] for j in self.resident)
            self.max_resident_bytes = max(self.max_resident_bytes, cur)
        return sim, st

    def done_event(self, stream):
        return FakeEvent(stream.sim.busy_until)

    def sync(self):
        pass


def make_jobs(n, seed=0, rate=400.0):
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, n))
    return [SV.Job(jid=k, arrival=float(arr[k]), network=None, trips=None,
                   params={"bytes": int(rng.integers(1, 10)) * 100}, horizon=int(rng.integers(1, 200)))
            for k in range(n)]


def test_all_jobs_complete_in_chunks():
    fac = FakeFactory()
    jobs = make_jobs(40)
    res = SV.ServeLoop(fac, hbm_budget=2000, steps_per_tick=30).run(jobs)
    assert len(res["jobs"]) == 40
    for j in res["jobs"]:
        assert j.steps_done == j.horizon
        assert j.metrics["vehicle_steps"] == 100 * j.horizon
        assert 0 <= j.arrival <= j.admitted <= j.started <= j.finished
    assert sorted(fac.closed) == list(range(40))
    assert not fac.resident


def test_budget_is_never_exceeded_and_admission_is_fifo():
    fac = FakeFactory(sec_per_step=1e-4)
    jobs = make_jobs(30, seed=1, rate=2000.0)
    budget = 1500
    res = SV.ServeLoop(fac, hbm_budget=budget, steps_per_tick=25).run(jobs)
    assert fac.max_resident_bytes <= budget
    assert res["peak_bytes"] <= budget
    by_arrival = sorted(res["jobs"], key=lambda j: j.arrival)
    adm = [j.admitted for j in by_arrival]
    assert adm == sorted(adm)
    # the budget binds: some job waited for memory to be released
    assert any(j.admitted - j.arrival > 1e-3 for j in by_arrival)


def test_chunks_are_bounded_by_tick():
    fac = FakeFactory()
    jobs = make_jobs(10, seed=2)
    k = 17
    SV.ServeLoop(fac, hbm_budget=10**6, steps_per_tick=k).run(jobs)
    assert len(fac.created) == 10
    for j in jobs:
        ch = fac.chunks[j.jid]
        assert sum(ch) == j.horizon
        assert all(c == k for c in ch[:-1]) and 0 < ch[-1] <= k


def test_late_short_job_overtakes_long_running_one():
    """Continuous batching: a short job arriving while a long one runs is
    admitted and finishes first instead of queueing behind it."""
    fac = FakeFactory(sec_per_step=2e-4)
    long_job = SV.Job(jid=0, arrival=0.0, network=None, trips=None, params={"bytes": 100}, horizon=600)
    short = SV.Job(jid=1, arrival=0.01, network=None, trips=None, params={"bytes": 100}, horizon=30)
    res = SV.ServeLoop(fac, hbm_budget=1000, steps_per_tick=30).run([long_job, short])
    d = {j.jid: j for j in res["jobs"]}
    assert d[1].finished < d[0].finished
    assert d[1].started < d[0].finished


def test_oversized_job_is_rejected():
    fac = FakeFactory()
    jobs = [SV.Job(jid=0, arrival=0.0, network=None, trips=None, params={"bytes": 5000}, horizon=10)]
    with pytest.raises(ValueError):
        SV.ServeLoop(fac, hbm_budget=1000).run(jobs)


def test_summarize_percentiles():
    fac = FakeFactory()
    jobs = make_jobs(50, seed=3)
    res = SV.ServeLoop(fac, hbm_budget=10**6, steps_per_tick=30).run(jobs)
    s = SV.summarize(res, skip=10)
    lat = sorted(j.finished - j.arrival for j in sorted(res["jobs"], key=lambda j: j.arrival)[10:])
    assert s["jobs"] == 40
    assert s["latency_p50_s"] == pytest.approx(float(np.percentile(lat, 50)))
    assert s["latency_p99_s"] == pytest.approx(float(np.percentile(lat, 99)))
    assert s["latency_p99_s"] >= s["latency_p50_s"] > 0
    assert s["jobs_per_s"] > 0


class FakeInstance:
    def __init__(self, job):
        self.job = job

    def capacity(self):
        return fake_capacity(self.job)

    def close(self):
        pass


def fake_capacity(job):
    c = {k: 1 for k in SV.CAP_KEYS}
    c["vehicles"] = job.params["bytes"]
    return c


class FakeBatch:
    """Library semantics of a reserved batch: instance ids in order of
    addition, removed trailing instances give their room back."""

    def __init__(self, fac, cap):
        self.fac, self.cap = fac, dict(cap)
        self.steps = 0
        self.inst = []          # [job, g0, horizon, removed]
        self.busy_until = time.perf_counter()

    def step(self, n):
        assert any(not e[3] for e in self.inst), "stepping a batch without live jobs"
        self.steps += n
        self.busy_until = max(self.busy_until, time.perf_counter()) + n * self.fac.sec_per_step

    def add(self, inst):
        assert SV.fits(inst.capacity(), self.capacity_left())
        self.inst.append([inst.job, self.steps, 1 << 30, False])
        with self.fac.lock:
            self.fac.resident.add(inst.job.jid)
            self.fac.joined_at[inst.job.jid] = self.steps
        return len(self.inst) - 1

    def set_horizon(self, k, h):
        self.inst[k][2] = h

    def metrics(self, k):
        job, g0, h, _ = self.inst[k]
        n = min(self.steps - g0, h)
        return {"vehicle_steps": 100 * n, "step": n}

    def remove(self, k):
        assert not self.inst[k][3]
        self.inst[k][3] = True
        with self.fac.lock:
            self.fac.resident.discard(self.inst[k][0].jid)
        while self.inst and self.inst[-1][3]:
            self.inst.pop()

    def capacity_left(self):
        left = dict(self.cap)
        for job, _, _, _ in self.inst:
            for k, v in fake_capacity(job).items():
                left[k] -= v
        return left

    def close(self):
        self.fac.closed += 1


class FakeBatchFactory(FakeFactory):
    def __init__(self, sec_per_step=2e-5):
        super().__init__(sec_per_step)
        self.closed = 0
        self.joined_at = {}

    def capacity_of(self, job):
        return fake_capacity(job)

    def instance(self, job):
        return FakeInstance(job)

    def reserve_footprint(self, cap):
        return cap["vehicles"]

    def reserve(self, cap, params):
        b = FakeBatch(self, cap)
        st = FakeStream()
        st.sim = b
        return b, st


def test_batched_loop_completes_every_job_at_its_horizon():
    fac = FakeBatchFactory()
    jobs = make_jobs(60, seed=4, rate=800.0)
    res = SV.BatchedServeLoop(fac, hbm_budget=3000, steps_per_tick=25, max_batches=3).run(jobs)
    assert len(res["jobs"]) == 60
    for j in res["jobs"]:
        assert j.metrics["step"] == j.horizon
        assert j.metrics["vehicle_steps"] == 100 * j.horizon
        assert 0 <= j.arrival <= j.admitted <= j.started <= j.finished
    assert res["peak_bytes"] <= 3000
    assert sorted(j.jid for j in res["jobs"]) == list(range(60))
    assert not fac.resident and fac.closed == 3
    # jobs joined batches that were already running
    assert sum(1 for g in fac.joined_at.values() if g > 0) >= 10


def test_batched_loop_short_job_leaves_before_long_batchmate():
    fac = FakeBatchFactory(sec_per_step=2e-4)
    a = SV.Job(jid=0, arrival=0.0, network=None, trips=None, params={"bytes": 10}, horizon=600)
    b = SV.Job(jid=1, arrival=0.0, network=None, trips=None, params={"bytes": 10}, horizon=30)
    c = SV.Job(jid=2, arrival=0.05, network=None, trips=None, params={"bytes": 10}, horizon=60)
    res = SV.BatchedServeLoop(fac, hbm_budget=100, steps_per_tick=30, max_batches=1).run([a, b, c])
    d = {j.jid: j for j in res["jobs"]}
    assert d[1].finished < d[0].finished        # delivered at its own horizon
    assert fac.joined_at[2] > 0                 # joined the running batch
    assert d[2].finished < d[0].finished
