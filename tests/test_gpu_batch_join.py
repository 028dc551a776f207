"""Instances joining and leaving a running batch (tsim_batch_reserve / add /
add_member / remove through the C ABI): a job that joins at some global step
follows exactly the trajectory it has alone, a joined instance passes the
one-step oracle comparison, removed instances stay frozen while the rest go
on, and the space of trailing removed instances is reused."""

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.parity import compare_one_step

pytestmark = pytest.mark.gpu

KEYS = ("status", "lane", "route_pos", "x", "v", "finish_step")


@pytest.fixture(scope="module")
def T():
    from paper_2406_10661_amd import tsim as T
    return T


@pytest.fixture(scope="module")
def jobs():
    return [W.config1(), W.config4_instance(7), W.config4_instance(13), W.config4_instance(21)]


def _cap(T, ws, extra=1.0):
    cap = {}
    for w in ws:
        cap = T.add_capacity(cap, T.Instance(w.network, w.trips, w.params).capacity(), extra)
    return cap


def _alone(T, w, steps):
    s = T.Sim(w.network, w.trips, w.params)
    s.step(steps)
    st, m = s.get_state(), s.metrics()
    s.close()
    return st, m


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


def test_join_running_batch_matches_alone(T, jobs):
    b = T.Batch.reserve(_cap(T, jobs), jobs[0].params)
    assert b.num_instances() == 0
    b.step(5)                                   # an empty batch steps nothing
    k0 = b.add(jobs[0].network, jobs[0].trips, jobs[0].params)
    b.step(40)
    k1 = b.add(jobs[1].network, jobs[1].trips, jobs[1].params)   # joins at the batch's step 40
    b.set_graph_steps(20)
    b.step(200)
    k2 = b.add(jobs[2].network, jobs[2].trips, jobs[2].params)   # joins after graphs were captured
    b.step(61)
    for k, w, n in ((k0, jobs[0], 301), (k1, jobs[1], 261), (k2, jobs[2], 61)):
        st, m = _alone(T, w, n)
        bs = b.get_state(k)
        assert bs["step"] == n
        _same(st, bs)
        bm = b.metrics(k)
        for key in ("vehicle_steps", "n_finished", "lane_changes", "transfers", "departures"):
            assert bm[key] == m[key], key
        assert bm["mean_speed_avg"] == m["mean_speed_avg"]


def test_joined_instance_oracle_one_step(T, jobs):
    from oracle import oracle as O
    O.build()
    b = T.Batch.reserve(_cap(T, jobs[:2]), jobs[0].params)
    b.add(jobs[0].network, jobs[0].trips, jobs[0].params)
    b.step(33)
    w = jobs[1]
    k = b.add(w.network, w.trips, w.params)
    st = W.synthetic_state(w.network, w.trips, 250, seed=5, p_active=0.7)
    b.set_state(k, st)
    b.step(1)
    rep = compare_one_step(O, None, w.network, w.trips, w.params, st, sim=b.instance(k), stepped=True)
    assert rep["active"] > 500


def test_remove_freezes_and_space_is_reused(T, jobs):
    b = T.Batch.reserve(_cap(T, jobs[:3]), jobs[0].params)
    ks = [b.add(w.network, w.trips, w.params) for w in jobs[:3]]
    b.step(50)
    frozen = b.get_state(ks[1])
    b.remove(ks[1])                 # a middle instance: frozen, its id stays
    assert b.num_instances() == 3
    b.step(30)
    _same(frozen, b.get_state(ks[1]))
    _same(_alone(T, jobs[2], 80)[0], b.get_state(ks[2]))
    left = b.capacity_left()
    b.remove(ks[2])                 # trailing: pops it and the frozen one before it
    assert b.num_instances() == 1
    more = b.capacity_left()
    assert more["vehicles"] == left["vehicles"] + jobs[1].trips.n_vehicles + jobs[2].trips.n_vehicles
    k = b.add(jobs[1].network, jobs[1].trips, jobs[1].params)   # fits the space given back
    assert k == 1
    b.step(25)
    _same(_alone(T, jobs[1], 25)[0], b.get_state(k))
    _same(_alone(T, jobs[0], 105)[0], b.get_state(ks[0]))
    with pytest.raises(T.TsimError) as e:
        for w in jobs * 4:
            b.add(w.network, w.trips, w.params)
    assert e.value.code == T.TSIM_ENOMEM


def test_add_member_continues_its_run(T, jobs):
    w = jobs[1]
    s = T.Sim(w.network, w.trips, w.params)
    s.step(70)
    b = T.Batch.reserve(_cap(T, jobs[:2]), jobs[0].params)
    b.add(jobs[0].network, jobs[0].trips, jobs[0].params)
    b.step(11)
    k = b.add_member(s)
    assert b.get_state(k)["step"] == 70
    m0 = s.metrics()
    b.step(45)
    s.step(45)
    _same(s.get_state(), b.get_state(k))
    # counters restart where the member joined (as after tsim_set_state); totals of trips do not
    bm, sm = b.metrics(k), s.metrics()
    assert bm["vehicle_steps"] == sm["vehicle_steps"] - m0["vehicle_steps"]
    assert bm["n_finished"] == sm["n_finished"] and bm["step"] == sm["step"] == 115
