"""The no-allocation entry point tsim_set_signal_phases_noalloc, called
through the C ABI, against tsim_set_signal_phases on two identical instances:
two calls in a row (every junction, then a few), each followed by steps;
states, held phases and metrics bit-identical.  Sizes beyond its staging
array are refused."""

import ctypes as C

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("status", "lane", "route_pos", "x", "v", "finish_step", "junc_policy", "junc_phase")


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def test_noalloc_phases_match_the_staged_entry_point():
    from paper_2406_10661_amd import tsim as T
    w = W.config1()
    a = T.Sim(w.network, w.trips, w.params)
    b = T.Sim(w.network, w.trips, w.params)
    L = T.lib()
    nj = w.network.n_junctions
    nph = np.diff(w.network.junc_phase_begin)
    rng = np.random.default_rng(17)
    a.step(50)
    b.step(50)
    for n in (nj, 5):
        ids = np.ascontiguousarray(rng.permutation(nj)[:n], np.int32)
        ph = np.ascontiguousarray(rng.integers(0, 1000, n) % nph[ids], np.int32)
        a.set_signal_phases(ids, ph)
        rc = L.tsim_set_signal_phases_noalloc(b.h, _p(ids), _p(ph), n)
        assert rc == T.TSIM_OK, L.tsim_last_error(b.h)
        a.step(37)
        b.step(37)
        sa, sb = a.get_state(), b.get_state()
        for k in KEYS:
            assert np.array_equal(sa[k], sb[k]), (n, k)
        assert np.all(sb["junc_policy"][ids] == W.POLICY_MANUAL)
        assert np.array_equal(sb["junc_phase"][ids], ph)
        ma, mb = a.metrics(), b.metrics()
        assert ma == mb


def test_noalloc_refuses_more_than_its_staging_array():
    from paper_2406_10661_amd import tsim as T
    w = W.config1()
    s = T.Sim(w.network, w.trips, w.params)
    n = (1 << 18) + 1
    ids = np.zeros(n, np.int32)
    ph = np.zeros(n, np.int32)
    rc = T.lib().tsim_set_signal_phases_noalloc(s.h, _p(ids), _p(ph), n)
    assert rc == T.TSIM_EINVAL
    assert b"262144" in T.lib().tsim_last_error(s.h)
