"""IDM pins (Appendix B.3 car-following equations) through the oracle's own
IDM routine: closed forms the equations fix, not a retyped formula.

  * free road: a(v = 0) = a_max, a(v = v0) = 0, and a(v) = 0 only at v0;
  * equilibrium gap: with dv = 0 and s = s_e(v) = (s0 + v T) / sqrt(1 - (v/v0)^4)
    the acceleration vanishes (delta = 4 enters through s_e);
  * standing queue: v = 0 at s = s0 gives a = 0, and a = a_max (1 - (s0/s)^2);
  * with a huge v0 the free term is 1, so a = 0 exactly at s = s_star, whose
    dynamic part v dv / (2 sqrt(a_max b)) is checked at two approach rates;
  * monotone in s, decreasing in the approach rate dv.
"""

import math

import numpy as np
import pytest

from paper_2406_10661_amd.workloads import Params


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


P = Params()


def test_free_road_ends(O):
    for v0 in (11.1, 13.9, 20.0):
        assert O.idm(P, 0.0, v0, math.inf, 0.0) == pytest.approx(P.a_max, abs=1e-15)
        assert O.idm(P, v0, v0, math.inf, 0.0) == pytest.approx(0.0, abs=1e-14)
        # half speed: 1 - 2^-4 of a_max (delta = 4)
        assert O.idm(P, v0 / 2, v0, math.inf, 0.0) == pytest.approx(P.a_max * (1 - 1 / 16), rel=1e-14)


@pytest.mark.parametrize("v", [0.5, 3.0, 7.0, 11.0, 13.0])
def test_equilibrium_gap(O, v):
    v0 = 13.9
    s_e = (P.s0 + v * P.T) / math.sqrt(1.0 - (v / v0) ** 4)
    assert O.idm(P, v, v0, s_e, 0.0) == pytest.approx(0.0, abs=1e-12)
    # slightly larger gap accelerates, smaller brakes
    assert O.idm(P, v, v0, s_e * 1.01, 0.0) > 0
    assert O.idm(P, v, v0, s_e * 0.99, 0.0) < 0


def test_standing_queue(O):
    assert O.idm(P, 0.0, 13.9, P.s0, 0.0) == pytest.approx(0.0, abs=1e-15)
    for s in (3.0, 10.0, 50.0):
        assert O.idm(P, 0.0, 13.9, s, 0.0) == pytest.approx(P.a_max * (1 - (P.s0 / s) ** 2), rel=1e-14)


@pytest.mark.parametrize("v,dv", [(10.0, 10.0), (10.0, 4.0), (5.0, -1.0)])
def test_desired_gap_root(O, v, dv):
    v0 = 1e12  # free term = 1
    s_star = P.s0 + max(0.0, v * P.T + v * dv / (2 * math.sqrt(P.a_max * P.b_comf)))
    assert O.idm(P, v, v0, s_star, dv) == pytest.approx(0.0, abs=1e-12)
    # 10 m/s closing at 10 m/s: s_star = 2 + 15 + 100/6
    if (v, dv) == (10.0, 10.0):
        assert s_star == pytest.approx(2 + 15 + 100 / 6)


def test_desired_gap_floor_s0(O):
    # a strongly opening gap cannot push s_star below s0: a = a_max(1-(s0/s)^2) at v0 huge
    v0 = 1e12
    for s in (4.0, 8.0):
        assert O.idm(P, 10.0, v0, s, -100.0) == pytest.approx(P.a_max * (1 - (P.s0 / s) ** 2), rel=1e-12)


def test_monotonicity(O):
    ss = np.linspace(2.5, 200, 50)
    a = [O.idm(P, 8.0, 13.9, s, 1.0) for s in ss]
    assert np.all(np.diff(a) > 0)
    dvs = np.linspace(-5, 5, 21)
    a = [O.idm(P, 8.0, 13.9, 30.0, d) for d in dvs]
    assert np.all(np.diff(a) <= 0)


def test_nonpositive_gap_is_minus_infinity(O):
    assert O.idm(P, 5.0, 13.9, 0.0, 0.0) == -math.inf
    assert O.idm(P, 5.0, 13.9, -1.0, 0.0) == -math.inf
