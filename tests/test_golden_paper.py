"""Pins against values the paper prints (fixture tests/golden/
paper_vehicle_model.txt, each value with its place in the paper): the IDM
exponent, the MOBIL politeness, the two end levels of the randomized
lane-change probability as the oracle computes them, and the scale of the
paper's largest run that the city workload and the benchmark's context
quote.

The middle branch of the lane-change probability is not pinned here: the
paper prints it in a form that is discontinuous at both ends, and the oracle
uses the continuous ramp between the two printed levels instead (the
binomial test of the randomized lane change covers it)."""

import inspect
import os

import numpy as np
import pytest

from paper_2406_10661_amd import workloads as W
from tests.scenes import line_network, trips_for, state_from

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_vehicle_model.txt")


def load_golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


G = load_golden()


def test_fixture_complete():
    assert set(G) == {"idm_delta", "mobil_politeness", "plc_high", "plc_floor", "paper_hz", "paper_vehicles"}


def test_model_defaults_are_the_papers():
    P = W.Params()
    assert P.delta == G["idm_delta"]
    assert P.politeness == G["mobil_politeness"]
    assert P.p_min == G["plc_floor"]
    # the workloads cap the probability at 0.5 (their stated change
    # probability); the paper's 0.9 is a parameter value
    assert W.Params(p_max=G["plc_high"]).p_max == G["plc_high"]


def _mobil_of_first(oracle_lib, n, lanes, xs, vs):
    params = W.Params(p_max=G["plc_high"])
    net = line_network(lanes=3, length=2000.0, policy=W.POLICY_NONE)
    o = oracle_lib.OracleSim(net, trips_for([[0, 2]] * n), params)
    o.set_state(state_from(n, lanes, xs, vs))
    o.step(1)
    return o.diag()["mobil"][0]


def test_plc_high_level(oracle_lib):
    """A vehicle at 12 m/s 15 m behind a stopped one, both side lanes empty:
    both utilities are large, u_T >= 1, and p_LC is the printed 0.9."""
    uL, uR, uT, plc = _mobil_of_first(oracle_lib, 2, [1, 1], [100.0, 115.0], [12.0, 0.0])
    assert uL > 1 and uR > 1 and uT >= 1
    assert plc == G["plc_high"]


def test_plc_floor_level(oracle_lib):
    """A lone vehicle at its desired speed on an empty three-lane road: no
    side gains anything (both utilities are -a_th), u_T = 0, and p_LC is the
    printed floor 2e-8."""
    uL, uR, uT, plc = _mobil_of_first(oracle_lib, 1, [1], [100.0], [float(np.float32(13.9))])
    assert uL == pytest.approx(-W.Params().a_th) and uR == pytest.approx(-W.Params().a_th)
    assert uT == 0.0
    assert plc == G["plc_floor"]


def test_city_scale_and_context_are_the_papers():
    n = inspect.signature(W.config3).parameters["n_vehicles"].default
    assert n == int(G["paper_vehicles"])
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py")).read()
    assert f'"hz": {G["paper_hz"]}' in src
    assert f'"vehicles": {int(G["paper_vehicles"])}' in src
