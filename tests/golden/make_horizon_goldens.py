"""Writes the oracle's horizon statistics used by the GPU horizon-parity
tests (tests/golden/horizon_*.json).  Calls only the oracle and the seeded
input generators; run from the repository root:

    python tests/golden/make_horizon_goldens.py [c2] [c3]

  c2: the 32x32 jittered grid with 100,000 vehicles over its whole 3,600-step
      horizon from t = 0;
  c3: the 2,464,950-vehicle city, 50 steps from a seeded synthetic state at
      t = 3,600 s (half of the due vehicles on the network).
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2406_10661_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
C3_STEP, C3_SEED, C3_P_ACTIVE, C3_STEPS = 3600, 61, 0.5, 50


def keep(m):
    return {k: m[k] for k in ("t", "finished", "sum_tt", "att", "mean_speed_avg", "vehicle_steps", "lane_changes",
                              "transfers", "departures", "speed_steps")}


def c2():
    w = W.config2()
    o = O.OracleSim(w.network, w.trips, w.params)
    t0 = time.time()
    for s in range(0, w.n_steps, 600):
        o.step(600)
        print(f"c2 step {s + 600}: {o.metrics()['finished']:.0f} finished, {time.time() - t0:.0f} s", flush=True)
    return {"workload": w.name, "from_step": 0, "steps": w.n_steps, "oracle": keep(o.metrics())}


def c3():
    w = W.config3()
    st = W.synthetic_state(w.network, w.trips, C3_STEP, seed=C3_SEED, p_active=C3_P_ACTIVE)
    o = O.OracleSim(w.network, w.trips, w.params)
    s64 = dict(st)
    s64["x"] = st["x"].astype("float64")
    s64["v"] = st["v"].astype("float64")
    o.set_state(s64)
    m0 = o.metrics()
    t0 = time.time()
    for s in range(C3_STEPS):
        o.step(1)
        if s % 10 == 9:
            print(f"c3 step {C3_STEP + s + 1}: {time.time() - t0:.0f} s", flush=True)
    return {"workload": w.name, "from_step": C3_STEP, "steps": C3_STEPS, "state_seed": C3_SEED,
            "p_active": C3_P_ACTIVE, "active_at_start": int((st["status"] == 1).sum()),
            "finished_at_start": m0["finished"], "oracle": keep(o.metrics())}


if __name__ == "__main__":
    O.build()
    which = sys.argv[1:] or ["c2", "c3"]
    for name in which:
        res = {"c2": c2, "c3": c3}[name]()
        with open(os.path.join(HERE, f"horizon_{name}.json"), "w") as f:
            json.dump(res, f, indent=1)
        print(name, json.dumps(res), flush=True)
