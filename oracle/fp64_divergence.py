"""How far the binary32 oracle drifts from its FP64 twin (same algorithm, same
random integers, every floating-point operation in double): the first step at
which a discrete decision differs, the share of vehicles whose arrival step
differs, and the largest position difference of a vehicle on the same edge
in both runs.  Test infrastructure; calls only the oracle and the seeded
input generators.

    python oracle/fp64_divergence.py [grid10x10|perturbed_grid_ring|metro_0800]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

DISCRETE = ("status", "edge", "lane", "cursor")


def compare(w, steps: int, init=None, every: int = 1) -> dict:
    """Run the two twins side by side for `steps` steps (from `init` if
    given), comparing their discrete state every `every` steps."""
    oracle.set_threads(0)
    a, b = oracle.OracleSim(w), oracle.OracleSim(w, fp64=True)
    t0 = 0
    if init is not None:
        t0 = int(init["t"])
        a.write_state(t0, init)
        b.write_state(t0, init)
    first = None
    done = 0
    while done < steps:
        k = min(every, steps - done)
        a.step(k)
        b.step(k)
        done += k
        if first is None:
            sa, sb = a.state(), b.state()
            if any(not np.array_equal(sa[q], sb[q]) for q in DISCRETE):
                first = t0 + done
    sa, sb = a.state(), b.state()
    dt = float(w.params.dt)
    # arrived in both runs, after the start (earlier arrivals are the same input)
    both = (sa["status"] == 2) & (sb["status"] == 2) & (np.minimum(sa["t_arr"], sb["t_arr"]) >= t0 * dt)
    arr_diff = np.floor(sa["t_arr"][both] / dt) != np.floor(sb["t_arr"][both] / dt)
    same_edge = (sa["status"] == 1) & (sb["status"] == 1) & (sa["edge"] == sb["edge"])
    dx = np.abs(sa["x"].astype(np.float64)[same_edge] - sb["x"][same_edge])
    ca, cb = a.counters(), b.counters()
    oracle.set_threads(1)
    return {"steps": steps, "from_step": t0, "first_divergent_step": first,
            "checked_every": every, "arrived_in_both": int(both.sum()),
            "arrival_step_changed_frac": float(arr_diff.mean()) if both.any() else 0.0,
            "max_abs_dx_same_edge_m": float(dx.max()) if dx.size else 0.0,
            "counters_equal": ca == cb,
            "counter_diff": {k: cb[k] - ca[k] for k in ca if ca[k] != cb[k]}}


def main(which: str) -> dict:
    t = time.time()
    if which == "grid10x10":
        rep = compare(W.config1(), 3600, every=1)
    elif which == "perturbed_grid_ring":
        rep = compare(W.config2(), 10_800, every=60)
    elif which == "metro_0800":
        w = W.config3()
        s0, _ = W.loaded_state(w, 21_600, speed_frac=0.4)
        rep = compare(w, 200, init=s0, every=1)
    else:
        raise SystemExit(f"unknown case {which}")
    rep["case"] = which
    rep["s"] = round(time.time() - t, 1)
    return rep


if __name__ == "__main__":
    for c in (sys.argv[1:] or ["grid10x10", "perturbed_grid_ring", "metro_0800"]):
        print(json.dumps(main(c)), flush=True)
