"""Writes oracle_snapshots.json: the CPU oracle's state at a few steps of
three seeded runs (two on the 10x10 grid, one on the full-size perturbed grid
with ring highway through its morning peak), as frozen expected values.

Every number in the file comes from ``oracle/`` run on inputs from the seeded
generators in ``workloads/`` (which hold none of the step's arithmetic).  The
oracle's own correctness rests on its pins (closed forms of Eq. (1), Eq. (2)
frequencies, brute-force admission, central differences); this file freezes
what it computes so that an unintended change of its arithmetic shows up as
a failed test, and gives the GPU path a stored target that does not need the
oracle at run time.

    python tests/golden/make_oracle_snapshots.py      # rewrites the file

A change of the oracle that changes these values must name, in its commit
message, the passage of the paper (or the reading of it) that justifies it."""
from __future__ import annotations

import hashlib
import json
import os
import re
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_snapshots.json")
INT_FIELDS = ("status", "edge", "lane", "cursor", "held_since", "mand", "ww")
F32_FIELDS = ("x", "v")
F64_FIELDS = ("tau_in", "t_arr")
N_SAMPLE = 16
ROW = ("id",) + INT_FIELDS + F32_FIELDS + F64_FIELDS   # one sampled vehicle per row


def case_workload(name: str):
    """The two seeded runs: case 2 (all-green nodes) with the config-1
    parameters, and case 1 (flashing red) with 4 jittered driver classes and
    a per-driver v0 spread of 0.05."""
    if name == "grid10x10_case2":
        return W.config1()
    if name == "grid10x10_case1_4classes_spread":
        w = W.config1(n_classes=4)
        w.params = W.jitter_params(w.params, 0.1, seed=5)
        w.params.v0_spread = 0.05
        w.params.intersection_mode = 1
        return w
    if name == "perturbed_grid_ring_peak":
        return W.config2()
    raise KeyError(name)


# checkpoints per case; config 2 at 07:45 and 08:00 (its departures peak at
# 08:00, about 110,000 vehicles active)
CASES = {"grid10x10_case2": [300, 1200, 3600],
         "grid10x10_case1_4classes_spread": [600, 1200, 2400],
         "perturbed_grid_ring_peak": [9900, 10800]}
# cases whose run is long: the oracle uses every thread for them (the result
# does not depend on the thread count)
LONG = ("perturbed_grid_ring_peak",)


def state_digest(s: dict, fields) -> str:
    """sha256 over the named fields of the state, in fixed dtypes and order."""
    h = hashlib.sha256()
    for k in fields:
        dt = np.float64 if k in F64_FIELDS else np.float32 if k in F32_FIELDS else np.int64
        h.update(np.ascontiguousarray(s[k], dt).tobytes())
    return h.hexdigest()


def sample_ids(n: int, k: int = N_SAMPLE) -> list:
    return np.random.default_rng(20070361).choice(n, k, replace=False).tolist()


def case_sample_ids(name: str, n: int) -> list:
    """The sampled vehicles of a case: 16, or 64 on the large network."""
    return sample_ids(n, 64 if name in LONG else N_SAMPLE)


def snapshot(s: dict, counters: dict, ids: list) -> dict:
    veh = []
    for i in ids:
        veh.append([int(i)] + [int(s[k][i]) for k in INT_FIELDS]
                   + [float(np.float32(s[k][i])).hex() for k in F32_FIELDS]
                   + [float(s[k][i]).hex() for k in F64_FIELDS])
    return {"t": int(s["t"]), "counters": counters, "vehicles": veh,
            # discrete fields and binary32 x, v (bitwise under the parity contract)
            "digest": state_digest(s, INT_FIELDS + F32_FIELDS),
            # FP64 entry and arrival times
            "digest_times": state_digest(s, F64_FIELDS)}


def main() -> None:
    import oracle
    oracle.build()
    out = {"about": "CPU oracle (binary32 build) state of three seeded runs; "
                    "written by make_oracle_snapshots.py; floats as C99 hex", "row": list(ROW), "cases": {}}
    for name, cps in CASES.items():
        w = case_workload(name)
        oracle.set_threads(0 if name in LONG else 1)
        sim = oracle.OracleSim(w)
        ids = case_sample_ids(name, w.n_vehicles)
        snaps, t = [], 0
        for cp in cps:
            sim.step(cp - t)
            t = cp
            snaps.append(snapshot(sim.state(), sim.counters(), ids))
        out["cases"][name] = {"n_vehicles": int(w.n_vehicles), "checkpoints": snaps}
        print(name, [c["counters"]["arrived"] for c in snaps])
    text = json.dumps(out, indent=1, sort_keys=True)
    # one vehicle row per line
    text = re.sub(r"\[\n\s+(\d+),\n([^\[\]]*?)\n\s+\]", lambda m: "[" + m.group(1) + ", " + ", ".join(
        x.strip() for x in m.group(2).split(",\n")) + "]", text)
    with open(OUT, "w") as f:
        f.write(text + "\n")


if __name__ == "__main__":
    main()
