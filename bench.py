#!/usr/bin/env python3
"""Benchmark of the per-timestep vehicle update on one MI355X.

A "step" is one simulated time step (dt = 0.5 s) of the whole hot path:
lane changes, leader search, IDM, integration, intersection admission and the
rebuild of the sorted vehicle layout.  The default workload is the
metropolitan-scale network (about 224k nodes, 549k directed edges, 3.2M
trips departing 05:00-10:00) timed at 08:00, the peak of its demand: the run
is stepped untimed from 05:00 to 08:00, `--warmup` steps follow untimed, then
`--steps` steps are timed, with every input resident in device memory.

value = vehicle-updates/s = sum over the timed steps of the vehicles active at
each step's start, divided by the device time of those steps (HIP events on
the simulation's stream around sim_step, which replays captured graphs of 8
steps).  The same window is then run again kernel by kernel between HIP
events to time each kernel.  The roofline object covers k_tile_step, which
does Phases 1-2 of every vehicle in a tile that fits one workgroup's LDS:
algorithmic bytes = 28 B per vehicle-update it does (read x, v, id and the
packed lane/flags word, write x, v and that word; updates in larger tiles,
done by k_big_admit, are counted by the library and left out), over its
event-measured time.  The CPU baseline is the oracle on an 08:00 state built
from the demand (which it can start from), on one thread and on every thread;
the GPU runs the same steps from the same state and the two are compared.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 28      # read x, v, id, meta (16 B), write x, v, meta (12 B)


def kernel_source_digest() -> str:
    """Digest of the HIP sources: byte counters taken on other sources no
    longer describe the kernel and are not reported."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2007_03614_amd", "csrc")
    for n in sorted(os.listdir(d)):
        with open(os.path.join(d, n), "rb") as f:
            h.update(n.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from(fetch_json: str, write_json: str, kernels=("k_tile_step",),
                 probe_mib: int = 256, workload: str = "metro", probe_jsons=None) -> dict:
    """HBM bytes per step of the tile kernel (launched once per step) from
    two --pmc summaries (FETCH_SIZE, WRITE_SIZE in KiB per dispatch),
    each counter scaled by what it reads for the copy probe (torch's add of
    probe_mib MiB: reads and writes probe_mib MiB each).  probe_jsons: the
    (fetch, write) summaries holding the probe when the kernel's runs
    collected counters over a window that leaves it out."""
    f = json.load(open(fetch_json))["kernels"]
    w = json.load(open(write_json))["kernels"]
    pfj, pwj = probe_jsons or (fetch_json, write_json)
    f_probe = json.load(open(pfj))["kernels"]
    w_probe = json.load(open(pwj))["kernels"]

    def probe(d, key):
        p = [k for k in d if "add" in k.lower() and "fill" not in k.lower() and key in d[k]]
        if len(p) != 1:
            raise SystemExit(f"cannot identify the copy probe in summary: {p}")
        return d[p[0]][key], p[0]

    def per_kernel(d, key):
        out = {}
        for kn in kernels:
            ks = [k for k in d if kn + "(" in k]
            if len(ks) != 1:
                raise SystemExit(f"cannot identify {kn} in summary: {ks}")
            out[kn] = d[ks[0]][key]
        return out

    pf, pname = probe(f_probe, "FETCH_SIZE")
    pw, _ = probe(w_probe, "WRITE_SIZE")
    kf, kw = per_kernel(f, "FETCH_SIZE"), per_kernel(w, "WRITE_SIZE")
    known = probe_mib * 1024.0
    fs, ws = known / pf, known / pw
    return {"workload": workload, "kernels": list(kernels), "sources": kernel_source_digest(),
            "bytes_per_step": 1024.0 * sum(kf[k] * fs + kw[k] * ws for k in kernels),
            "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
            "probe": pname[:80], "probe_fetch_kib": pf, "probe_write_kib": pw,
            "probe_from": [os.path.basename(os.path.dirname(os.path.abspath(x))) + "/" + os.path.basename(x)
                           for x in (pfj, pwj)],
            "fetch_scale": fs, "write_scale": ws}


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"tile_kernels_traffic_{workload}.json")


def stored_traffic(workload: str, v0_spread: float = 0.0, intersection_mode: int = 0, path: str = None):
    """HBM bytes per step of k_tile_step from the committed counter record, or
    None when there is no record or it was taken on other HIP sources, another
    workload or other options (its bytes then describe another kernel)."""
    path = path or traffic_file(workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f)
    if (tr.get("workload") == workload and tr.get("sources") == kernel_source_digest()
            and tr.get("v0_spread", 0.0) == v0_spread and tr.get("intersection_mode", 0) == intersection_mode):
        return tr.get("bytes_per_step")
    return None


# step at which each plain workload is timed: 08:00, the morning peak of its demand
PEAK_STEP = {"metro": 21600, "perturbed_grid_ring": 10800, "grid10x10": 600}
# assumed mean speed, as a fraction of each edge's limit, of the vehicles placed
# on their routes to build the 08:00 state the oracle starts from
SPEED_FRAC = 0.4


def make_workload(name: str):
    import workloads as W
    if name == "metro":
        return W.config3()
    if name == "perturbed_grid_ring":
        return W.config2()
    if name == "grid10x10":
        return W.config1()
    raise SystemExit(f"unknown workload {name}")


def cpu_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable}


def cpu_baseline(w, state0, warmup: int, steps: int, threads: int):
    """The oracle as it stands, from the same written state as the GPU run:
    `warmup` untimed steps, then `steps` timed steps, with `threads` OpenMP
    threads in its parallel phases.  Returns the figures and the oracle's
    counters and state at the end (for the window's parity check)."""
    import oracle
    used = oracle.set_threads(threads)
    s = oracle.OracleSim(w)
    s.write_state(int(state0["t"]), state0)
    s.step(warmup)
    before = s.counters()["active_sum"]
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    upd = s.counters()["active_sum"] - before
    return {"value": upd / dt, "unit": "vehicle-updates/s", "cores": used, "kind": "oracle",
            "vehicle_updates": int(upd), "s": dt}, s.counters(), s.state()


def summarize_pmc(directory: str, last: int = 0) -> dict:
    """Per-kernel means of the counters in a `rocprofv3 --pmc --output-format
    csv` directory: {kernel: {"dispatches": n, counter: mean per dispatch}};
    with last > 0 over each kernel's last `last` dispatches only (the timed
    window of a run stepped untimed to its start).  Device copies
    (`__amd_rocclr_copyBuffer`) are kept per grid size, so a copy of known
    size can calibrate byte counters."""
    import csv
    import glob
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    rows = {}
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                name = row.get("Kernel_Name", "?")
                if "copyBuffer" in name:
                    name = f"{name} grid={row.get('Grid_Size', '?')}"
                did = next((row[k] for k in row if k and k.lower() in ("dispatch_id", "dispatch_index")), "0")
                rows.setdefault((name, row.get("Counter_Name", "?")), []).append(
                    (int(did), float(row.get("Counter_Value", 0.0))))
    out = {}
    for (name, ctr), vals in rows.items():
        vals.sort()
        if last > 0:
            vals = vals[-last:]
        k = out.setdefault(name, {})
        k["dispatches"] = max(k.get("dispatches", 0), len(vals))
        k[ctr] = sum(v for _, v in vals) / len(vals)
    return {"files": len(files), "kernels": out}


def summarize_trace(directory: str, last: int = 0) -> dict:
    """Per-kernel dispatch counts and mean durations (us) from a `rocprofv3
    --kernel-trace --output-format csv` directory, over every dispatch and
    over the last `last` dispatches of each kernel (the timed window of a run
    that is first stepped untimed to its start)."""
    import csv
    import glob
    files = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)
    per = {}
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                name = row.get("Kernel_Name", "?")
                per.setdefault(name, []).append((int(row["Start_Timestamp"]), int(row["End_Timestamp"])))
    out = {}
    for name, ev in per.items():
        ev.sort()
        dur = [(b - a) / 1e3 for a, b in ev]
        k = {"dispatches": len(dur), "mean_us": sum(dur) / len(dur)}
        if last > 0:
            tail = dur[-last:]
            k[f"mean_us_last_{len(tail)}"] = sum(tail) / len(tail)
        out[name] = k
    return {"files": len(files), "kernels": out}


def bench_ensemble(args, M, torch, stream):
    """64 what-if scenarios on the 10x10 grid (demand U[0.8, 1.2] x 200,000 of
    a 240,000 master list, 1 % of edges cut to one lane each), 2 h: one
    ensemble handle (autotuned schedule, captured graph) against the 64
    scenarios run one after another, each on its own graph-captured handle."""
    import workloads as W
    master, scen = W.config4(n_scen=args.scenarios)
    steps = args.steps if args.steps_given else master.n_steps
    cache = os.path.join("/tmp", "manta_schedule_cache.txt")
    tune = M.Sim(master, scenarios=scen, stream=stream)
    tune.step(args.tune_at)
    sched = tune.autotune(cache, steps_per_trial=10)
    tune.close()
    ens = M.Sim(master, scenarios=scen, stream=stream)
    ens.autotune(cache)   # read back from the cache
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ens.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    c = ens.counters()
    upd = c["active_sum"]
    ens.close()
    seq_ms, seq_upd = 0.0, 0
    for k, (n, red) in enumerate(scen):
        if k % 8 == 0:
            print(f"sequential handles: {k}/{len(scen)}", file=sys.stderr, flush=True)
        solo = M.Sim(W.scenario_workload(master, n, red), stream=stream)
        torch.cuda.synchronize()
        e0.record(stream)
        solo.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        seq_ms += e0.elapsed_time(e1)
        seq_upd += solo.counters()["active_sum"]
        solo.close()
    assert seq_upd == upd, (seq_upd, upd)
    return {
        "metric": "vehicle-updates/sec (1 GPU)", "value": upd / (ms / 1e3), "unit": "vehicle-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": args.tune_at, "ms_per_step": ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"ensemble{args.scenarios}_grid10x10", "scenarios": args.scenarios,
                   "vehicles": int(sum(n for n, _ in scen)), "steps": steps, "vehicle_updates": int(upd),
                   "arrived": int(c["arrived"]), "schedule": sched},
        "sequential": {"value": seq_upd / (seq_ms / 1e3), "ms": seq_ms, "handles": args.scenarios},
        "ensemble_speedup": (upd / ms) / (seq_upd / seq_ms),
    }


def bench_calibration(args, M, torch, stream):
    """Differentiable form on the 10x10 grid at 1 h (7,200 steps), 4 classes:
    loss = sum over edges of (mean traversal time - target)^2, targets from a
    run at hidden parameters theta* = base * (1 + U[-0.1, 0.1]); gradient with
    respect to the 20 class parameters at theta0 = base, checkpoint every 120
    steps.  Reports sim_backward wall time (segment re-runs included) over the
    recording forward's wall time."""
    import workloads as W
    steps = args.steps if args.steps_given else 7200
    w = W.config1(n_classes=4, n_steps=steps)
    hidden = W.jitter_params(w.params, 0.1, seed=5)
    tw = M.with_class_params(w, np.stack([hidden.v0_factor, hidden.T, hidden.a, hidden.b, hidden.s0], 1))
    ref = M.Sim(tw, stream=stream)
    ref.step(steps)
    target, tcnt = ref.mean_travel_times()
    ref.close()
    w.params.record_every = 120
    res = []
    for rep in range(1 + args.reps):
        sim = M.Sim(w, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mean, cnt = sim.mean_travel_times()
        use = (cnt > 0) & (tcnt > 0)
        dl = np.where(use, 2.0 * (mean - target), 0.0)
        t2 = time.perf_counter()
        g = sim.backward(dl)
        t3 = time.perf_counter()
        sim.close()
        if rep > 0 or args.reps == 0:
            res.append((t1 - t0, t3 - t2, float(np.sum(np.where(use, (mean - target) ** 2, 0.0))), g))
    fwd = min(r[0] for r in res)
    bwd = min(r[1] for r in res)
    return {
        "metric": "backward/forward time ratio", "value": bwd / fwd, "unit": "ratio", "n_gpus": 1,
        "steps": steps, "warmup": 1 if args.reps else 0, "ms_per_step": 1e3 * fwd / steps,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32 state, f64 adjoint",
        "data": "synthetic",
        "config": {"workload": "calibration_grid10x10_4classes", "vehicles": w.n_vehicles, "params": 20,
                   "record_every": 120, "forward_s": fwd, "backward_s": bwd, "loss": res[-1][2],
                   "grad_norm": float(np.linalg.norm(res[-1][3]))},
    }


def bench_calibration_search(args, M, torch, stream):
    """The paper's calibration loop (Sec. IV-A) on the 10x10 grid with
    flashing-red intersections (case 1, where stops and queues make speeds
    depend on the parameters), one class, 1 h (7,200 steps): observed edge
    speeds from a run at hidden (a, b, T, s0) = config-1 values * (1 + U[-0.3,
    0.3]) (clipped to the bounds); the search starts from (2, 2.5, 1, 3).
    5 iterations of 5 parameter sets, each iteration one ensemble handle,
    against the same loop with 5 handles run one after another (identical
    decisions, checked), and against 5 iterations of adjoint gradient descent
    on the same L1 loss."""
    import workloads as W
    from paper_2007_03614_amd import calibrate as C
    steps = args.steps if args.steps_given else 7200
    w = W.config1(n_steps=steps)
    w.params.intersection_mode = 1
    rng = np.random.default_rng(11)
    ref_p = np.array([w.params.a[0], w.params.b[0], w.params.T[0], w.params.s0[0]], np.float64)
    lo, hi = C._bounds_arrays()
    hidden = np.clip(ref_p * (1.0 + rng.uniform(-0.3, 0.3, 4)), lo, hi)
    base = np.array([2.0, 2.5, 1.0, 3.0])
    ref = M.Sim(M.with_class_params(w, C.class_params(w, hidden).astype(np.float64)), stream=stream)
    ref.step(steps)
    mean, cnt = ref.mean_travel_times()
    ref.close()
    observed = C.edge_speeds(mean, cnt, w.net.length)
    deltas = rng.uniform(-1.0, 1.0, (5, 4, 4))

    def sequential(sets):
        out = []
        for th in sets:
            sim = M.Sim(M.with_class_params(w, C.class_params(w, th).astype(np.float64)), stream=stream)
            sim.step(steps)
            mm, cc = sim.mean_travel_times()
            sim.close()
            out.append(C.l1_speed_loss(C.edge_speeds(mm, cc, w.net.length), observed))
        return out

    C.random_search(w, observed, steps, deltas[:1], theta0=base, tol=0.0, stream=stream)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th_e, h_e = C.random_search(w, observed, steps, deltas, theta0=base, tol=0.0, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    th_s, h_s = C.random_search(w, observed, steps, deltas, theta0=base, tol=0.0, evaluate=sequential)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert all(a["losses"] == b["losses"] for a, b in zip(h_e, h_s)), "ensemble and sequential runs differ"
    th_g, h_g = C.gradient_descent(w, observed, steps, iterations=5, lr=0.05, decay=0.7, theta0=base,
                                   stream=stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    it = len(h_e)
    return {
        "metric": "calibration search: seconds per iteration (5 parameter sets in one ensemble)",
        "value": (t1 - t0) / it, "unit": "s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": 1e3 * (t1 - t0) / (it * steps), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "calibration_search_grid10x10_case1", "vehicles": w.n_vehicles, "sets": 5,
                   "iterations": it, "hidden_abTs0": hidden.tolist(), "start_abTs0": base.tolist(),
                   "random_search": {"abTs0": th_e.tolist(),
                                     "mean_diff_mph": [h["mean_diff_mps"] / C.MPH for h in h_e],
                                     "s": t1 - t0},
                   "sequential_handles_s": t2 - t1, "ensemble_speedup": (t2 - t1) / (t1 - t0),
                   "gradient_descent": {"abTs0": th_g.tolist(),
                                        "mean_diff_mph": [h["mean_diff_mps"] / C.MPH for h in h_g],
                                        "s": t3 - t2}},
    }


def bench_metro_scale(args, M, torch, stream):
    """Config 2 at metropolitan size: 16 copies of the perturbed grid + ring
    and its 200,000-vehicle demand in one ensemble handle -- 3.2M vehicles on
    572,800 edges, the sizes of the metropolitan config -- over the same 3 h.
    Measures the step where tiles no longer fit in one round of resident
    workgroups: vehicle-updates/s from the graph path, and the tile kernel
    against the HBM roofline (48 B per vehicle-update) from the event pass."""
    import workloads as W
    copies = 16
    w = W.config2()
    steps = args.steps if args.steps_given else w.n_steps
    n = int(w.depart_step.shape[0])
    scen = [(n, np.zeros(0, np.int32))] * copies
    warm = M.Sim(w, scenarios=scen, stream=stream)
    warm.step(args.warmup)
    warm.close()
    sim = M.Sim(w, scenarios=scen, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    done = 0
    chunk = 2400
    while done < steps:                           # progress lines for long runs
        k = min(chunk, steps - done)
        sim.step(k)
        done += k
        if args.progress:
            torch.cuda.synchronize()
            print(f"graph pass: {done}/{steps}", file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    upd = sim.counters()["active_sum"]
    sim.close()
    ev = M.Sim(w, scenarios=scen, stream=stream)
    kernel_ms, tot = {}, 0.0
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        kms, t = ev.step_timed(k)
        for key, v in kms.items():
            kernel_ms[key] = kernel_ms.get(key, 0.0) + v
        tot += t
        done += k
        if args.progress:
            print(f"event pass: {done}/{steps}", file=sys.stderr, flush=True)
    big = ev.big_tile_updates()
    assert ev.counters()["active_sum"] == upd
    ev.close()
    tile_ms = kernel_ms["k_tile_step"]
    achieved = BYTES_PER_UPDATE * (upd - big) / (tile_ms / 1e3) / 1e9
    return {
        "metric": "vehicle-updates/sec (1 GPU)", "value": upd / (ms / 1e3), "unit": "vehicle-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "perturbed_grid_ring_x16", "copies": copies, "vehicles": n * copies,
                   "edges": w.net.n_edges * copies, "steps": steps, "vehicle_updates": int(upd)},
        "roofline": {"bound": "hbm", "kernel": "k_tile_step", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "us_per_launch": 1e3 * tile_ms / steps, "big_tile_updates": big},
        "kernel_us_per_step": {k: round(1e3 * v / steps, 3) for k, v in kernel_ms.items()},
        "event_path_ms_per_step": tot / steps,
    }


def bench_reroute(args, M, torch, stream):
    """Routes on travel times for every vehicle of config 2 (200,000 O/D
    pairs, about 9,900 distinct destinations, 10,040 nodes): edge costs are the
    mean traversal times after 1.5 h of the plain run (free-flow time where
    nothing traversed); sim_shortest_routes on the GPU, timed end to end (host
    copies included), against the oracle's routing on a sample of pairs."""
    import workloads as W
    w = W.config2()
    sim = M.Sim(w, stream=stream)
    sim.step(10800)
    mean, cnt = sim.mean_travel_times()
    sim.close()
    net = w.net
    cost = np.where(cnt > 0, mean, net.length / net.limit).astype(np.float32)
    o = net.edge_from[w.route_edges[w.route_off[:-1]]].astype(np.int32)
    d = net.edge_to[w.route_edges[w.route_off[1:] - 1]].astype(np.int32)
    M.shortest_routes(net, cost, o[:1000], d[:1000])           # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    off, edges = M.shortest_routes(net, cost, o, d)
    t1 = time.perf_counter()
    changed = sum(1 for q in range(0, o.size, 97)
                  if not np.array_equal(edges[off[q]:off[q + 1]], w.route_edges[w.route_off[q]:w.route_off[q + 1]]))
    line = {
        "metric": "routes/s (sim_shortest_routes, 1 GPU)", "value": o.size / (t1 - t0), "unit": "routes/s",
        "n_gpus": 1, "steps": 10800, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "reroute_perturbed_grid_ring", "queries": int(o.size),
                   "destinations": int(np.unique(d).size), "nodes": int(net.n_nodes), "edges": int(net.n_edges),
                   "route_edges": int(edges.size), "s": t1 - t0,
                   "changed_vs_free_flow_routes_sampled": changed / len(range(0, o.size, 97))},
    }
    if args.cpu_steps > 0:
        import oracle
        k = 12
        t2 = time.perf_counter()
        for q in range(k):
            r = oracle.route(net, cost, int(o[q]), int(d[q]))
            assert r == edges[off[q]:off[q + 1]].tolist()
        t3 = time.perf_counter()
        line["cpu_baseline"] = {"value": k / (t3 - t2), "unit": "routes/s", "cores": 1, "kind": "oracle",
                                "sample": f"the first {k} O/D pairs (one O(V^2) Dijkstra each), same routes"}
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="metro",
                    choices=["metro", "perturbed_grid_ring", "grid10x10", "ensemble", "calibration",
                             "calibration_search", "metro_scale", "reroute", "probe_r", "reroute_metro"])
    ap.add_argument("--start", type=int, default=-1,
                    help="plain workloads: step of the written start state (default: 08:00, the demand peak)")
    ap.add_argument("--reps", type=int, default=2, help="calibration: timed repetitions after one warm-up")
    ap.add_argument("--scenarios", type=int, default=64, help="ensemble: number of scenarios")
    ap.add_argument("--tune-at", type=int, default=3000, help="ensemble: step at which the schedule is tuned")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="plain workloads: most steps the oracle times (0: skip); reroute: on if > 0")
    ap.add_argument("--intersection-mode", type=int, default=0, choices=[0, 1],
                    help="0: all green (case 2); 1: flashing red at every node (case 1)")
    ap.add_argument("--v0-spread", type=float, default=0.0,
                    help="per-driver free-flow speed spread (sigma_s / limit; drivers drawn at 2 sigma_s)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="skip the graph-replayed pass (hardware-counter runs); value then comes from the "
                         "kernel-by-kernel pass")
    ap.add_argument("--progress", type=int, default=0, metavar="STEPS",
                    help="print a line every STEPS steps (for profiler runs; adds synchronizations)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of this many MiB before the timed region "
                         "(a known-size reference for hardware byte counters)")
    ap.add_argument("--summarize-pmc", metavar="DIR", help="summarize a rocprofv3 --pmc csv directory and exit")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="summarize a rocprofv3 --kernel-trace csv directory (see --last) and exit")
    ap.add_argument("--last", type=int, default=0, help="--summarize-trace / --summarize-pmc: the mean of each "
                                                         "kernel's last LAST dispatches")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_JSON", "WRITE_JSON"),
                    help="combine two --summarize-pmc outputs into the traffic record and exit")
    ap.add_argument("--probe-from", nargs=2, metavar=("FETCH_JSON", "WRITE_JSON"),
                    help="--traffic-from: the summaries that hold the copy probe, if not those two")
    args = ap.parse_args()
    args.steps_given = "--steps" in sys.argv
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(args.summarize_pmc, args.last), indent=1))
        return
    if args.summarize_trace:
        print(json.dumps(summarize_trace(args.summarize_trace, args.last), indent=1))
        return
    if args.traffic_from:
        print(json.dumps(traffic_from(*args.traffic_from, probe_mib=args.copy_probe or 256,
                                      workload=args.workload, probe_jsons=args.probe_from), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the simulation is single-device; "
              "sharding it by edges over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2007_03614_amd as M

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload == "ensemble":
        print(json.dumps(bench_ensemble(args, M, torch, stream)), flush=True)
        return
    if args.workload == "calibration":
        print(json.dumps(bench_calibration(args, M, torch, stream)), flush=True)
        return
    if args.workload == "reroute":
        print(json.dumps(bench_reroute(args, M, torch, stream)), flush=True)
        return
    if args.workload == "metro_scale":
        print(json.dumps(bench_metro_scale(args, M, torch, stream)), flush=True)
        return
    if args.workload == "reroute_metro":
        print(json.dumps(bench_reroute_metro(args, M, torch, stream)), flush=True)
        return
    if args.workload == "probe_r":
        print(json.dumps(bench_probe_r(args, M, torch, stream)), flush=True)
        return
    if args.workload == "calibration_search":
        print(json.dumps(bench_calibration_search(args, M, torch, stream)), flush=True)
        return
    print(json.dumps(bench_plain(args, M, torch, stream)), flush=True)


def _window(sim, M, torch, stream, steps, progress, kernels_only):
    """`steps` steps from the handle's current state, twice: on the graph path
    between two HIP events, then (state restored) kernel by kernel between HIP
    events.  Returns (graph ms or None, vehicle-updates, per-kernel ms, event
    path ms, big-tile updates, state at the end)."""
    start_state = sim.state()
    before = int(start_state["counters"][0])
    # both passes start from the written state (with flashing-red intersections a written state
    # restarts the round-robin, so a pass that continued the run could take other decisions)
    sim.write_state(start_state)
    total_ms = None
    if not kernels_only:                     # counter runs: the event-timed pass below is enough
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        if progress:                         # profiling runs only: these syncs cost time
            for k0 in range(0, steps, progress):
                sim.step(min(progress, steps - k0))
                torch.cuda.synchronize()
                print(f"graph path: step {k0 + min(progress, steps - k0)}", flush=True)
        else:
            sim.step(steps)                  # the production path: captured graphs of 8 steps
        e1.record(stream)
        torch.cuda.synchronize()
        total_ms = e0.elapsed_time(e1)
    end_state = sim.state()
    upd = int(end_state["counters"][0]) - before
    sim.write_state(start_state)
    big0 = sim.big_tile_updates()
    if progress:
        kernel_ms, event_ms = None, 0.0
        for k0 in range(0, steps, progress):
            km, tm = sim.step_timed(min(progress, steps - k0))
            kernel_ms = km if kernel_ms is None else {k: kernel_ms[k] + km[k] for k in km}
            event_ms += tm
            print(f"event path: step {k0 + min(progress, steps - k0)}", flush=True)
    else:
        kernel_ms, event_ms = sim.step_timed(steps)
    upd_t = sim.counters()["active_sum"] - before
    big = sim.big_tile_updates() - big0
    if kernels_only:
        upd, total_ms, end_state = upd_t, event_ms, sim.state()
    assert upd_t == upd, (upd_t, upd)
    return total_ms, upd, kernel_ms, event_ms, big, end_state


def bench_reroute_metro(args, M, torch, stream):
    """Routes of the metropolitan demand on the GPU: every one of its 3.2M
    trips routed by sim_shortest_routes on free-flow costs (224,202 nodes,
    16,321 distinct destinations, labels in device memory), timed end to end
    (host copies included).  The CPU side is the generator's multithreaded
    Dijkstra (per destination) on a sample of the trips."""
    import workloads as W
    w = W.config3()
    net = w.net
    cost = (net.length / net.limit).astype(np.float32)
    o = net.edge_from[w.route_edges[w.route_off[:-1]]].astype(np.int32)
    d = net.edge_to[w.route_edges[w.route_off[1:] - 1]].astype(np.int32)
    M.shortest_routes(net, cost, o[:2000], d[:2000])            # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    off, edges = M.shortest_routes(net, cost, o, d)
    t1 = time.perf_counter()
    line = {
        "metric": "routes/s (sim_shortest_routes, 1 GPU)", "value": o.size / (t1 - t0), "unit": "routes/s",
        "n_gpus": 1, "steps": 0, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "reroute_metro", "queries": int(o.size), "destinations": int(np.unique(d).size),
                   "nodes": int(net.n_nodes), "edges": int(net.n_edges), "route_edges": int(edges.size),
                   "s": t1 - t0},
    }
    if args.cpu_steps > 0:
        k = 200_000
        t2 = time.perf_counter()
        W.shortest_routes_to(net, o[:k], d[:k])
        t3 = time.perf_counter()
        line["cpu_baseline"] = {"value": k / (t3 - t2), "unit": "routes/s", "cores": min(16, os.cpu_count() or 1),
                                "kind": "generator Dijkstra (per destination, binary heap, FP64 costs)",
                                "sample": f"the first {k} trips", **cpu_info()}
    return line


def bench_probe_r(args, M, torch, stream):
    """Roofline probe: the metropolitan network 8 times over in one ensemble
    handle, every lane filled in steady state at 30 % of jam density (about
    46M vehicles, every one active), so that the step's data (about 1.3 GB of
    vehicle records read and written per step) cannot stay in the 256 MB
    last-level cache.  The state is written, `warmup` steps run untimed, then
    `steps` steps are timed on the graph path and again kernel by kernel."""
    import workloads as W
    t0 = time.perf_counter()
    copies = 8
    w, st = W.probe_r(density=0.3)
    n = w.n_vehicles
    scen = [(n, np.zeros(0, np.int32))] * copies
    print(f"probe R: {copies} x {n} vehicles on {copies} x {w.net.n_edges} edges "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 0.5, out=dst)
        torch.cuda.synchronize()
        del src, dst
    sim = M.Sim(w, scenarios=scen, stream=stream)
    sim.write_state(W.replicate_state(st, w.net.n_edges, copies))
    print(f"handle created and state written ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    active0 = sim.n_active
    total_ms, upd, kernel_ms, event_ms, big_upd, _ = _window(sim, M, torch, stream, args.steps, args.progress,
                                                               args.kernels_only)
    sim.close()
    tile_ms = kernel_ms["k_tile_step"]
    achieved = BYTES_PER_UPDATE * (upd - big_upd) / (tile_ms / 1e3) / 1e9
    return {
        "metric": "vehicle-updates/sec (1 GPU)", "value": upd / (total_ms / 1e3), "unit": "vehicle-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "probe_r", "copies": copies, "vehicles": n * copies,
                   "edges": w.net.n_edges * copies, "density": 0.3, "active_at_timed_start": int(active0),
                   "steps": args.steps, "vehicle_updates": int(upd)},
        "roofline": {"bound": "hbm", "kernel": "k_tile_step", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic("probe_r"),
                     "bytes_per_update": BYTES_PER_UPDATE, "us_per_launch": 1e3 * tile_ms / args.steps,
                     "big_tile_updates": big_upd},
        "kernel_us_per_step": {k: round(1e3 * v / args.steps, 3) for k, v in kernel_ms.items()},
        "event_path_ms_per_step": event_ms / args.steps,
    }


def bench_plain(args, M, torch, stream):
    """The plain step on one workload, timed at 08:00, the peak of its
    demand.  The run starts at the workload's first step and is stepped
    untimed on the graph path to 08:00 (setup); `warmup` steps follow untimed,
    then `steps` steps are timed with HIP events on the handle's stream, and
    the same window runs again kernel by kernel for per-kernel times.

    The oracle cannot reach 08:00 of the metropolitan run in a bench's time,
    so the CPU baseline and the parity check of a timed window start from the
    08:00 state built from the demand (workloads.loaded_state), written into
    both the oracle and a GPU handle: the oracle runs `warmup` + min(steps,
    cpu_steps) steps on one thread and on every thread, and its counters and
    end state are compared with the GPU's over the same steps."""
    import workloads as W
    t_setup = time.perf_counter()
    w = make_workload(args.workload)
    w.params.v0_spread = args.v0_spread
    w.params.intersection_mode = args.intersection_mode
    start = PEAK_STEP[args.workload] if args.start < 0 else args.start
    print(f"{args.workload}: {w.n_vehicles} vehicles, {w.net.n_edges} edges "
          f"({time.perf_counter() - t_setup:.1f} s)", file=sys.stderr, flush=True)
    if args.copy_probe > 0:
        # a plain streaming kernel of known size: reads MIB MiB, writes MIB MiB
        # (torch's elementwise add; a device-to-device copy_ would use the DMA engine)
        src = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 0.5, out=dst)
        torch.cuda.synchronize()
        del src, dst

    sim = M.Sim(w, stream=stream)
    t_ff = time.perf_counter()
    done = 0
    while done < start:                      # untimed: the run from its first step to 08:00
        k = min(2400, start - done)
        sim.step(k)
        done += k
        if args.progress:
            torch.cuda.synchronize()
            print(f"run to 08:00: step {done}", flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    active0 = sim.n_active
    print(f"run to step {start} + {args.warmup} warm-up steps: {active0} active "
          f"({time.perf_counter() - t_ff:.1f} s)", file=sys.stderr, flush=True)
    total_ms, upd, kernel_ms, event_ms, big_upd, _ = _window(sim, M, torch, stream, args.steps, args.progress,
                                                               args.kernels_only)
    value = upd / (total_ms / 1e3)

    # roofline of k_tile_step: 28 algorithmic bytes per vehicle-update it does
    # (all but those in tiles above one workgroup's LDS) over its event time
    tile_ms = kernel_ms["k_tile_step"]
    achieved = BYTES_PER_UPDATE * (upd - big_upd) / (tile_ms / 1e3) / 1e9
    traffic = stored_traffic(args.workload, args.v0_spread, args.intersection_mode)
    clock0 = {"metro": 5.0, "perturbed_grid_ring": 6.5}.get(args.workload)
    hh = None if clock0 is None else clock0 + start * 0.5 / 3600
    line = {
        "metric": "vehicle-updates/sec (1 GPU)",
        "value": value,
        "unit": "vehicle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "vehicles": w.n_vehicles, "edges": w.net.n_edges,
                   "lanes": int(w.net.lanes.sum()), "dt_s": 0.5,
                   "timed_from_step": start + args.warmup,
                   **({"clock": f"{int(hh):02d}:{int(round(hh % 1 * 60)):02d}"} if hh is not None else {}),
                   "active_at_timed_start": int(active0), "steps": args.steps,
                   "vehicle_updates": int(upd), **({"v0_spread": args.v0_spread} if args.v0_spread else {}),
                   **({"intersection_mode": 1} if args.intersection_mode else {})},
        "roofline": {"bound": "hbm", "kernel": "k_tile_step", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_update": BYTES_PER_UPDATE, "us_per_launch": 1e3 * tile_ms / args.steps,
                     "big_tile_updates": big_upd},
        "kernel_us_per_step": {k: round(1e3 * v / args.steps, 3) for k, v in kernel_ms.items()},
        "event_path_ms_per_step": event_ms / args.steps,
    }
    if args.cpu_steps > 0:
        k = min(args.steps, args.cpu_steps)
        state0, info = W.loaded_state(w, start, speed_frac=SPEED_FRAC)
        one, _, _ = cpu_baseline(w, state0, args.warmup, k, 1)
        allc, oc, os_ = cpu_baseline(w, state0, args.warmup, k, 0)
        sample = (f"{k} steps after {args.warmup} from the 08:00 state built from the demand "
                  f"({info['active']} active, mean speed {SPEED_FRAC} x limit; "
                  f"{allc['vehicle_updates']} vehicle-updates)")
        line["cpu_baseline"] = {"value": allc["value"], "unit": "vehicle-updates/s", "cores": allc["cores"],
                                "kind": "oracle", "sample": sample,
                                "single_thread": {"value": one["value"], "cores": 1, "s": one["s"]},
                                "all_threads_s": allc["s"], **cpu_info()}
        # the same steps on the GPU from the same written state: its rate
        # beside the oracle's, and the window's parity (counters exact,
        # discrete state bit for bit, x and v within 1e-5 relative)
        sim.write_state(dict(state0, counters=np.zeros(len(M.COUNTERS), np.int64)))
        sim.step(args.warmup)
        torch.cuda.synchronize()
        g_ms, g_upd, _, _, _, g_end = _window(sim, M, torch, stream, k, 0, False)
        gc = dict(zip(M.COUNTERS, g_end["counters"].tolist()))
        same = all(np.array_equal(g_end[q], os_[q].astype(g_end[q].dtype))
                   for q in ("status", "edge", "lane", "cursor", "held_since", "mand", "ww"))
        rel = max(float(np.max(np.abs(g_end[q].astype(np.float64) - os_[q].astype(np.float64))
                               / np.maximum(np.abs(os_[q].astype(np.float64)), 1.0), initial=0.0))
                  for q in ("x", "v"))
        line["built_state_window"] = {"gpu_value": g_upd / (g_ms / 1e3), "vehicle_updates": g_upd,
                                      "counters_equal": gc == oc, "discrete_state_equal": bool(same),
                                      "max_rel_xv": rel}
    sim.close()
    return line


if __name__ == "__main__":
    main()
