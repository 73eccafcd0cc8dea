"""Host-side parts of bench.py: the one-GPU refusal, the arithmetic that turns
two hardware-counter summaries (FETCH_SIZE, WRITE_SIZE in KiB per dispatch)
into HBM bytes per step with the copy probe's scale, and the rule that a
stored counter record only counts for the kernel sources it was taken on."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PROBE = "void at::native::vectorized_elementwise_kernel<4, at::native::AddFunctor<float> >(int, float*)"
TILE = "k_tile_step(Dev)"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _pmc_dir(tmp_path, name, counter, rows):
    d = tmp_path / name / "host" / "pid"
    d.mkdir(parents=True)
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kernel, value in rows:
            w.writerow({"Kernel_Name": kernel, "Grid_Size": 256000, "Counter_Name": counter, "Counter_Value": value})
    return str(tmp_path / name)


def test_traffic_from_counter_summaries(tmp_path):
    # fetch counts half the probe's bytes (scale 2), write counts all of them
    fdir = _pmc_dir(tmp_path, "fetch", "FETCH_SIZE",
                    [(PROBE, 128 * 1024.0), (TILE, 5000.0), (TILE, 7000.0)])
    wdir = _pmc_dir(tmp_path, "write", "WRITE_SIZE", [(PROBE, 256 * 1024.0), (TILE, 1500.0), (TILE, 2500.0)])
    fs, ws = bench.summarize_pmc(fdir), bench.summarize_pmc(wdir)
    assert fs["kernels"][TILE] == {"dispatches": 2, "FETCH_SIZE": 6000.0}
    fj, wj = tmp_path / "f.json", tmp_path / "w.json"
    fj.write_text(json.dumps(fs))
    wj.write_text(json.dumps(ws))
    tr = bench.traffic_from(str(fj), str(wj), probe_mib=256)
    assert tr["fetch_scale"] == 2.0 and tr["write_scale"] == 1.0
    assert tr["bytes_per_step"] == 1024.0 * (6000.0 * 2.0 + 2000.0 * 1.0)
    assert tr["sources"] == bench.kernel_source_digest()


def test_stored_traffic_needs_the_same_sources_and_workload(tmp_path):
    rec = {"workload": "perturbed_grid_ring", "sources": bench.kernel_source_digest(), "bytes_per_step": 123.0}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    assert bench.stored_traffic("perturbed_grid_ring", path=str(p)) == 123.0
    assert bench.stored_traffic("grid10x10", path=str(p)) is None
    assert bench.stored_traffic("perturbed_grid_ring", v0_spread=0.05, path=str(p)) is None
    assert bench.stored_traffic("perturbed_grid_ring", intersection_mode=1, path=str(p)) is None
    p.write_text(json.dumps(dict(rec, sources="0" * 16)))
    assert bench.stored_traffic("perturbed_grid_ring", path=str(p)) is None
    assert bench.stored_traffic("perturbed_grid_ring", path=str(tmp_path / "missing.json")) is None


def test_committed_records_are_well_formed():
    """Each committed record: counters of k_tile_step on the workload its file
    is named for, probe scales near what a plain add reads and writes, and
    bytes per step that follow from the two counters and their scales."""
    import glob
    files = glob.glob(os.path.join(ROOT, "profiles", "tile_kernels_traffic_*.json"))
    for fn in files:
        with open(fn) as f:
            tr = json.load(f)
        assert fn == bench.traffic_file(tr["workload"]) and tr["kernels"] == ["k_tile_step"]
        assert len(tr["sources"]) == 16
        assert 0.9 <= tr["write_scale"] <= 1.1 and 0.9 <= tr["fetch_scale"] / 2.0 <= 1.1
        assert tr["bytes_per_step"] == pytest.approx(
            1024.0 * (tr["fetch_kib_per_dispatch"]["k_tile_step"] * tr["fetch_scale"]
                      + tr["write_kib_per_dispatch"]["k_tile_step"] * tr["write_scale"]), rel=1e-12)
        assert tr["bytes_per_step"] > 0.0


def test_cpu_info_names_the_host():
    info = bench.cpu_info()
    assert info["nproc"] >= 1 and isinstance(info["cpu_model"], str)


def test_summarize_trace_means_and_last_window(tmp_path):
    d = tmp_path / "tr" / "host"
    d.mkdir(parents=True)
    with open(d / "x_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        # five dispatches (listed out of start order) and one of another kernel
        for k, us in [(3, 3), (0, 1), (4, 5), (1, 2), (2, 4)]:
            w.writerow({"Kernel_Name": TILE, "Start_Timestamp": 1000 * k * 10, "End_Timestamp": 1000 * (k * 10 + us)})
        w.writerow({"Kernel_Name": "k_commit(Dev)", "Start_Timestamp": 0, "End_Timestamp": 7000})
    out = bench.summarize_trace(str(tmp_path / "tr"), last=2)
    t = out["kernels"][TILE]
    assert t["dispatches"] == 5 and t["mean_us"] == 3.0 and t["mean_us_last_2"] == 4.0   # in start order: 1 2 4 3 5
    assert out["kernels"]["k_commit(Dev)"]["mean_us_last_1"] == 7.0
