"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle, built with gcc -fsanitize=address,undefined, runs a case-1 run
  with 4 classes and the adjoint replay, a run from a built metropolitan
  state, and a route.
* libmanta.so, built with the host half of hipcc under the same sanitizers
  (the device code is not instrumented), runs every host-side check of
  sim_create, sim_create_ensemble and sim_shortest_routes on invalid inputs,
  and the allocator hook; with no GPU here each valid input stops at the
  first device allocation with SIM_ENOMEM.
Each runs in a child process with the sanitizer runtime preloaded; a report
fails the test."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_HOST = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer".split()

ORACLE_RUN = r'''
import sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle, workloads as W
lib = oracle._load(LIBPATH)
oracle.lib = lambda fp64=False: lib
w = W.config1(n_vehicles=600, n_steps=900, n_classes=4)
w.params.intersection_mode = 1
w.params.v0_spread = 0.05
o = oracle.OracleSim(w)
o.enable_record()
o.step(900)
loss, mean, g = o.replay(o.theta(w), np.zeros(w.net.n_edges), None, grad=True)
assert np.isfinite(g).all()
w2 = W.config3(n_vehicles=5000, rows=25, cols=26, pool_size=200, cache=False)
s, _ = W.loaded_state(w2, 21600)
o2 = oracle.OracleSim(w2)
o2.write_state(21600, s)
o2.step(100)
assert o2.counters()["active_sum"] > 0
assert len(oracle.route(w.net, (w.net.length / w.net.limit).astype(np.float32), 0, 99)) > 0
print("oracle ok")
'''

LIB_RUN = r'''
import copy, sys
sys.path.insert(0, PKGROOT)
sys.path.insert(1, ROOT)
import numpy as np
import workloads as W
import paper_2007_03614_amd as M
assert M.LIB_PATH.startswith(PKGROOT), M.LIB_PATH
base = W.config1(n_vehicles=50)

def status(w, **kw):
    try:
        M.Sim(w, allocator="hip", **kw)
    except M.SimError as e:
        return e.name
    return "SIM_OK"

def mutate(f):
    w = copy.deepcopy(base)
    f(w)
    return w

cases = [
    lambda w: w.net.lanes.__setitem__(3, 0),
    lambda w: w.net.length.__setitem__(5, 19.5),
    lambda w: w.net.limit.__setitem__(2, -1.0),
    lambda w: w.route_edges.__setitem__(int(w.route_off[1]) - 1, 0),
    lambda w: w.depart_step.__setitem__(0, -3),
    lambda w: w.vclass.__setitem__(0, 9),
    lambda w: w.alpha.__setitem__(0, 0.9),
    lambda w: setattr(w.params, "T", np.array([5.0], np.float32)),
    lambda w: setattr(w.params, "dt", 0.0),
]
for k, f in enumerate(cases):
    got = status(mutate(f))
    assert got in ("SIM_EINVAL", "SIM_EUNSUPPORTED"), (k, got)
# a valid input gets through every check and stops at the first device allocation
assert status(base) in ("SIM_ENOMEM", "SIM_EDEVICE"), status(base)
assert status(base, scenarios=[(50, np.array([1, 2], np.int32)), (30, np.zeros(0, np.int32))]) in \
    ("SIM_ENOMEM", "SIM_EDEVICE")
# (the no-allocation form resolves its device region first: no device here)
for fn, ok in ((M.shortest_routes, ("SIM_EINVAL",)), (M.shortest_routes_noalloc, ("SIM_EINVAL", "SIM_EDEVICE"))):
    try:
        fn(base.net, np.full(base.net.n_edges, -1.0, np.float32), np.array([0], np.int32), np.array([5], np.int32))
        raise AssertionError("negative cost accepted")
    except M.SimError as e:
        assert e.name in ok, e.name
M.use_hip_allocator()
print("library ok")
'''


def _run(code, env_extra, **subst):
    for k, v in subst.items():
        code = code.replace(k, repr(v))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               **env_extra)
    r = subprocess.run([sys.executable, "-c", code.replace("ROOT", repr(ROOT))], capture_output=True, text=True,
                       env=env, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "Sanitizer" not in out and "runtime error" not in out, out[-3000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "manta_oracle.c"), "-o", so, "-lm"])
    pre = " ".join(subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
                   for n in ("libasan.so", "libubsan.so"))
    out = _run(ORACLE_RUN, {"LD_PRELOAD": pre}, LIBPATH=so)
    assert "oracle ok" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no clang sanitizer runtime or hipcc")
    pkg = tmp_path / "pkg"
    shutil.copytree(os.path.join(ROOT, "paper_2007_03614_amd"), pkg / "paper_2007_03614_amd",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
             "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN_HOST
    subprocess.check_call(["/opt/rocm/bin/hipcc", *flags, "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "paper_2007_03614_amd", "csrc", "manta.hip"),
                           "-o", str(pkg / "paper_2007_03614_amd" / "libmanta.so")],
                          stderr=subprocess.DEVNULL)
    out = _run(LIB_RUN, {"LD_PRELOAD": rt[0]}, PKGROOT=str(pkg))
    assert "library ok" in out
