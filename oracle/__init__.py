"""CPU oracle for the per-timestep vehicle update (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does: it shares
no code with the oracle, which is written separately from the paper's model
(IDM, Eq. (1); mandatory lane change, Eq. (2); gap acceptance, Eqs. (3)-(4);
case-2 intersections, Sec. II-D) in plain C (``manta_oracle.c``).

Two builds of the same source:
  * ``liboracle32.so`` — FP32, operation order of the step contract, no
    contraction: the parity oracle;
  * ``liboracle64.so`` — the FP64 twin, used only to report FP32 drift.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "manta_oracle.c")
LIB32 = os.path.join(_HERE, "liboracle32.so")
LIB64 = os.path.join(_HERE, "liboracle64.so")

COUNTERS = ["active_sum", "departed", "arrived", "lane_changes", "transfers", "holds",
            "insert_denied", "mand_triggers", "stop_branch", "clamp", "wrong_lane_holds",
            "waived_exits", "gridlock_steps"]
EV = dict(REQ=1, WIN=2, ARRIVE=4, WHOLD=8, CLAMP=16, STOPB=32, ELIG=64, INSERT_REQ=128,
          MOVED=256, MAND_TRIG=512)
KIND = dict(FREE=0, VEH=1, STOP=2, LOOK=3)

_CFLAGS = ["-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fno-unsafe-math-optimizations"]


def build(force: bool = False) -> None:
    """Compile both oracle builds with gcc (x86-64 SSE2 arithmetic, no FMA)."""
    for out, extra in ((LIB32, []), (LIB64, ["-DREAL=double", "-DORACLE_FP64"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp"
            subprocess.check_call(["gcc", *_CFLAGS, *extra, _SRC, "-o", tmp, "-lm"])
            os.replace(tmp, out)


def _load(path):
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    P, I32, I64, U64, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                           ctypes.c_double)
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [I32, I32, P, P, P, P, P, P, P, P, I32, P, P, P, P, P, I32,
                               P, P, P, P, P, P, ctypes.c_float, U64]
    lib.orc_destroy.argtypes = [P]
    lib.orc_step.argtypes = [P, I32]
    lib.orc_time.argtypes = [P]
    lib.orc_time.restype = I32
    lib.orc_read_state.argtypes = [P] + [P] * 11
    lib.orc_write_state.argtypes = [P, I32] + [P] * 11
    lib.orc_counters.argtypes = [P, P]
    lib.orc_edge_stats.argtypes = [P, P, P]
    lib.orc_last_events.argtypes = [P] + [P] * 7
    lib.orc_last_partner.argtypes = [P, P]
    lib.orc_real_bytes.restype = I32
    lib.orc_set_threads.argtypes = [I32]
    lib.orc_set_threads.restype = I32
    lib.orc_set_threads(1)          # one thread unless asked: test runners start many processes
    lib.orc_enable_record.argtypes = [P]
    lib.orc_enable_record.restype = I32
    lib.orc_replay.argtypes = [P, P, P, P, P, P]
    lib.orc_replay.restype = D
    lib.orc_philox4x64.argtypes = [P, P, P]
    lib.orc_expf_c_batch.argtypes = [P, P, I64]
    lib.orc_mand_trigger.argtypes = [U64, I64, I64, D]
    lib.orc_mand_trigger.restype = I32
    lib.orc_idm_d.argtypes = [D, D, D, D, D, D, D, D, I32, P]
    lib.orc_idm_d.restype = D
    lib.orc_crit_gap_d.argtypes = [D, D, D, D, D]
    lib.orc_crit_gap_d.restype = D
    lib.orc_desired_gap_d.argtypes = [D]
    lib.orc_desired_gap_d.restype = D
    lib.orc_uniform_d.argtypes = [U64, I64, I64, I32]
    lib.orc_uniform_d.restype = D
    lib.orc_normal_d.argtypes = [U64, I64, I64, I32]
    lib.orc_normal_d.restype = D
    lib.orc_set_v0_spread.argtypes = [P, ctypes.c_float]
    lib.orc_route.argtypes = [I32, I32, P, P, P, I32, I32, P, I32]
    lib.orc_route.restype = I32
    lib.orc_route_dist.argtypes = [I32, I32, P, P, P, I32, P]
    lib.orc_set_intersection_mode.argtypes = [P, I32]
    lib.orc_set_intersection_mode.restype = I32
    lib.orc_driver_limit_d.argtypes = [U64, I64, I64, ctypes.c_float, ctypes.c_float]
    lib.orc_driver_limit_d.restype = D
    return lib


@functools.lru_cache(maxsize=2)
def lib(fp64: bool = False):
    return _load(LIB64 if fp64 else LIB32)


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class OracleSim:
    """One simulation held by the C oracle."""

    def __init__(self, w, fp64: bool = False):
        self._lib = lib(fp64)
        self.fp64 = fp64
        self.n = w.n_vehicles
        self.n_edges = w.net.n_edges
        net, p = w.net, w.params
        self._keep = [
            _c(net.edge_from, np.int32), _c(net.edge_to, np.int32), _c(net.length, np.float32),
            _c(net.limit, np.float32), _c(net.lanes, np.uint8), _c(net.conn_off, np.int32),
            _c(net.conn_to, np.int32), _c(net.conn_mask, np.uint8), _c(w.route_off, np.int64),
            _c(w.route_edges, np.int32), _c(w.depart_step, np.int32), _c(w.vclass, np.uint8),
            _c(w.alpha, np.float32), _c(p.v0_factor, np.float32), _c(p.T, np.float32),
            _c(p.a, np.float32), _c(p.b, np.float32), _c(p.s0, np.float32), _c(p.veh_len, np.float32)]
        k = self._keep
        self._h = self._lib.orc_create(net.n_nodes, net.n_edges, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]),
                                       _p(k[4]), _p(k[5]), _p(k[6]), _p(k[7]), self.n, _p(k[8]),
                                       _p(k[9]), _p(k[10]), _p(k[11]), _p(k[12]), p.n_classes,
                                       _p(k[13]), _p(k[14]), _p(k[15]), _p(k[16]), _p(k[17]),
                                       _p(k[18]), float(p.dt), int(p.seed))
        if not self._h:
            raise MemoryError("oracle create failed")
        if getattr(p, "v0_spread", 0.0):
            self._lib.orc_set_v0_spread(self._h, float(p.v0_spread))
        if getattr(p, "intersection_mode", 0):
            if self._lib.orc_set_intersection_mode(self._h, int(p.intersection_mode)) != 0:
                raise ValueError("case 1 intersections need at most 64 (in, out) pairs per node")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def step(self, n: int = 1) -> None:
        self._lib.orc_step(self._h, int(n))

    @property
    def t(self) -> int:
        return int(self._lib.orc_time(self._h))

    def state(self) -> dict:
        n = self.n
        s = dict(status=np.empty(n, np.uint8), edge=np.empty(n, np.int32), lane=np.empty(n, np.int32),
                 cursor=np.empty(n, np.int32), x=np.empty(n, np.float64), v=np.empty(n, np.float64),
                 held_since=np.empty(n, np.int32), mand=np.empty(n, np.uint8), ww=np.empty(n, np.int32),
                 tau_in=np.empty(n, np.float64), t_arr=np.empty(n, np.float64))
        self._lib.orc_read_state(self._h, *[_p(s[k]) for k in ("status", "edge", "lane", "cursor", "x", "v",
                                                                 "held_since", "mand", "ww", "tau_in",
                                                                 "t_arr")])
        if not self.fp64:
            s["x"] = s["x"].astype(np.float32)
            s["v"] = s["v"].astype(np.float32)
        s["t"] = self.t
        return s

    def write_state(self, t: int, s: dict) -> None:
        a = [_c(s["status"], np.uint8), _c(s["edge"], np.int32), _c(s["lane"], np.int32),
             _c(s["cursor"], np.int32), _c(s["x"], np.float64), _c(s["v"], np.float64),
             _c(s["held_since"], np.int32), _c(s["mand"], np.uint8), _c(s["ww"], np.int32),
             _c(s["tau_in"], np.float64),
             _c(s["t_arr"], np.float64) if s.get("t_arr") is not None else None]
        self._lib.orc_write_state(self._h, int(t), *[_p(q) for q in a])

    def counters(self) -> dict:
        c = np.empty(len(COUNTERS), np.int64)
        self._lib.orc_counters(self._h, _p(c))
        return dict(zip(COUNTERS, c.tolist()))

    def edge_stats(self):
        s = np.empty(self.n_edges, np.float64)
        c = np.empty(self.n_edges, np.int64)
        self._lib.orc_edge_stats(self._h, _p(s), _p(c))
        return s, c

    def enable_record(self) -> None:
        """Record every discrete decision from step 0 on (differentiable form)."""
        if self._lib.orc_enable_record(self._h) != 0:
            raise RuntimeError("recording must start at step 0")

    def theta(self, w) -> np.ndarray:
        """Class parameters of a workload as [5 * n_classes] (v0_factor, T, a, b, s0)."""
        p = w.params
        return np.stack([p.v0_factor, p.T, p.a, p.b, p.s0], axis=1).astype(np.float64).ravel()

    def replay(self, theta, target=None, use=None, grad: bool = False):
        """FP64 replay of the recorded run with its decisions frozen, at the
        class parameters theta.  Returns (loss, per-edge mean traversal time,
        dL/dtheta or None)."""
        th = np.ascontiguousarray(theta, np.float64)
        tg = None if target is None else np.ascontiguousarray(target, np.float64)
        us = None if use is None else np.ascontiguousarray(use, np.uint8)
        mean = np.empty(self.n_edges, np.float64)
        g = np.empty(th.size, np.float64) if grad else None
        loss = self._lib.orc_replay(self._h, _p(th), _p(tg), _p(us), _p(mean), _p(g))
        return loss, mean, g

    def last_events(self) -> dict:
        n = self.n
        ev = dict(leader=np.empty(n, np.int32), kind=np.empty(n, np.int32), flags=np.empty(n, np.int32),
                  post_lane=np.empty(n, np.int32), xnew=np.empty(n, np.float64), vnew=np.empty(n, np.float64),
                  target_lane=np.empty(n, np.int32))
        self._lib.orc_last_events(self._h, *[_p(ev[k]) for k in ("leader", "kind", "flags", "post_lane",
                                                                   "xnew", "vnew", "target_lane")])
        ev["partner"] = np.empty(n, np.int32)
        self._lib.orc_last_partner(self._h, _p(ev["partner"]))
        return ev


def all_threads() -> int:
    """OMP_NUM_THREADS if set, else every CPU this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def set_threads(n: int = 1, fp64: bool = False) -> int:
    """Threads of the oracle's parallel phases (the library starts with one;
    n <= 0: all_threads()); returns the count in use."""
    return int(lib(fp64).orc_set_threads(int(n) if n > 0 else all_threads()))


# ---------------------------------------------------------------- scalar hooks for pins
def philox4x64(counter, key, fp64=False):
    c = np.asarray(counter, np.uint64)
    k = np.asarray(key, np.uint64)
    out = np.empty(4, np.uint64)
    lib(fp64).orc_philox4x64(_p(c), _p(k), _p(out))
    return out


def expf_c(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, np.float32)
    out = np.empty_like(y)
    lib(False).orc_expf_c_batch(_p(y), _p(out), int(y.size))
    return out


def idm(v, v0, vl, s, T, a, b, s0, kind, fp64=False):
    fl = np.zeros(1, np.int32)
    acc = lib(fp64).orc_idm_d(v, v0, vl, s, T, a, b, s0, int(kind), _p(fl))
    return acc, int(fl[0])


def crit_gap(g0, alpha_first, v_i, alpha_second, v_other, fp64=False):
    return lib(fp64).orc_crit_gap_d(g0, alpha_first, v_i, alpha_second, v_other)


def desired_gap(v_i, fp64=False):
    return lib(fp64).orc_desired_gap_d(v_i)


def uniform(seed, t, vid, stream, fp64=False):
    return lib(fp64).orc_uniform_d(seed, t, vid, stream)


def normal(seed, t, vid, stream, fp64=False):
    return lib(fp64).orc_normal_d(seed, t, vid, stream)


def driver_limit(seed, edge, vid, lim, spread, fp64=False):
    """Free-flow limit of one driver on one edge under a per-driver v0 spread."""
    return lib(fp64).orc_driver_limit_d(seed, edge, vid, lim, spread)


def mand_trigger(seed, t, vid, d, fp64=False):
    return lib(fp64).orc_mand_trigger(seed, t, vid, d)


def route(net, cost, o, d, fp64=False):
    """Shortest route from node o to node d on binary32 edge costs (list of
    edge ids), or None (o == d or unreachable)."""
    ef, et = _c(net.edge_from, np.int32), _c(net.edge_to, np.int32)
    c = _c(cost, np.float32)
    out = np.empty(net.n_edges, np.int32)
    n = lib(fp64).orc_route(net.n_nodes, net.n_edges, _p(ef), _p(et), _p(c), int(o), int(d), _p(out), out.size)
    return None if n < 0 else out[:n].tolist()


def route_dist(net, cost, d, fp64=False):
    """dist_d(v) for every node v (binary32 in the FP32 build)."""
    ef, et = _c(net.edge_from, np.int32), _c(net.edge_to, np.int32)
    c = _c(cost, np.float32)
    dist = np.empty(net.n_nodes, np.float32 if not fp64 else np.float64)
    if fp64:
        raise NotImplementedError("route_dist is binary32")
    lib(False).orc_route_dist(net.n_nodes, net.n_edges, _p(ef), _p(et), _p(c), int(d), _p(dist))
    return dist
