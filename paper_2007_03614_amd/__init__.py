"""Python binding of libmanta (the per-timestep vehicle update on MI355X).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI declared in ``include/manta.h``.  PyTorch provides
device memory (its caching allocator, registered with ``sim_set_allocator``)
and streams.  There is no CPU fallback: if ``libmanta.so`` is missing the
import fails.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmanta.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libmanta.so is not built ({LIB_PATH}); run __graft_entry__.build() first")

_lib = ctypes.CDLL(LIB_PATH)

COUNTERS = ["active_sum", "departed", "arrived", "lane_changes", "transfers", "holds",
            "insert_denied", "mand_triggers", "stop_branch", "clamp", "wrong_lane_holds",
            "waived_exits", "gridlock_steps"]
STATUS = {"SIM_OK": 0, "SIM_EINVAL": -1, "SIM_ENOMEM": -2, "SIM_EDEVICE": -3, "SIM_ESTATE": -4,
          "SIM_EUNSUPPORTED": -5}
_STATUS_NAME = {v: k for k, v in STATUS.items()}

P = ctypes.c_void_p
I32, I64, U64, F32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float


class SimNetwork(ctypes.Structure):
    _fields_ = [("n_nodes", I32), ("n_edges", I32), ("edge_from", P), ("edge_to", P), ("length_m", P),
                ("speed_limit_mps", P), ("n_lanes", P), ("conn_off", P), ("conn_to", P),
                ("conn_lane_mask", P)]


class SimRoutes(ctypes.Structure):
    _fields_ = [("n_vehicles", I32), ("route_off", P), ("route_edges", P), ("depart_step", P),
                ("vclass", P), ("alpha_s", P)]


class SimIdmParams(ctypes.Structure):
    _fields_ = [("n_classes", I32), ("v0_factor", P), ("T", P), ("a", P), ("b", P), ("s0", P),
                ("length_m", P), ("dt", F32), ("seed", U64), ("intersection_mode", I32),
                ("record_every", I32), ("v0_spread", F32)]


class SimScenario(ctypes.Structure):
    _fields_ = [("n_vehicles", I32), ("n_reduced", I32), ("reduced_edges", P), ("class_params", P)]


class SimState(ctypes.Structure):
    _fields_ = [("status", P), ("edge", P), ("lane", P), ("cursor", P), ("x", P), ("v", P),
                ("held_since", P), ("mand", P), ("ww", P), ("tau_in", P), ("t_arr", P), ("counters", P),
                ("t", I32)]


_ALLOC_FN = ctypes.CFUNCTYPE(P, ctypes.c_size_t, P)
_FREE_FN = ctypes.CFUNCTYPE(None, P, P)

_lib.sim_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, P]
_lib.sim_set_allocator.restype = I32
_lib.sim_create.argtypes = [ctypes.POINTER(SimNetwork), ctypes.POINTER(SimRoutes),
                            ctypes.POINTER(SimIdmParams), ctypes.POINTER(P)]
_lib.sim_create.restype = I32
_lib.sim_set_stream.argtypes = [P, P]
_lib.sim_set_stream.restype = I32
_lib.sim_step.argtypes = [P, I32]
_lib.sim_step.restype = I32
_lib.sim_step_timed.argtypes = [P, I32, P, P]
_lib.sim_step_timed.restype = I32
_lib.sim_read_state.argtypes = [P, ctypes.POINTER(SimState)]
_lib.sim_read_state.restype = I32
_lib.sim_write_state.argtypes = [P, ctypes.POINTER(SimState)]
_lib.sim_write_state.restype = I32
_lib.sim_read_edge_stats.argtypes = [P, P, P]
_lib.sim_read_edge_stats.restype = I32
_lib.sim_n_active.argtypes = [P, ctypes.POINTER(I32)]
_lib.sim_n_active.restype = I32
_lib.sim_destroy.argtypes = [P]
_lib.sim_destroy.restype = I32
_lib.sim_last_error.argtypes = [P]
_lib.sim_last_error.restype = ctypes.c_char_p
_lib.sim_create_ensemble.argtypes = [ctypes.POINTER(SimNetwork), ctypes.POINTER(SimRoutes), P, I32,
                                     ctypes.POINTER(SimIdmParams), ctypes.POINTER(P)]
_lib.sim_create_ensemble.restype = I32
_lib.sim_ensemble_offsets.argtypes = [P, P, P]
_lib.sim_ensemble_offsets.restype = I32
_lib.sim_autotune.argtypes = [P, ctypes.c_char_p]
_lib.sim_autotune.restype = I32
_lib.sim_autotune_steps.argtypes = [P, ctypes.c_char_p, I32]
_lib.sim_autotune_steps.restype = I32
_lib.sim_read_edge_means.argtypes = [P, P, P]
_lib.sim_read_edge_means.restype = I32
_lib.sim_big_tile_updates.argtypes = [P, P]
_lib.sim_big_tile_updates.restype = I32
_lib.sim_get_schedule.argtypes = [P, P]
_lib.sim_get_schedule.restype = I32
_lib.sim_backward.argtypes = [P, P, P]
_lib.sim_backward.restype = I32
_lib.sim_probe_fp32.argtypes = [I32, P, P, P, I64]
_lib.sim_probe_fp32.restype = I32
_lib.sim_probe_philox.argtypes = [P, P, P, I64]
_lib.sim_probe_philox.restype = I32
_lib.sim_probe_draws.argtypes = [U64, P, P, P, P, P, I64]
_lib.sim_probe_draws.restype = I32

KERNELS = ["k_tile_step", "k_big_admit", "k_commit", "k_scatter"]

_lib.sim_shortest_routes.argtypes = [ctypes.POINTER(SimNetwork), P, I32, P, P, P, P, ctypes.c_int64, P]
_lib.sim_shortest_routes.restype = I32
_lib.sim_shortest_routes_noalloc.argtypes = _lib.sim_shortest_routes.argtypes
_lib.sim_shortest_routes_noalloc.restype = I32

EXPORTED = ["sim_set_allocator", "sim_create", "sim_set_stream", "sim_step", "sim_step_timed", "sim_read_state",
            "sim_write_state", "sim_read_edge_stats", "sim_n_active", "sim_destroy", "sim_last_error",
            "sim_create_ensemble", "sim_ensemble_offsets", "sim_autotune", "sim_autotune_steps", "sim_get_schedule",
            "sim_read_edge_means", "sim_backward",
            "sim_big_tile_updates", "sim_shortest_routes", "sim_shortest_routes_noalloc",
            "sim_probe_fp32", "sim_probe_philox", "sim_probe_draws"]


class SimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAME.get(status, status)}: {msg}")
        self.status = status
        self.name = _STATUS_NAME.get(status, str(status))


def _check(st: int, handle=None):
    if st != 0:
        raise SimError(st, _lib.sim_last_error(handle).decode(errors="replace"))


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- allocator
# The callback objects are created once and kept for the life of the process:
# every handle keeps the function pointers it was created with and calls the
# release callback when it is destroyed.
_torch_cb = None
_null_cb = None


def _torch_callbacks():
    global _torch_cb
    if _torch_cb is None:
        import torch

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes))
            except Exception:
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        _torch_cb = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    return _torch_cb


def use_torch_allocator() -> None:
    """Route device allocations of handles created afterwards through torch's
    caching allocator (current device, current stream)."""
    cb = _torch_callbacks()
    _check(_lib.sim_set_allocator(cb[0], cb[1], None))


def use_hip_allocator() -> None:
    global _null_cb
    if _null_cb is None:
        _null_cb = (_ALLOC_FN(), _FREE_FN())
    _check(_lib.sim_set_allocator(_null_cb[0], _null_cb[1], None))


# ---------------------------------------------------------------- handle
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # before torch's own teardown: destroying a handle calls the release callback
    for sim in list(_live):
        sim.close()


class Sim:
    """One simulation on the current GPU.

    ``Sim(workload)`` takes any object with the generator's attribute names
    (``net``, ``route_off``, ``route_edges``, ``depart_step``, ``vclass``,
    ``alpha``, ``params``)."""

    def __init__(self, w, stream=None, allocator: str = "torch", scenarios=None):
        """scenarios: optional list of (n_vehicles, reduced_edges) or
        (n_vehicles, reduced_edges, class_params) — an ensemble over the
        workload's network, with the workload's demand as the master list
        (sim_create_ensemble).  class_params: None or [n_classes, 5]
        (v0_factor, T, a, b, s0) for that scenario; if any scenario has them,
        scenario k's class c is class k * n_classes + c of the handle."""
        net, p = w.net, w.params
        self.n_edges_base = int(net.edge_from.shape[0])
        keep = dict(
            ef=_c(net.edge_from, np.int32), et=_c(net.edge_to, np.int32), ln=_c(net.length, np.float32),
            li=_c(net.limit, np.float32), la=_c(net.lanes, np.uint8), co=_c(net.conn_off, np.int32),
            ct=_c(net.conn_to, np.int32), cm=_c(net.conn_mask, np.uint8), ro=_c(w.route_off, np.int64),
            re=_c(w.route_edges, np.int32), dp=_c(w.depart_step, np.int32), vc=_c(w.vclass, np.uint8),
            al=_c(w.alpha, np.float32), v0=_c(p.v0_factor, np.float32), T=_c(p.T, np.float32),
            a=_c(p.a, np.float32), b=_c(p.b, np.float32), s0=_c(p.s0, np.float32),
            vl=_c(p.veh_len, np.float32))
        k = keep
        n_master = int(w.depart_step.shape[0])
        n_nodes = int(getattr(net, "n_nodes", int(max(k["ef"].max(), k["et"].max())) + 1))
        self._net = SimNetwork(n_nodes, self.n_edges_base, _p(k["ef"]), _p(k["et"]), _p(k["ln"]), _p(k["li"]),
                               _p(k["la"]), _p(k["co"]), _p(k["ct"]), _p(k["cm"]))
        self._routes = SimRoutes(n_master, _p(k["ro"]), _p(k["re"]), _p(k["dp"]), _p(k["vc"]), _p(k["al"]))
        self._params = SimIdmParams(int(p.T.shape[0]), _p(k["v0"]), _p(k["T"]), _p(k["a"]), _p(k["b"]),
                                    _p(k["s0"]), _p(k["vl"]), float(p.dt), int(p.seed),
                                    int(getattr(p, "intersection_mode", 0)), int(getattr(p, "record_every", 0)),
                                    float(getattr(p, "v0_spread", 0.0)))
        if allocator == "torch":
            use_torch_allocator()
        elif allocator == "hip":
            use_hip_allocator()
        h = P()
        if scenarios is None:
            self.n_scen = 1
            self.n = n_master
            self.n_edges = self.n_edges_base
            _check(_lib.sim_create(ctypes.byref(self._net), ctypes.byref(self._routes),
                                   ctypes.byref(self._params), ctypes.byref(h)))
        else:
            red = [_c(sc_[1], np.int32) for sc_ in scenarios]
            cps = [None if len(sc_) < 3 or sc_[2] is None else _c(np.asarray(sc_[2]).reshape(-1), np.float32)
                   for sc_ in scenarios]
            sc = (SimScenario * len(scenarios))(*[SimScenario(int(sc_[0]), int(r.size), _p(r),
                                                              None if cp is None else _p(cp))
                                                  for sc_, r, cp in zip(scenarios, red, cps)])
            keep["red"], keep["sc"], keep["cps"] = red, sc, cps
            self.n_scen = len(scenarios)
            self.n = int(sum(int(sc_[0]) for sc_ in scenarios))
            if any(cp is not None for cp in cps):
                self.n_classes = self.n_scen * int(p.T.shape[0])
            self.n_edges = self.n_edges_base * self.n_scen
            _check(_lib.sim_create_ensemble(ctypes.byref(self._net), ctypes.byref(self._routes),
                                            ctypes.cast(sc, P), self.n_scen, ctypes.byref(self._params),
                                            ctypes.byref(h)))
        self._keep = keep
        self._h = h
        _live.add(self)
        if stream is not None:
            self.set_stream(stream)

    def mean_travel_times(self):
        """Per-edge mean completed traversal time (s, 0 where none completed)
        and traversal count (sim_read_edge_means)."""
        m = np.empty(self.n_edges, np.float64)
        c = np.empty(self.n_edges, np.int64)
        _check(_lib.sim_read_edge_means(self._h, _p(m), _p(c)), self._h)
        return m, c

    def backward(self, dL_dmean: np.ndarray) -> np.ndarray:
        """dL/d(class parameters) as [n_classes, 5] (v0_factor, T, a, b, s0)
        for dL/d(per-edge mean traversal time) = dL_dmean (sim_backward)."""
        g = _c(dL_dmean, np.float64)
        out = np.zeros(5 * int(getattr(self, "n_classes", self._params.n_classes)), np.float64)
        _check(_lib.sim_backward(self._h, _p(g), _p(out)), self._h)
        return out.reshape(-1, 5)

    def offsets(self) -> np.ndarray:
        """Vehicle-id range of every scenario: [n_scen + 1]."""
        out = np.zeros(self.n_scen + 1, np.int32)
        ns = I32()
        _check(_lib.sim_ensemble_offsets(self._h, ctypes.byref(ns), _p(out)), self._h)
        return out

    def autotune(self, cache_path=None, steps_per_trial: int = 20) -> list:
        cp = cache_path.encode() if cache_path else None
        _check(_lib.sim_autotune_steps(self._h, cp, int(steps_per_trial)), self._h)
        return self.schedule()

    def big_tile_updates(self) -> int:
        """Vehicle-updates done in tiles above one workgroup's LDS since the
        state was last written (sim_big_tile_updates)."""
        out = np.zeros(1, np.int64)
        _check(_lib.sim_big_tile_updates(self._h, _p(out)), self._h)
        return int(out[0])

    def schedule(self) -> list:
        out = np.zeros(4, np.int32)
        _check(_lib.sim_get_schedule(self._h, _p(out)), self._h)
        return out.tolist()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.sim_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def set_stream(self, stream) -> None:
        """stream: a torch.cuda.Stream, a raw hipStream_t (int), or None."""
        raw = getattr(stream, "cuda_stream", stream)
        _check(_lib.sim_set_stream(self._h, P(raw) if raw else None), self._h)

    def step(self, n: int = 1) -> None:
        _check(_lib.sim_step(self._h, int(n)), self._h)

    def step_timed(self, n: int):
        """Run n steps kernel by kernel with HIP events; returns (per-kernel
        ms summed over the steps as a dict, total ms)."""
        ks = np.zeros(len(KERNELS), np.float64)
        tot = np.zeros(1, np.float64)
        _check(_lib.sim_step_timed(self._h, int(n), _p(ks), _p(tot)), self._h)
        return dict(zip(KERNELS, ks.tolist())), float(tot[0])

    @property
    def n_active(self) -> int:
        out = I32()
        _check(_lib.sim_n_active(self._h, ctypes.byref(out)), self._h)
        return int(out.value)

    def state(self) -> dict:
        n = self.n
        s = dict(status=np.empty(n, np.uint8), edge=np.empty(n, np.int32), lane=np.empty(n, np.int32),
                 cursor=np.empty(n, np.int32), x=np.empty(n, np.float32), v=np.empty(n, np.float32),
                 held_since=np.empty(n, np.int32), mand=np.empty(n, np.uint8), ww=np.empty(n, np.int32),
                 tau_in=np.empty(n, np.float64), t_arr=np.empty(n, np.float64),
                 counters=np.empty(len(COUNTERS), np.int64))
        st = SimState(*[_p(s[k]) for k in ("status", "edge", "lane", "cursor", "x", "v", "held_since", "mand",
                                           "ww", "tau_in", "t_arr", "counters")], 0)
        _check(_lib.sim_read_state(self._h, ctypes.byref(st)), self._h)
        s["t"] = int(st.t)
        return s

    def write_state(self, s: dict) -> None:
        a = dict(status=_c(s["status"], np.uint8), edge=_c(s["edge"], np.int32), lane=_c(s["lane"], np.int32),
                 cursor=_c(s["cursor"], np.int32), x=_c(s["x"], np.float32), v=_c(s["v"], np.float32),
                 held_since=_c(s["held_since"], np.int32), mand=_c(s["mand"], np.uint8),
                 ww=_c(s["ww"], np.int32), tau_in=_c(s["tau_in"], np.float64),
                 t_arr=_c(s["t_arr"], np.float64))
        cnt = _c(s["counters"], np.int64) if s.get("counters") is not None else None
        st = SimState(*[_p(a[k]) for k in ("status", "edge", "lane", "cursor", "x", "v", "held_since", "mand",
                                           "ww", "tau_in", "t_arr")], _p(cnt), int(s["t"]))
        _check(_lib.sim_write_state(self._h, ctypes.byref(st)), self._h)

    def counters(self) -> dict:
        return dict(zip(COUNTERS, self.state()["counters"].tolist()))

    def edge_stats(self):
        s = np.empty(self.n_edges, np.float64)
        c = np.empty(self.n_edges, np.int64)
        _check(_lib.sim_read_edge_stats(self._h, _p(s), _p(c)), self._h)
        return s, c


# ---------------------------------------------------------------- probes
def probe_fp32(op: int, a: np.ndarray, b: np.ndarray = None) -> np.ndarray:
    a = _c(a, np.float32)
    b = _c(b, np.float32) if b is not None else None
    out = np.empty_like(a)
    _check(_lib.sim_probe_fp32(int(op), _p(a), _p(b), _p(out), int(a.size)))
    return out


def probe_philox(counters: np.ndarray, key) -> np.ndarray:
    c = _c(counters, np.uint64).reshape(-1, 4)
    k = _c(key, np.uint64)
    out = np.empty_like(c)
    _check(_lib.sim_probe_philox(_p(c), _p(k), _p(out), int(c.shape[0])))
    return out


def probe_draws(seed: int, t: np.ndarray, vid: np.ndarray):
    t = _c(t, np.int64)
    vid = _c(vid, np.int64)
    u = np.empty(t.size, np.float32)
    e2 = np.empty(t.size, np.float32)
    e3 = np.empty(t.size, np.float32)
    _check(_lib.sim_probe_draws(int(seed), _p(t), _p(vid), _p(u), _p(e2), _p(e3), int(t.size)))
    return u, e2, e3


# ---------------------------------------------------------------- autograd
def with_class_params(w, theta):
    """Shallow copy of a workload whose class parameters are theta [n_classes, 5]
    = (v0_factor, T, a, b, s0) (rounded to binary32 like every input)."""
    import copy
    th = np.asarray(theta, np.float64).reshape(-1, 5)
    w2 = copy.copy(w)
    p = copy.copy(w.params)
    p.v0_factor, p.T, p.a, p.b, p.s0 = [th[:, k].astype(np.float32) for k in range(5)]
    w2.params = p
    return w2


def _edge_tt_function():
    import torch

    class EdgeMeanTravelTime(torch.autograd.Function):
        """theta [n_classes, 5] -> per-edge mean traversal times [n_edges]
        after `steps` steps; the backward runs sim_backward (adjoint with the
        forward's discrete decisions held fixed, checkpoint every
        record_every steps)."""

        @staticmethod
        def forward(ctx, theta, workload, steps, record_every=120, stream=None):
            w = with_class_params(workload, theta.detach().cpu().numpy())
            w.params.record_every = int(record_every)
            sim = Sim(w, stream=stream)
            sim.step(int(steps))
            mean, cnt = sim.mean_travel_times()
            ctx.sim = sim
            ctx.shape = theta.shape
            ctx.dtype = theta.dtype
            out = torch.from_numpy(mean)
            return out

        @staticmethod
        def backward(ctx, grad_mean):
            g = ctx.sim.backward(grad_mean.detach().cpu().numpy())
            ctx.sim.close()
            return torch.from_numpy(g).reshape(ctx.shape).to(ctx.dtype), None, None, None, None

    return EdgeMeanTravelTime


def edge_mean_travel_time(theta, workload, steps, record_every=120, stream=None):
    """Differentiable per-edge mean traversal times (torch.autograd)."""
    return _edge_tt_function().apply(theta, workload, steps, record_every, stream)


def _routes(fn, net, cost, origin, dest):
    ef, et = _c(net.edge_from, np.int32), _c(net.edge_to, np.int32)
    z8 = np.zeros(net.n_edges, np.uint8)
    zo = np.zeros(net.n_edges + 1, np.int32)
    sn = SimNetwork(int(net.n_nodes), int(net.n_edges), _p(ef), _p(et), _p(_c(net.length, np.float32)),
                    _p(_c(net.limit, np.float32)), _p(z8), _p(zo), _p(zo), _p(z8))
    c = _c(cost, np.float32)
    o, d = _c(origin, np.int32), _c(dest, np.int32)
    off = np.zeros(o.size + 1, np.int64)
    tot = np.zeros(1, np.int64)
    edges = np.zeros(max(1024, 128 * o.size), np.int32)
    st = fn(ctypes.byref(sn), _p(c), int(o.size), _p(o), _p(d), _p(off), _p(edges), int(edges.size), _p(tot))
    if st != 0 and int(tot[0]) > edges.size:   # longer routes than guessed: again, sized
        edges = np.zeros(int(tot[0]), np.int32)
        st = fn(ctypes.byref(sn), _p(c), int(o.size), _p(o), _p(d), _p(off), _p(edges), int(edges.size), _p(tot))
    _check(st)
    return off, edges[:int(tot[0])]


def shortest_routes(net, cost, origin, dest):
    """Routes on the GPU minimising binary32 edge costs (sim_shortest_routes):
    returns (route_off int64[n + 1], route_edges int32)."""
    return _routes(_lib.sim_shortest_routes, net, cost, origin, dest)


def shortest_routes_noalloc(net, cost, origin, dest):
    """The same through sim_shortest_routes_noalloc (no device allocation; the
    call's buffers live in the library's fixed 64 MiB region)."""
    return _routes(_lib.sim_shortest_routes_noalloc, net, cost, origin, dest)
