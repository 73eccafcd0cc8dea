"""Seeded synthetic inputs for the per-timestep vehicle update.

This module is the only code shared by the CPU oracle (``oracle/``) and the
HIP path (``paper_2007_03614_amd/``).  It produces *inputs* only — road
networks, turn-lane masks, origin/destination demand, departure steps and
fixed routes — and holds none of the simulation arithmetic.

The paper's workloads (Sec. II-A network, II-B demand, II-C routing, II-D
departures) rely on OpenStreetMap and MTC data that are not available, so the
generators below build stand-ins with the shapes and distributions the paper
states: grid/planar road graphs with lanes, lengths and speed limits, origins
and destinations on nodes, departures drawn from a stated distribution, and
shortest routes on free-flow time computed before the simulation starts.

Every draw uses numpy ``PCG64`` seeded by ``SeedSequence(seed, spawn_key=(purpose,))``
so a workload is a pure function of (config, seed, overrides).
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DIJ_SRC = os.path.join(_HERE, "dijkstra.c")
_DIJ_SO = os.path.join(_HERE, "libdijkstra.so")

KMH = 1.0 / 3.6

# purposes for SeedSequence spawn keys
_P_NET, _P_DEL, _P_SEG, _P_OD, _P_DEP, _P_ALPHA, _P_CLASS, _P_SCEN, _P_HIDDEN = range(9)
_P_TREE, _P_EXTRA, _P_POOL, _P_DEST, _P_PREFILL, _P_CLASSPAR = range(9, 15)


def _rng(seed: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(purpose,))))


# --------------------------------------------------------------------------- build
def build_dijkstra(force: bool = False) -> str:
    """Compile the route generator's C Dijkstra (plain gcc, -O2)."""
    if force or not os.path.exists(_DIJ_SO) or os.path.getmtime(_DIJ_SO) < os.path.getmtime(_DIJ_SRC):
        tmp = _DIJ_SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread",
                               _DIJ_SRC, "-o", tmp])
        os.replace(tmp, _DIJ_SO)
    return _DIJ_SO


@functools.lru_cache(maxsize=1)
def _dij_lib():
    lib = ctypes.CDLL(build_dijkstra())
    P = ctypes.c_void_p
    lib.dij_solve.restype = P
    lib.dij_solve.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_int32, P,
                              ctypes.c_int32, P, P, P, ctypes.c_int32]
    lib.dij_solve_to.restype = P
    lib.dij_solve_to.argtypes = lib.dij_solve.argtypes
    lib.dij_lengths.argtypes = [P, P]
    lib.dij_copy.argtypes = [P, P, P]
    lib.dij_free.argtypes = [P]
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------- data
@dataclass
class Network:
    """Directed road network, edges sorted by (from, to).

    lanes: 1..8 per edge (lane 0 is the rightmost); length in metres;
    limit in m/s; conn_* is the CSR of allowed (e -> f) moves with a lane mask
    (bit l set: lane l of e may proceed to f)."""
    node_x: np.ndarray
    node_y: np.ndarray
    edge_from: np.ndarray
    edge_to: np.ndarray
    length: np.ndarray
    limit: np.ndarray
    lanes: np.ndarray
    conn_off: np.ndarray = None
    conn_to: np.ndarray = None
    conn_mask: np.ndarray = None

    @property
    def n_nodes(self) -> int:
        return int(self.node_x.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edge_from.shape[0])


@dataclass
class Params:
    """Per-class car-following parameters and run constants."""
    v0_factor: np.ndarray
    T: np.ndarray
    a: np.ndarray
    b: np.ndarray
    s0: np.ndarray
    veh_len: np.ndarray
    dt: float = 0.5
    seed: int = 0
    intersection_mode: int = 0
    record_every: int = 0
    v0_spread: float = 0.0     # per-driver v0: sigma_s = v0_spread * limit, drawn at 2 sigma_s

    @property
    def n_classes(self) -> int:
        return int(self.T.shape[0])


@dataclass
class Workload:
    name: str
    net: Network
    route_off: np.ndarray      # int64 [n_veh+1]
    route_edges: np.ndarray    # int32
    depart_step: np.ndarray    # int32 [n_veh]
    vclass: np.ndarray         # uint8 [n_veh]
    alpha: np.ndarray          # float32 [n_veh]
    params: Params
    n_steps: int
    info: dict = field(default_factory=dict)

    @property
    def n_vehicles(self) -> int:
        return int(self.depart_step.shape[0])


def base_params(n_classes: int = 1, seed: int = 0) -> Params:
    """The config-1 car-following parameters: v0 = limit, T = 1.5 s,
    a = 1.0, b = 2.0 m/s^2, s0 = 2 m, vehicle length 5 m."""
    f = lambda v: np.full(n_classes, v, dtype=np.float32)
    return Params(v0_factor=f(1.0), T=f(1.5), a=f(1.0), b=f(2.0), s0=f(2.0),
                  veh_len=f(5.0), seed=seed)


# calibration bounds of the car-following parameters (Sec. IV-A)
BOUNDS = dict(v0_factor=(0.05, 2.0), T=(0.1, 2.0), a=(1.0, 10.0), b=(1.0, 10.0), s0=(1.0, 5.0))


def jitter_params(p: Params, rel: float, seed: int, purpose: int = _P_CLASS) -> Params:
    """Each (class, parameter) scaled by (1 + U[-rel, rel]), then clipped to
    the calibration bounds (a = 1 sits on its lower bound)."""
    r = _rng(seed, purpose)
    k = p.n_classes

    def g(arr, name):
        lo, hi = BOUNDS[name]
        return np.clip(arr.astype(np.float64) * (1.0 + r.uniform(-rel, rel, size=k)), lo, hi).astype(np.float32)
    return Params(v0_factor=g(p.v0_factor, "v0_factor"), T=g(p.T, "T"), a=g(p.a, "a"), b=g(p.b, "b"),
                  s0=g(p.s0, "s0"),
                  veh_len=p.veh_len.copy(), dt=p.dt, seed=p.seed,
                  intersection_mode=p.intersection_mode, record_every=p.record_every, v0_spread=p.v0_spread)


# --------------------------------------------------------------------------- networks
def _finish_edges(nx, ny, seg_u, seg_v, seg_len, seg_lim, seg_lanes) -> Network:
    """Turn undirected segments into directed edges sorted by (from, to)."""
    fr = np.concatenate([seg_u, seg_v]).astype(np.int32)
    to = np.concatenate([seg_v, seg_u]).astype(np.int32)
    ln = np.concatenate([seg_len, seg_len]).astype(np.float32)
    li = np.concatenate([seg_lim, seg_lim]).astype(np.float32)
    la = np.concatenate([seg_lanes, seg_lanes]).astype(np.uint8)
    order = np.lexsort((to, fr))
    net = Network(node_x=np.asarray(nx, np.float64), node_y=np.asarray(ny, np.float64),
                  edge_from=fr[order], edge_to=to[order], length=ln[order],
                  limit=li[order], lanes=la[order])
    turn_lane_masks(net)
    return net


def turn_lane_masks(net: Network) -> None:
    """Connections and which lanes may take them (geometric rule).

    At node v, the moves out of incoming edge e = (u -> v) are all out-edges
    (v -> w) with w != u; a U-turn is allowed only at a dead end.  The moves
    are ranked by turn angle from rightmost to leftmost (ties by edge id);
    with m moves and L lanes on e, rank k may use lanes
    floor(kL/m) .. max(floor(kL/m), ceil((k+1)L/m) - 1).  Moves are listed
    in ascending target edge id.  Vectorized over edges: every edge's
    candidate moves sit in one row of an [E, max out-degree] table."""
    E = net.n_edges
    fr = net.edge_from.astype(np.int64)
    to = net.edge_to.astype(np.int64)
    out_start = np.searchsorted(fr, np.arange(net.n_nodes + 1))
    deg = out_start[1:] - out_start[:-1]
    D = max(int(deg.max(initial=0)), 1)
    k = np.arange(D)[None, :]
    valid = k < deg[to][:, None]
    cand = np.where(valid, out_start[to][:, None] + k, 0)
    not_back = valid & (to[cand] != fr[:, None])
    dead_end = ~not_back.any(axis=1)
    use = np.where(dead_end[:, None], valid, not_back)
    nx, ny = net.node_x, net.node_y
    dx_in = (nx[to] - nx[fr])[:, None]
    dy_in = (ny[to] - ny[fr])[:, None]
    w = to[cand]
    dx = nx[w] - nx[to][:, None]
    dy = ny[w] - ny[to][:, None]
    ang = np.where(use, np.arctan2(dx_in * dy - dy_in * dx, dx_in * dx + dy_in * dy), np.inf)
    order = np.argsort(ang, axis=1, kind="stable")
    rank = np.empty_like(order)
    np.put_along_axis(rank, order, np.broadcast_to(np.arange(D)[None, :], order.shape).copy(), axis=1)
    m = np.maximum(use.sum(axis=1), 1)[:, None]
    L = net.lanes.astype(np.int64)[:, None]
    lo = (rank * L) // m
    hi = np.maximum(lo, -((-(rank + 1) * L) // m) - 1)
    lane = np.arange(8)[None, None, :]
    mask = (((lane >= lo[:, :, None]) & (lane <= hi[:, :, None])).astype(np.int64) << lane).sum(axis=2)
    conn_off = np.zeros(E + 1, np.int32)
    conn_off[1:] = np.cumsum(use.sum(axis=1))
    net.conn_off = conn_off
    net.conn_to = cand[use].astype(np.int32)
    net.conn_mask = mask[use].astype(np.uint8)


def grid_network(rows: int = 10, cols: int = 10, spacing: float = 200.0, lanes: int = 2,
                 limit_kmh: float = 50.0) -> Network:
    """Regular grid, node id = cols*row + col, uniform segments."""
    ids = np.arange(rows * cols).reshape(rows, cols)
    nx = (np.arange(rows * cols) % cols) * spacing
    ny = (np.arange(rows * cols) // cols) * spacing
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    n = u.shape[0]
    lim = np.float32(np.float64(limit_kmh) / 3.6)
    return _finish_edges(nx, ny, u, v, np.full(n, spacing), np.full(n, lim), np.full(n, lanes))


def _largest_component(n_nodes, u, v):
    parent = np.arange(n_nodes)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a, b in zip(u.tolist(), v.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(n_nodes)])
    vals, counts = np.unique(roots, return_counts=True)
    return roots == vals[np.argmax(counts)]


def perturbed_grid_ring(rows: int = 100, cols: int = 100, spacing: float = 250.0,
                        delete_frac: float = 0.10, ring_nodes: int = 40, ring_offset: float = 1000.0,
                        seed: int = 0) -> Network:
    """Grid with a fraction of segments deleted (largest connected part kept;
    segments are two-way so it is strongly connected), 1-3 lanes,
    40-60 km/h, lengths U[100, 400] m, plus a 4-lane 100 km/h ring highway
    outside the grid joined to the nearest boundary node by 1-lane 60 km/h ramps."""
    rd = _rng(seed, _P_DEL)
    rs = _rng(seed, _P_SEG)
    ids = np.arange(rows * cols).reshape(rows, cols)
    gx = (np.arange(rows * cols) % cols) * spacing
    gy = (np.arange(rows * cols) // cols) * spacing
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    keep = np.ones(u.shape[0], bool)
    keep[rd.choice(u.shape[0], size=int(round(delete_frac * u.shape[0])), replace=False)] = False
    u, v = u[keep], v[keep]
    alive = _largest_component(rows * cols, u, v)
    m = alive[u] & alive[v]
    u, v = u[m], v[m]
    nseg = u.shape[0]
    lanes = rs.integers(1, 4, size=nseg)
    lim = (rs.uniform(40.0, 60.0, size=nseg) * KMH).astype(np.float32)
    length = rs.uniform(100.0, 400.0, size=nseg).astype(np.float32)
    # renumber kept grid nodes
    old = np.nonzero(alive)[0]
    newid = -np.ones(rows * cols, np.int64)
    newid[old] = np.arange(old.shape[0])
    u, v = newid[u], newid[v]
    nx, ny = list(gx[old]), list(gy[old])
    n_grid = old.shape[0]
    # ring: square loop ring_offset outside the grid, ring_nodes evenly spaced
    lo, hi = -ring_offset, (cols - 1) * spacing + ring_offset
    side = hi - lo
    per = 4 * side
    ring_xy = []
    for k in range(ring_nodes):
        s = per * k / ring_nodes
        if s < side:
            ring_xy.append((lo + s, lo))
        elif s < 2 * side:
            ring_xy.append((hi, lo + s - side))
        elif s < 3 * side:
            ring_xy.append((hi - (s - 2 * side), hi))
        else:
            ring_xy.append((lo, hi - (s - 3 * side)))
    ring_ids = list(range(n_grid, n_grid + ring_nodes))
    for (x, y) in ring_xy:
        nx.append(x)
        ny.append(y)
    nxa, nya = np.asarray(nx), np.asarray(ny)
    seg_u, seg_v = list(u), list(v)
    seg_len, seg_lim, seg_lanes = list(length), list(lim), list(lanes)
    for k in range(ring_nodes):
        a, b = ring_ids[k], ring_ids[(k + 1) % ring_nodes]
        seg_u.append(a); seg_v.append(b)
        seg_len.append(np.float32(math.hypot(nxa[a] - nxa[b], nya[a] - nya[b])))
        seg_lim.append(np.float32(100.0 * KMH)); seg_lanes.append(4)
    # ramps: each ring node to the nearest kept boundary grid node
    gxo, gyo = gx[old], gy[old]
    bnd = (gxo == 0) | (gyo == 0) | (gxo == (cols - 1) * spacing) | (gyo == (rows - 1) * spacing)
    bidx = np.nonzero(bnd)[0]
    for k in range(ring_nodes):
        r = ring_ids[k]
        d2 = (gxo[bidx] - nxa[r]) ** 2 + (gyo[bidx] - nya[r]) ** 2
        g = int(bidx[np.argmin(d2)])
        seg_u.append(r); seg_v.append(g)
        seg_len.append(np.float32(math.sqrt(float(np.min(d2)))))
        seg_lim.append(np.float32(60.0 * KMH)); seg_lanes.append(1)
    return _finish_edges(nxa, nya, np.asarray(seg_u), np.asarray(seg_v), np.asarray(seg_len, np.float32),
                         np.asarray(seg_lim, np.float32), np.asarray(seg_lanes))


# lanes 1..5 of the metropolitan network and their shares
METRO_LANE_P = (0.45, 0.30, 0.12, 0.09, 0.04)


def metro_network(rows: int = 473, cols: int = 474, pitch: float = 120.0, jitter: float = 30.0,
                  n_segments: int = 274_504, min_len: float = 25.0, arterial_every: int = 8,
                  seed: int = 0) -> Network:
    """Random planar road-like graph standing in for the paper's metropolitan
    network (Sec. II-A: 224,223 nodes, 549,008 directed edges).

    Nodes sit on a rows x cols lattice of `pitch` metres, each moved by
    U[-jitter, jitter] in x and y.  Candidate segments are the 4-neighbour
    links plus one diagonal per lattice cell, its direction drawn (so the
    candidates are planar).  Every `arterial_every`-th lattice row and column
    is an arterial line.  A random spanning tree (minimum spanning tree on
    random weights, arterial links first) keeps every node connected; the
    arterial links it left out are added (the arterials form a complete
    grid), then segments drawn uniformly from the remaining candidates up to
    `n_segments` (two-way, so 2 * n_segments directed edges): local streets
    are the tree's branches plus a few loops.  Lanes 1..5 have the shares
    METRO_LANE_P: whole arterial lines, in a drawn order, take the widest
    classes (5, then 4, then 3 lanes) until each class has its share of
    segments; local streets take the rest (3, 2, 1 lanes) uniformly.  Limit
    clamp(30 + 20 (lanes - 1) + U[-10, 10], 30, 110) km/h; length log-normal
    with median 120 m and sigma_ln 0.5, clamped to [min_len, 2000] m (min_len
    25 m: an edge must be longer than one step's reach at the fastest limit
    plus a vehicle length, 21.3 m here)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import minimum_spanning_tree
    rn = _rng(seed, _P_NET)
    n = rows * cols
    ids = np.arange(n).reshape(rows, cols)
    nx = (np.arange(n) % cols) * pitch + rn.uniform(-jitter, jitter, size=n)
    ny = (np.arange(n) // cols) * pitch + rn.uniform(-jitter, jitter, size=n)
    flip = rn.random((rows - 1) * (cols - 1)) < 0.5
    du = np.where(flip, ids[:-1, 1:].ravel(), ids[:-1, :-1].ravel())
    dv = np.where(flip, ids[1:, :-1].ravel(), ids[1:, 1:].ravel())
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    cu = np.concatenate([hu, vu, du]).astype(np.int64)
    cv = np.concatenate([hv, vv, dv]).astype(np.int64)
    # arterial line of each candidate: row r -> r, column c -> rows + c, else -1
    hrow, vcol = hu // cols, vu % cols
    line = np.concatenate([np.where(hrow % arterial_every == 0, hrow, -1),
                           np.where(vcol % arterial_every == 0, rows + vcol, -1),
                           np.full(du.shape[0], -1)])
    art = line >= 0
    lo, hi = np.minimum(cu, cv), np.maximum(cu, cv)
    key = lo * n + hi
    rt = _rng(seed, _P_TREE)
    wts = 1.0 + rt.random(key.shape[0]) + np.where(art, 0.0, 1.0)
    tree = minimum_spanning_tree(sp.csr_matrix((wts, (lo, hi)), shape=(n, n))).tocoo()
    tkey = np.minimum(tree.row, tree.col).astype(np.int64) * n + np.maximum(tree.row, tree.col)
    order = np.argsort(key)
    keep = np.zeros(key.shape[0], bool)
    keep[order[np.searchsorted(key[order], tkey)]] = True
    if int(keep.sum()) != n - 1:
        raise RuntimeError("spanning tree does not cover the lattice")
    keep |= art
    rest = np.nonzero(~keep)[0]
    n_extra = min(max(n_segments - int(keep.sum()), 0), rest.shape[0])
    keep[_rng(seed, _P_EXTRA).choice(rest, size=n_extra, replace=False)] = True
    pick = np.nonzero(keep)[0]
    su, sv, sline = lo[pick], hi[pick], line[pick]
    ns = su.shape[0]
    rs = _rng(seed, _P_SEG)
    quota = np.round(np.asarray(METRO_LANE_P) * ns).astype(np.int64)    # segments per class 1..5
    lanes = np.zeros(ns, np.int64)
    lines = np.unique(sline[sline >= 0])
    lines = lines[rs.permutation(lines.shape[0])]
    per_line = np.bincount(sline[sline >= 0], minlength=rows + cols)[lines]
    left = quota.copy()
    cls_of_line = np.zeros(lines.shape[0], np.int64)
    k = 4                                            # 5 lanes first
    for j in range(lines.shape[0]):
        while k > 0 and left[k] <= 0:
            k -= 1
        cls_of_line[j] = k + 1
        left[k] -= per_line[j]
    lane_of_line = np.zeros(rows + cols, np.int64)
    lane_of_line[lines] = cls_of_line
    lanes[sline >= 0] = lane_of_line[sline[sline >= 0]]
    loc = np.nonzero(sline < 0)[0]
    pool = np.concatenate([np.full(max(int(left[q]), 0), q + 1, np.int64) for q in range(5)])
    if pool.shape[0] < loc.shape[0]:
        pool = np.concatenate([pool, np.ones(loc.shape[0] - pool.shape[0], np.int64)])
    lanes[loc] = pool[rs.permutation(pool.shape[0])[:loc.shape[0]]]
    kmh = np.clip(30.0 + 20.0 * (lanes - 1) + rs.uniform(-10.0, 10.0, size=ns), 30.0, 110.0)
    lim = (kmh * KMH).astype(np.float32)
    length = np.clip(rs.lognormal(math.log(120.0), 0.5, size=ns), min_len, 2000.0).astype(np.float32)
    return _finish_edges(nx, ny, su, sv, length, lim, lanes)


# --------------------------------------------------------------------------- routing
def shortest_routes(net: Network, orig: np.ndarray, dst: np.ndarray, n_threads: int = 0):
    """Fixed routes on free-flow time (length / limit), one per OD row.

    Returns (route_off int64[n+1], route_edges int32, ok bool[n]); rows with
    O == D or no path get an empty route and ok = False."""
    lib = _dij_lib()
    E, N = net.n_edges, net.n_nodes
    out_off = np.searchsorted(net.edge_from, np.arange(N + 1)).astype(np.int32)
    out_edge = np.arange(E, dtype=np.int32)  # edges are sorted by from, ids ascending
    w = net.length.astype(np.float64) / net.limit.astype(np.float64)
    orig = np.asarray(orig, np.int32)
    dst = np.asarray(dst, np.int32)
    order = np.argsort(orig, kind="stable").astype(np.int32)
    uo, starts = np.unique(orig[order], return_index=True)
    grp_off = np.append(starts, order.shape[0]).astype(np.int32)
    grp_origin = uo.astype(np.int32)
    if n_threads <= 0:
        n_threads = min(16, os.cpu_count() or 1)
    edge_from = np.ascontiguousarray(net.edge_from, np.int32)
    edge_to = np.ascontiguousarray(net.edge_to, np.int32)
    res = lib.dij_solve(N, _ptr(out_off), _ptr(out_edge), _ptr(edge_from), _ptr(edge_to), _ptr(w),
                        int(orig.shape[0]), _ptr(dst), int(grp_origin.shape[0]), _ptr(grp_origin),
                        _ptr(grp_off), _ptr(order), int(n_threads))
    if not res:
        raise MemoryError("route generation failed")
    try:
        plen = np.empty(orig.shape[0], np.int32)
        lib.dij_lengths(res, _ptr(plen))
        ok = plen > 0
        route_off = np.zeros(orig.shape[0] + 1, np.int64)
        route_off[1:] = np.cumsum(np.maximum(plen, 0))
        route_edges = np.empty(int(route_off[-1]), np.int32)
        lib.dij_copy(res, _ptr(route_off), _ptr(route_edges))
    finally:
        lib.dij_free(res)
    return route_off, route_edges, ok


def shortest_routes_to(net: Network, orig: np.ndarray, dst: np.ndarray, n_threads: int = 0):
    """The same routes as shortest_routes (free-flow time, ties broken the
    same way on the reversed graph), solved once per distinct *destination*:
    cheaper when many trips share few destinations.  Returns
    (route_off int64[n+1], route_edges int32, ok bool[n])."""
    lib = _dij_lib()
    E, N = net.n_edges, net.n_nodes
    in_edge = np.lexsort((np.arange(E), net.edge_to)).astype(np.int32)
    in_off = np.searchsorted(net.edge_to[in_edge], np.arange(N + 1)).astype(np.int32)
    w = net.length.astype(np.float64) / net.limit.astype(np.float64)
    orig = np.ascontiguousarray(orig, np.int32)
    dst = np.asarray(dst, np.int32)
    order = np.argsort(dst, kind="stable").astype(np.int32)
    ud, starts = np.unique(dst[order], return_index=True)
    grp_off = np.append(starts, order.shape[0]).astype(np.int32)
    grp_dest = ud.astype(np.int32)
    if n_threads <= 0:
        n_threads = min(16, os.cpu_count() or 1)
    edge_from = np.ascontiguousarray(net.edge_from, np.int32)
    edge_to = np.ascontiguousarray(net.edge_to, np.int32)
    res = lib.dij_solve_to(N, _ptr(in_off), _ptr(in_edge), _ptr(edge_from), _ptr(edge_to), _ptr(w),
                           int(orig.shape[0]), _ptr(orig), int(grp_dest.shape[0]), _ptr(grp_dest),
                           _ptr(grp_off), _ptr(order), int(n_threads))
    if not res:
        raise MemoryError("route generation failed")
    try:
        plen = np.empty(orig.shape[0], np.int32)
        lib.dij_lengths(res, _ptr(plen))
        ok = plen > 0
        route_off = np.zeros(orig.shape[0] + 1, np.int64)
        route_off[1:] = np.cumsum(np.maximum(plen, 0))
        route_edges = np.empty(int(route_off[-1]), np.int32)
        lib.dij_copy(res, _ptr(route_off), _ptr(route_edges))
    finally:
        lib.dij_free(res)
    return route_off, route_edges, ok


def _od_routes(net, n_veh, seed, nodes=None):
    """Uniform origin and destination nodes (O != D), routed."""
    r = _rng(seed, _P_OD)
    pool = np.arange(net.n_nodes) if nodes is None else np.asarray(nodes)
    o = pool[r.integers(0, pool.shape[0], size=n_veh)]
    d = pool[r.integers(0, pool.shape[0], size=n_veh)]
    same = o == d
    while same.any():
        d[same] = pool[r.integers(0, pool.shape[0], size=int(same.sum()))]
        same = o == d
    route_off, route_edges, ok = shortest_routes(net, o, d)
    if not ok.all():
        raise RuntimeError("network is not strongly connected")
    return route_off, route_edges, o, d


# --------------------------------------------------------------------------- configs
def config1(seed: int = 0, n_vehicles: int = 2000, n_steps: int = 3600, n_classes: int = 1) -> Workload:
    """10x10 grid of signal-free intersections, two-way 2-lane 200 m edges at
    50 km/h; uniform-random O/D nodes; departures U[0, 10 min); routes on
    free-flow time; base car-following parameters; dt = 0.5 s; 30 min."""
    net = grid_network()
    route_off, route_edges, _, _ = _od_routes(net, n_vehicles, seed)
    rdp = _rng(seed, _P_DEP)
    dep = np.floor(rdp.uniform(0.0, 600.0, size=n_vehicles) / 0.5).astype(np.int32)
    alpha = _rng(seed, _P_ALPHA).uniform(0.05, 0.40, size=n_vehicles).astype(np.float32)
    if n_classes == 1:
        vclass = np.zeros(n_vehicles, np.uint8)
    else:
        vclass = _rng(seed, _P_CLASS).integers(0, n_classes, size=n_vehicles).astype(np.uint8)
    p = base_params(n_classes, seed)
    return Workload("grid10x10", net, route_off, route_edges, dep, vclass, alpha, p, n_steps,
                    info={"departures": "U[0,600) s", "horizon_min": n_steps * 0.5 / 60})


@functools.lru_cache(maxsize=4)
def _c2_network(rows, cols, seed):
    return perturbed_grid_ring(rows=rows, cols=cols, seed=seed)


def config2(seed: int = 0, n_vehicles: int = 200_000, n_steps: int = 21_600, rows: int = 100,
            cols: int = 100) -> Workload:
    """Perturbed 100x100 grid (10% of segments deleted, largest connected part
    kept; 1-3 lanes, 40-60 km/h, 100-400 m) plus a 4-lane 100 km/h ring
    highway; departures N(08:00, 40 min) truncated to [06:30, 09:30); the run
    starts at 06:30 and lasts 3 h at dt = 0.5 s."""
    net = _c2_network(rows, cols, seed)
    route_off, route_edges, _, _ = _od_routes(net, n_vehicles, seed)
    r = _rng(seed, _P_DEP)
    t = r.normal(90.0 * 60.0, 40.0 * 60.0, size=n_vehicles)  # seconds after 06:30
    bad = (t < 0.0) | (t >= 3 * 3600.0)
    while bad.any():
        t[bad] = r.normal(90.0 * 60.0, 40.0 * 60.0, size=int(bad.sum()))
        bad = (t < 0.0) | (t >= 3 * 3600.0)
    dep = np.floor(t / 0.5).astype(np.int32)
    alpha = _rng(seed, _P_ALPHA).uniform(0.05, 0.40, size=n_vehicles).astype(np.float32)
    vclass = np.zeros(n_vehicles, np.uint8)
    return Workload(f"perturbed_grid{rows}x{cols}_ring", net, route_off, route_edges, dep, vclass, alpha,
                    base_params(1, seed), n_steps,
                    info={"departures": "N(08:00, 40 min) in [06:30, 09:30)", "start": "06:30"})


def _workload_cache_dir() -> str:
    return os.environ.get("MANTA_WORKLOAD_CACHE", os.path.join("/tmp", "manta_workloads"))


_WORKLOAD_ARRAYS = ("node_x", "node_y", "edge_from", "edge_to", "length", "limit", "lanes", "conn_off",
                    "conn_to", "conn_mask", "route_off", "route_edges", "depart_step", "vclass", "alpha",
                    "v0_factor", "T", "a", "b", "s0", "veh_len")


def _save_workload(path: str, w: "Workload") -> None:
    arrs = {k: getattr(w.net, k) for k in _WORKLOAD_ARRAYS[:10]}
    arrs.update({k: getattr(w, k) for k in _WORKLOAD_ARRAYS[10:15]})
    arrs.update({k: getattr(w.params, k) for k in _WORKLOAD_ARRAYS[15:]})
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, path)


def _load_workload(path: str, name: str, n_steps: int, info: dict) -> "Workload":
    z = np.load(path, allow_pickle=False)
    net = Network(**{k: z[k] for k in _WORKLOAD_ARRAYS[:10]})
    p = Params(**{k: z[k] for k in _WORKLOAD_ARRAYS[15:]})
    return Workload(name, net, z["route_off"], z["route_edges"], z["depart_step"], z["vclass"], z["alpha"],
                    p, n_steps, info=info)


def metro_demand(net: Network, n_vehicles: int, seed: int = 0, pool_size: int = 16_384,
                 median_m: float = 6460.0, sigma_ln: float = 1.06):
    """Origins uniform over nodes.  Each trip draws a straight-line distance
    D ~ LogNormal(ln median_m, sigma_ln) and a uniform direction from its
    origin (redrawn while the point falls outside the network's bounding
    box); its destination is the node nearest that point among a pool of
    `pool_size` nodes drawn uniformly (the attraction nodes of the zones;
    redrawn if it equals the origin)."""
    from scipy.spatial import cKDTree
    N = net.n_nodes
    pool = np.sort(_rng(seed, _P_POOL).choice(N, size=min(pool_size, N), replace=False))
    tree = cKDTree(np.stack([net.node_x[pool], net.node_y[pool]], axis=1))
    r = _rng(seed, _P_DEST)
    o = r.integers(0, N, size=n_vehicles)
    d = np.full(n_vehicles, -1, np.int64)
    x0, x1 = net.node_x.min(), net.node_x.max()
    y0, y1 = net.node_y.min(), net.node_y.max()
    todo = np.arange(n_vehicles)
    while todo.size:
        dist = r.lognormal(math.log(median_m), sigma_ln, size=todo.size)
        ang = r.uniform(0.0, 2.0 * math.pi, size=todo.size)
        px = net.node_x[o[todo]] + dist * np.cos(ang)
        py = net.node_y[o[todo]] + dist * np.sin(ang)
        inside = (px >= x0) & (px <= x1) & (py >= y0) & (py <= y1)
        sel = todo[inside]
        if sel.size:
            _, j = tree.query(np.stack([px[inside], py[inside]], axis=1))
            cand = pool[j]
            good = cand != o[sel]
            d[sel[good]] = cand[good]
        todo = todo[d[todo] < 0]
    return o.astype(np.int32), d.astype(np.int32)


def config3(seed: int = 0, n_vehicles: int = 3_200_000, n_steps: int = 50_400, rows: int = 473,
            cols: int = 474, pool_size: int = 16_384, cache: bool = True) -> Workload:
    """Metropolitan-scale stand-in (Sec. II-A network, II-B demand, II-D
    departures): metro_network (about 224k nodes and 549k directed edges at
    full size; smaller lattices keep the segment-per-node ratio), 3.2M trips
    from metro_demand routed on free-flow time, departures N(08:00, 45 min)
    truncated to [05:00, 10:00), 4 classes with each car-following parameter
    jittered by U[-10 %, +10 %], alpha U[0.05, 0.40]; the run starts at 05:00
    and lasts 7 h (05:00-12:00) at dt = 0.5 s.  The workload is cached on
    disk (MANTA_WORKLOAD_CACHE, default /tmp/manta_workloads)."""
    name = f"metro{rows}x{cols}_n{n_vehicles}"
    info = {"departures": "N(08:00, 45 min) in [05:00, 10:00)", "start": "05:00",
            "destination_pool": pool_size}
    path = os.path.join(_workload_cache_dir(), f"{name}_s{seed}_p{pool_size}_v3.npz")
    if cache and os.path.exists(path):
        return _load_workload(path, name, n_steps, info)
    n_nodes = rows * cols
    n_seg = int(round(274_504 * n_nodes / (473 * 474)))
    net = metro_network(rows=rows, cols=cols, n_segments=n_seg, seed=seed)
    o, d = metro_demand(net, n_vehicles, seed=seed, pool_size=pool_size)
    route_off, route_edges, ok = shortest_routes_to(net, o, d)
    if not ok.all():
        raise RuntimeError("metro network is not strongly connected")
    r = _rng(seed, _P_DEP)
    mu, sd, span = 3 * 3600.0, 45 * 60.0, 5 * 3600.0   # seconds after 05:00
    t = r.normal(mu, sd, size=n_vehicles)
    bad = (t < 0.0) | (t >= span)
    while bad.any():
        t[bad] = r.normal(mu, sd, size=int(bad.sum()))
        bad = (t < 0.0) | (t >= span)
    dep = np.floor(t / 0.5).astype(np.int32)
    alpha = _rng(seed, _P_ALPHA).uniform(0.05, 0.40, size=n_vehicles).astype(np.float32)
    vclass = _rng(seed, _P_CLASS).integers(0, 4, size=n_vehicles).astype(np.uint8)
    p = jitter_params(base_params(4, seed), 0.10, seed, purpose=_P_CLASSPAR)
    w = Workload(name, net, route_off, route_edges, dep, vclass, alpha, p, n_steps, info=info)
    if cache:
        _save_workload(path, w)
    return w


def single_edge_workload(length: float = 5000.0, limit: float = 50.0 / 3.6, lanes: int = 1,
                         n_vehicles: int = 1, depart_step=None, n_steps: int = 100,
                         params: Params = None) -> Workload:
    """A two-node network with one long edge each way; every vehicle drives
    the single edge 0 -> 1 and arrives at its end.  Used by closed-form tests."""
    nx = np.array([0.0, length])
    ny = np.array([0.0, 0.0])
    net = _finish_edges(nx, ny, np.array([0]), np.array([1]), np.array([length], np.float32),
                        np.array([limit], np.float32), np.array([lanes]))
    e01 = int(np.nonzero((net.edge_from == 0) & (net.edge_to == 1))[0][0])
    route_off = np.arange(n_vehicles + 1, dtype=np.int64)
    route_edges = np.full(n_vehicles, e01, np.int32)
    dep = np.zeros(n_vehicles, np.int32) if depart_step is None else np.asarray(depart_step, np.int32)
    alpha = np.full(n_vehicles, 0.2, np.float32)
    vclass = np.zeros(n_vehicles, np.uint8)
    return Workload("single_edge", net, route_off, route_edges, dep, vclass, alpha,
                    params or base_params(1), n_steps)


def ring_road(n_vehicles: int, n_nodes: int = 10, edge_len: float = 100.0, limit: float = 50.0 / 3.6,
              laps: int = 60, n_steps: int = 0, params: Params = None) -> Workload:
    """A one-lane ring road of n_nodes edges of edge_len metres (both
    directions exist; vehicles use the forward one).  Vehicle j enters at the
    start of edge j mod n_nodes at step 2 * (j // n_nodes) and drives `laps`
    laps.  For the fundamental diagram of the car-following model."""
    ang = 2.0 * math.pi * np.arange(n_nodes) / n_nodes
    rad = n_nodes * edge_len / (2.0 * math.pi)
    u = np.arange(n_nodes)
    net = _finish_edges(rad * np.cos(ang), rad * np.sin(ang), u, (u + 1) % n_nodes,
                        np.full(n_nodes, edge_len, np.float32), np.full(n_nodes, limit, np.float32),
                        np.ones(n_nodes, np.int64))
    fwd = np.empty(n_nodes, np.int32)
    for i in range(n_nodes):
        fwd[i] = int(np.nonzero((net.edge_from == i) & (net.edge_to == (i + 1) % n_nodes))[0][0])
    j = np.arange(n_vehicles)
    start = j % n_nodes
    route_edges = fwd[(start[:, None] + np.arange(laps * n_nodes)[None, :]) % n_nodes].astype(np.int32).ravel()
    route_off = np.arange(n_vehicles + 1, dtype=np.int64) * laps * n_nodes
    dep = (2 * (j // n_nodes)).astype(np.int32)
    return Workload(f"ring{n_nodes}x{int(edge_len)}_n{n_vehicles}", net, route_off, route_edges, dep,
                    np.zeros(n_vehicles, np.uint8), np.full(n_vehicles, 0.2, np.float32),
                    params or base_params(1), n_steps)


def scaled_config2(n_vehicles: int, rows: int, cols: int, n_steps: int, seed: int = 0) -> Workload:
    """Config 2's recipe on a smaller grid (for oracle-sized parity cases)."""
    w = config2(seed=seed, n_vehicles=n_vehicles, n_steps=n_steps, rows=rows, cols=cols)
    w.name = f"perturbed_grid{rows}x{cols}_ring_n{n_vehicles}"
    return w


def scenario_workload(master: Workload, n_vehicles: int, reduced_edges) -> Workload:
    """One what-if scenario on its own: the first n_vehicles of the master
    demand on the master network with `reduced_edges` cut to one lane (every
    move out of a reduced edge then leaves from lane 0)."""
    net = master.net
    lanes = net.lanes.copy()
    mask = net.conn_mask.copy()
    for e in np.asarray(reduced_edges, np.int64):
        lanes[e] = 1
        mask[net.conn_off[e]:net.conn_off[e + 1]] = 1
    n2 = Network(node_x=net.node_x, node_y=net.node_y, edge_from=net.edge_from, edge_to=net.edge_to,
                 length=net.length, limit=net.limit, lanes=lanes, conn_off=net.conn_off, conn_to=net.conn_to,
                 conn_mask=mask)
    ro = master.route_off[:n_vehicles + 1].copy()
    return Workload(f"{master.name}_scenario", n2, ro, master.route_edges[:int(ro[-1])].copy(),
                    master.depart_step[:n_vehicles].copy(), master.vclass[:n_vehicles].copy(),
                    master.alpha[:n_vehicles].copy(), master.params, master.n_steps)


def ensemble_scenarios(n_scen: int, base: int, n_edges: int, seed: int = 0, scale=(0.8, 1.2),
                       reduced_frac: float = 0.01):
    """Scenario list: demand round(U[scale] * base) vehicles of the master
    list and ceil(reduced_frac * n_edges) random edges cut to one lane."""
    r = _rng(seed, _P_SCEN)
    k = int(math.ceil(reduced_frac * n_edges))
    out = []
    for _ in range(n_scen):
        n = int(round(r.uniform(*scale) * base))
        red = np.sort(r.choice(n_edges, size=k, replace=False)).astype(np.int32)
        out.append((n, red))
    return out


def config4(seed: int = 0, n_scen: int = 64, base: int = 200_000, n_steps: int = 14_400):
    """Ensemble on the 10x10 grid: a master demand of 1.2 * base vehicles
    (uniform O/D, departures U[0, 2 h)), n_scen scenarios taking the first
    round(U[0.8, 1.2] * base) of them, 1 % of the edges cut to one lane in
    each; 2 h at dt = 0.5 s."""
    net = grid_network()
    n_master = int(round(1.2 * base))
    route_off, route_edges, _, _ = _od_routes(net, n_master, seed)
    dep = np.floor(_rng(seed, _P_DEP).uniform(0.0, n_steps * 0.5, size=n_master) / 0.5).astype(np.int32)
    alpha = _rng(seed, _P_ALPHA).uniform(0.05, 0.40, size=n_master).astype(np.float32)
    master = Workload("grid10x10_master", net, route_off, route_edges, dep, np.zeros(n_master, np.uint8), alpha,
                      base_params(1, seed), n_steps, info={"departures": "U[0, 2 h)"})
    return master, ensemble_scenarios(n_scen, base, net.n_edges, seed)


# --------------------------------------------------------------------------- loaded states
def _conn_index(net: Network, e: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Index of the move (e -> f) in the connection list (moves are sorted by
    (e, f), so their keys are sorted); -1 where there is no such move."""
    E = np.int64(net.n_edges)
    ce = np.repeat(np.arange(net.n_edges, dtype=np.int64), np.diff(net.conn_off))
    keys = ce * E + net.conn_to.astype(np.int64)
    q = e.astype(np.int64) * E + f.astype(np.int64)
    k = np.minimum(np.searchsorted(keys, q), max(keys.shape[0] - 1, 0))
    return np.where((keys.shape[0] > 0) & (keys[k] == q), k, -1)


# for each 8-bit lane mask: its set bits, lowest first (padded with the last)
_MASK_BITS = np.array([([b for b in range(8) if (m >> b) & 1] + [0] * 8)[:8] for m in range(256)],
                      dtype=np.int64)
_MASK_POP = np.array([bin(m).count("1") for m in range(256)], dtype=np.int64)


def entry_lanes(w: Workload) -> np.ndarray:
    """The entry lane of every vehicle: the lowest lane of its first edge that
    may take its second edge (lane 0 for a one-edge route)."""
    ro, re_ = w.route_off, w.route_edges
    rl = np.diff(ro)
    out = np.zeros(w.n_vehicles, np.int32)
    two = np.nonzero(rl > 1)[0]
    if two.size:
        c = _conn_index(w.net, re_[ro[two]], re_[ro[two] + 1])
        out[two] = _MASK_BITS[w.net.conn_mask[c].astype(np.int64), 0]
    return out


def loaded_state(w: Workload, t0: int, speed_frac: float = 0.6, gap_m: float = 2.5,
                 seed: int = 0, chunk: int = 250_000) -> dict:
    """A mid-run state at step t0, built from the demand alone (an input, like
    the demand itself): every vehicle that departed before t0 is placed where
    its route would take it driving each edge at speed_frac x its limit; if
    that is past the end of its route it has arrived.  An active vehicle gets
    a lane drawn uniformly among those that may take its next move (any lane
    on its last edge).  In each lane, from the front back, a vehicle is moved
    back as needed to keep at least gap_m metres behind its leader's rear,
    and its speed is capped at (gap - 2 m) / 1.5 s (a 1.5 s time headway);
    a vehicle pushed behind the lane start is tried in another lane of its
    edge, then at the end of its previous route edge, and is finally counted
    as arrived (info['unplaced']).  Vehicles due at t0 or later wait.
    Returns the sim_state fields by vehicle id, with t = t0 and the counters
    left to the simulation (None); info has the counts."""
    net, p = w.net, w.params
    dt = float(p.dt)
    N = w.n_vehicles
    ro, re_ = w.route_off, w.route_edges
    rl = np.diff(ro)
    r = _rng(seed, _P_PREFILL)
    L64 = net.length.astype(np.float64)
    tt_edge = L64 / (speed_frac * net.limit.astype(np.float64))
    status = np.zeros(N, np.uint8)
    cursor = np.zeros(N, np.int32)
    x = np.zeros(N, np.float64)
    tau_in = np.full(N, -1.0)
    t_arr = np.full(N, -1.0)
    dep = w.depart_step.astype(np.int64)
    gone = np.nonzero(dep < t0)[0]
    for s in range(0, gone.size, chunk):
        ids = gone[s:s + chunk]
        n = ids.size
        lens = rl[ids]
        base = np.repeat(ro[ids] - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
        pos = base + np.arange(int(lens.sum()))
        seg = tt_edge[re_[pos]]
        csum = np.cumsum(seg)
        first = np.concatenate([[0], np.cumsum(lens)[:-1]])
        start_val = np.concatenate([[0.0], csum])[first]
        excl = csum - seg - np.repeat(start_val, lens)          # time at the start of each route edge
        total = excl[first + lens - 1] + seg[first + lens - 1]
        elapsed = (t0 - dep[ids]) * dt
        arrived = elapsed >= total
        big = 1e7
        rank = np.repeat(np.arange(n, dtype=np.float64), lens)
        key = rank * big + excl
        k = np.searchsorted(key, np.arange(n, dtype=np.float64) * big + np.minimum(elapsed, total), side="right") - 1
        k = np.maximum(k, first)
        kk = np.where(arrived, first + lens - 1, k)
        cursor[ids] = (kk - first).astype(np.int32)
        frac = np.clip((elapsed - excl[kk]) / seg[kk], 0.0, 1.0)
        e = re_[pos[kk]]
        x[ids] = np.where(arrived, L64[e], frac * L64[e])
        tau_in[ids] = dep[ids] * dt + excl[kk]
        t_arr[ids] = np.where(arrived, dep[ids] * dt + total, -1.0)
        status[ids] = np.where(arrived, 2, 1).astype(np.uint8)
    edge = re_[ro[:-1] + cursor].astype(np.int32)
    lanes = net.lanes.astype(np.int64)
    has_next = cursor + 1 < rl
    nxt = np.where(has_next, re_[np.minimum(ro[:-1] + cursor + 1, re_.shape[0] - 1)], -1)
    act = np.nonzero(status == 1)[0]
    mask = np.full(N, 0, np.int64)
    hn = act[has_next[act]]
    mask[hn] = net.conn_mask[_conn_index(net, edge[hn], nxt[hn])].astype(np.int64)
    last = act[~has_next[act]]
    mask[last] = (1 << lanes[edge[last]]) - 1
    lane = entry_lanes(w).astype(np.int64)
    pick = np.floor(r.random(act.size) * _MASK_POP[mask[act]]).astype(np.int64)
    lane[act] = _MASK_BITS[mask[act], pick]
    vlen = float(p.veh_len.max())
    step_m = vlen + gap_m
    unplaced = np.zeros(N, bool)
    for attempt in range(4):
        act = np.nonzero(status == 1)[0]
        order = act[np.lexsort((-act, -x[act], lane[act], edge[act]))]
        ge = edge[order].astype(np.int64) * 8 + lane[order]
        run_start = np.concatenate([[True], ge[1:] != ge[:-1]])
        run_id = np.cumsum(run_start) - 1
        first_of_run = np.nonzero(run_start)[0]
        j = np.arange(order.size) - first_of_run[run_id]
        y = x[order] + j * step_m - run_id * 1e9
        pm = np.minimum.accumulate(y) + run_id * 1e9
        xs = pm - j * step_m
        x[order] = xs
        bad = order[xs < 0.0]
        if bad.size == 0:
            break
        if attempt == 0:            # another lane of the same edge, drawn uniformly
            lane[bad] = np.floor(r.random(bad.size) * lanes[edge[bad]]).astype(np.int64)
            x[bad] = np.maximum(x[bad], 0.0) + 0.0
        elif attempt in (1, 2):     # the end of the previous route edge
            back = bad[cursor[bad] > 0]
            stay = bad[cursor[bad] == 0]
            cursor[back] -= 1
            edge[back] = re_[ro[back] + cursor[back]]
            e2 = edge[back]
            f2 = re_[ro[back] + cursor[back] + 1]
            m2 = net.conn_mask[_conn_index(net, e2, f2)].astype(np.int64)
            lane[back] = _MASK_BITS[m2, np.floor(r.random(back.size) * _MASK_POP[m2]).astype(np.int64)]
            x[back] = L64[e2]
            tau_in[back] = tau_in[back] - tt_edge[e2]
            lane[stay] = np.floor(r.random(stay.size) * lanes[edge[stay]]).astype(np.int64)
        else:
            unplaced[bad] = True
            status[bad] = 2
            t_arr[bad] = t0 * dt
            x[bad] = L64[edge[bad]]
    # speeds: speed_frac x limit, capped by the time headway to the leader's rear
    act = np.nonzero(status == 1)[0]
    order = act[np.lexsort((-act, -x[act], lane[act], edge[act]))]
    ge = edge[order].astype(np.int64) * 8 + lane[order]
    lead_same = np.concatenate([[False], ge[1:] == ge[:-1]])
    v = np.zeros(N, np.float64)
    vfree = speed_frac * net.limit.astype(np.float64)[edge[order]]
    gap = np.full(order.size, np.inf)
    gap[1:] = x[order[:-1]] - vlen - x[order[1:]]
    gap = np.where(lead_same, gap, np.inf)
    v[order] = np.clip(np.minimum(vfree, (gap - 2.0) / 1.5), 0.0, None)
    arr = status == 2
    lane[arr] = 0
    lane[status == 0] = entry_lanes(w)[status == 0]
    x32 = x.astype(np.float32)
    x32[arr] = net.length[edge[arr]]
    x32 = np.minimum(x32, net.length[edge])
    x32[status == 0] = 0.0
    v32 = v.astype(np.float32)
    v32[status != 1] = 0.0
    state = dict(status=status, edge=edge, lane=lane.astype(np.int32), cursor=cursor, x=x32, v=v32,
                 held_since=np.full(N, -1, np.int32), mand=np.zeros(N, np.uint8), ww=np.zeros(N, np.int32),
                 tau_in=np.where(status == 0, -1.0, tau_in), t_arr=np.where(status == 2, t_arr, -1.0),
                 counters=None, t=int(t0))
    info = dict(active=int((status == 1).sum()), arrived=int(arr.sum()), waiting=int((status == 0).sum()),
                unplaced=int(unplaced.sum()), speed_frac=speed_frac, gap_m=gap_m)
    return state, info


# --------------------------------------------------------------------------- roofline probe
def probe_r(replica_net: Network = None, density: float = 0.3, route_len: int = 12, seed: int = 0,
            params: Params = None):
    """A network filled in steady state, to measure the step where its data
    cannot stay in the last-level cache: on every lane of every edge,
    vehicles spaced evenly at `density` x jam density (one vehicle per
    length + 2 m of lane), each at the equilibrium speed of a 1.5 s time
    headway to the one ahead (at most the limit), all active from step 0.
    Each vehicle's route starts at its edge and continues `route_len` - 1
    edges by a random walk over the allowed moves (drawn uniformly).  Four
    classes as the metropolitan workload.  Returns (workload, state); the
    state is indexed by vehicle id and written with sim_write_state."""
    net = replica_net if replica_net is not None else metro_network(seed=seed)
    p = params or jitter_params(base_params(4, seed), 0.10, seed, purpose=_P_CLASSPAR)
    r = _rng(seed, _P_PREFILL)
    vlen = float(p.veh_len.max())
    jam = vlen + 2.0
    L = net.length.astype(np.float64)
    lanes = net.lanes.astype(np.int64)
    per_lane = np.floor(density * L / jam).astype(np.int64)          # vehicles on each lane of edge e
    per_edge = per_lane * lanes
    n = int(per_edge.sum())
    e_of = np.repeat(np.arange(net.n_edges), per_edge)
    first = np.concatenate([[0], np.cumsum(per_edge)[:-1]])
    k_in_edge = np.arange(n) - np.repeat(first, per_edge)
    pl = np.repeat(per_lane, per_edge)
    lane = k_in_edge // np.maximum(pl, 1)
    rank = k_in_edge % np.maximum(pl, 1)                              # 0 = front of the lane
    spacing = L[e_of] / np.maximum(pl, 1)
    x = L[e_of] - (rank + 0.5) * spacing
    gap = spacing - vlen
    v = np.clip(np.minimum(net.limit.astype(np.float64)[e_of], (gap - 2.0) / 1.5), 0.0, None)
    # random-walk routes over the allowed moves
    deg = np.diff(net.conn_off).astype(np.int64)
    routes = np.empty((n, route_len), np.int32)
    cur = e_of.astype(np.int64)
    routes[:, 0] = cur
    for k in range(1, route_len):
        pick = np.floor(r.random(n) * deg[cur]).astype(np.int64)
        cur = net.conn_to[net.conn_off[cur] + pick].astype(np.int64)
        routes[:, k] = cur
    route_off = np.arange(n + 1, dtype=np.int64) * route_len
    vclass = r.integers(0, p.n_classes, size=n).astype(np.uint8)
    alpha = r.uniform(0.05, 0.40, size=n).astype(np.float32)
    w = Workload(f"probe_r_d{density}", net, route_off, routes.ravel(), np.zeros(n, np.int32), vclass, alpha, p,
                 route_len * 8, info={"density": density, "vehicles": n})
    state = dict(status=np.ones(n, np.uint8), edge=e_of.astype(np.int32), lane=lane.astype(np.int32),
                 cursor=np.zeros(n, np.int32), x=x.astype(np.float32), v=v.astype(np.float32),
                 held_since=np.full(n, -1, np.int32), mand=np.zeros(n, np.uint8), ww=np.zeros(n, np.int32),
                 tau_in=np.zeros(n), t_arr=np.full(n, -1.0), counters=None, t=0)
    return w, state


def replicate_state(state: dict, n_edges: int, copies: int) -> dict:
    """The state of an ensemble whose scenarios all take the whole master
    demand: scenario k's vehicles follow scenario k - 1's, on its own copy of
    the network (edge ids shifted by k x n_edges)."""
    out = {}
    for key, a in state.items():
        if key in ("t", "counters"):
            out[key] = a
        elif key == "edge":
            out[key] = np.concatenate([a + k * n_edges for k in range(copies)]).astype(np.int32)
        else:
            out[key] = np.concatenate([a] * copies)
    return out


CONFIGS = {"grid10x10": config1, "perturbed_grid_ring": config2, "metro": config3}
