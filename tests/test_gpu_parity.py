"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  The bar: discrete state (status, edge, lane, route
cursor, held/mandatory/wait flags) and event counters bit-exact; x and v
within 1e-5 relative (the contract makes them bitwise equal, which is also
reported); per-edge travel-time sums equal."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

DISCRETE = ("status", "edge", "lane", "cursor", "held_since", "mand", "ww")


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2007_03614_amd as M
    return M


def compare_states(g, o, where=""):
    for k in DISCRETE:
        a, b = np.asarray(g[k]), np.asarray(o[k]).astype(np.asarray(g[k]).dtype)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"{where}: {k} differs for vehicles {bad[:10].tolist()} gpu={a[bad[:5]]} oracle={b[bad[:5]]}"
    for k in ("x", "v"):
        a = np.asarray(g[k], np.float32)
        b = np.asarray(o[k], np.float32)
        err = np.abs(a.astype(np.float64) - b) / np.maximum(np.abs(b.astype(np.float64)), 1.0)
        assert err.max(initial=0.0) <= 1e-5, f"{where}: {k} max rel err {err.max()}"
    for k in ("tau_in", "t_arr"):
        a, b = np.asarray(g[k]), np.asarray(o[k])
        assert np.allclose(a, b, rtol=1e-9, atol=1e-9), f"{where}: {k}"
    return all(np.array_equal(np.asarray(g[k], np.float32), np.asarray(o[k], np.float32)) for k in ("x", "v"))


def run_pair(M, oracle_mod, w, checkpoints, init=None):
    g = M.Sim(w)
    o = oracle_mod.OracleSim(w)
    t = 0
    if init is not None:   # both sides start from the same written state
        g.write_state(init)
        o.write_state(init["t"], init)
        t = init["t"]
    bitwise = True
    for cp in checkpoints:
        g.step(cp - t)
        o.step(cp - t)
        t = cp
        gs, os_ = g.state(), o.state()
        assert gs["t"] == os_["t"] == t
        bitwise &= compare_states(gs, os_, f"step {t}")
        gc = dict(zip(M.COUNTERS, gs["counters"].tolist()))
        assert gc == o.counters(), f"step {t}: counters {gc} vs {o.counters()}"
    gsum, gcnt = g.edge_stats()
    osum, ocnt = o.edge_stats()
    assert np.array_equal(gcnt, ocnt)
    assert np.array_equal(gsum, osum), np.abs(gsum - osum).max()
    return g, o, bitwise


# ---------------------------------------------------------------- arithmetic
def test_fp32_division_sqrt_bitwise(M):
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.uniform(-50, 50, 1 << 20), rng.standard_normal(1 << 18) * 1e-30,
                        rng.uniform(1e-3, 1e3, 1 << 18)]).astype(np.float32)
    b = np.concatenate([rng.uniform(0.01, 40, 1 << 20), rng.uniform(0.1, 10, 1 << 18),
                        rng.uniform(-1e3, 1e3, 1 << 18)]).astype(np.float32)
    b[b == 0] = 1.0
    assert np.array_equal(M.probe_fp32(0, a, b), a / b)
    pos = np.abs(a)
    assert np.array_equal(M.probe_fp32(1, pos), np.sqrt(pos))
    assert np.array_equal(M.probe_fp32(2, a, b), a * b)
    assert np.array_equal(M.probe_fp32(3, a, b), a + b)


def test_eq2_exp_bitwise_vs_oracle(M, oracle_mod):
    bits_lo = int(np.float32(-17.0).view(np.uint32))
    ys = np.arange(0x80000000, bits_lo, 13, dtype=np.uint64).astype(np.uint32).view(np.float32)
    assert np.array_equal(M.probe_fp32(4, ys).view(np.uint32), oracle_mod.expf_c(ys).view(np.uint32))


def test_philox_vs_numpy_and_draws_vs_oracle(M, oracle_mod):
    from test_oracle_math import numpy_philox_block
    rng = np.random.default_rng(2)
    ctr = rng.integers(0, 2**63, size=(64, 4), dtype=np.uint64)
    key = np.array([987654321, 0], np.uint64)
    got = M.probe_philox(ctr, key)
    for k in range(ctr.shape[0]):
        assert got[k].tolist() == numpy_philox_block(ctr[k], key).tolist()
    t = rng.integers(0, 60000, 4000)
    vid = rng.integers(0, 3_000_000, 4000)
    u, e2, e3 = M.probe_draws(77, t, vid)
    for k in range(0, 4000, 7):
        assert u[k] == np.float32(oracle_mod.uniform(77, int(t[k]), int(vid[k]), 1))
        assert e2[k] == np.float32(oracle_mod.normal(77, int(t[k]), int(vid[k]), 2))
        assert e3[k] == np.float32(oracle_mod.normal(77, int(t[k]), int(vid[k]), 3))


# ---------------------------------------------------------------- trajectories
def test_parity_single_edge_free_road(M, oracle_mod):
    w = W.single_edge_workload(length=5000.0, n_vehicles=3, depart_step=[0, 0, 40], n_steps=600)
    _, _, bitwise = run_pair(M, oracle_mod, w, [1, 2, 5, 50, 200, 600])
    assert bitwise


@pytest.mark.parametrize("n", [30, 100])
def test_parity_ring_road(M, oracle_mod, n):
    """A closed one-lane ring: every vehicle crosses a node every few steps,
    so look-ahead across edge ends and admission run on every lap; n = 100
    keeps a stop-and-go wave alive."""
    w = W.ring_road(n)
    _, _, bitwise = run_pair(M, oracle_mod, w, [1, 25, 200, 1000, 3000])
    assert bitwise


def test_parity_config1_full(M, oracle_mod, c1):
    """10x10 grid, 2,000 vehicles, 3,600 steps: every 100 steps."""
    g, o, bitwise = run_pair(M, oracle_mod, c1, list(range(1, 20)) + list(range(100, 3601, 100)))
    assert bitwise
    st = g.state()
    assert (st["status"] == 2).all()


def test_parity_config1_four_classes(M, oracle_mod):
    w = W.config1(n_classes=4)
    w.params = W.jitter_params(w.params, 0.1, seed=5)
    _, _, bitwise = run_pair(M, oracle_mod, w, [10, 500, 1000, 2000, 3600])
    assert bitwise


def test_parity_long_edge_two_classes(M, oracle_mod):
    """One 8 km two-lane edge fed with 1,500 vehicles of two classes (v0
    factor 1 and 0.6): fast vehicles pass slow ones by the lane-change
    incentive."""
    p = W.base_params(2)
    p.v0_factor[1] = np.float32(0.6)
    w = W.single_edge_workload(length=8000.0, lanes=2, n_vehicles=1500, depart_step=np.arange(1500) // 2,
                               n_steps=2400, params=p)
    w.vclass[::3] = 1
    g, o, bitwise = run_pair(M, oracle_mod, w, [100, 600, 1200, 1800, 2400])
    assert bitwise
    assert o.counters()["lane_changes"] > 100


def test_parity_dense_queue_big_tiles(M, oracle_mod):
    """A 16 km two-lane edge that starts as a dense queue of 2,600 vehicles
    (7.5 m apart, speeds U[0, 6] m/s, written as the state at step 0).  As the
    queue discharges (about 0.4 vehicles per step), the edge runs first from
    the global-memory tile scratch (above 1,408 vehicles), then from the LDS
    of the 1,024-thread kernel; the first steps brake hard (stop branch)."""
    n = 2600
    w = W.single_edge_workload(length=16000.0, lanes=2, n_vehicles=n, depart_step=np.zeros(n, np.int32),
                               n_steps=0)
    rng = np.random.default_rng(3)
    i = np.arange(n)
    init = dict(status=np.ones(n, np.uint8), edge=np.full(n, int(w.route_edges[0]), np.int32),
                lane=(i % 2).astype(np.int32), cursor=np.zeros(n, np.int32),
                x=(16000.0 - 1.0 - 7.5 * (i // 2)).astype(np.float32),
                v=rng.uniform(0.0, 6.0, n).astype(np.float32), held_since=np.full(n, -1, np.int32),
                mand=np.zeros(n, np.uint8), ww=np.zeros(n, np.int32), tau_in=np.zeros(n),
                t_arr=np.full(n, -1.0), counters=None, t=0)
    g, o, bitwise = run_pair(M, oracle_mod, w, [1, 2, 10, 100, 400, 1000, 2000, 3000, 4000], init=init)
    assert bitwise
    c = o.counters()
    assert c["stop_branch"] > 0 and c["lane_changes"] > 0, c
    assert 384 < n - c["arrived"] < 1408, c   # started above the LDS of one workgroup, ends inside it
    # every step had a big tile: the big-tile part and the grid barrier of k_big_admit ran
    assert g.big_tile_updates() == c["active_sum"]


def _long_edge_grid(n=12000, t0=2400, seed=7):
    """A 3x3 grid of 2,500 m two-lane edges (a lane holds up to 333 vehicles
    7.5 m apart), uniform O/D routes, departures U[0, 1,500 s).  The state at
    t0 is built from the demand at 15 % of the limit, so most edges are dense
    queues: tiles above the LDS cap ask to move into other big tiles and into
    ordinary tiles, ordinary lanes ask to move into big tiles, and departures
    still due wait at the entry lanes of big tiles."""
    net = W.grid_network(rows=3, cols=3, spacing=2500.0, lanes=2)
    r = np.random.default_rng(seed)
    o = r.integers(0, net.n_nodes, n)
    d = (o + r.integers(1, net.n_nodes, n)) % net.n_nodes
    route_off, route_edges, ok = W.shortest_routes(net, o, d)
    assert ok.all()
    dep = r.integers(0, 3000, n).astype(np.int32)
    w = W.Workload("long_edge_grid", net, route_off, route_edges, dep, np.zeros(n, np.uint8),
                   r.uniform(0.05, 0.40, n).astype(np.float32), W.base_params(1), 0)
    init, _ = W.loaded_state(w, t0, speed_frac=0.15)
    return w, init


def _schedule_cache(tmp_path, w, g):
    """A schedule cache whose lines (one per size of the admission grid, the
    largest valid one applied last) give k_big_admit more workgroups than the
    network has edges, hence than big tiles."""
    p = tmp_path / "sched.txt"
    sch = g.schedule()
    with open(p, "w") as f:
        for g2 in (2, 4, 8, 16, 32, 64, 128, 256, 512, 1024):
            f.write(f"manta-schedule E={w.net.n_edges} L={int(w.net.lanes.sum())} N={w.n_vehicles} S=1 -> "
                    f"0 {sch[1]} {g2} {sch[3]}\n")
    return str(p)


@pytest.mark.parametrize("spread_admission", [False, True])
@pytest.mark.parametrize("intersection_mode", [0, 1])
def test_parity_big_tiles_with_transfers(M, oracle_mod, tmp_path, spread_admission, intersection_mode):
    """Big tiles that exchange vehicles with each other and with ordinary
    tiles, and take departures, bit for bit with the oracle: with one
    admission workgroup (every workgroup has a big tile: grid barrier, then
    admission) and with more admission workgroups than big tiles (admission
    of the other lanes alongside the big tiles, the rest by each tile's own
    workgroup); all green, and flashing red at every node (admission sets
    each request's node key)."""
    w, init = _long_edge_grid()
    w.params.intersection_mode = intersection_mode
    g = M.Sim(w)
    if spread_admission:
        g.autotune(_schedule_cache(tmp_path, w, g))
        assert g.schedule()[2] > w.net.n_edges
    else:
        assert g.schedule()[2] == 1
    o = oracle_mod.OracleSim(w)
    g.write_state(init)
    o.write_state(init["t"], init)
    t = init["t"]
    c0 = o.counters()
    for cp in (t + 1, t + 2, t + 50, t + 200, t + 600):
        g.step(cp - t)
        o.step(cp - t)
        t = cp
        gs, os_ = g.state(), o.state()
        assert compare_states(gs, os_, f"step {t}")
        gc = dict(zip(M.COUNTERS, gs["counters"].tolist()))
        assert gc == o.counters(), f"step {t}: counters {gc} vs {o.counters()}"
    c = o.counters()
    assert g.big_tile_updates() > 0
    assert c["transfers"] > c0["transfers"] and c["departed"] > c0["departed"], (c0, c)
    gsum, gcnt = g.edge_stats()
    osum, ocnt = o.edge_stats()
    assert np.array_equal(gcnt, ocnt) and np.array_equal(gsum, osum)


@pytest.mark.parametrize("g1", [16, 5])
def test_parity_tile_counters(M, oracle_mod, tmp_path, g1):
    """Few tile workgroups, set through a schedule cache, so that a step has
    more rounds of tiles than the threshold above which k_tile_step hands
    out the tiles after each workgroup's first from its counters: full-size
    config 2 from the state its demand gives at 08:00 (about 60,000 active,
    20 or 60 rounds), 100 steps bit for bit with the oracle; with 5
    workgroups, fewer workgroups than counter groups."""
    w = W.config2()
    init, _ = W.loaded_state(w, 10_800, speed_frac=0.4)
    n_act = int((init["status"] == 1).sum())
    rounds = -(-n_act // (192 * g1))
    assert rounds > 8, (n_act, rounds)
    g = M.Sim(w)
    sch = g.schedule()
    p = tmp_path / "sched.txt"
    p.write_text(f"manta-schedule E={w.net.n_edges} L={int(w.net.lanes.sum())} N={w.n_vehicles} S=1 -> "
                 f"0 {g1} {sch[2]} {sch[3]}\n")
    assert g.autotune(str(p))[1] == g1
    o = oracle_mod.OracleSim(w)
    g.write_state(init)
    o.write_state(init["t"], init)
    t = init["t"]
    oracle_mod.set_threads(0)
    try:
        for cp in (t + 1, t + 2, t + 30, t + 100):
            g.step(cp - t)
            o.step(cp - t)
            t = cp
            gs, os_ = g.state(), o.state()
            assert compare_states(gs, os_, f"g1 {g1} step {t}")
            gc = dict(zip(M.COUNTERS, gs["counters"].tolist()))
            assert gc == o.counters(), f"step {t}: counters {gc} vs {o.counters()}"
    finally:
        oracle_mod.set_threads(1)
    gsum, gcnt = g.edge_stats()
    osum, ocnt = o.edge_stats()
    assert np.array_equal(gcnt, ocnt) and np.array_equal(gsum, osum)


def test_parity_scaled_config2(M, oracle_mod):
    """Config 2's recipe on a 30x30 grid + ring with 15,000 vehicles, full 3 h."""
    w = W.scaled_config2(n_vehicles=15000, rows=30, cols=30, n_steps=21600)
    _, _, bitwise = run_pair(M, oracle_mod, w, [1000, 5000, 9000, 13000, 17000, 21600])
    assert bitwise


def test_parity_config2_full_size_prefix(M, oracle_mod):
    """Full-size config 2 (200,000 vehicles, 35,800 edges): parity over the
    first 2,400 steps, which the oracle finishes in seconds."""
    w = W.config2()
    _, _, bitwise = run_pair(M, oracle_mod, w, [600, 1200, 2400])
    assert bitwise


def test_edge_means_on_the_device(M, oracle_mod, c1):
    """sim_read_edge_means: sum / count per edge computed on the device equals
    the division of sim_read_edge_stats' arrays and the oracle's means, bit
    for bit, with 0 where no traversal completed."""
    g = M.Sim(c1)
    o = oracle_mod.OracleSim(c1)
    g.step(1500)
    o.step(1500)
    mean, cnt = g.mean_travel_times()
    s, c = g.edge_stats()
    assert np.array_equal(cnt, c) and (c == 0).any() and (c > 0).any()
    assert np.array_equal(mean, np.where(c > 0, s / np.maximum(c, 1), 0.0))
    os_, oc = o.edge_stats()
    assert np.array_equal(mean, np.where(oc > 0, os_ / np.maximum(oc, 1), 0.0))


def test_gridlock_detector(M, oracle_mod):
    """The stopped ring of the oracle's detector tests (60 vehicles on 400 m,
    every gap below s0): both sides count a step from the 600th stalled one
    on, and the run restarts at a written state."""
    from test_oracle_sim import stopped_ring
    w, st = stopped_ring()
    g, o, bitwise = run_pair(M, oracle_mod, w, [599, 600, 700], init=st)
    assert bitwise and o.counters()["gridlock_steps"] == 101
    s = g.state()
    g.write_state(dict(s, counters=None))
    g.step(599)
    assert g.counters()["gridlock_steps"] == 101
    g.step(1)
    assert g.counters()["gridlock_steps"] == 102


def test_determinism_and_resume(M, c1):
    a = M.Sim(c1)
    a.step(2000)
    sa = a.state()
    b = M.Sim(c1)
    b.step(1000)
    mid = b.state()
    c = M.Sim(c1)
    c.write_state(mid)
    c.step(1000)
    b.step(1000)
    for s in (b.state(), c.state()):
        for k in sa:
            if k == "t":
                assert s[k] == sa[k]
            else:
                assert np.array_equal(np.asarray(s[k]), np.asarray(sa[k])), k


def test_empty_and_tiny_inputs(M, oracle_mod):
    w = W.single_edge_workload(length=100.0, n_vehicles=1, depart_step=[5], n_steps=50)
    run_pair(M, oracle_mod, w, [1, 5, 6, 7, 50])
    w0 = W.single_edge_workload(length=100.0, n_vehicles=0, n_steps=5)
    g = M.Sim(w0)
    g.step(5)
    assert g.state()["t"] == 5 and g.n_active == 0
