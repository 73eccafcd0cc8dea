"""Error paths of the C ABI that need a device: an allocator that runs out
(SIM_ENOMEM, with every block it handed out given back), and states that
sim_write_state must refuse (SIM_EINVAL, the handle unchanged)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

# callbacks live for the whole process: a handle keeps the pointers it was
# created with and calls the release callback when it is destroyed
_cb = {}


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03614_amd as M
    return M


class Budget:
    """torch's caching allocator behind a counter: the first `limit` calls
    succeed, later ones return NULL."""

    def __init__(self):
        self.limit, self.calls, self.live = 0, 0, {}

    def alloc(self, nbytes, ctx):
        import torch
        self.calls += 1
        if self.calls > self.limit:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes))
        self.live[int(p)] = int(nbytes)
        return p

    def free(self, ptr, ctx):
        import torch
        self.live.pop(int(ptr))
        torch.cuda.caching_allocator_delete(int(ptr))


def _install(M, budget):
    if "fns" not in _cb:
        _cb["budget"] = budget
        _cb["fns"] = (M._ALLOC_FN(lambda n, c: _cb["budget"].alloc(n, c)),
                      M._FREE_FN(lambda p, c: _cb["budget"].free(p, c)))
    _cb["budget"] = budget
    M._check(M._lib.sim_set_allocator(_cb["fns"][0], _cb["fns"][1], None))


def test_out_of_memory_at_every_allocation_gives_enomem_and_no_leak(M):
    w = W.config1(n_vehicles=300, n_steps=100)
    w.params.record_every = 20
    probe = Budget()
    probe.limit = 10 ** 9
    _install(M, probe)
    sim = M.Sim(w, allocator="keep")
    sim.step(100)                      # creation and five checkpoints
    n_create = probe.calls
    sim.close()
    assert probe.live == {} and n_create > 10
    def attempt():
        s = None
        try:
            s = M.Sim(w, allocator="keep")
            s.step(100)
        finally:
            if s is not None:
                s.close()

    try:
        for limit in sorted({0, 1, 2, 5, n_create // 2, n_create - 1}):
            b = Budget()
            b.limit = limit
            _install(M, b)
            with pytest.raises(M.SimError) as ei:
                attempt()
            assert ei.value.name == "SIM_ENOMEM", (limit, str(ei.value))
            assert b.live == {}, (limit, len(b.live))
    finally:
        M.use_torch_allocator()


def _state(M, w, steps):
    sim = M.Sim(w)
    sim.step(steps)
    return sim, sim.state()


@pytest.mark.parametrize("what", ["overlap", "edge_not_at_cursor", "lane", "x_beyond_edge", "negative_v",
                                  "queue_order", "bad_status", "cursor"])
def test_write_state_refuses_inconsistent_states(M, what):
    w = W.config1(n_vehicles=400, n_steps=400)
    sim, s = _state(M, w, 400)
    act = np.nonzero(s["status"] == 1)[0]
    assert act.size > 20
    bad = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in s.items()}
    i = int(act[0])
    if what == "overlap":
        # the follower of a lane moved up to 1 m behind its leader's front
        key = s["edge"][act].astype(np.int64) * 8 + s["lane"][act]
        order = np.lexsort((-s["x"][act], key))
        pair = next(k for k in range(order.size - 1) if key[order[k]] == key[order[k + 1]])
        lead, fol = int(act[order[pair]]), int(act[order[pair + 1]])
        bad["x"][fol] = np.float32(s["x"][lead] - 1.0)
    elif what == "edge_not_at_cursor":
        bad["edge"][i] = (s["edge"][i] + 1) % w.net.n_edges
    elif what == "lane":
        bad["lane"][i] = int(w.net.lanes[s["edge"][i]])
    elif what == "x_beyond_edge":
        bad["x"][i] = np.float32(w.net.length[s["edge"][i]] + 1.0)
    elif what == "negative_v":
        bad["v"][i] = np.float32(-1.0)
    elif what == "queue_order":
        # the first vehicle of a departure queue back to waiting while a later
        # one of the same queue has left it
        gone = np.nonzero(s["status"] != 0)[0]
        q = W.entry_lanes(w)
        first = w.route_edges[w.route_off[:-1]]
        key = (first[gone].astype(np.int64) * 8 + q[gone]) * 16 + w.vclass[gone]
        order = np.lexsort((gone, w.depart_step[gone], key))
        k = next(j for j in range(order.size - 1) if key[order[j]] == key[order[j + 1]])
        v = int(gone[order[k]])
        bad["status"][v] = 0
        bad["edge"][v], bad["lane"][v], bad["cursor"][v] = int(first[v]), int(q[v]), 0
        bad["x"][v], bad["v"][v] = 0.0, 0.0
        bad["tau_in"][v], bad["t_arr"][v] = -1.0, -1.0
    elif what == "bad_status":
        bad["status"][i] = 3
    elif what == "cursor":
        bad["cursor"][i] = int(w.route_off[i + 1] - w.route_off[i])
    with pytest.raises(M.SimError) as ei:
        sim.write_state(bad)
    assert ei.value.name == "SIM_EINVAL", str(ei.value)
    # the handle is unchanged: it continues exactly like an untouched twin
    twin, _ = _state(M, w, 400)
    sim.step(50)
    twin.step(50)
    a, b = sim.state(), twin.state()
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
