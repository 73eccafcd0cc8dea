"""Host logic of the calibration loop (Sec. IV-A), on a stand-in objective:
the range schedule (1, 0.1, 0.01, ...), clipping to the bounds, binary32
parameters, the nominal set kept, first-on-ties choice and the stopping rule;
and the speed and L1 loss of Eq. (5)."""
import numpy as np

import workloads as W


def test_speeds_and_l1_loss():
    from paper_2007_03614_amd import calibrate as C
    sp = C.edge_speeds(np.array([10.0, 0.0, 20.0, 5.0]), np.array([2, 0, 1, 3]), np.array([100.0, 50.0, 100.0, 10.0]))
    assert np.isnan(sp[1]) and sp[0] == 10.0 and sp[2] == 5.0 and sp[3] == 2.0
    loss, n = C.l1_speed_loss(sp, np.array([9.0, 3.0, np.nan, 4.0]))
    assert n == 2 and loss == 1.0 + 2.0


def test_random_search_schedule_on_a_stand_in_objective():
    from paper_2007_03614_amd import calibrate as C
    w = W.config1(n_vehicles=10, n_steps=10)
    target = np.array([2.0, 3.0, 1.2, 2.5])
    calls = []

    def evaluate(sets):
        calls.append([np.array(s) for s in sets])
        return [(float(np.abs(np.asarray(s) - target).sum()), 1) for s in sets]

    deltas = np.random.default_rng(0).uniform(-1, 1, (4, 4, 4))
    deltas[0, 0] = [-50.0, -50.0, 50.0, 50.0]          # clipped to (lo, lo, hi, hi)
    th, hist = C.random_search(w, None, 0, deltas, tol=0.0, evaluate=evaluate)
    lo, hi = C._bounds_arrays()
    assert [h["range"] for h in hist] == [1.0, 0.1, 0.01, 0.001]
    assert np.array_equal(calls[0][1], np.array([lo[0], lo[1], hi[2], hi[3]]))
    for it, sets in enumerate(calls):
        nom = sets[0]
        for j in range(1, 5):
            exp = np.clip(nom + 10.0 ** -it * deltas[it][j - 1], lo, hi).astype(np.float32).astype(np.float64)
            assert np.array_equal(sets[j], exp)
        if it + 1 < len(calls):
            best = int(np.argmin([np.abs(s - target).sum() for s in sets]))
            assert np.array_equal(calls[it + 1][0], sets[best])
    best = [h["losses"][h["best"]] for h in hist]
    assert all(x >= y for x, y in zip(best, best[1:]))
    # stopping rule: a tolerance above the first best loss ends after one iteration
    _, h1 = C.random_search(w, None, 0, deltas, tol=1e9, evaluate=evaluate)
    assert len(h1) == 1
