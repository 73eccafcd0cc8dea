"""Calibration of the car-following parameters against observed per-edge
speeds (Sec. IV-A, Eqs. (5)-(6)).

* ``random_search``: the paper's loop.  Each iteration runs several parameter
  sets of (a, b, T, s0) -- here all of them in one ensemble handle, one
  scenario per set -- scores each by the L1 distance between simulated and
  observed edge speeds, keeps the best as the nominal set, and perturbs it by
  uniform draws whose range shrinks tenfold per iteration.
* ``gradient_descent``: the same loss minimised with the adjoint of the step
  (``Sim.backward``), one recorded forward run and one reverse sweep per
  iteration.

Simulated edge speed: edge length over the mean completed traversal time
(the statistic the step keeps per edge); edges without a traversal in the
simulation or without an observation are left out of the loss."""
from __future__ import annotations

import numpy as np

from . import Sim

# (T, a, b, s0) bounds of Sec. IV-A; v0_factor is not calibrated
BOUNDS = {"T": (0.1, 2.0), "a": (1.0, 10.0), "b": (1.0, 10.0), "s0": (1.0, 5.0)}
CALIBRATED = ("a", "b", "T", "s0")            # the parameters of Eq. (6), in this order
_COL = {"v0_factor": 0, "T": 1, "a": 2, "b": 3, "s0": 4}
MPH = 0.44704                                  # m/s


def edge_speeds(mean_tt: np.ndarray, cnt: np.ndarray, length: np.ndarray) -> np.ndarray:
    """Length over mean traversal time; NaN where nothing completed the edge."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where((cnt > 0) & (mean_tt > 0), np.asarray(length, np.float64) / mean_tt, np.nan)


def l1_speed_loss(speed: np.ndarray, observed: np.ndarray):
    """Eq. (5): sum over matched edges of |simulated - observed| speed, and the
    number of matched edges."""
    m = np.isfinite(speed) & np.isfinite(observed)
    return float(np.abs(speed[m] - observed[m]).sum()), int(m.sum())


def _bounds_arrays():
    lo = np.array([BOUNDS[k][0] for k in CALIBRATED])
    hi = np.array([BOUNDS[k][1] for k in CALIBRATED])
    return lo, hi


def class_params(workload, theta) -> np.ndarray:
    """[1, 5] (v0_factor, T, a, b, s0) of the workload's single class with
    (a, b, T, s0) = theta, as binary32."""
    p = workload.params
    row = np.array([p.v0_factor[0], p.T[0], p.a[0], p.b[0], p.s0[0]], np.float64)
    for k, name in enumerate(CALIBRATED):
        row[_COL[name]] = theta[k]
    return row.astype(np.float32).reshape(1, 5)


def evaluate_sets(workload, sets, observed, steps: int, stream=None):
    """One ensemble handle, one scenario per parameter set (the workload's
    whole demand on its network); returns the L1 loss and matched-edge count
    of every set."""
    n = int(workload.depart_step.shape[0])
    scen = [(n, np.zeros(0, np.int32), class_params(workload, th)) for th in sets]
    sim = Sim(workload, stream=stream, scenarios=scen)
    sim.step(steps)
    mean, cnt = sim.mean_travel_times()
    sim.close()
    E = workload.net.n_edges
    out = []
    for k in range(len(sets)):
        sp = edge_speeds(mean[k * E:(k + 1) * E], cnt[k * E:(k + 1) * E], workload.net.length)
        out.append(l1_speed_loss(sp, observed))
    return out


def random_search(workload, observed, steps: int, deltas: np.ndarray, theta0=None, tol: float = 0.05 * MPH,
                  evaluate=None, stream=None):
    """The paper's calibration loop for a one-class workload.

    deltas: [iterations, n_sets - 1, 4] draws of U[-1, 1] for (a, b, T, s0),
    from the caller's seeded generator.  Iteration i (from 0) evaluates the
    nominal set and nominal + 10^-i * deltas[i][j], clipped to the bounds,
    with parameters rounded to binary32; the set of smallest loss (first on
    ties) becomes the nominal.  Stops once the mean difference per matched
    edge falls below tol (0.05 mph).  evaluate(sets) -> [(loss, matched)]
    defaults to one GPU ensemble per iteration.
    Returns (theta, history)."""
    p = workload.params
    lo, hi = _bounds_arrays()
    nominal = (np.array([p.a[0], p.b[0], p.T[0], p.s0[0]], np.float64) if theta0 is None
               else np.asarray(theta0, np.float64))
    nominal = nominal.astype(np.float32).astype(np.float64)
    if evaluate is None:
        def evaluate(sets):
            return evaluate_sets(workload, sets, observed, steps, stream)
    hist = []
    for it in range(deltas.shape[0]):
        r = 10.0 ** (-it)
        sets = [nominal] + [np.clip(nominal + r * deltas[it][j], lo, hi).astype(np.float32).astype(np.float64)
                            for j in range(deltas.shape[1])]
        res = evaluate(sets)
        losses = np.array([x[0] for x in res])
        best = int(np.argmin(losses))
        nominal = sets[best]
        mean_diff = losses[best] / max(res[best][1], 1)
        hist.append({"iteration": it + 1, "range": r, "sets": [s.tolist() for s in sets],
                     "losses": losses.tolist(), "best": best, "mean_diff_mps": mean_diff})
        if mean_diff < tol:
            break
    return nominal, hist


def gradient_descent(workload, observed, steps: int, iterations: int, lr: float = 0.2, decay: float = 0.5,
                     theta0=None, record_every: int = 120, stream=None):
    """Projected descent on the Eq. (5) loss with the adjoint gradient.  Each
    step moves every parameter by lr * decay^i of its bounds range, scaled by
    its share of the largest range-scaled gradient component.
    Returns (theta, history)."""
    import copy
    lo, hi = _bounds_arrays()
    p = workload.params
    th = (np.array([p.a[0], p.b[0], p.T[0], p.s0[0]], np.float64) if theta0 is None
          else np.asarray(theta0, np.float64)).astype(np.float32).astype(np.float64)
    cols = [_COL[k] for k in CALIBRATED]
    hist = []
    for it in range(iterations):
        w = copy.copy(workload)
        w.params = copy.copy(workload.params)
        cp = class_params(workload, th)[0]
        w.params.v0_factor, w.params.T, w.params.a, w.params.b, w.params.s0 = (
            cp[0:1].copy(), cp[1:2].copy(), cp[2:3].copy(), cp[3:4].copy(), cp[4:5].copy())
        w.params.record_every = record_every
        sim = Sim(w, stream=stream)
        sim.step(steps)
        mean, cnt = sim.mean_travel_times()
        sp = edge_speeds(mean, cnt, workload.net.length)
        loss, nm = l1_speed_loss(sp, observed)
        use = np.isfinite(sp) & np.isfinite(observed)
        # d|L/m - u|/dm = -sign(L/m - u) L / m^2
        dl = np.zeros_like(mean)
        L = np.asarray(workload.net.length, np.float64)
        dl[use] = -np.sign(sp[use] - observed[use]) * L[use] / (mean[use] ** 2)
        g = sim.backward(dl)[0][cols]
        sim.close()
        hist.append({"iteration": it + 1, "theta": th.tolist(), "loss": loss, "mean_diff_mps": loss / max(nm, 1),
                     "grad": g.tolist()})
        scaled = g * (hi - lo)
        m = np.abs(scaled).max()
        if m == 0.0:
            break
        th = np.clip(th - lr * decay ** it * (hi - lo) * scaled / m, lo, hi).astype(np.float32).astype(np.float64)
    return th, hist
