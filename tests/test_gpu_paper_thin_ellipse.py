"""The paper's thin-ellipse study on the GPU stepper (FP64): errors and
convergence rates of u, p and X and the divergence error, at N = 64 ... 512,
for sigma = 0.1, 1 and 10, against the GM-IB columns the paper prints
(tests/golden/thin_ellipse_gm.json; Sec. "Thin Ellipse").

The four grids of one stiffness run as one batched ensemble (one context per
grid size, replayed from a hipGraph).  Restrictions follow the paper's
I^{2N->N}: a coarse face averages the fine faces that coincide with it, a
coarse cell the four fine cells, and the Lagrangian points are every other
fine point (N_s = 19N/4 doubles with N).  Norms are the paper's discrete l2
norms (h^2 weights on the grid, h_s on the membrane).  The paper's errors use
a BCM-IB run at N = 512 as the exact solution; here the GM run at N = 512
plays that part, so the errors are compared within a factor, the rates and
the divergence error (which need no reference) more closely."""
import json
import math
import os

import numpy as np
import pytest

from paper_1305_3976_amd import inputs
from helpers import LazyModule

ensemble = LazyModule("paper_1305_3976_amd.ensemble")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thin_ellipse_gm.json")
SIZES = (64, 128, 256, 512)


class Member:
    def __init__(self, n, dt, sigma, r1, r2, ppn):
        self.n, self.dt, self.sigma = n, dt, sigma
        self.structure = inputs.ellipse(int(round(ppn * n)), r1, r2, sigma)


def restrict_faces(u):
    """u[0] on x-faces (i h, (j + 1/2) h), u[1] on y-faces; arrays [y][x]."""
    return [0.5 * (u[0][0::2, 0::2] + u[0][1::2, 0::2]),
            0.5 * (u[1][0::2, 0::2] + u[1][0::2, 1::2])]


def restrict_cells(p):
    return 0.25 * (p[0::2, 0::2] + p[1::2, 0::2] + p[0::2, 1::2] + p[1::2, 1::2])


def down(field, kind, times):
    for _ in range(times):
        field = restrict_faces(field) if kind == "u" else restrict_cells(field)
    return field


def norm_grid(q, n):
    h2 = 1.0 / n ** 2
    if isinstance(q, list):
        return math.sqrt(h2 * sum(float(np.sum(c ** 2)) for c in q))
    return math.sqrt(h2 * float(np.sum(q ** 2)))


def norm_points(X):
    """(h_s sum_k |X_k|^2)^(1/2), h_s = 1/N_s: the paper's Lagrangian l2 norm."""
    return math.sqrt(float(np.sum(X ** 2)) / X.shape[1])


def printed_x_error(X):
    """The printed X errors equal h_s (sum_k |X_k|^2)^(1/2): N_s^(1/2) below the
    norm above at every N (the printed X rates follow the norm above)."""
    return math.sqrt(float(np.sum(X ** 2))) / X.shape[1]


def divergence(u, n):
    return (np.roll(u[0], -1, axis=1) - u[0] + np.roll(u[1], -1, axis=0) - u[1]) * n


def diff(qa, qb):
    if isinstance(qa, list):
        return [a - b for a, b in zip(qa, qb)]
    return qa - qb


@pytest.fixture(scope="module")
def study():
    g = json.load(open(GOLDEN))
    s = g["setup"]
    out = {}
    for key, case in g["cases"].items():
        sigma = float(key)
        steps = int(round(case["t"] / case["dt"]))
        members = [Member(n, case["dt"], sigma, s["r1"], s["r2"], s["points_per_N"]) for n in SIZES]
        ens = ensemble.Ensemble(members, rho=s["rho"], mu=s["mu"], precision=0)
        ens.run(steps, steps_per_launch=2)
        assert ens.sync() == [steps] * len(SIZES)
        out[key] = {m.n: ens.member_state(m) for m in members}
        ens.close()
    return g, out


def measured(states):
    """Errors (against the N = 512 run), divergence errors and rates."""
    err, rate = {}, {}
    ref = states[512]
    for n in (64, 128, 256):
        k = int(round(math.log2(512 // n)))
        st = states[n]
        e = {"u": norm_grid(diff(st["u"], down(ref["u"], "u", k)), n),
             "p": norm_grid(st["p"] - down(ref["p"], "p", k), n),
             "X": printed_x_error(st["X"] - ref["X"][:, ::2 ** k])}
        err[n] = e
    for n in SIZES:
        err.setdefault(n, {})["div"] = norm_grid(divergence(states[n]["u"], n), n)
    for n in (64, 128):
        a, b, c = states[n], states[2 * n], states[4 * n]
        r = {}
        for q in ("u", "p"):
            num = norm_grid(diff(a[q], down(b[q], q, 1)), n)
            den = norm_grid(diff(b[q], down(c[q], q, 1)), 2 * n)
            r[q] = math.log2(num / den)
        num = norm_points(a["X"] - b["X"][:, ::2])
        den = norm_points(b["X"] - c["X"][:, ::2])
        r["X"] = math.log2(num / den)
        rate[n] = r
    return err, rate


@pytest.mark.parametrize("key", ["0.1", "1", "10"])
def test_thin_ellipse_against_printed_gm_columns(study, key):
    g, out = study
    paper = g["cases"][key]
    err, rate = measured(out[key])
    print("sigma", key)
    for n in (64, 128):
        print("  rate N=%d ours %s paper %s" % (n, {q: round(v, 2) for q, v in rate[n].items()},
                                               paper["rate"][str(n)]))
    for n in SIZES:
        print("  error N=%d ours %s paper %s" % (n, {q: "%.3g" % v for q, v in err[n].items()},
                                                paper["error"][str(n)]))
    # divergence error: same definition, no reference solution -- the paper
    # prints three digits, which the stepper reproduces
    for n in SIZES:
        mine, theirs = err[n]["div"], paper["error"][str(n)]["div"]
        assert abs(mine - theirs) <= 0.01 * theirs, (key, n, mine, theirs)
    # rates: same scheme, same estimator (no reference solution involved)
    for n in (64, 128):
        for q in ("u", "p", "X"):
            assert abs(rate[n][q] - paper["rate"][str(n)][q]) <= 0.15, (key, n, q, rate[n][q])
    # errors against the finest run: the paper's reference is a BCM-IB run at
    # N = 512, ours the GM run; the membrane position hardly depends on it
    # (within 15 %), u and p are compared within a factor 2
    for n in (64, 128):
        for q in ("u", "p", "X"):
            mine, theirs = err[n][q], paper["error"][str(n)][q]
            f = 1.15 if q == "X" else 2.0
            assert theirs / f <= mine <= theirs * f, (key, n, q, mine, theirs)


def polygon_area(X):
    """Shoelace area of the closed polygon through the points (unwrapped)."""
    x, y = X[0], X[1]
    return 0.5 * abs(float(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1))))


def test_thin_ellipse_area_loss_and_leak_rate():
    """sigma = 1, dt = 0.04/512 to t = 4 at N = 64 ... 512: the relative loss
    of enclosed area at t = 4 and the leak rate (least-squares slope of the
    relative area loss over t in [2, 4]) against the paper's GM column."""
    g = json.load(open(GOLDEN))
    s, a = g["setup"], g["area"]
    members = [Member(n, a["dt"], a["sigma"], s["r1"], s["r2"], s["points_per_N"]) for n in SIZES]
    ens = ensemble.Ensemble(members, rho=s["rho"], mu=s["mu"], precision=0)
    a0 = math.pi * s["r1"] * s["r2"]
    every = 640                                     # samples every 0.05 time units
    total = int(round(a["t_end"] / a["dt"]))
    times, areas = [], {m.n: [] for m in members}
    done = 0
    while done < total:
        ens.run(min(every, total - done), steps_per_launch=2)
        done += min(every, total - done)
        t = done * a["dt"]
        if t >= a["leak_window"][0] - 1e-9:
            times.append(t)
            for m in members:
                areas[m.n].append(polygon_area(ens.member_state(m)["X"]))
    ens.close()
    times = np.array(times)
    for m in members:
        loss = (a0 - np.array(areas[m.n])) / a0
        slope = float(np.polyfit(times, loss, 1)[0])
        pl, pr = a["loss_at_t_end"][str(m.n)], a["leak_rate"][str(m.n)]
        print("N=%d area loss at t=4 %.3g (paper %.3g), leak rate %.3g (paper %.3g)"
              % (m.n, loss[-1], pl, slope, pr))
        assert loss[-1] < 0.01                      # "less than one percent"
        # the stepper reproduces the printed three digits of both columns
        assert abs(slope - pr) <= 0.03 * pr, (m.n, slope, pr)
        assert abs(loss[-1] - pl) <= 0.03 * pl, (m.n, loss[-1], pl)
