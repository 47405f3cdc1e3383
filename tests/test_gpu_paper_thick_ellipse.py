"""The paper's thick elliptical shell on the GPU stepper (FP64): a nested
family of closed fibers with stiffness sigma(r) = 1 - cos(2 pi r) across the
shell (Sec. "Thick Elliptical Shell").  Against the GM-IB row of the
convergence-rate table at t = 0.4 (three viscosities) and the table of
divergence errors (mu = 0.01, N = 64 ... 512, six time steps), stored in
tests/golden/thick_ellipse_gm.json.

Readings: fiber l of N_r sits at r_l = (l + 1/2)/N_r (the paper gives
s, r in [0, 1] and N_s = 75N/16, N_r = 3N/8 without the placement), so the
fibers of grid N are the means of fiber pairs (2l, 2l + 1) of grid 2N at
every other point s -- the Lagrangian restriction used by the rates.  The
grid restrictions and norms are those of the thin-ellipse study (faces
averaged over the coinciding fine faces, cells over four fine cells, h^2
weights); the Lagrangian norm weighs each point by h_s h_r."""
import json
import math
import os

import numpy as np
import pytest

from paper_1305_3976_amd import inputs
from helpers import LazyModule

ensemble = LazyModule("paper_1305_3976_amd.ensemble")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thick_ellipse_gm.json")


class Member:
    def __init__(self, n, dt, s):
        self.n, self.dt = n, dt
        self.ns = int(round(s["ns_per_N"] * n))
        self.nr = int(round(s["nr_per_N"] * n))
        self.structure = inputs.thick_ellipse(self.ns, self.nr, s["r1"], s["r2"], s["gamma"])


def restrict_faces(u):
    return [0.5 * (u[0][0::2, 0::2] + u[0][1::2, 0::2]),
            0.5 * (u[1][0::2, 0::2] + u[1][0::2, 1::2])]


def restrict_cells(p):
    return 0.25 * (p[0::2, 0::2] + p[1::2, 0::2] + p[0::2, 1::2] + p[1::2, 1::2])


def restrict_points(X, nr, ns):
    """Fine shell (nr fibers of ns points) -> coarse shell (nr/2 by ns/2)."""
    Xf = X.reshape(2, nr, ns)
    return (0.5 * (Xf[:, 0::2, 0::2] + Xf[:, 1::2, 0::2])).reshape(2, -1)


def norm_grid(q, n):
    h2 = 1.0 / n ** 2
    if isinstance(q, list):
        return math.sqrt(h2 * sum(float(np.sum(c ** 2)) for c in q))
    return math.sqrt(h2 * float(np.sum(q ** 2)))


def divergence(u, n):
    return (np.roll(u[0], -1, axis=1) - u[0] + np.roll(u[1], -1, axis=0) - u[1]) * n


def run(members, s, mu, steps):
    ens = ensemble.Ensemble(members, rho=s["rho"], mu=mu, precision=0)
    ens.run(steps, steps_per_launch=2)
    assert ens.sync() == [steps] * len(members)
    out = {m.n: ens.member_state(m) for m in members}
    ens.close()
    return out


@pytest.mark.parametrize("mu", ["0.05", "0.01", "0.005"])
def test_thick_ellipse_rates(mu):
    g = json.load(open(GOLDEN))
    s = g["setup"]
    steps = int(round(s["t"] / s["dt"]))
    members = [Member(n, s["dt"], s) for n in (128, 256, 512)]
    st = run(members, s, float(mu), steps)
    a, b, c = st[128], st[256], st[512]
    mb, mc = members[1], members[2]
    rate = {}
    num = norm_grid([x - y for x, y in zip(a["u"], restrict_faces(b["u"]))], 128)
    den = norm_grid([x - y for x, y in zip(b["u"], restrict_faces(c["u"]))], 256)
    rate["u"] = math.log2(num / den)
    num = norm_grid(a["p"] - restrict_cells(b["p"]), 128)
    den = norm_grid(b["p"] - restrict_cells(c["p"]), 256)
    rate["p"] = math.log2(num / den)
    wa = 1.0 / (members[0].ns * members[0].nr)
    wb = 1.0 / (mb.ns * mb.nr)
    num = math.sqrt(wa * float(np.sum((a["X"] - restrict_points(b["X"], mb.nr, mb.ns)) ** 2)))
    den = math.sqrt(wb * float(np.sum((b["X"] - restrict_points(c["X"], mc.nr, mc.ns)) ** 2)))
    rate["X"] = math.log2(num / den)
    paper = g["rates"][mu]
    print("mu", mu, "rates ours", {k: round(v, 3) for k, v in rate.items()}, "paper", paper)
    for q in ("u", "p", "X"):
        assert abs(rate[q] - paper[q]) <= 0.15, (mu, q, rate[q], paper[q])


def test_thick_ellipse_divergence_errors():
    g = json.load(open(GOLDEN))
    s, d = g["setup"], g["divergence"]
    worst = 0.0
    for j, f in enumerate(d["dt_times_512"]):
        dt = f / 512
        steps = int(round(d["t"] / dt))
        members = [Member(n, dt, s) for n in (64, 128, 256, 512)]
        st = run(members, s, d["mu"], steps)
        for n in (64, 128, 256, 512):
            mine = norm_grid(divergence(st[n]["u"], n), n)
            theirs = d["error"][str(n)][j]
            rel = abs(mine - theirs) / theirs
            worst = max(worst, rel)
            print("dt=%g/512 N=%d div error %.4g (paper %.3g) rel %.3g" % (f, n, mine, theirs, rel))
            assert rel <= 0.02, (f, n, mine, theirs)
    print("worst relative difference", worst)
