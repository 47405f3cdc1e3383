"""Pins of the oracle's Lagrangian parts (Steps 1a, 2a, 2b): brute-force
double sums over all cells and points, exactness on constant and linear
fields, the spread/interp adjoint identity, force conservation and the closed
form of a discrete circle, and the fiber formula written with D_s^+-."""
import numpy as np
import pytest

import oracle
from paper_1305_3976_amd import inputs


def stag_coords(P, c):
    """Physical coordinates (per axis, broadcast to the grid) of MAC component c."""
    d = P.dim
    h = P.h
    n = [P.n[0], P.n[1], P.n[2]]
    out = []
    for a in range(3):
        idx = np.arange(n[a], dtype=float)
        if a < d:
            x = (idx + (0.0 if a == c else 0.5)) * h
        else:
            x = np.zeros(1)
        shape = [1, 1, 1]
        shape[2 - a] = len(x)
        out.append(x.reshape(shape))
    return out


def brute_spread(P, X, F, w):
    d = P.dim
    L = [P.n[a] * P.h for a in range(d)]
    f = []
    for c in range(d):
        xs = stag_coords(P, c)
        acc = np.zeros((P.n[2], P.n[1], P.n[0]))
        for k in range(X.shape[1]):
            wt = np.ones_like(acc)
            for a in range(d):
                dx = xs[a] - X[a, k]
                dx = (dx + L[a] / 2) % L[a] - L[a] / 2  # periodic image nearest
                wt = wt * oracle.phi(dx / P.h)
            acc += F[c, k] * w[k] * wt / P.h ** d
        f.append(acc)
    return f


@pytest.mark.parametrize("dim", [2, 3])
def test_spread_equals_brute_force(dim):
    n = (8, 8, 8 if dim == 3 else 1)
    P = oracle.make_params(dim, n, 1.0 / 8)
    rng = np.random.default_rng(5 + dim)
    npts = 5
    X = rng.uniform(-0.3, 1.3, size=(dim, npts))  # includes unwrapped points
    X[:, 0] = 0.25  # exactly on grid lines
    F = rng.standard_normal((dim, npts))
    w = rng.uniform(0.5, 2.0, npts)
    f = oracle.spread(P, X, F, w)
    ref = brute_spread(P, X, F, w)
    for c in range(dim):
        assert np.abs(f[c] - ref[c]).max() <= 1e-13 * np.abs(ref[c]).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_brute_force_and_adjoint(dim):
    N = 8
    n = (N, N, N if dim == 3 else 1)
    P = oracle.make_params(dim, n, 1.0 / N)
    rng = np.random.default_rng(21 + dim)
    u = [rng.standard_normal((n[2], n[1], n[0])) for _ in range(dim)]
    X = rng.uniform(0, 1, size=(dim, 7))
    F = rng.standard_normal((dim, 7))
    w = rng.uniform(0.1, 1.0, 7)
    U = oracle.interp(P, u, X)
    # brute force: U_c(k) = sum_cells u_c delta_h(x - X_k) h^d
    for c in range(dim):
        xs = stag_coords(P, c)
        for k in range(X.shape[1]):
            wt = np.ones_like(u[c])
            for a in range(dim):
                dx = xs[a] - X[a, k]
                dx = (dx + 0.5) % 1.0 - 0.5
                wt = wt * oracle.phi(dx / P.h)
            assert abs((u[c] * wt).sum() - U[c, k]) < 1e-13
    # adjoint: <S F, u>_h = <F, J u>_w
    f = oracle.spread(P, X, F, w)
    lhs = sum((f[c] * u[c]).sum() for c in range(dim)) * P.h ** dim
    rhs = sum((w * F[c] * U[c]).sum() for c in range(dim))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(rhs))
    # total force is preserved
    for c in range(dim):
        assert abs(f[c].sum() * P.h ** dim - (w * F[c]).sum()) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_exact_on_linear_fields(dim):
    """Zero first moments: a field linear in x (sampled at its staggered
    positions) is interpolated exactly away from the periodic seam.  A wrong
    staggering offset would fail this."""
    N = 16
    n = (N, N, N if dim == 3 else 1)
    P = oracle.make_params(dim, n, 1.0 / N)
    rng = np.random.default_rng(9)
    coef = rng.standard_normal((dim, dim + 1))
    u = []
    for c in range(dim):
        xs = stag_coords(P, c)
        q = coef[c, 0] + sum(coef[c, 1 + a] * xs[a] for a in range(dim))
        u.append(np.broadcast_to(q, (n[2], n[1], n[0])).copy())
    X = rng.uniform(0.3, 0.7, size=(dim, 11))
    U = oracle.interp(P, u, X)
    for c in range(dim):
        ref = coef[c, 0] + sum(coef[c, 1 + a] * X[a] for a in range(dim))
        assert np.abs(U[c] - ref).max() < 1e-13
    # constants are exact everywhere, seam included
    X2 = rng.uniform(-1, 2, size=(dim, 11))
    U2 = oracle.interp(P, [np.full((n[2], n[1], n[0]), 3.25)] * dim, X2)
    assert np.abs(U2 - 3.25).max() < 1e-14


def test_link_force_circle_closed_form():
    """Discrete circle of radius R with L = 0: every point feels
    -sigma R (2 - 2 cos(2 pi h_s)) / h_s^2 along its radius; total is zero."""
    npts, R, sigma = 64, 0.25, 1.7
    S = inputs.ellipse(npts, R, R, sigma)
    F = oracle.link_force(S.X, S.links)
    hs = 1.0 / npts
    rad = (S.X - 0.5) / R
    mag = -sigma * R * (2 - 2 * np.cos(2 * np.pi * hs)) / hs ** 2
    assert np.abs(F - mag * rad).max() < 1e-10 * abs(mag)
    assert np.abs(F.sum(axis=1)).max() < 1e-9


def test_link_force_equals_fiber_formula():
    """F_k = sigma D_s^-( D_s^+ X_k (1 - L / |D_s^+ X_k|) ) (Step 2a), written
    with numpy differences, equals the force-connection form for L != 0."""
    npts, sigma, L = 40, 2.0, 0.8
    rng = np.random.default_rng(4)
    S = inputs.ellipse(npts, 0.3, 0.2, sigma, L)
    X = S.X + 1e-3 * rng.standard_normal(S.X.shape)
    hs = 1.0 / npts
    Dp = (np.roll(X, -1, axis=1) - X) / hs
    T = Dp * (1 - L / np.linalg.norm(Dp, axis=0))
    Fref = sigma * (T - np.roll(T, 1, axis=1)) / hs
    F = oracle.link_force(X, S.links)
    assert np.abs(F - Fref).max() < 1e-11 * np.abs(Fref).max()


def test_link_force_periodic_image():
    """A fiber that closes through the periodic box (Sec. "Cylindrical Shell
    in 3D"): with nearest-image link vectors the force does not depend on
    which periodic copy of each point is stored.  Reference: the same fiber
    unwrapped (all links short) with no images."""
    rng = np.random.default_rng(11)
    box = np.array([1.25, 0.8])
    S = inputs.ellipse(96, 0.2, 0.15, 1.3, L=0.5, center=(0.05, 0.75))
    X = S.X + 1e-3 * rng.standard_normal(S.X.shape)
    Fref = oracle.link_force(X, S.links)
    Xw = np.mod(X, box[:, None])                       # wrapped into the box
    Xw[:, :7] += box[:, None] * rng.integers(-2, 3, size=(2, 7))  # other copies
    F = oracle.link_force(Xw, S.links, period=box)
    assert np.abs(F - Fref).max() < 1e-9 * np.abs(Fref).max()
    # without images the wrapped fiber is torn apart
    assert np.abs(oracle.link_force(Xw, S.links) - Fref).max() > np.abs(Fref).max()


def test_cylinder_initial_force_is_the_ring_force():
    """At t = 0 every axial fiber of the cylinder sits at its rest length
    (|X_r| = L = 1, through the periodic seam), so the force is the zero-
    rest-length ring force of each elliptical cross-section, in y-z, with no
    x component (Sec. "Cylindrical Shell in 3D")."""
    N = 16
    S = inputs.cylinder_shell(N)
    ns, nr = 19 * N // 4, 3 * N
    F = oracle.link_force(S.X, S.links, period=(1.0, 1.0, 1.0))
    ring = inputs.ellipse(ns, 5 / 28, 7 / 20, 1.0)
    Fr = oracle.link_force(ring.X, ring.links)
    scale = np.abs(Fr).max()
    Fc = F.reshape(3, nr, ns)
    assert np.abs(Fc[0]).max() < 1e-9 * scale
    assert np.abs(Fc[1:] - Fr[:, None, :]).max() < 1e-9 * scale
    # the seam links are what the images fix
    assert np.abs(oracle.link_force(S.X, S.links)[0]).max() > scale


def test_link_force_network_conserves_momentum():
    S = inputs.ellipsoid_shell(200)
    F = oracle.link_force(S.X, S.links)
    assert np.abs(F.sum(axis=1)).max() < 1e-12
    # zero-rest-length links under a uniform scaling about the centre pull
    # every point inward
    r = S.X - 0.5
    assert ((F * r).sum(axis=0) < 0).all()
