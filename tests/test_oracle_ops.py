"""Pins of the oracle's difference operators (Sec. "Spatial Finite Difference
Operators") and of the skew-symmetric advection stencil (Sec. "IB-GM
Algorithm"): exact discrete identities, energy neutrality of the skew form
for arbitrary fields, and second-order agreement with the analytic u.grad u
(+ 1/2 u div u) on smooth fields."""
import numpy as np
import pytest

import oracle


def grid_fields(dim, N, seed):
    rng = np.random.default_rng(seed)
    shp = (N if dim == 3 else 1, N, N)
    return [rng.standard_normal(shp) for _ in range(dim)]


@pytest.mark.parametrize("dim", [2, 3])
def test_skew_advection_energy_neutral(dim):
    N = 12
    P = oracle.make_params(dim, (N, N, N if dim == 3 else 1), 1.0 / N)
    u = grid_fields(dim, N, 30 + dim)  # arbitrary, not divergence-free
    Nu = oracle.advection(P, u)
    e = sum((u[c] * Nu[c]).sum() for c in range(dim))
    scale = sum(np.abs(u[c] * Nu[c]).sum() for c in range(dim))
    assert abs(e) < 1e-14 * scale
    # constants are not advected
    Nc = oracle.advection(P, [np.full_like(u[c], 0.7 + c) for c in range(dim)])
    assert max(np.abs(q).max() for q in Nc) < 1e-12


def _analytic_fields(dim, N):
    """A smooth, non-divergence-free field and the exact value of the skew
    form u.grad u + 1/2 u (div u) at each MAC location."""
    h = 1.0 / N
    k = 2 * np.pi

    def U(x, y, z):
        return [np.sin(k * x + 0.3) * np.cos(k * y) + (0.2 * np.sin(k * z) if dim == 3 else 0),
                np.cos(k * x) * np.sin(2 * k * y + 0.1) + (0.3 * np.cos(k * z) if dim == 3 else 0),
                np.sin(k * x + k * y) * np.cos(k * z + 0.2)][:dim]

    def grad(x, y, z, eps=1e-6):
        base = U(x, y, z)
        g = []
        for a in range(dim):
            dx = [0, 0, 0]
            dx[a] = eps
            up = U(x + dx[0], y + dx[1], z + dx[2])
            dn = U(x - dx[0], y - dx[1], z - dx[2])
            g.append([(up[c] - dn[c]) / (2 * eps) for c in range(dim)])
        return base, g  # g[a][c] = d u_c / d x_a

    u, exact = [], []
    for c in range(dim):
        coords = []
        for a in range(3):
            if a < dim:
                idx = np.arange(N) + (0.0 if a == c else 0.5)
                coords.append(idx * h)
            else:
                coords.append(np.array([0.0]))
        Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
        base, g = grad(X, Y, Z)
        div = sum(g[a][a] for a in range(dim))
        exact.append(sum(base[a] * g[a][c] for a in range(dim)) + 0.5 * base[c] * div)
        u.append(base[c])
    return u, exact


@pytest.mark.parametrize("dim", [2, 3])
def test_skew_advection_second_order(dim):
    Ns = [16, 32, 64]
    errs = []
    for N in Ns:
        P = oracle.make_params(dim, (N, N, N if dim == 3 else 1), 1.0 / N)
        u, ex = _analytic_fields(dim, N)
        Nu = oracle.advection(P, u)
        errs.append(max(np.abs(Nu[c] - ex[c]).max() for c in range(dim)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (rates > 1.8).all(), (errs, rates)


@pytest.mark.parametrize("dim", [2, 3])
def test_div_grad_is_compact_laplacian(dim):
    N = 10
    P = oracle.make_params(dim, (N, N, N if dim == 3 else 1), 0.1)
    p = grid_fields(dim, N, 3)[0]
    dg = oracle.divergence(P, oracle.gradient(P, p))
    lap = oracle.laplacian(P, p)
    assert np.abs(dg - lap).max() < 1e-11 * np.abs(lap).max()
    # the (2d+1)-point Laplacian written with numpy rolls
    ref = sum(np.roll(p, 1, axis=2 - a) - 2 * p + np.roll(p, -1, axis=2 - a)
              for a in range(dim)) / 0.1 ** 2
    assert np.abs(lap - ref).max() < 1e-11 * np.abs(ref).max()
    # divergence and gradient of constants vanish
    assert np.abs(oracle.divergence(P, [np.full_like(p, 2.0)] * dim)).max() == 0
    assert max(np.abs(g).max() for g in oracle.gradient(P, np.full_like(p, 5.0))) == 0


def test_split_order_rotation():
    P2 = oracle.make_params(2, (8, 8, 1), 0.125)
    assert [oracle.split_order(P2, n) for n in range(3)] == [[0, 1], [1, 0], [0, 1]]
    P3 = oracle.make_params(3, (8, 8, 8), 0.125)
    assert [oracle.split_order(P3, n) for n in range(4)] == [
        [0, 1, 2], [1, 2, 0], [2, 0, 1], [0, 1, 2]]
    P3n = oracle.make_params(3, (8, 8, 8), 0.125, rotate=False)
    assert oracle.split_order(P3n, 1) == [0, 1, 2]
