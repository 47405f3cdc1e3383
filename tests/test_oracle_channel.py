"""Pins of the oracle's channel (no-slip walls at y = 0 and y = 1, periodic in
x and z) against what the mathematics fixes: the bounded line systems against
the periodic solve of the mirrored (odd or even) extension and against dense
solves; the exact decay factor of a shear mode between the walls; energy
neutrality of the skew advection with walls; v stays zero on the wall faces,
rest stays at rest and the mean pressure stays zero with a membrane between
the walls.  (The paper notes
the solver is not tied to periodic boundaries, Sec. "Comparison with Poisson
Solvers"; the walls here are its periodic channel.)"""
import math

import numpy as np
import pytest

import oracle
from paper_1305_3976_amd import inputs

NO_LINKS = (np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0))


def dense(N, diag, off, bc):
    A = np.diag(np.full(N, diag)) + np.diag(np.full(N - 1, off), 1) + np.diag(np.full(N - 1, off), -1)
    if bc == oracle.BC_DIRICHLET_CELL:
        A[0, 0] -= off
        A[-1, -1] -= off
    elif bc == oracle.BC_NEUMANN_CELL:
        A[0, 0] += off
        A[-1, -1] += off
    return A


@pytest.mark.parametrize("bc", [oracle.BC_DIRICHLET_CELL, oracle.BC_DIRICHLET_FACE,
                                oracle.BC_NEUMANN_CELL])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_bounded_line_solves_are_mirrored_periodic_solves(bc, axis):
    """Method of images: with the ghost value -x (+x) across a wall between
    cells, the bounded system is the periodic system of twice the length
    applied to the odd (even) extension about the wall; a face unknown on the
    wall extends oddly about that face (x_0 = x_N = 0)."""
    rng = np.random.default_rng(3 + bc + 7 * axis)
    shape = [5, 6, 7]
    N = shape[2 - axis]
    diag, off = 1.0 + 2.0 * 37.0, -37.0
    f = rng.standard_normal(shape)
    if bc == oracle.BC_DIRICHLET_FACE:
        idx = [slice(None)] * 3
        idx[2 - axis] = 0
        f[tuple(idx)] = 0.0
    got = oracle.line_solve_bc(f, axis, diag, off, bc)
    g = np.moveaxis(f, 2 - axis, -1)
    if bc == oracle.BC_DIRICHLET_CELL:
        ext = np.concatenate([g, -g[..., ::-1]], axis=-1)
    elif bc == oracle.BC_NEUMANN_CELL:
        ext = np.concatenate([g, g[..., ::-1]], axis=-1)
    else:  # face: x_0 = 0, x_{N+m} = -x_{N-m}
        ext = np.concatenate([g, np.zeros(g.shape[:-1] + (1,)), -g[..., :0:-1]], axis=-1)[..., :2 * N]
    ext_sol = oracle.line_solve(np.moveaxis(ext, -1, 2 - axis), axis, diag, off)
    want = np.moveaxis(np.moveaxis(ext_sol, 2 - axis, -1)[..., :N], -1, 2 - axis)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # and the written-out bounded matrix, solved densely, line by line
    gl = np.moveaxis(got, 2 - axis, -1).reshape(-1, N)
    fl = g.reshape(-1, N)
    if bc == oracle.BC_DIRICHLET_FACE:
        A = dense(N - 1, diag, off, bc)
        assert np.abs(gl[:, 0]).max() == 0.0
        ref = np.linalg.solve(A, fl[:, 1:].T).T
        assert np.abs(gl[:, 1:] - ref).max() < 1e-12 * np.abs(ref).max()
    else:
        ref = np.linalg.solve(dense(N, diag, off, bc), fl.T).T
        assert np.abs(gl - ref).max() < 1e-12 * np.abs(ref).max()


def channel_sim(dim, n, u, structure=None, mu=0.05, dt=1e-3, no_advection=False, rotate=True):
    P = oracle.make_params(dim, n, 1.0 / n[0], mu=mu, dt=dt, no_advection=no_advection,
                           rotate=rotate, walls_y=True)
    if structure is None:
        return oracle.Sim(P, u, np.full((dim, 1), 0.5), NO_LINKS, np.ones(1))
    return oracle.Sim(P, u, structure.X, structure.links, structure.w)


@pytest.mark.parametrize("dim,comp,k", [(2, 0, 1), (2, 0, 3), (3, 0, 2), (3, 2, 1)])
def test_shear_mode_decay_between_walls(dim, comp, k):
    """u_c(y) = sin(k pi (j + 1/2)/n1), all else 0: divergence-free, its
    advection vanishes, and it is an eigenvector of the wall second
    difference with lambda = -(4/h^2) sin^2(k pi/(2 n1)).  The explicit step
    and the Douglas sweeps then give exactly
    u^{n+1} = (1 + nu lambda)/(1 - nu lambda) u^n,  nu = mu dt/(2 rho);
    psi and p stay zero."""
    n = (8, 16, 6 if dim == 3 else 1)
    h = 1.0 / n[0]
    mu, dt, steps = 0.05, 2e-3, 7
    y = (np.arange(n[1]) + 0.5) / n[1]
    prof = np.sin(k * math.pi * y)
    shp = (n[2], n[1], n[0])
    u = [np.zeros(shp) for _ in range(dim)]
    u[comp] = np.broadcast_to(prof[None, :, None], shp).copy()
    s = channel_sim(dim, n, u, mu=mu, dt=dt).advance(steps)
    lam = -(4 / h ** 2) * math.sin(k * math.pi / (2 * n[1])) ** 2
    nu = mu * dt / 2
    g = (1 + nu * lam) / (1 - nu * lam)
    assert np.abs(s.u[comp] - g ** steps * u[comp]).max() < 1e-13
    for c in range(dim):
        if c != comp:
            assert np.abs(s.u[c]).max() < 1e-13
    assert np.abs(s.p).max() < 1e-11 and np.abs(s.psi).max() < 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_advection_with_walls_is_energy_neutral(dim):
    n = (8, 12, 6 if dim == 3 else 1)
    P = oracle.make_params(dim, n, 1.0 / n[0], walls_y=True)
    rng = np.random.default_rng(5)
    u = [rng.standard_normal((n[2], n[1], n[0])) for _ in range(dim)]
    u[1][:, 0, :] = 0.0
    N = oracle.advection(P, u)
    e = sum(float(np.sum(u[c] * N[c])) for c in range(dim))
    scale = sum(float(np.sum(np.abs(u[c] * N[c]))) for c in range(dim))
    assert abs(e) < 1e-13 * scale
    assert np.abs(N[1][:, 0, :]).max() == 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_channel_invariants(dim):
    n = (16, 16, 8 if dim == 3 else 1)
    shp = (n[2], n[1], n[0])
    s = channel_sim(dim, n, [np.zeros(shp)] * dim).advance(3)
    assert max(np.abs(c).max() for c in s.u[:dim]) == 0.0
    u0 = inputs.channel_velocity(dim, n, seed=1)
    P = oracle.make_params(dim, n, 1.0 / n[0], walls_y=True)
    assert np.abs(oracle.divergence(P, u0)).max() < 1e-12
    if dim == 2:
        S = inputs.ellipse(64, 0.2, 0.15, 1.0)
    else:
        S = inputs.ellipsoid_shell(300, axes=(0.2, 0.15, 0.1), center=(0.5, 0.5, 0.25))
    s = channel_sim(dim, n, u0, structure=S, mu=0.05, dt=1e-3).advance(20)
    assert np.abs(s.u[1][:, 0, :]).max() == 0.0          # v on the walls
    assert abs(float(np.mean(s.p))) < 1e-10 * max(1.0, np.abs(s.p).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_body_force_drives_discrete_poiseuille_flow(dim):
    """A uniform body force g along x between the walls, from rest: the
    steady state of the discrete scheme solves mu D_yy u = -g with the
    no-slip ghosts, whose exact solution is the parabola shifted by the
    ghost condition: u_j = g/(2 mu) (y_j (L - y_j) + h^2/4), y_j = (j + 1/2) h,
    L = n1 h; v, w, psi vanish and p stays zero."""
    n = (8, 16, 4 if dim == 3 else 1)
    h = 1.0 / 16
    mu, g, dt, steps = 1.0, 2.0, 0.01, 400
    P = oracle.make_params(dim, n, h, mu=mu, dt=dt, walls_y=True, body_force=(g, 0.0, 0.0))
    shp = (n[2], n[1], n[0])
    s = oracle.Sim(P, [np.zeros(shp) for _ in range(dim)], np.full((dim, 1), 0.5), NO_LINKS,
                   np.zeros(1)).advance(steps)
    y = (np.arange(n[1]) + 0.5) * h
    L = n[1] * h
    want = g / (2 * mu) * (y * (L - y) + h * h / 4)
    assert np.abs(s.u[0] - want[None, :, None]).max() < 1e-12 * want.max()
    for c in range(1, dim):
        assert np.abs(s.u[c]).max() < 1e-13
    assert np.abs(s.p).max() < 1e-11 and np.abs(s.psi).max() < 1e-11


def test_tether_is_a_link_to_a_fixed_point():
    """kappa (Y - X) on a tethered point is the pull of a zero-rest-length
    link of stiffness kappa to a point held at Y (link force brute force),
    also across the periodic box."""
    rng = np.random.default_rng(9)
    n = 40
    X = rng.uniform(0, 1, size=(2, n))
    Y = X + 0.02 * rng.standard_normal((2, n))
    Y[:, :5] += np.array([[1.0], [-1.0]])              # targets stored as other copies
    kap = rng.uniform(0, 50, size=n)
    F = oracle.tether_force(X, kap, Y, period=(1.0, 1.0))
    XX = np.concatenate([X, Y], axis=1)
    links = (np.arange(n, dtype=np.int32), np.arange(n, 2 * n, dtype=np.int32), kap, np.zeros(n))
    ref = oracle.link_force(XX, links, period=(1.0, 1.0))[:, :n]
    assert np.abs(F - ref).max() < 1e-12 * np.abs(ref).max()


def test_tethered_ring_holds_in_driven_channel():
    """A tethered ring in a channel driven by a body force: the fluid goes
    round it and the ring stays within a small fraction of a cell of its
    targets, while a free ring in the same flow is carried downstream."""
    n = (32, 32, 1)
    h = 1.0 / 32
    P = oracle.make_params(2, n, h, mu=0.1, dt=1e-3, walls_y=True, body_force=(5.0, 0.0, 0.0))
    shp = (1, 32, 32)
    moved = {}
    for kt in (0.0, 2e4):
        S = inputs.tethered_ring(48, 0.1, (0.5, 0.5), 1.0, kt)
        s = oracle.Sim(P, [np.zeros(shp)] * 2, S.X, S.links, S.w, tether=S.tether).advance(150)
        moved[kt] = float(np.abs(s.X - S.X).max())
        if kt:
            assert np.abs(s.u[1][:, 0, :]).max() == 0.0
    assert moved[2e4] < 0.05 * h
    assert moved[0.0] > 20 * moved[2e4]


@pytest.mark.parametrize("dim", [2, 3])
def test_moving_wall_drives_discrete_couette_flow(dim):
    """The upper wall moving with U (tangential: x, and z in 3-D), the lower
    at rest, from rest: the steady state of the discrete scheme is the linear
    profile u_j = U y_j / L, y_j = (j + 1/2) h -- with the ghost -u below and
    2U - u above it continues linearly across both walls, so D_yy u = 0 --
    and v, p, psi stay zero.  A wrong ghost (-u above) would leave the fluid
    at rest; a y solve without the wall's known term would bend the profile
    next to the wall."""
    n = (8, 16, 4 if dim == 3 else 1)
    h = 1.0 / 16
    mu, dt, steps = 1.0, 0.01, 400
    U = (0.7, 0.0, -0.4 if dim == 3 else 0.0)
    P = oracle.make_params(dim, n, h, mu=mu, dt=dt, walls_y=True, wall_velocity=U)
    shp = (n[2], n[1], n[0])
    s = oracle.Sim(P, [np.zeros(shp) for _ in range(dim)], np.full((dim, 1), 0.5), NO_LINKS,
                   np.zeros(1)).advance(steps)
    y = (np.arange(n[1]) + 0.5) * h
    L = n[1] * h
    for c in (0, 2) if dim == 3 else (0,):
        want = U[c] * y / L
        assert np.abs(s.u[c] - want[None, :, None]).max() < 1e-12 * abs(U[c])
    assert np.abs(s.u[1]).max() < 1e-13
    assert np.abs(s.p).max() < 1e-11 and np.abs(s.psi).max() < 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_couette_profile_is_a_fixed_point(dim):
    """Started on the linear profile of a moving upper wall, with the
    advection term on, the scheme leaves it in place to rounding (it is an
    exact steady solution of every step of the method)."""
    n = (8, 32, 4 if dim == 3 else 1)
    h = 1.0 / 32
    U = (1.3, 0.0, 0.5 if dim == 3 else 0.0)
    P = oracle.make_params(dim, n, h, mu=0.01, dt=1e-3, walls_y=True, wall_velocity=U)
    shp = (n[2], n[1], n[0])
    y = (np.arange(n[1]) + 0.5) * h
    u0 = [np.broadcast_to((U[c] * y / (n[1] * h))[None, :, None], shp).copy() for c in range(dim)]
    u0[1][:] = 0.0
    s = oracle.Sim(P, [a.copy() for a in u0], np.full((dim, 1), 0.5), NO_LINKS,
                   np.zeros(1)).advance(5)
    for c in range(dim):
        assert np.abs(s.u[c] - u0[c]).max() < 1e-14
    assert np.abs(s.p).max() < 1e-12


def test_wall_velocity_needs_tangential_walls():
    """A wall velocity without walls, or along y, is refused."""
    S = (np.full((2, 1), 0.5), NO_LINKS, np.zeros(1))
    for kw in ({"walls_y": False, "wall_velocity": (1.0, 0.0, 0.0)},
               {"walls_y": True, "wall_velocity": (0.0, 1.0, 0.0)}):
        P = oracle.make_params(2, (8, 16), 1.0 / 16, mu=0.1, **kw)
        with pytest.raises(Exception):
            oracle.Sim(P, [np.zeros((1, 16, 8))] * 2, *S).advance(1)
