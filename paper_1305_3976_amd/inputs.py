"""Seeded synthetic inputs for the IB-GM path (membranes, link networks and
initial velocity fields).

This module holds no arithmetic of the method itself: it only builds initial
positions, connectivity, per-point weights and initial fluid fields.  Both the
HIP path and the CPU oracle consume what it returns, so it lives on its own.

Conventions: grid arrays have shape (n2, n1, n0) (x fastest; n2 = 1 in 2D) and
the MAC component c lives on the faces normal to axis c (integer index along c,
half-integer along the others).  Lagrangian arrays have shape (dim, np).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Structure:
    """Lagrangian points joined by elastic links.

    X       (dim, np) float64 initial positions
    links   (a, b, kappa, l0): int32, int32, float64, float64 arrays; each link
            pulls a and b together with kappa (X_b - X_a)(1 - l0/|X_b - X_a|)
    w       (np,) float64 spreading weight of each point (h_s for a fiber
            force density, 1 for a total nodal force)
    tether  optional (kappa, Y): point k is pulled by kappa[k] (Y[:, k] - X_k)
            towards a fixed target (tether points)
    """
    X: np.ndarray
    links: tuple
    w: np.ndarray
    tether: tuple = None  # (kappa [np], fixed target [dim][np]) or None

    @property
    def np(self) -> int:
        return int(self.X.shape[1])

    @property
    def nlinks(self) -> int:
        return int(len(self.links[0]))


def closed_fiber_links(npts: int, sigma: float, L: float = 0.0, offset: int = 0):
    """Links of one closed fiber with points offset..offset+npts-1 and
    parameter spacing h_s = 1/npts.  The fiber force density
    sigma D_s^-(D_s^+ X (1 - L/|D_s^+ X|)) equals the link form with
    kappa = sigma/h_s^2 and l0 = L h_s (force-connection form)."""
    hs = 1.0 / npts
    a = np.arange(npts, dtype=np.int32) + offset
    b = (np.arange(npts, dtype=np.int32) + 1) % npts + offset
    k = np.full(npts, sigma / hs ** 2)
    l0 = np.full(npts, L * hs)
    return a, b.astype(np.int32), k, l0


def ellipse(npts: int, r1: float, r2: float, sigma: float, L: float = 0.0,
            center=(0.5, 0.5)) -> Structure:
    """Closed elliptical fiber X(s) = (c_x + r1 cos 2 pi s, c_y + r2 sin 2 pi s),
    s_k = k/npts (thin-ellipse problem of the paper), spread with w = h_s."""
    s = np.arange(npts) / npts
    X = np.stack([center[0] + r1 * np.cos(2 * np.pi * s),
                  center[1] + r2 * np.sin(2 * np.pi * s)])
    w = np.full(npts, 1.0 / npts)
    return Structure(X, closed_fiber_links(npts, sigma, L), w)


def tethered_ring(npts: int, radius: float, center, sigma: float, kappa_t: float) -> Structure:
    """A rigid-ish obstacle: a closed circular fiber (stiffness sigma, w = h_s)
    whose points are tied to their initial positions by tethers of stiffness
    kappa_t (force density per unit displacement)."""
    S = ellipse(npts, radius, radius, sigma, center=center)
    S.tether = (np.full(npts, float(kappa_t)), S.X.copy())
    return S


def thick_ellipse(ns: int, nr: int, r1: float, r2: float, gamma: float,
                  center=(0.5, 0.5)) -> Structure:
    """Nested closed fibers r_l = (l + 1/2)/nr of the thick elliptical shell,
    stiffness sigma(r) = 1 - cos(2 pi r), spread with w = h_s h_r."""
    Xs, A, B, K, L0 = [], [], [], [], []
    s = np.arange(ns) / ns
    for l in range(nr):
        r = (l + 0.5) / nr
        Xs.append(np.stack([center[0] + (r1 + gamma * (r - 0.5)) * np.cos(2 * np.pi * s),
                            center[1] + (r2 + gamma * (r - 0.5)) * np.sin(2 * np.pi * s)]))
        a, b, k, l0 = closed_fiber_links(ns, 1.0 - math.cos(2 * math.pi * r),
                                         0.0, offset=l * ns)
        A.append(a); B.append(b); K.append(k); L0.append(l0)
    X = np.concatenate(Xs, axis=1)
    w = np.full(ns * nr, (1.0 / ns) * (1.0 / nr))
    return Structure(X, (np.concatenate(A), np.concatenate(B),
                         np.concatenate(K), np.concatenate(L0)), w)


def fibonacci_sphere(npts: int) -> np.ndarray:
    """Quasi-uniform unit-sphere points (golden-angle spiral), shape (3, np)."""
    i = np.arange(npts) + 0.5
    z = 1.0 - 2.0 * i / npts
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = np.pi * (3.0 - math.sqrt(5.0)) * np.arange(npts)
    return np.stack([r * np.cos(th), r * np.sin(th), z])


def _cotan_weights(P: np.ndarray, tris: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Cotangent weights (cot a + cot b)/2 of each edge of a triangulated unit
    sphere, a and b being the angles opposite the edge in its two triangles
    (measured on the flat triangles of the parameter mesh)."""
    pts = P.T
    tris = np.asarray(tris)
    n = pts.shape[0]
    keys, vals = [], []
    for k in range(3):
        i, j, o = tris[:, k], tris[:, (k + 1) % 3], tris[:, (k + 2) % 3]
        a, b = pts[i] - pts[o], pts[j] - pts[o]
        cot = np.einsum("ij,ij->i", a, b) / np.linalg.norm(np.cross(a, b), axis=1)
        keys.append(np.minimum(i, j).astype(np.int64) * n + np.maximum(i, j))
        vals.append(0.5 * cot)
    keys = np.concatenate(keys)
    vals = np.concatenate(vals)
    ekeys = E[:, 0].astype(np.int64) * n + E[:, 1]
    order = np.argsort(keys)
    sk, sv = keys[order], vals[order]
    uk, start = np.unique(sk, return_index=True)
    sums = np.add.reduceat(sv, start)
    pos = np.searchsorted(uk, ekeys)
    assert np.array_equal(uk[pos], ekeys)
    return sums[pos]


def ellipsoid_shell(npts: int, axes=(0.3, 0.25, 0.2), kappa: float = 1.0,
                    center=(0.5, 0.5, 0.5), weights: str = "uniform") -> Structure:
    """Triangulated ellipsoidal shell: Fibonacci-sphere points and the edges
    of their convex hull as zero-rest-length links, scaled to the semi-axes
    and centred; the links carry a total nodal force (w = 1).

    weights = "uniform": every link has stiffness kappa.
    weights = "cotan":   kappa is the modulus sigma of the membrane energy
        (sigma/2) int |grad X|^2 over the unit-sphere parameterisation -- the
        triangulated analogue of the fiber-sheet energy behind the paper's
        force density sigma (X_ss + X_rr) -- discretised with cotangent
        weights, so link ij has stiffness sigma (cot a_ij + cot b_ij)/2."""
    from scipy.spatial import ConvexHull

    P = fibonacci_sphere(npts)
    hull = ConvexHull(P.T)
    e = set()
    for t in hull.simplices:
        for u, v in ((t[0], t[1]), (t[1], t[2]), (t[0], t[2])):
            e.add((min(u, v), max(u, v)))
    E = np.array(sorted(e), dtype=np.int32)
    X = np.stack([center[a] + axes[a] * P[a] for a in range(3)])
    if weights == "cotan":
        k = kappa * _cotan_weights(P, hull.simplices, E)
    else:
        k = np.full(len(E), float(kappa))
    links = (E[:, 0].copy(), E[:, 1].copy(), k, np.zeros(len(E)))
    return Structure(X, links, np.ones(npts))


def cylinder_shell(N: int, r1: float = 5 / 28, r2: float = 7 / 20,
                   sigma_s: float = 1.0, sigma_r: float = 1.0, L: float = 1.0):
    """3-D cylindrical shell of the paper's performance test: N_s = 19N/4
    circumferential fibers around the x axis crossed by N_r = 3N axial fibers,
    X(s, r) = (r, 1/2 + r1 cos 2 pi s, 1/2 + r2 sin 2 pi s); periodic in r.
    Fiber sheet weights w = h_s h_r."""
    ns, nr = 19 * N // 4, 3 * N
    hs, hr = 1.0 / ns, 1.0 / nr
    s = np.arange(ns) * hs
    r = np.arange(nr) * hr
    S, R = np.meshgrid(s, r)  # (nr, ns): point id = l*ns + k
    X = np.stack([R.ravel(), 0.5 + r1 * np.cos(2 * np.pi * S.ravel()),
                  0.5 + r2 * np.sin(2 * np.pi * S.ravel())])
    ids = np.arange(nr * ns, dtype=np.int32).reshape(nr, ns)
    a_s = ids.ravel()
    b_s = np.roll(ids, -1, axis=1).ravel()
    a_r = ids.ravel()
    b_r = np.roll(ids, -1, axis=0).ravel()
    A = np.concatenate([a_s, a_r]).astype(np.int32)
    B = np.concatenate([b_s, b_r]).astype(np.int32)
    K = np.concatenate([np.full(a_s.size, sigma_s / hs ** 2),
                        np.full(a_r.size, sigma_r / hr ** 2)])
    L0 = np.concatenate([np.zeros(a_s.size), np.full(a_r.size, L * hr)])
    return Structure(X, (A, B, K, L0), np.full(nr * ns, hs * hr))


# ----------------------------------------------------------- fluid fields --

def zero_velocity(dim: int, n) -> list:
    shp = (n[2] if dim == 3 else 1, n[1], n[0])
    return [np.zeros(shp) for _ in range(dim)]


def random_streamfunction_velocity_2d(n: int, kmax: int = 4, amp: float = 0.1,
                                      seed: int = 2):
    """Smooth, discretely divergence-free 2-D velocity: a streamfunction s at
    the cell corners built from integer wave vectors 1 <= |k|_inf <= kmax with
    N(0,1) cosine/sine coefficients, then u = (s[j+1] - s[j])/h on x-faces and
    v = -(s[i+1] - s[i])/h on y-faces, scaled so max |u|, |v| = amp."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    x = np.arange(n) * h
    Xn, Yn = np.meshgrid(x, x)  # (j, i)
    s = np.zeros((n, n))
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            if max(abs(kx), abs(ky)) == 0 or (ky == 0 and kx < 0):
                continue
            a, b = rng.standard_normal(2)
            ph = 2 * np.pi * (kx * Xn + ky * Yn)
            s += a * np.cos(ph) + b * np.sin(ph)
    u = (np.roll(s, -1, axis=0) - s) / h
    v = -(np.roll(s, -1, axis=1) - s) / h
    scale = amp / max(np.abs(u).max(), np.abs(v).max())
    return [(u * scale)[None], (v * scale)[None]]


def random_vector_potential_velocity_3d(n: int, kmax: int = 4, amp: float = 0.1,
                                        seed: int = 5):
    """3-D analogue: a vector potential A on the cell edges (A_c at integer
    indices except along c), u = curl A with one-cell differences, which is
    discretely divergence-free on the MAC grid; scaled to max |u| = amp."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = np.arange(n) * h
    A = []
    for c in range(3):
        off = [0.0, 0.0, 0.0]
        off[c] = 0.5 * h
        acc = np.zeros((n, n, n))
        for _ in range(6):
            k = rng.integers(-kmax, kmax + 1, size=3)
            if not k.any():
                continue
            a, b = rng.standard_normal(2)
            # a cos(phase) + b sin(phase) = Re((a - i b) e^{i phase}), the
            # phase 2 pi k.(x + off) separating into one factor per axis
            e = [np.exp(2j * np.pi * k[ax] * (g + off[ax])) for ax in range(3)]
            acc += ((a - 1j * b) * e[2][:, None, None] * e[1][None, :, None]
                    * e[0][None, None, :]).real
        A.append(acc)
    # axis numbering: array axes (2, 1, 0) = (z, y, x)
    def d(q, ax):  # forward difference along grid axis ax (0 = x)
        return (np.roll(q, -1, axis=2 - ax) - q) / h
    u = d(A[2], 1) - d(A[1], 2)
    v = d(A[0], 2) - d(A[2], 0)
    w = d(A[1], 0) - d(A[0], 1)
    scale = amp / max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    return [u * scale, v * scale, w * scale]


# ---------------------------------------------------------- named configs --

@dataclass
class Workload:
    name: str
    dim: int
    n: tuple
    rho: float
    mu: float
    dt: float
    steps: int
    structure: Structure
    u0: list
    chi: float = 0.6

    @property
    def h(self) -> float:
        return 1.0 / self.n[0]


def channel_velocity(dim: int, n, seed: int = 1, amp: float = 0.2) -> list:
    """Smooth, discretely divergence-free velocity for a channel with walls at
    y = 0 and y = n1 h (v = 0 on the wall faces, rows j = 0): a stream
    function (2-D) or vector potential (3-D, A_y = 0) built from
    cos/sin(2 pi (kx x + kz z)) sin(m pi y) modes with N(0,1) coefficients,
    which vanishes on the wall rows, differenced with one-cell stencils and
    scaled to max |u| = amp."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n[0]
    ny = n[1]
    x = np.arange(n[0]) * h
    yw = np.arange(ny) / ny                         # wall-face rows y = j h
    z = np.arange(n[2]) * h if dim == 3 else np.zeros(1)
    Z, Y, Xg = np.meshgrid(z, yw, x, indexing="ij")

    def potential():
        s = np.zeros(Xg.shape)
        for kx in range(0, 3):
            for m in range(1, 4):
                for kz in (range(0, 2) if dim == 3 else [0]):
                    a, b = rng.standard_normal(2)
                    ph = 2 * math.pi * (kx * Xg + kz * Z)
                    s += (a * np.cos(ph) + b * np.sin(ph)) * np.sin(m * math.pi * Y)
        return s                                     # zero on the wall rows j = 0

    if dim == 2:
        s = potential()                               # at corners (i h, j h)
        u = (np.roll(s, -1, axis=1) - s) / h          # x-faces (i h, (j+1/2) h)
        v = -(np.roll(s, -1, axis=2) - s) / h         # y-faces (j = 0 rows stay 0)
        vel = [u, v]
    else:
        A0, A2 = potential(), potential()              # A_x on x-edges, A_z on z-edges
        # u = curl A with A_y = 0: u = dA_z/dy, v = dA_x/dz - dA_z/dx, w = -dA_x/dy
        u = (np.roll(A2, -1, axis=1) - A2) / h
        v = (np.roll(A0, -1, axis=0) - A0) / h - (np.roll(A2, -1, axis=2) - A2) / h
        w = -(np.roll(A0, -1, axis=1) - A0) / h
        vel = [u, v, w]
    scale = amp / max(np.abs(c).max() for c in vel)
    return [c * scale for c in vel]


def config_ellipse_64(steps: int = 100) -> Workload:
    """2-D periodic unit square, 64^2, rho=1, mu=0.1, dt=1e-3; closed ellipse
    (semi-axes 0.3/0.2, centred), 256 points, sigma=1, L=0, fluid at rest."""
    n = 64
    return Workload("ellipse2d_64", 2, (n, n, 1), 1.0, 0.1, 1e-3, steps,
                    ellipse(256, 0.3, 0.2, 1.0), zero_velocity(2, (n, n, 1)))


def config_ellipse_512(steps: int = 1000, seed: int = 2, dt: float = 0.01 / 512) -> Workload:
    """2-D periodic, 512^2, mu=0.01; ellipse with 2048 points and sigma=10,
    plus a seeded random smooth velocity (|k| <= 4, amplitude 0.1).  The time
    step is the paper's for sigma = 10 at N = 512 (0.01/512, Sec. "Thin
    Ellipse"): the 1e-4 often quoted with this configuration makes the
    membrane blow up within ~20 steps on the oracle."""
    n = 512
    return Workload("ellipse2d_512", 2, (n, n, 1), 1.0, 0.01, dt, steps,
                    ellipse(2048, 0.3, 0.2, 10.0),
                    random_streamfunction_velocity_2d(n, 4, 0.1, seed))


def config_shell_256(steps: int = 200, n: int = 256, npts: int = 65536) -> Workload:
    """3-D periodic unit cube, 256^3, mu=0.01, dt=5e-4; ellipsoidal shell
    (semi-axes 0.3/0.25/0.2) triangulated into 65,536 points, zero-rest-length
    links whose stiffness 1 is the modulus of the membrane energy (cotangent
    link weights, see ellipsoid_shell), fluid at rest."""
    return Workload("shell3d_%d" % n, 3, (n, n, n), 1.0, 0.01, 5e-4, steps,
                    ellipsoid_shell(npts, weights="cotan"), zero_velocity(3, (n, n, n)))


# ------------------------------------------------------- batched ensemble --

def config_cylinder(n: int = 256, steps: int = 100) -> Workload:
    """3-D cylindrical shell of Sec. "Cylindrical Shell in 3D": N^3 periodic
    unit cube, rho = 1, mu = 0.01, dt = 0.04/N, sigma_s = sigma_r = 1, L = 1,
    r1 = 5/28, r2 = 7/20, N_s = 19N/4 circumferential by N_r = 3N axial
    fibers (933,888 points at N = 256), fluid at rest; the paper times the
    first 100 steps."""
    return Workload("cylinder3d_%d" % n, 3, (n, n, n), 1.0, 0.01, 0.04 / n, steps,
                    cylinder_shell(n), zero_velocity(3, (n, n, n)))


def stiffness_time_step(sigma: float) -> float:
    """Time step for a thin ellipse of stiffness sigma, from the step sizes the
    paper uses for its thin-ellipse runs at N = 512 (Sec. "Thin Ellipse":
    0.08/512, 0.04/512 and 0.01/512 for sigma = 0.1, 1 and 10), taken
    piecewise linear in (log10 sigma, log2 dt), with the last factor (1/4 per
    decade) continued above sigma = 10 and the first (1/2 per decade) below
    sigma = 0.1."""
    ls = math.log10(sigma)
    if ls <= 0.0:
        l2 = math.log2(0.04 / 512) - ls * 1.0          # x2 per decade downwards
    else:
        l2 = math.log2(0.04 / 512) - ls * 2.0          # x1/4 per decade upwards
    return 2.0 ** l2


@dataclass
class EnsembleMember:
    """One independent 2-D problem of a batched ensemble."""
    index: int
    n: int
    sigma: float
    dt: float
    structure: Structure


def config_ensemble(nsims: int = 64, seed: int = 4, steps: int = 500,
                    sizes=(128, 192, 256, 384, 512), sigma_range=(0.1, 100.0),
                    points_per_cell: int = 4, rho: float = 1.0, mu: float = 0.01):
    """Batched ensemble of independent 2-D periodic problems: grid size drawn
    uniformly from `sizes`, a centred 0.3 x 0.2 ellipse with 4N points and
    stiffness log-uniform in sigma_range, fluid at rest, time step from
    stiffness_time_step.  Returns (members, dict of shared parameters)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=nsims)
    lo, hi = math.log(sigma_range[0]), math.log(sigma_range[1])
    sig = np.exp(rng.uniform(lo, hi, size=nsims))
    members = []
    for i in range(nsims):
        n = int(ns[i])
        sg = float(sig[i])
        members.append(EnsembleMember(i, n, sg, stiffness_time_step(sg),
                                      ellipse(points_per_cell * n, 0.3, 0.2, sg)))
    return members, {"rho": rho, "mu": mu, "steps": steps, "chi": 0.6}


# -------------------------------------------------- closure training family --

@dataclass
class ClosureCase:
    """One fine trajectory of the closure's training family."""
    seed: int
    sigma: float
    axes: tuple
    dt_fine: float
    structure: Structure
    u0: list


def closure_family(ntraj: int, seed: int = 5, n_fine: int = 256, npts: int = None):
    """Ellipsoidal shells with seeded semi-axes in [0.15, 0.3], membrane
    modulus log-uniform in [0.1, 10] (cotangent links) and a seeded random
    smooth divergence-free velocity (|k| <= 4, max |u| = 0.1) on the n_fine^3
    grid; the fine time step is (64 / n_fine) min(1e-3, 6e-4 / sigma): the
    explicit membrane force limits it to about 6 mu h / sigma on the oracle
    for this family (so the coarse companion, at twice h, takes twice the
    step).  npts defaults to 65,536 (n_fine / 256)^2 points."""
    rng = np.random.default_rng(seed)
    if npts is None:
        npts = max(256, int(65536 * (n_fine / 256) ** 2))
    cases = []
    for i in range(ntraj):
        axes = tuple(float(a) for a in rng.uniform(0.15, 0.3, size=3))
        sigma = float(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
        vseed = int(rng.integers(0, 2 ** 31 - 1))
        dt = (64.0 / n_fine) * min(1e-3, 6e-4 / sigma)
        cases.append(ClosureCase(i, sigma, axes, dt,
                                 ellipsoid_shell(npts, axes, sigma, weights="cotan"),
                                 random_vector_potential_velocity_3d(n_fine, 4, 0.1, vseed)))
    return cases
