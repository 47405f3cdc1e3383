"""Plain FP64 CPU oracle for the IB-GM time step (ctypes binding of ibo.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product path never imports it.  It shares no code
with the HIP library.

Grid arrays are numpy float64 arrays of shape (n2, n1, n0) (x fastest), so the
flat index is i + n0*(j + n1*k).  Lagrangian arrays have shape (dim, np).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibo.c")
_LIB = os.path.join(_HERE, "libibo.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile ibo.c into libibo.so with gcc (OpenMP over independent loops)."""
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                             os.path.getmtime(os.path.join(_HERE, "ibo.h"))))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall", "-o", tmp,
             _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("h", ctypes.c_double), ("rho", ctypes.c_double),
                ("mu", ctypes.c_double), ("dt", ctypes.c_double),
                ("chi", ctypes.c_double), ("rotate", ctypes.c_int32),
                ("no_advection", ctypes.c_int32), ("walls_y", ctypes.c_int32),
                ("body_force", ctypes.c_double * 3),
                ("wall_velocity", ctypes.c_double * 3)]


class _Sim(ctypes.Structure):
    _fields_ = [("prm", Params), ("step", ctypes.c_int64),
                ("u", _dp * 3), ("nl_prev", _dp * 3), ("p", _dp),
                ("psi", _dp), ("np", ctypes.c_int64), ("X", _dp),
                ("U_prev", _dp), ("nlinks", ctypes.c_int64),
                ("link_a", _ip), ("link_b", _ip), ("link_k", _dp),
                ("link_l0", _dp), ("w", _dp), ("tether_k", _dp), ("tether_Y", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.ibo_phi.restype = ctypes.c_double
        L.ibo_phi.argtypes = [ctypes.c_double]
        L.ibo_cyclic_solve.argtypes = [ctypes.c_int32, _dp, _dp, _dp, _dp, _dp]
        L.ibo_line_solve.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_double]
        L.ibo_interp.argtypes = [ctypes.POINTER(Params), _dp * 3, _dp,
                                 ctypes.c_int64, _dp]
        L.ibo_spread.argtypes = [ctypes.POINTER(Params), _dp, _dp, _dp,
                                 ctypes.c_int64, _dp * 3]
        L.ibo_link_force.argtypes = [ctypes.c_int32, ctypes.c_int64, _dp, _dp,
                                     ctypes.c_int64, _ip, _ip, _dp, _dp, _dp]
        L.ibo_advection.argtypes = [ctypes.POINTER(Params), _dp * 3, _dp * 3]
        L.ibo_tether_force.argtypes = [ctypes.c_int32, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp]
        L.ibo_vel_laplacian.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, _dp, _dp]
        L.ibo_line_solve_bc.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int32]
        L.ibo_laplacian.argtypes = [ctypes.POINTER(Params), _dp, _dp]
        L.ibo_divergence.argtypes = [ctypes.POINTER(Params), _dp * 3, _dp]
        L.ibo_gradient.argtypes = [ctypes.POINTER(Params), _dp, _dp * 3]
        L.ibo_split_order.argtypes = [ctypes.POINTER(Params), ctypes.c_int64,
                                      _ip]
        L.ibo_step.argtypes = [ctypes.POINTER(_Sim)]
        L.ibo_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _pi(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


def make_params(dim, n, h, rho=1.0, mu=0.0, dt=1e-3, chi=0.6, rotate=True,
                no_advection=False, walls_y=False, body_force=(0.0, 0.0, 0.0),
                wall_velocity=(0.0, 0.0, 0.0)) -> Params:
    nn = list(n) + [1] * (3 - len(n))
    P = Params()
    P.dim = dim
    for a in range(3):
        P.n[a] = nn[a]
    P.h, P.rho, P.mu, P.dt, P.chi = h, rho, mu, dt, chi
    P.rotate = 1 if rotate else 0
    P.no_advection = 1 if no_advection else 0
    P.walls_y = 1 if walls_y else 0
    for a in range(3):
        P.body_force[a] = float(body_force[a]) if a < len(body_force) else 0.0
        P.wall_velocity[a] = float(wall_velocity[a]) if a < len(wall_velocity) else 0.0
    return P


def grid_shape(P: Params):
    return (P.n[2], P.n[1], P.n[0])


def num_threads() -> int:
    return lib().ibo_num_threads()


def phi(r):
    f = lib().ibo_phi
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda x: f(float(x)))(r) if r.ndim else f(float(r))


def cyclic_solve(a, b, c, d):
    """Solve a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i] (indices mod n)."""
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    x = np.empty_like(d)
    rc = lib().ibo_cyclic_solve(len(d), _p(a), _p(b), _p(c), _p(d), _p(x))
    if rc != 0:
        raise ValueError("cyclic solve failed")
    return x


def line_solve(field_, axis: int, diag: float, off: float):
    """Return a copy of `field_` (shape (n2,n1,n0) or (n1,n0)) with every line
    along `axis` (0 = x) solved against the periodic (off, diag, off) matrix."""
    f = np.ascontiguousarray(field_, dtype=np.float64).copy()
    shp = f.shape[::-1] + (1,) * (3 - f.ndim)
    n = np.array(shp, dtype=np.int32)
    rc = lib().ibo_line_solve(_p(f), _pi(n), axis, diag, off)
    if rc != 0:
        raise ValueError("line solve failed")
    return f


BC_PERIODIC, BC_DIRICHLET_CELL, BC_DIRICHLET_FACE, BC_NEUMANN_CELL = 0, 1, 2, 3


def line_solve_bc(field_, axis: int, diag: float, off: float, bc: int):
    """line_solve with a channel boundary kind along `axis` (the BC_* values:
    periodic, Dirichlet for cell-centred unknowns (ghost -x), Dirichlet for a
    face unknown on the wall (element 0 held at 0), Neumann for cell-centred
    unknowns (ghost +x))."""
    f = np.ascontiguousarray(field_, dtype=np.float64).copy()
    shp = f.shape[::-1] + (1,) * (3 - f.ndim)
    n = np.array(shp, dtype=np.int32)
    rc = lib().ibo_line_solve_bc(_p(f), _pi(n), axis, diag, off, bc)
    if rc != 0:
        raise ValueError("line solve failed")
    return f


def _ptr3(arrs):
    out = (_dp * 3)()
    for i, a in enumerate(arrs):
        out[i] = _p(a)
    return out


def interp(P: Params, u, X):
    u = [np.ascontiguousarray(c, dtype=np.float64) for c in u]
    X = np.ascontiguousarray(X, dtype=np.float64)
    U = np.zeros_like(X)
    lib().ibo_interp(ctypes.byref(P), _ptr3(u), _p(X), X.shape[1], _p(U))
    return U


def spread(P: Params, X, F, w):
    X = np.ascontiguousarray(X, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    f = [np.zeros(grid_shape(P)) for _ in range(P.dim)]
    lib().ibo_spread(ctypes.byref(P), _p(X), _p(F), _p(w), X.shape[1], _ptr3(f))
    return f


def link_force(X, links, period=None):
    """Step 2a; period = box lengths per axis for nearest-image link vectors
    (None: no images)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    a, b, k, l0 = links
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    k = np.ascontiguousarray(k, dtype=np.float64)
    l0 = np.ascontiguousarray(l0, dtype=np.float64)
    per = None if period is None else np.ascontiguousarray(period, dtype=np.float64)
    F = np.zeros_like(X)
    lib().ibo_link_force(X.shape[0], X.shape[1], _p(X), None if per is None else _p(per),
                         len(a), _pi(a), _pi(b), _p(k), _p(l0), _p(F))
    return F


def tether_force(X, kappa, Y, period=None):
    """Tether pulls kappa_k (Y_k - X_k) alone (nearest image if period)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    per = None if period is None else np.ascontiguousarray(period, dtype=np.float64)
    F = np.zeros_like(X)
    lib().ibo_tether_force(X.shape[0], X.shape[1], _p(X), None if per is None else _p(per),
                           _p(kappa), _p(Y), _p(F))
    return F


def advection(P: Params, u):
    u = [np.ascontiguousarray(c, dtype=np.float64) for c in u]
    N = [np.zeros(grid_shape(P)) for _ in range(P.dim)]
    lib().ibo_advection(ctypes.byref(P), _ptr3(u), _ptr3(N))
    return N


def laplacian(P: Params, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros_like(q)
    lib().ibo_laplacian(ctypes.byref(P), _p(q), _p(out))
    return out


def vel_laplacian(P: Params, c: int, q):
    """Laplacian of velocity component c, with the channel's walls if set."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros_like(q)
    lib().ibo_vel_laplacian(ctypes.byref(P), c, _p(q), _p(out))
    return out


def divergence(P: Params, u):
    u = [np.ascontiguousarray(c, dtype=np.float64) for c in u]
    out = np.zeros(grid_shape(P))
    lib().ibo_divergence(ctypes.byref(P), _ptr3(u), _p(out))
    return out


def gradient(P: Params, p):
    p = np.ascontiguousarray(p, dtype=np.float64)
    g = [np.zeros(grid_shape(P)) for _ in range(P.dim)]
    lib().ibo_gradient(ctypes.byref(P), _p(p), _ptr3(g))
    return g


def split_order(P: Params, n: int):
    o = np.zeros(3, dtype=np.int32)
    lib().ibo_split_order(ctypes.byref(P), n, _pi(o))
    return [int(v) for v in o[:P.dim]]


@dataclass
class Sim:
    """Full IB-GM state advanced by ibo_step (Steps 1a-3f)."""
    P: Params
    u: list
    X: np.ndarray
    links: tuple
    w: np.ndarray
    p: np.ndarray = None
    psi: np.ndarray = None
    nl_prev: list = None
    U_prev: np.ndarray = None
    step: int = 0
    tether: tuple = None  # (kappa [np], target [dim][np]) or None
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        shp = grid_shape(self.P)
        d = self.P.dim
        self.u = [np.ascontiguousarray(c, dtype=np.float64).reshape(shp).copy()
                  for c in self.u]
        while len(self.u) < 3:
            self.u.append(np.zeros(1))
        if self.p is None:
            self.p = np.zeros(shp)
        if self.psi is None:
            self.psi = np.zeros(shp)
        if self.nl_prev is None:
            self.nl_prev = [np.zeros(shp) for _ in range(d)]
        while len(self.nl_prev) < 3:
            self.nl_prev.append(np.zeros(1))
        self.p = np.ascontiguousarray(self.p, dtype=np.float64).reshape(shp).copy()
        self.psi = np.ascontiguousarray(self.psi, dtype=np.float64).reshape(shp).copy()
        self.X = np.ascontiguousarray(self.X, dtype=np.float64).copy()
        if self.U_prev is None:
            self.U_prev = np.zeros_like(self.X)
        a, b, k, l0 = self.links
        self.links = (np.ascontiguousarray(a, dtype=np.int32),
                      np.ascontiguousarray(b, dtype=np.int32),
                      np.ascontiguousarray(k, dtype=np.float64),
                      np.ascontiguousarray(l0, dtype=np.float64))
        self.w = np.ascontiguousarray(self.w, dtype=np.float64)
        if self.tether is not None:
            self.tether = (np.ascontiguousarray(self.tether[0], dtype=np.float64),
                           np.ascontiguousarray(self.tether[1], dtype=np.float64))

    def _struct(self) -> _Sim:
        s = _Sim()
        s.prm = self.P
        s.step = self.step
        s.u = _ptr3(self.u)
        s.nl_prev = _ptr3(self.nl_prev)
        s.p = _p(self.p)
        s.psi = _p(self.psi)
        s.np = self.X.shape[1]
        s.X = _p(self.X)
        s.U_prev = _p(self.U_prev)
        a, b, k, l0 = self.links
        s.nlinks = len(a)
        s.link_a, s.link_b = _pi(a), _pi(b)
        s.link_k, s.link_l0 = _p(k), _p(l0)
        s.w = _p(self.w)
        if self.tether is not None:
            s.tether_k, s.tether_Y = _p(self.tether[0]), _p(self.tether[1])
        return s

    def advance(self, nsteps: int = 1):
        L = lib()
        for _ in range(nsteps):
            s = self._struct()
            if L.ibo_step(ctypes.byref(s)) != 0:
                raise RuntimeError("ibo_step failed")
            self.step = int(s.step)
        return self

    def fields(self):
        d = self.P.dim
        return {"u": [c.copy() for c in self.u[:d]], "p": self.p.copy(),
                "psi": self.psi.copy(), "X": self.X.copy()}
