"""ctypes binding of libibgm.so (the C ABI in include/ibgm.h and
include/ibgm_closure.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  Importing this
module loads the library and raises if it has not been built -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibgm.so")

IB_OK, IB_E_INVALID, IB_E_UNSUPPORTED, IB_E_DEVICE, IB_E_NONFINITE, IB_E_STATE = range(6)
IB_F64, IB_F32 = 0, 1
IB_PREC_FP64, IB_PREC_MIXED, IB_PREC_MIXED_STATE64 = 0, 1, 2
IB_FLAG_NO_ADVECTION = 1
IB_FLAG_WALLS_Y = 2
IB_FLAG_DETERMINISTIC_SPREAD = 4
IB_SPREAD_STATIC_MAX_BYTES = 32 << 20  # the static array of ib_spread_static
IB_GRAPH_BRANCHES = 1

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class GridParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("h", ctypes.c_double),
                ("rho", ctypes.c_double), ("mu", ctypes.c_double), ("dt", ctypes.c_double),
                ("chi", ctypes.c_double), ("precision", ctypes.c_int32),
                ("rotate_split", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("step0", ctypes.c_int64), ("layer_dt", _dp),
                ("body_force", ctypes.c_double * 3),
                ("wall_velocity", ctypes.c_double * 3)]


class Buffers(ctypes.Structure):
    _fields_ = [("u", _vp * 3), ("nl_prev", _vp * 3), ("psi", _vp), ("div_prev", _vp),
                ("p", _vp), ("X", _vp), ("U_prev", _vp), ("n_points", ctypes.c_int64),
                ("workspace", _vp), ("workspace_bytes", ctypes.c_size_t)]


class Structure(ctypes.Structure):
    _fields_ = [("n_links", ctypes.c_int64), ("a", ctypes.POINTER(ctypes.c_int32)),
                ("b", ctypes.POINTER(ctypes.c_int32)), ("kappa", _dp), ("l0", _dp),
                ("w", _dp), ("layer", ctypes.POINTER(ctypes.c_int32)),
                ("tether_kappa", _dp), ("tether_target", _dp)]


class IBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("ibgm status %d: %s" % (status, msg))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libibgm.so is not built (run python -m paper_1305_3976_amd.build); "
                          "there is no non-HIP fallback")
    L = ctypes.CDLL(LIB_PATH)
    L.ib_last_error.restype = ctypes.c_char_p
    L.ib_workspace_size.argtypes = [ctypes.POINTER(GridParams), ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_size_t)]
    L.ib_init.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(GridParams),
                          ctypes.POINTER(Buffers), ctypes.POINTER(Structure), _vp]
    L.ib_step.argtypes = [_vp, ctypes.c_int32]
    L.ib_restart.argtypes = [_vp, ctypes.c_int64]
    L.ib_sync.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
    L.ib_spread.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp * 3, ctypes.c_int32]
    L.ib_spread_static.argtypes = [ctypes.POINTER(GridParams), _vp, _vp, _vp, ctypes.c_int64,
                                   _vp * 3, ctypes.c_int32, _vp]
    L.ib_interp.argtypes = [_vp, _vp, ctypes.c_int64, _vp * 3, _vp]
    L.ib_refresh_divergence.argtypes = [_vp]
    L.ib_check_fields.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
    L.ib_force.argtypes = [_vp, _vp, _vp]
    L.ib_step_force.argtypes = [_vp, _vp * 3]
    L.ib_line_solve.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_double, ctypes.c_double, _vp]
    L.ib_destroy.argtypes = [_vp]
    L.ib_profile_enable.argtypes = [_vp, ctypes.c_int32]
    L.ib_profile_count.restype = ctypes.c_int32
    L.ib_profile_name.restype = ctypes.c_char_p
    L.ib_profile_name.argtypes = [ctypes.c_int32]
    L.ib_profile_read.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64)]
    L.ib_tune.argtypes = [_vp, ctypes.c_int32]
    _ip = ctypes.POINTER(ctypes.c_int32)
    L.ib_tune_read.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _ip, _ip, _ip]
    L.ib_graph_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, _vp]
    L.ib_graph_launch.argtypes = [_vp, ctypes.c_int32]
    L.ib_graph_destroy.argtypes = [_vp]
    # learned closure (include/ibgm_closure.h)
    i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.ib_conv3d_pack.argtypes = [_vp, i32, i32, i32, i32, _vp, _vp]
    L.ib_conv3d_fwd.argtypes = [_vp, i32, _ip, i32, _vp, _vp, i32, i32, _vp, i32, i32, _vp]
    L.ib_conv3d_bwd_data.argtypes = [_vp, i32, _ip, _vp, i32, _vp, _vp, _vp]
    L.ib_conv3d_bwd_weight.argtypes = [_vp, _vp, i32, _ip, i32, i32, i32, i32, _vp, _vp, _vp, _vp]
    L.ib_mse_grad.argtypes = [_vp, _vp, i64, i32, _vp, _vp, _vp, _vp]
    L.ib_adam_step.argtypes = [_vp, _vp, _vp, _vp, i64, f32, f32, f32, f32, i32, _vp]
    L.ib_restrict.argtypes = [_vp, i32, _ip, i32, _vp, _vp]
    L.ib_closure_gather.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(f32), _ip, i32, _ip, _vp,
                                    i32, _ip, i32, i32, _vp, _vp]
    L.ib_closure_apply.argtypes = [ctypes.POINTER(_vp), _ip, _vp, f32, _vp]
    L.ib_closure_conv_apply.argtypes = [_vp, _ip, _vp, _vp, f32, ctypes.POINTER(_vp), _vp]
    # streaming-rate probe (include/ibgm_probe.h)
    L.ib_probe_stream_rate.argtypes = [ctypes.POINTER(_vp), i32, ctypes.POINTER(_vp), i32, i64,
                                       i32, _vp, ctypes.POINTER(ctypes.c_double)]
    L.ib_probe_stream_rate.restype = ctypes.c_int
    for f in ("ib_workspace_size", "ib_init", "ib_step", "ib_restart", "ib_sync", "ib_spread",
              "ib_spread_static", "ib_interp", "ib_refresh_divergence", "ib_check_fields",
              "ib_force", "ib_step_force", "ib_line_solve", "ib_destroy", "ib_profile_enable",
              "ib_profile_read", "ib_tune", "ib_tune_read", "ib_graph_create", "ib_graph_launch",
              "ib_graph_destroy") + CLOSURE_EXPORTED:
        getattr(L, f).restype = ctypes.c_int
    return L


CLOSURE_EXPORTED = ("ib_conv3d_pack", "ib_conv3d_fwd", "ib_conv3d_bwd_data",
                    "ib_conv3d_bwd_weight", "ib_mse_grad", "ib_adam_step", "ib_restrict",
                    "ib_closure_gather", "ib_closure_apply", "ib_closure_conv_apply")


lib = _load()

EXPORTED = ("ib_workspace_size", "ib_init", "ib_step", "ib_restart", "ib_sync", "ib_spread",
            "ib_spread_static", "ib_interp", "ib_refresh_divergence", "ib_check_fields",
            "ib_force", "ib_step_force", "ib_line_solve", "ib_destroy", "ib_last_error",
            "ib_profile_enable",
            "ib_profile_count", "ib_profile_name", "ib_profile_read", "ib_tune", "ib_tune_read",
            "ib_graph_create", "ib_graph_launch", "ib_graph_destroy",
            "ib_probe_stream_rate") + CLOSURE_EXPORTED


def check(status: int):
    if status != IB_OK:
        raise IBError(status, lib.ib_last_error().decode())
    return status


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous()
    return _vp(t.data_ptr())


def spread_static(cfg, X: torch.Tensor, F: torch.Tensor, w: torch.Tensor, out=None,
                  accumulate=False, stream=None):
    """Step 2b without a context or workspace (ib_spread_static): the force F
    at points X (FP64 [dim][npts]) with weights w spread onto the grid of
    `cfg` (one problem), the tables in the library's static device array."""
    d = cfg.dim
    if out is None:
        out = [torch.empty(cfg.shape, dtype=cfg.grid_dtype, device=X.device) for _ in range(d)]
    P = cfg.params()
    ptrs = (_vp * 3)(*[out[c].data_ptr() if c < d else None for c in range(3)])
    npts = X.shape[1]
    args = [_ptr(X), _ptr(F), _ptr(w)] if npts > 0 else [None, None, None]
    check(lib.ib_spread_static(ctypes.byref(P), *args, npts, ptrs, 1 if accumulate else 0,
                               _stream_handle(stream)))
    return out


def stream_rate(nsrc: int, ndst: int, mib_per_stream: int = 512, reps: int = 5, stream=None):
    """HBM bytes per second that a plain elementwise kernel reaches reading
    nsrc and writing ndst FP32 streams of mib_per_stream MiB each
    (ib_probe_stream_rate): the practical ceiling for streaming kernels."""
    n = mib_per_stream * 2 ** 20 // 4
    src = [torch.ones(n, dtype=torch.float32, device="cuda") for _ in range(nsrc)]
    dst = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(ndst)]
    S = (_vp * max(1, nsrc))(*[t.data_ptr() for t in src])
    D = (_vp * max(1, ndst))(*[t.data_ptr() for t in dst])
    rate = ctypes.c_double()
    check(lib.ib_probe_stream_rate(S, nsrc, D, ndst, n, reps, _stream_handle(stream),
                                   ctypes.byref(rate)))
    del src, dst
    return rate.value


def line_solve(t: torch.Tensor, axis: int, diag: float, off: float, stream=None):
    """In-place periodic (off, diag, off) solve along `axis` (0 = x, the last
    tensor dimension) of a CUDA tensor of shape (n2, n1, n0), (n1, n0) or
    (nf, n2, n1, n0) (nf fields)."""
    if t.dtype not in (torch.float64, torch.float32):
        raise TypeError("line_solve needs float64 or float32")
    shp = list(t.shape)
    nf = 1
    if len(shp) == 4:
        nf = shp[0]
        shp = shp[1:]
    n = (ctypes.c_int32 * 3)(*([shp[-1], shp[-2] if len(shp) > 1 else 1,
                                 shp[-3] if len(shp) > 2 else 1]))
    stride = n[0] * n[1] * n[2]
    check(lib.ib_line_solve(_ptr(t), IB_F64 if t.dtype == torch.float64 else IB_F32, n, axis,
                            nf, stride, diag, off, _stream_handle(stream)))
    return t


@dataclass
class Config:
    dim: int
    n: tuple
    h: float
    rho: float = 1.0
    mu: float = 0.0
    dt: float = 1e-3
    chi: float = 0.6
    precision: int = IB_PREC_FP64
    rotate_split: bool = True
    no_advection: bool = False
    layer_dt: tuple = None  # 2-D batches: time step of each layer
    walls_y: bool = False   # channel: no-slip walls at y = 0 and y = n[1] h
    body_force: tuple = (0.0, 0.0, 0.0)  # uniform force density added to f
    wall_velocity: tuple = (0.0, 0.0, 0.0)  # walls_y: the upper wall's velocity (x, z)
    deterministic_spread: bool = False  # bitwise-reproducible spreading (slower)

    def params(self, step0: int = 0) -> GridParams:
        P = GridParams()
        P.dim = self.dim
        nn = list(self.n) + [1] * (3 - len(self.n))
        if self.dim == 2 and len(self.n) < 3:
            nn[2] = 1
        for a in range(3):
            P.n[a] = nn[a]
        P.h, P.rho, P.mu, P.dt, P.chi = self.h, self.rho, self.mu, self.dt, self.chi
        P.precision = self.precision
        P.rotate_split = 1 if self.rotate_split else 0
        P.flags = ((IB_FLAG_NO_ADVECTION if self.no_advection else 0)
                   | (IB_FLAG_WALLS_Y if self.walls_y else 0)
                   | (IB_FLAG_DETERMINISTIC_SPREAD if self.deterministic_spread else 0))
        P.step0 = step0
        for a in range(3):
            P.body_force[a] = float(self.body_force[a]) if a < len(self.body_force) else 0.0
            P.wall_velocity[a] = (float(self.wall_velocity[a]) if a < len(self.wall_velocity)
                                  else 0.0)
        if self.layer_dt is not None:
            self._ldt = np.ascontiguousarray(self.layer_dt, dtype=np.float64)
            P.layer_dt = self._ldt.ctypes.data_as(_dp)
        return P

    @property
    def grid_dtype(self):
        """dtype of the work arrays (nl_prev, psi, div_prev, spread forces)."""
        return torch.float64 if self.precision == IB_PREC_FP64 else torch.float32

    @property
    def velocity_dtype(self):
        return torch.float32 if self.precision == IB_PREC_MIXED else torch.float64

    @property
    def shape(self):
        nn = list(self.n) + [1] * (3 - len(self.n))
        return (nn[2], nn[1], nn[0])


class Simulation:
    """Device state of one IB-GM problem plus its library context.

    u0: list of dim numpy arrays of shape Config.shape; structure: an object
    with X (dim, np), links (a, b, kappa, l0) and w (np,).  Optional state
    (for restarts): p, psi, nl_prev, div_prev, U_prev and step0.
    """

    def __init__(self, cfg: Config, u0, structure, device="cuda", p=None, psi=None,
                 nl_prev=None, div_prev=None, U_prev=None, step0: int = 0, stream=None):
        self.cfg = cfg
        d = cfg.dim
        dev = torch.device(device)
        gd = cfg.grid_dtype
        shp = cfg.shape
        to = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).reshape(shp).to(dev).contiguous()
        self.u = [to(u0[c], cfg.velocity_dtype) for c in range(d)]
        self.nl_prev = [to(nl_prev[c], gd) if nl_prev is not None else torch.zeros(shp, dtype=gd, device=dev)
                        for c in range(d)]
        self.psi = to(psi, gd) if psi is not None else torch.zeros(shp, dtype=gd, device=dev)
        self.div_prev = to(div_prev, gd) if div_prev is not None else torch.zeros(shp, dtype=gd, device=dev)
        self.p = to(p, torch.float64) if p is not None else torch.zeros(shp, dtype=torch.float64, device=dev)
        X = np.ascontiguousarray(structure.X, dtype=np.float64)
        self.np = X.shape[1]
        self.X = torch.as_tensor(X).to(dev).contiguous()
        self.U_prev = (torch.as_tensor(np.ascontiguousarray(U_prev, dtype=np.float64)).to(dev).contiguous()
                       if U_prev is not None else torch.zeros_like(self.X))
        P = cfg.params(step0)
        nbytes = ctypes.c_size_t()
        check(lib.ib_workspace_size(ctypes.byref(P), self.np, ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        B = Buffers()
        for c in range(3):
            B.u[c] = self.u[c].data_ptr() if c < d else None
            B.nl_prev[c] = self.nl_prev[c].data_ptr() if c < d else None
        B.psi = self.psi.data_ptr()
        B.div_prev = self.div_prev.data_ptr()
        B.p = self.p.data_ptr()
        B.X = self.X.data_ptr()
        B.U_prev = self.U_prev.data_ptr()
        B.n_points = self.np
        B.workspace = self.workspace.data_ptr() + off
        B.workspace_bytes = nbytes.value
        a, b, k, l0 = structure.links
        self._host = [np.ascontiguousarray(a, dtype=np.int32), np.ascontiguousarray(b, dtype=np.int32),
                      np.ascontiguousarray(k, dtype=np.float64), np.ascontiguousarray(l0, dtype=np.float64),
                      np.ascontiguousarray(structure.w, dtype=np.float64)]
        layer = getattr(structure, "layer", None)
        if layer is not None:
            self._host.append(np.ascontiguousarray(layer, dtype=np.int32))
        S = Structure()
        S.n_links = len(self._host[0])
        S.a = self._host[0].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        S.b = self._host[1].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        S.kappa = self._host[2].ctypes.data_as(_dp)
        S.l0 = self._host[3].ctypes.data_as(_dp)
        S.w = self._host[4].ctypes.data_as(_dp)
        if len(self._host) > 5:
            S.layer = self._host[5].ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        tether = getattr(structure, "tether", None)
        if tether is not None:
            self._tether = (np.ascontiguousarray(tether[0], dtype=np.float64),
                            np.ascontiguousarray(tether[1], dtype=np.float64))
            S.tether_kappa = self._tether[0].ctypes.data_as(_dp)
            S.tether_target = self._tether[1].ctypes.data_as(_dp)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        ctx = _vp()
        check(lib.ib_init(ctypes.byref(ctx), ctypes.byref(P), ctypes.byref(B), ctypes.byref(S),
                          _vp(self.stream.cuda_stream)))
        self.ctx = ctx

    # -- stepping --------------------------------------------------------
    def step(self, nsteps: int = 1):
        check(lib.ib_step(self.ctx, nsteps))
        return self

    def restart(self, step0: int = 0):
        """Continue from whatever the state tensors now hold, as step step0."""
        check(lib.ib_restart(self.ctx, step0))
        return self

    def refresh_divergence(self):
        """Recompute div_prev = D.u after the caller changed u between steps."""
        check(lib.ib_refresh_divergence(self.ctx))
        return self

    def max_velocity(self) -> float:
        """Grid-field watchdog: max |u| over all faces (raises IBError with
        IB_E_NONFINITE if u or p holds a non-finite value)."""
        m = ctypes.c_double()
        check(lib.ib_check_fields(self.ctx, ctypes.byref(m)))
        return m.value

    def sync(self) -> int:
        n = ctypes.c_int64()
        check(lib.ib_sync(self.ctx, ctypes.byref(n)))
        return n.value

    # -- single steps of the method on given buffers ------------------------
    def spread(self, X: torch.Tensor, F: torch.Tensor, w: torch.Tensor, out=None, accumulate=False):
        d = self.cfg.dim
        if out is None:
            out = [torch.zeros(self.cfg.shape, dtype=self.cfg.grid_dtype, device=X.device)
                   for _ in range(d)]
        ptrs = (_vp * 3)(*[out[c].data_ptr() if c < d else None for c in range(3)])
        check(lib.ib_spread(self.ctx, _ptr(X), _ptr(F), _ptr(w), X.shape[1], ptrs,
                            1 if accumulate else 0))
        return out

    def interp(self, X: torch.Tensor, u):
        d = self.cfg.dim
        U = torch.empty_like(X)
        ptrs = (_vp * 3)(*[u[c].data_ptr() if c < d else None for c in range(3)])
        check(lib.ib_interp(self.ctx, _ptr(X), X.shape[1], ptrs, _ptr(U)))
        return U

    def force(self, X: torch.Tensor):
        F = torch.empty_like(X)
        check(lib.ib_force(self.ctx, _ptr(X), _ptr(F)))
        return F

    def step_force(self, out=None):
        """The force density spread in the last step (grid dtype, dense)."""
        d = self.cfg.dim
        if out is None:
            out = [torch.empty(self.cfg.shape, dtype=self.cfg.grid_dtype, device=self.X.device)
                   for _ in range(d)]
        ptrs = (_vp * 3)(*[out[c].data_ptr() if c < d else None for c in range(3)])
        check(lib.ib_step_force(self.ctx, ptrs))
        return out

    # -- tuning --------------------------------------------------------------
    def tune(self, reps: int = 3):
        check(lib.ib_tune(self.ctx, reps))
        out = {}
        for axis in range(self.cfg.dim):
            for r64 in (0, 1):
                v = [ctypes.c_int32() for _ in range(3)]
                check(lib.ib_tune_read(self.ctx, axis, r64, *[ctypes.byref(x) for x in v]))
                out[(axis, r64)] = tuple(x.value for x in v)
        return out

    # -- profiling ---------------------------------------------------------
    def profile(self, enable: bool = True):
        check(lib.ib_profile_enable(self.ctx, 1 if enable else 0))

    def profile_read(self):
        out = {}
        for i in range(lib.ib_profile_count()):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            check(lib.ib_profile_read(self.ctx, i, ctypes.byref(ms), ctypes.byref(n)))
            if n.value:
                out[lib.ib_profile_name(i).decode()] = (ms.value, n.value)
        return out

    # -- state -------------------------------------------------------------
    def state(self):
        torch.cuda.synchronize()
        d = self.cfg.dim
        f = lambda t: t.detach().double().cpu().numpy()
        return {"u": [f(self.u[c]) for c in range(d)], "p": f(self.p), "psi": f(self.psi),
                "X": f(self.X), "U_prev": f(self.U_prev),
                "nl_prev": [f(self.nl_prev[c]) for c in range(d)], "div_prev": f(self.div_prev)}

    def close(self):
        if getattr(self, "ctx", None):
            lib.ib_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """One hipGraph replaying `steps_per_launch` steps of several simulations
    that share a (non-null) stream (ib_graph_create / ib_graph_launch).
    branches=True records each simulation as an independent graph branch."""

    def __init__(self, sims, steps_per_launch: int, branches: bool = False, stream=None):
        self.sims = list(sims)
        arr = (_vp * len(self.sims))(*[s.ctx.value for s in self.sims])
        st = stream if stream is not None else self.sims[0].stream
        g = _vp()
        check(lib.ib_graph_create(ctypes.byref(g), arr, len(self.sims), steps_per_launch,
                                  IB_GRAPH_BRANCHES if branches else 0, _vp(st.cuda_stream)))
        self.g = g
        self.steps_per_launch = steps_per_launch

    def launch(self, nlaunches: int = 1):
        check(lib.ib_graph_launch(self.g, nlaunches))

    def close(self):
        if getattr(self, "g", None):
            lib.ib_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
