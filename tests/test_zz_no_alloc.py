"""ib_spread_static -- Step 2b (spreading) without a context or workspace,
its point sort and tile tables in the library's fixed device array -- through
the C ABI against ib_spread on a context (the existing entry point, same
points, forces and weights), and against the oracle's spreading.

Two calls in a row on one GPU, the second with a smaller grid and fewer
points, so stale tables of the first call would show; both grid dtypes;
accumulate mode; a call with no points.  Spreading adds in LDS with
atomics, so the two entry points agree to the rounding of the sums' order:
FP64 within 1e-13 of the largest value, FP32 grids (one rounding of an FP64
sum) within 2^-22 of it."""
import numpy as np
import pytest
import torch

import oracle
from helpers import LazyModule

ibgm = LazyModule("paper_1305_3976_amd.ibgm")
inputs = LazyModule("paper_1305_3976_amd.inputs")

pytestmark = pytest.mark.gpu


def make_case(dim, n, npts, seed):
    """Points spread over the box and beyond it (unwrapped), seeded forces
    and weights."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n[0]
    box = np.array([n[a] * h for a in range(dim)])
    X = rng.uniform(-0.3, 1.3, (dim, npts)) * box[:, None]
    F = rng.standard_normal((dim, npts))
    w = rng.uniform(0.5, 2.0, npts)
    return h, X, F, w


def tol_for(precision):
    return 1e-13 if precision == ibgm.IB_PREC_FP64 else 2.0 ** -22


def context_spread(cfg, X, F, w, accumulate_onto=None):
    """ib_spread on a context built for these points (no links)."""
    npts = X.shape[1]
    links = (np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0))
    S = inputs.Structure(X, links, w)
    u0 = [np.zeros(cfg.shape) for _ in range(cfg.dim)]
    sim = ibgm.Simulation(cfg, u0, S)
    Xd = torch.as_tensor(X).cuda()
    Fd = torch.as_tensor(F).cuda()
    wd = torch.as_tensor(w).cuda()
    out = None if accumulate_onto is None else [t.clone() for t in accumulate_onto]
    f = sim.spread(Xd, Fd, wd, out=out, accumulate=accumulate_onto is not None)
    torch.cuda.synchronize()
    res = [t.cpu().numpy().astype(np.float64) for t in f]
    sim.close()
    assert npts == X.shape[1]
    return res


def static_spread(cfg, X, F, w, accumulate_onto=None):
    Xd = torch.as_tensor(X).cuda()
    Fd = torch.as_tensor(F).cuda()
    wd = torch.as_tensor(w).cuda()
    out = None
    if accumulate_onto is not None:
        out = [t.clone() for t in accumulate_onto]
    else:
        # poison the output: the call must clear it
        out = [torch.full(cfg.shape, 7.0, dtype=cfg.grid_dtype, device="cuda")
               for _ in range(cfg.dim)]
    f = ibgm.spread_static(cfg, Xd, Fd, wd, out=out, accumulate=accumulate_onto is not None)
    torch.cuda.synchronize()
    return [t.cpu().numpy().astype(np.float64) for t in f]


def compare(a, b, tol, label):
    for c in range(len(b)):
        scale = max(np.abs(b[c]).max(), 1e-300)
        err = np.abs(a[c] - b[c]).max() / scale
        print(label, "component", c, "max rel diff", err)
        assert err <= tol, (label, c, err, tol)


@pytest.mark.parametrize("precision", [0, 1])
def test_static_equals_context_spread_two_calls(precision):
    """Two calls in a row: 3-D 64 x 48 x 40 with 6000 points, then 32 x 24 x
    20 with 700 points; each equals ib_spread on a context of its own, and
    the first also equals the oracle's spreading."""
    cases = [((64, 48, 40), 6000, 1), ((32, 24, 20), 700, 2)]
    for k, (n, npts, seed) in enumerate(cases):
        h, X, F, w = make_case(3, n, npts, seed)
        cfg = ibgm.Config(3, n, h, mu=0.01, dt=1e-3, precision=precision)
        print("call", k, "grid", n, "points", npts, "precision", precision, flush=True)
        got = static_spread(cfg, X, F, w)
        ref = context_spread(cfg, X, F, w)
        compare(got, ref, tol_for(precision), "static vs ib_spread call %d" % k)
        if k == 0:
            P = oracle.make_params(3, n, h, rho=1.0, mu=0.01, dt=1e-3)
            orc = oracle.spread(P, X, F, w)
            # FP32 grids hold FP32 stencil weights and values: a few units of
            # 2^-24 per term
            compare(got, orc, 1e-13 if precision == 0 else 1e-6, "static vs oracle")


@pytest.mark.parametrize("precision", [0, 1])
def test_static_2d_accumulate_and_empty(precision):
    """2-D 96 x 80: a first call of 1500 points, then accumulate 400 more on
    top (against ib_spread in accumulate mode), then a call with no points
    (the output is cleared and nothing else happens)."""
    n = (96, 80, 1)
    h, X, F, w = make_case(2, n, 1500, 5)
    cfg = ibgm.Config(2, n, h, mu=0.01, dt=1e-3, precision=precision)
    first = static_spread(cfg, X, F, w)
    ref1 = context_spread(cfg, X, F, w)
    compare(first, ref1, tol_for(precision), "2-D first")
    _, X2, F2, w2 = make_case(2, n, 400, 6)
    base = [torch.as_tensor(a).to(cfg.grid_dtype).cuda() for a in ref1]
    got = static_spread(cfg, X2, F2, w2, accumulate_onto=base)
    ref = context_spread(cfg, X2, F2, w2, accumulate_onto=base)
    compare(got, ref, tol_for(precision), "2-D accumulate")
    empty = static_spread(cfg, X2[:, :0], F2[:, :0], w2[:0])
    for c in range(2):
        assert np.all(empty[c] == 0.0)


def test_static_rejects_what_it_cannot_hold():
    """Beyond the static array, a batch of 2-D layers, bad pointers: refused
    on the host with nothing enqueued."""
    import ctypes
    cfg = ibgm.Config(3, (256, 256, 256), 1 / 256, mu=0.01, dt=5e-4,
                      precision=ibgm.IB_PREC_FP64)
    P = cfg.params()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    ptrs = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    # more points than the static array has bytes: whatever the tables hold
    # per point (the point sort alone keeps several ints), this is refused on
    # the host -- a count that fits would enqueue kernels on the fake pointers
    too_many = ibgm.IB_SPREAD_STATIC_MAX_BYTES + 1
    st = ibgm.lib.ib_spread_static(ctypes.byref(P), fake, fake, fake, too_many, ptrs, 0, None)
    assert st == ibgm.IB_E_UNSUPPORTED
    assert b"static array" in ibgm.lib.ib_last_error()
    Q = ibgm.Config(2, (64, 64, 3), 1 / 64, mu=0.01, dt=1e-3).params()
    assert ibgm.lib.ib_spread_static(ctypes.byref(Q), fake, fake, fake, 10, ptrs, 0,
                                     None) == ibgm.IB_E_INVALID
    assert ibgm.lib.ib_spread_static(ctypes.byref(P), None, fake, fake, 10, ptrs, 0,
                                     None) == ibgm.IB_E_INVALID
