"""Learned closure: a three-layer 3-D convolutional network that corrects a
2x coarser IB-GM solve (mesh 2h, time step 2 dt) toward the restriction of the
fine solve, trained on pairs the method itself generates.

Everything that computes runs in libibgm.so (include/ibgm_closure.h): the
convolutions and their gradients on the matrix cores, the loss, Adam, the MAC
restriction, the gathering of inputs and targets, and applying the
correction.  PyTorch only holds the buffers.

Network: 9 input channels (the coarse velocity u, v, w after one coarse
step, the spread elastic force f on the coarse grid, and the coarse step's
velocity increment, each scaled), 32 -> 32
hidden channels with ReLU, 3 output channels (the scaled correction
R(u_fine) - u_coarse), 3x3x3 taps, BF16 weights and activations, FP32
accumulation and FP32 master weights.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import ibgm
from .ibgm import _vp, check, lib

CIN, HID, COUT = 9, 32, 3
PERIODIC, VALID, FULL = 0, 1, 2
RELU, OUT_F32, NARROW = 1, 2, 4
PACK_FORWARD, PACK_ADJOINT, PACK_NARROW = 0, 1, 2
WGRAD_WS = 256 * (27 * 32 * 32 + 32) * 4


def packed_bytes(ci_pad):
    return 27 * (ci_pad // 16) * 64 * 16


def _i3(d):
    return (ctypes.c_int32 * 3)(*[int(v) for v in d])


def _p(t):
    return _vp(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def out_dims(dims, mode, layers=1):
    g = {PERIODIC: 0, VALID: -2, FULL: 2}[mode] * layers
    return tuple(int(d) + g for d in dims)


class ConvNet:
    """FP32 master parameters in one flat tensor (theta), their gradient and
    Adam moments; packed BF16 operand tiles for the forward and adjoint
    convolutions are refreshed after every update."""

    LAYERS = ((CIN, HID, 16), (HID, HID, 32), (HID, COUT, 32))  # (ci, co, ci_pad)

    def __init__(self, seed: int = 0, device="cuda"):
        self.device = torch.device(device)
        shapes = []
        for ci, co, _ in self.LAYERS:
            shapes += [(27, ci, co), (co,)]
        sizes = [int(np.prod(s)) for s in shapes]
        self.n_params = sum(sizes)
        rng = np.random.default_rng(seed)
        host = []
        for li, (ci, co, _) in enumerate(self.LAYERS):
            std = math.sqrt(2.0 / (27 * ci)) * (0.1 if li == 2 else 1.0)
            host.append(rng.standard_normal((27, ci, co)) * std)
            host.append(np.zeros(co))
        flat = np.concatenate([h.ravel() for h in host]).astype(np.float32)
        dev = self.device
        self.theta = torch.as_tensor(flat).to(dev)
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.offsets = np.cumsum([0] + sizes)
        self.W = [self._view(self.theta, 2 * i) for i in range(3)]
        self.b = [self._view(self.theta, 2 * i + 1) for i in range(3)]
        self.gW = [self._view(self.grad, 2 * i) for i in range(3)]
        self.gb = [self._view(self.grad, 2 * i + 1) for i in range(3)]
        # the output layer (3 channels) uses the 16-wide matrix-core packing
        self.P = [torch.empty(packed_bytes(cp) if i < 2 else 27 * 64 * 16, dtype=torch.uint8,
                              device=dev) for i, (_, _, cp) in enumerate(self.LAYERS)]
        self.T = [None] + [torch.empty(packed_bytes(32), dtype=torch.uint8, device=dev)
                           for _ in range(2)]
        self.wg_ws = torch.empty(WGRAD_WS, dtype=torch.uint8, device=dev)
        self.mse_ws = torch.empty(4096, dtype=torch.uint8, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.t = 0
        self._buf = {}
        self.pack()

    def _view(self, t, k):
        o0, o1 = int(self.offsets[k]), int(self.offsets[k + 1])
        ci, co, _ = self.LAYERS[k // 2]
        return t[o0:o1].view((27, ci, co) if k % 2 == 0 else (co,))

    def pack(self, stream=None):
        st = _stream(stream)
        for i, (ci, co, cp) in enumerate(self.LAYERS):
            check(lib.ib_conv3d_pack(_p(self.W[i]), ci, co, cp,
                                     PACK_NARROW if i == 2 else PACK_FORWARD, _p(self.P[i]), st))
            if i > 0:
                check(lib.ib_conv3d_pack(_p(self.W[i]), ci, co, 32, PACK_ADJOINT, _p(self.T[i]), st))

    def _buffers(self, batch, dims, mode):
        key = (batch, tuple(dims), mode)
        if key not in self._buf:
            d1 = out_dims(dims, mode, 1)
            d2 = out_dims(dims, mode, 2)
            d3 = out_dims(dims, mode, 3)
            nv = lambda d: batch * d[0] * d[1] * d[2]
            dev = self.device
            bf = torch.bfloat16
            self._buf[key] = {
                "dims": (tuple(dims), d1, d2, d3),
                "a1": torch.empty(nv(d1) * 32, dtype=bf, device=dev),
                "a2": torch.empty(nv(d2) * 32, dtype=bf, device=dev),
                "y": torch.empty(nv(d3) * COUT, dtype=torch.float32, device=dev),
                "gy": torch.empty(nv(d3) * 32, dtype=bf, device=dev),
                "g2": torch.empty(nv(d2) * 32, dtype=bf, device=dev),
                "g1": torch.empty(nv(d1) * 32, dtype=bf, device=dev),
            }
        return self._buf[key]

    def forward(self, x, batch, dims, mode, stream=None):
        """x: BF16 [batch][d2][d1][d0][16] (dims = (d0, d1, d2)).  Returns the
        FP32 output [batch][..][3] (a view of an internal buffer)."""
        B = self._buffers(batch, dims, mode)
        st = _stream(stream)
        d0, d1, d2, _ = B["dims"]
        check(lib.ib_conv3d_fwd(_p(x), batch, _i3(d0), 16, _p(self.P[0]), _p(self.b[0]), mode,
                                RELU, _p(B["a1"]), 32, 32, st))
        check(lib.ib_conv3d_fwd(_p(B["a1"]), batch, _i3(d1), 32, _p(self.P[1]), _p(self.b[1]),
                                mode, RELU, _p(B["a2"]), 32, 32, st))
        check(lib.ib_conv3d_fwd(_p(B["a2"]), batch, _i3(d2), 32, _p(self.P[2]), _p(self.b[2]),
                                mode, OUT_F32 | NARROW, _p(B["y"]), COUT, COUT, st))
        return B["y"]

    def correct(self, x, n, u, scale, stream=None):
        """The periodic forward pass over a whole grid n = (n0, n1, n2) with
        its output added in place: u[c] += scale * y[..., c] (three FP32
        component arrays).  Layers 1 and 2 as in forward(); the last layer
        adds to u as it goes (ib_closure_conv_apply), the same arithmetic as
        forward() followed by apply_correction()."""
        B = self._buffers(1, n, PERIODIC)
        st = _stream(stream)
        d = _i3(n)
        check(lib.ib_conv3d_fwd(_p(x), 1, d, 16, _p(self.P[0]), _p(self.b[0]), PERIODIC, RELU,
                                _p(B["a1"]), 32, 32, st))
        check(lib.ib_conv3d_fwd(_p(B["a1"]), 1, d, 32, _p(self.P[1]), _p(self.b[1]), PERIODIC,
                                RELU, _p(B["a2"]), 32, 32, st))
        U = (_vp * 3)(*[t.data_ptr() for t in u])
        check(lib.ib_closure_conv_apply(_p(B["a2"]), d, _p(self.P[2]), _p(self.b[2]),
                                        float(scale), U, st))

    def backward(self, x, target, batch, dims, mode, stream=None):
        """Loss (device scalar) and the gradient of every parameter into
        self.grad, after forward() on the same x."""
        B = self._buffers(batch, dims, mode)
        st = _stream(stream)
        d0, d1, d2, d3 = B["dims"]
        nv3 = batch * d3[0] * d3[1] * d3[2]
        check(lib.ib_mse_grad(_p(B["y"]), _p(target), nv3, COUT, _p(self.loss), _p(B["gy"]),
                              _p(self.mse_ws), st))
        check(lib.ib_conv3d_bwd_weight(_p(B["a2"]), _p(B["gy"]), batch, _i3(d2), 32, mode, HID,
                                       COUT, _p(self.gW[2]), _p(self.gb[2]), _p(self.wg_ws), st))
        check(lib.ib_conv3d_bwd_data(_p(B["gy"]), batch, _i3(d3), _p(self.T[2]), mode,
                                     _p(B["a2"]), _p(B["g2"]), st))
        check(lib.ib_conv3d_bwd_weight(_p(B["a1"]), _p(B["g2"]), batch, _i3(d1), 32, mode, HID,
                                       HID, _p(self.gW[1]), _p(self.gb[1]), _p(self.wg_ws), st))
        check(lib.ib_conv3d_bwd_data(_p(B["g2"]), batch, _i3(d2), _p(self.T[1]), mode,
                                     _p(B["a1"]), _p(B["g1"]), st))
        check(lib.ib_conv3d_bwd_weight(_p(x), _p(B["g1"]), batch, _i3(d0), 16, mode, CIN, HID,
                                       _p(self.gW[0]), _p(self.gb[0]), _p(self.wg_ws), st))
        return self.loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.t += 1
        check(lib.ib_adam_step(_p(self.theta), _p(self.grad), _p(self.m), _p(self.v),
                               self.n_params, lr, beta1, beta2, eps, self.t, _stream(stream)))
        self.pack(stream)

    def train_step(self, x, target, batch, dims, mode, lr, stream=None):
        self.forward(x, batch, dims, mode, stream)
        loss = self.backward(x, target, batch, dims, mode, stream)
        self.adam(lr, stream=stream)
        return loss

    def params_numpy(self):
        """[(W, b)] per layer as float64 numpy arrays (for checks)."""
        return [(self.W[i].detach().double().cpu().numpy(), self.b[i].detach().double().cpu().numpy())
                for i in range(3)]

    def grads_numpy(self):
        return [(self.gW[i].detach().double().cpu().numpy(), self.gb[i].detach().double().cpu().numpy())
                for i in range(3)]

    def load_numpy(self, params):
        flat = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])
        self.theta.copy_(torch.as_tensor(flat.astype(np.float32)))
        self.pack()


# ---------------------------------------------------------- field helpers --

def restrict(fine: torch.Tensor, kind: int, out: torch.Tensor = None, stream=None):
    """ib_restrict of a (n2, n1, n0) fine tensor; kind 0-2 = face normal to
    that axis, 3 = cell centred."""
    n2, n1, n0 = fine.shape
    if out is None:
        out = torch.empty((n2 // 2, n1 // 2, n0 // 2), dtype=fine.dtype, device=fine.device)
    dt = ibgm.IB_F64 if fine.dtype == torch.float64 else ibgm.IB_F32
    check(lib.ib_restrict(_p(fine), dt, _i3((n0, n1, n2)), kind, _p(out), _stream(stream)))
    return out


def gather(srcs, scales, chans, n, origins: torch.Tensor, dims, out_f32: bool, out_ch: int,
           out: torch.Tensor, stream=None):
    """ib_closure_gather into `out` (see the header)."""
    k = len(srcs)
    S = (_vp * k)(*[s.data_ptr() for s in srcs])
    F = (ctypes.c_float * k)(*scales)
    C = (ctypes.c_int32 * k)(*chans)
    check(lib.ib_closure_gather(S, F, C, k, _i3(n), _p(origins), origins.shape[0], _i3(dims),
                                1 if out_f32 else 0, out_ch, _p(out), _stream(stream)))
    return out


def apply_correction(u, y, scale, stream=None):
    n2, n1, n0 = u[0].shape
    U = (_vp * 3)(*[t.data_ptr() for t in u])
    check(lib.ib_closure_apply(U, _i3((n0, n1, n2)), _p(y), float(scale), _stream(stream)))


# ------------------------------------------------------------ pair maker --

@dataclass
class Scales:
    u: float
    f: float
    du: float
    target: float


class CoarseFine:
    """A fine IB-GM run (n_fine^3, dt) and a coarse companion (n_fine/2, 2 dt)
    restarted from the restricted fine state; one coarse step against two fine
    steps gives one training pair (input: coarse velocity and spread force;
    target: restricted fine velocity minus coarse velocity)."""

    def __init__(self, case, n_fine: int, precision=ibgm.IB_PREC_MIXED, mu=0.01, rho=1.0,
                 device="cuda"):
        if precision != ibgm.IB_PREC_MIXED:
            raise ValueError("the closure works on the FP32 grids of the mixed policy")
        nf, nc = n_fine, n_fine // 2
        self.nf, self.nc = nf, nc
        dev = torch.device(device)
        cf = ibgm.Config(3, (nf, nf, nf), 1.0 / nf, rho=rho, mu=mu, dt=case.dt_fine,
                         precision=precision)
        cc = ibgm.Config(3, (nc, nc, nc), 1.0 / nc, rho=rho, mu=mu, dt=2 * case.dt_fine,
                         precision=precision)
        self.fine = ibgm.Simulation(cf, case.u0, case.structure, device=dev)
        zero = [np.zeros((nc, nc, nc))] * 3
        self.coarse = ibgm.Simulation(cc, zero, case.structure, device=dev)
        self.w = torch.as_tensor(np.asarray(case.structure.w, dtype=np.float64)).to(dev)
        self.Ru = [torch.empty((nc, nc, nc), dtype=torch.float32, device=dev) for _ in range(3)]
        self.ub = [torch.empty((nc, nc, nc), dtype=torch.float32, device=dev) for _ in range(3)]
        self.f = None

    def sync_coarse_to_fine(self):
        """Coarse state := restriction of the fine state, restarted at step 0."""
        c, f = self.coarse, self.fine
        for k in range(3):
            restrict(f.u[k], k, c.u[k])
        restrict(f.p, 3, c.p)
        c.psi.zero_()
        c.X.copy_(f.X)
        c.restart(0)

    def coarse_step(self, net: ConvNet = None, scales: Scales = None):
        """One coarse step (2 dt), optionally followed by the learned correction."""
        # the velocity before the step, for the input's increment channels (one
        # multi-tensor copy launch for the three components)
        torch._foreach_copy_(self.ub, list(self.coarse.u))
        self.coarse.step(1)
        self.spread_force()
        if net is not None:
            nc = self.nc
            x = self.inputs_full(scales)
            net.correct(x, (nc, nc, nc), self.coarse.u, 1.0 / scales.target)
            # the next step's pressure update averages D.u^{n+1} with D.u^n:
            # recompute the latter from the corrected velocity
            self.coarse.refresh_divergence()

    def spread_force(self):
        """The force density the coarse step spread (FP32 grid arrays)."""
        if self.f is None:
            self.f = self.coarse.step_force()
        else:
            self.coarse.step_force(self.f)
        return self.f

    def fine_steps(self, k=2):
        self.fine.step(k)

    def restricted_fine(self):
        for k in range(3):
            restrict(self.fine.u[k], k, self.Ru[k])
        return self.Ru

    def inputs_full(self, scales: Scales, out=None):
        """The network input over the whole coarse grid (BF16, 16 channels);
        into `out`, or into a buffer kept for the next call."""
        nc = self.nc
        if out is None:
            if getattr(self, "_x_full", None) is None:
                self._x_full = torch.empty(nc ** 3 * 16, dtype=torch.bfloat16,
                                           device=self.Ru[0].device)
            out = self._x_full
        if getattr(self, "_org0", None) is None:
            self._org0 = torch.zeros((1, 3), dtype=torch.int32, device=out.device)
        srcs, sc, ch = self.input_sources(scales)
        gather(srcs, sc, ch, (nc, nc, nc), self._org0, (nc, nc, nc), False, 16, out)
        return out

    def input_sources(self, scales: Scales):
        """Sources, scales and channels of the network input: u_c, f and
        u_c - u_c(before the step)."""
        u = list(self.coarse.u)
        return (u + list(self.f) + u + list(self.ub),
                [scales.u] * 3 + [scales.f] * 3 + [scales.du] * 3 + [-scales.du] * 3,
                [0, 1, 2, 3, 4, 5, 6, 7, 8, 6, 7, 8])

    def close(self):
        self.fine.close()
        self.coarse.close()


def estimate_scales(cf: CoarseFine):
    """Input and target scales (1 / rms) from one pair on the host."""
    cf.sync_coarse_to_fine()
    cf.coarse_step()
    cf.fine_steps(2)
    Ru = cf.restricted_fine()
    torch.cuda.synchronize()
    host = lambda ts: [t.double().cpu().numpy() for t in ts]
    rms = lambda arrs: float(np.sqrt(np.mean([np.mean(a ** 2) for a in arrs])))
    uc, ru, ub = host(cf.coarse.u), host(Ru), host(cf.ub)
    su = rms(uc)
    sf = rms(host(cf.f))
    sd = rms([uc[k] - ub[k] for k in range(3)])
    st = rms([ru[k] - uc[k] for k in range(3)])
    inv = lambda v: 1.0 / max(v, 1e-30)
    return Scales(inv(su), inv(sf), inv(sd), inv(st))


class PairSet:
    """Training pairs on the device.  Periodic mode stores whole coarse fields
    (bricks = the grid); valid mode stores crops of `crop` output voxels per
    side with a 3-voxel input margin, `crops` per pair."""

    def __init__(self, capacity: int, nc: int, mode=PERIODIC, crop: int = 32, device="cuda"):
        self.mode = mode
        self.nc = nc
        if mode == PERIODIC:
            self.in_dims = self.out_dims = (nc, nc, nc)
        else:
            self.out_dims = (crop, crop, crop)
            self.in_dims = (crop + 6,) * 3
        nin = int(np.prod(self.in_dims))
        nout = int(np.prod(self.out_dims))
        self.x = torch.zeros(capacity * nin * 16, dtype=torch.bfloat16, device=device)
        self.t = torch.zeros(capacity * nout * 3, dtype=torch.float32, device=device)
        self.nin, self.nout = nin, nout
        self.capacity = capacity
        self.count = 0
        self.slot_of = np.random.default_rng(1234).permutation(capacity)

    def add(self, cf: CoarseFine, scales: Scales, crops: int, rng):
        """Append `crops` bricks of the current pair (coarse step taken, fine
        advanced): inputs from the coarse fields, targets R(u_f) - u_c."""
        nc = self.nc
        Ru = cf.restricted_fine()
        for _ in range(crops):
            if self.count >= self.capacity:
                return
            s = int(self.slot_of[self.count])
            if self.mode == PERIODIC:
                o_in = np.zeros(3, dtype=np.int32)
                o_out = o_in
            else:
                o_out = rng.integers(0, nc, size=3).astype(np.int32)
                o_in = (o_out - 3).astype(np.int32)
            dev = self.x.device
            oi = torch.as_tensor(o_in.reshape(1, 3)).to(dev)
            oo = torch.as_tensor(o_out.reshape(1, 3)).to(dev)
            xs = self.x[s * self.nin * 16:(s + 1) * self.nin * 16]
            ts = self.t[s * self.nout * 3:(s + 1) * self.nout * 3]
            srcs, sc, ch = cf.input_sources(scales)
            gather(srcs, sc, ch, (nc, nc, nc), oi, self.in_dims, False, 16, xs)
            gather(list(Ru) + list(cf.coarse.u), [scales.target] * 3 + [-scales.target] * 3,
                   [0, 1, 2, 0, 1, 2], (nc, nc, nc), oo, self.out_dims, True, 3, ts)
            self.count += 1

    def batch(self, first: int, size: int):
        """Slots [first, first + size): inputs and targets as views."""
        return (self.x[first * self.nin * 16:(first + size) * self.nin * 16],
                self.t[first * self.nout * 3:(first + size) * self.nout * 3])


def collect(cases, n_fine, snapshots, every, warmup, pairs: PairSet, scales: Scales = None,
            crops: int = 1, seed: int = 0, precision=ibgm.IB_PREC_MIXED):
    """Run each case's fine trajectory and add `snapshots` pairs taken every
    `every` fine steps after `warmup` steps.  Returns the scales used."""
    rng = np.random.default_rng(seed)
    for case in cases:
        cf = CoarseFine(case, n_fine, precision)
        cf.fine_steps(warmup)
        if scales is None:
            scales = estimate_scales(cf)
        for _ in range(snapshots):
            cf.sync_coarse_to_fine()
            cf.coarse_step()
            cf.fine_steps(2)
            pairs.add(cf, scales, crops, rng)
            if every > 2:
                cf.fine_steps(every - 2)
        cf.fine.sync()
        cf.close()
    return scales


def collect_rollouts(cases, n_fine, net: ConvNet, scales: Scales, pairs: PairSet, syncs: int,
                     horizon: int, every: int, warmup: int, crops: int = 1, seed: int = 2):
    """Pairs along corrected coarse runs (the states the network meets in
    service): from each of `syncs` restarts at the restricted fine state,
    `horizon` coarse intervals, each a plain coarse step whose input and
    target R(u_f) - u_c make a pair, after which the current network's
    correction is applied before the next interval; the fine run advances two
    steps per interval and `every` more between restarts."""
    rng = np.random.default_rng(seed)
    nc = n_fine // 2
    for case in cases:
        cf = CoarseFine(case, n_fine)
        cf.fine_steps(warmup)
        for _ in range(syncs):
            cf.sync_coarse_to_fine()
            for _ in range(horizon):
                cf.coarse_step()
                cf.fine_steps(2)
                pairs.add(cf, scales, crops, rng)
                x = cf.inputs_full(scales)
                net.correct(x, (nc, nc, nc), cf.coarse.u, 1.0 / scales.target)
                cf.coarse.refresh_divergence()
            if every:
                cf.fine_steps(every)
        cf.fine.sync()
        cf.close()


def train(net: ConvNet, pairs, iters: int, batch: int, lr: float = 1e-3,
          stream=None, lr_decay_to: float = 0.1):
    """Adam over contiguous slot batches (slots are a random permutation of
    the pairs) of one PairSet or of several (same crop shape; batches drawn
    from all of them in one shuffled plan), linear decay of the learning
    rate.  Returns the loss of every iteration (host floats, read once at
    the end)."""
    sets = list(pairs) if isinstance(pairs, (list, tuple)) else [pairs]
    plan = [(i, k) for i, ps in enumerate(sets) for k in range(max(1, ps.count // batch))]
    losses = torch.empty(iters, dtype=torch.float32, device=net.device)
    order = np.random.default_rng(99).permutation(len(plan))
    for it in range(iters):
        i, k = plan[int(order[it % len(plan)])]
        ps = sets[i]
        x, t = ps.batch(k * batch, batch)
        frac = it / max(1, iters - 1)
        l = net.train_step(x, t, batch, ps.in_dims, ps.mode,
                           lr * (1.0 - (1.0 - lr_decay_to) * frac), stream)
        losses[it:it + 1].copy_(l)
    return losses.cpu().numpy()


def evaluate(net: ConvNet, pairs: PairSet, first: int, count: int, batch: int = 1):
    """Relative l2 error of the coarse velocity against the restricted fine one
    over pairs [first, first + count), without and with the correction."""
    num0 = num1 = 0.0
    for k in range(first, first + count, batch):
        b = min(batch, first + count - k)
        x, t = pairs.batch(k, b)
        y = net.forward(x, b, pairs.in_dims, pairs.mode)
        yy = y[:b * pairs.nout * 3]
        num0 += float(torch.sum(t.double() ** 2))
        num1 += float(torch.sum((t.double() - yy.double()) ** 2))
    return math.sqrt(num0), math.sqrt(num1)


# -------------------------------------------------------------- rollout --

def rollout(case, n_fine: int, steps: int, net: ConvNet, scales: Scales, warmup: int = 6,
            snap: dict = None):
    """Coarse runs with and without the correction, both restarted from the
    restricted fine state after `warmup` fine steps, against the restricted
    fine run: relative l2 velocity error after each coarse step, and the mean
    time per coarse step of each (HIP events on the current stream).  With
    `snap` = {"interval": k}, the three velocities after interval k (FP64
    host arrays: restricted fine, plain coarse, corrected coarse) are stored
    in it under "fine", "plain" and "corrected"."""
    cf = CoarseFine(case, n_fine)
    plain = CoarseFine.__new__(CoarseFine)
    plain.__dict__.update(cf.__dict__)
    nc = cf.nc
    cc = cf.coarse.cfg
    plain.coarse = ibgm.Simulation(cc, [np.zeros((nc, nc, nc))] * 3, case.structure,
                                   device=cf.w.device)
    plain.ub = [torch.empty_like(t) for t in cf.ub]
    plain.f = None
    cf.fine_steps(warmup)
    cf.sync_coarse_to_fine()
    plain.sync_coarse_to_fine()
    errs = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_plain = t_corr = 0.0
    for _ in range(steps):
        ev[0].record()
        plain.coarse_step()
        ev[1].record()
        cf.coarse_step(net, scales)
        ev[2].record()
        cf.fine_steps(2)
        ev[3].record()
        Ru = cf.restricted_fine()
        torch.cuda.synchronize()
        t_plain += ev[0].elapsed_time(ev[1])
        t_corr += ev[1].elapsed_time(ev[2])
        h = lambda ts: [t.double().cpu().numpy() for t in ts]
        r, a, b = h(Ru), h(plain.coarse.u), h(cf.coarse.u)
        if snap is not None and len(errs) + 1 == snap.get("interval"):
            snap.update(fine=r, plain=a, corrected=b)
        nr = math.sqrt(sum(float(np.sum(x ** 2)) for x in r))
        ea = math.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, r))) / nr
        eb = math.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(b, r))) / nr
        errs.append((ea, eb))
    plain.coarse.close()
    cf.close()
    return errs, t_plain / steps, t_corr / steps


def interval_times(case, n_fine: int, net: ConvNet, scales: Scales, reps: int = 20,
                   warmup: int = 6):
    """GPU time per coarse interval, plain and corrected, each over `reps`
    consecutive intervals enqueued back to back (HIP events on the current
    stream, no host round trip between intervals -- the way the fine steps
    are timed), from the restricted fine state after `warmup` fine steps."""
    cf = CoarseFine(case, n_fine)
    cf.fine_steps(warmup)
    cf.sync_coarse_to_fine()
    out = []
    for corrected in (False, True):
        step = (lambda: cf.coarse_step(net, scales)) if corrected else cf.coarse_step
        step()  # first call allocates the step's buffers
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / reps)
    cf.close()
    return out[0], out[1]


# ------------------------------------------------- guarded rollout (judge) --

def guarded_rollout(case, n_fine: int, steps: int, net: ConvNet, scales: Scales,
                    check_every: int = 4, warmup: int = 6):
    """The closure in service, with the plain fine solve as its judge and its
    fallback.  Three coarse runs start from the restricted fine state after
    `warmup` fine steps: plain, corrected after every step, and guarded
    (corrected too, but audited).  Every `check_every` coarse intervals the
    judge compares the guarded and the plain coarse velocities with the
    restricted fine one; where the correction has stopped winning (guarded
    error above plain), the guarded run falls back on the fine solve: it
    restarts from the restricted fine state, with the correction kept on.
    Returns per interval (plain, corrected, guarded) relative l2 errors
    against the restricted fine velocity, and the intervals where the
    fallback fired."""
    runs = [CoarseFine(case, n_fine)]
    nc = runs[0].nc
    cc = runs[0].coarse.cfg
    for _ in range(2):
        r = CoarseFine.__new__(CoarseFine)
        r.__dict__.update(runs[0].__dict__)
        r.coarse = ibgm.Simulation(cc, [np.zeros((nc, nc, nc))] * 3, case.structure,
                                   device=runs[0].w.device)
        r.ub = [torch.empty_like(t) for t in runs[0].ub]
        r.f = None
        runs.append(r)
    judge, plain, corr = runs[0], runs[1], runs[2]
    guard = judge  # the guarded run is the judge's own coarse companion
    judge.fine_steps(warmup)
    for r in (guard, plain, corr):
        r.sync_coarse_to_fine()
    host = lambda ts: [t.double().cpu().numpy() for t in ts]

    def err(u, ref, nr):
        return math.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(host(u), ref))) / nr

    errs, fired = [], []
    for k in range(steps):
        plain.coarse_step()
        corr.coarse_step(net, scales)
        guard.coarse_step(net, scales)
        judge.fine_steps(2)
        ref = host(judge.restricted_fine())
        nr = math.sqrt(sum(float(np.sum(x ** 2)) for x in ref))
        e = (err(plain.coarse.u, ref, nr), err(corr.coarse.u, ref, nr),
             err(guard.coarse.u, ref, nr))
        errs.append(e)
        if (k + 1) % check_every == 0 and e[2] > e[0]:
            guard.sync_coarse_to_fine()   # fall back on the fine solve
            fired.append(k)
    for r in (plain, corr):
        r.coarse.close()
    judge.close()
    return errs, fired
