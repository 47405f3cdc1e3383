"""Plain FP64 CPU oracle of the learned closure: a three-layer 3-D
convolutional network, its gradients, the Adam update, and the fine-to-coarse
restriction of MAC-grid fields that builds its training pairs.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests, the smoke
check and the CPU-baseline leg of the benchmark use it; the product path never
imports it, and it shares no code with the HIP library.

Conventions
  Activations are float64 arrays of shape (B, D2, D1, D0, C): a batch of 3-D
  bricks, x fastest, channels last.  A layer's weights have shape (27, Ci, Co)
  with tap t = 9 tz + 3 ty + tx (tz, ty, tx in {0, 1, 2}) and bias shape (Co,).
  Output voxel p of a layer reads input voxel p + (tz, ty, tx) + off:
    "periodic":  off = -1 and indices wrap (same size out as in),
    "valid":     off = 0, output D - 2 per axis (no padding),
    "full":      off = -2 and voxels outside the input read 0 (output D + 2);
                 the transpose of "valid".
Parity is pinned by brute-force sums, the adjoint identity, central
differences and closed forms (see the tests); the network itself is not in the
paper (its gain is measured, not pinned).
"""
from __future__ import annotations

import numpy as np

OFFSETS = {"periodic": -1, "valid": 0, "full": -2}


def taps():
    """(t, tz, ty, tx) for the 27 taps in storage order."""
    return [(9 * tz + 3 * ty + tx, tz, ty, tx)
            for tz in range(3) for ty in range(3) for tx in range(3)]


def _shifted(x, tz, ty, tx, mode):
    """x[:, p + t + off] for every output voxel p of the given mode."""
    B, D2, D1, D0, C = x.shape
    off = OFFSETS[mode]
    if mode == "periodic":
        return np.roll(x, shift=(-(tz + off), -(ty + off), -(tx + off)), axis=(1, 2, 3))
    if mode == "valid":
        return x[:, tz:tz + D2 - 2, ty:ty + D1 - 2, tx:tx + D0 - 2, :]
    pad = np.zeros((B, D2 + 4, D1 + 4, D0 + 4, C))
    pad[:, 2:-2, 2:-2, 2:-2, :] = x
    return pad[:, tz:tz + D2 + 2, ty:ty + D1 + 2, tx:tx + D0 + 2, :]


def conv3d(x, W, b, mode):
    """y[p, co] = b[co] + sum_t sum_ci x[p + t + off, ci] W[t, ci, co]."""
    y = None
    for t, tz, ty, tx in taps():
        term = _shifted(x, tz, ty, tx, mode) @ W[t]
        y = term if y is None else y + term
    return y + b


def conv3d_transpose(g, W, mode):
    """Adjoint of conv3d (without bias) with respect to its input:
    x_grad[q, ci] = sum_t sum_co g[q - t - off, co] W[t, ci, co]."""
    B = g.shape[0]
    if mode == "periodic":
        out = np.zeros(g.shape[:4] + (W.shape[1],))
        for t, tz, ty, tx in taps():
            out += np.roll(g @ W[t].T, shift=(tz - 1, ty - 1, tx - 1), axis=(1, 2, 3))
        return out
    if mode == "valid":
        E2, E1, E0 = g.shape[1:4]
        out = np.zeros((B, E2 + 2, E1 + 2, E0 + 2, W.shape[1]))
        for t, tz, ty, tx in taps():
            out[:, tz:tz + E2, ty:ty + E1, tx:tx + E0, :] += g @ W[t].T
        return out
    raise ValueError(mode)


def conv3d_weight_grad(x, g, mode):
    """dW[t, ci, co] = sum_p x[p + t + off, ci] g[p, co];  db[co] = sum_p g[p, co]."""
    dW = np.zeros((27, x.shape[-1], g.shape[-1]))
    for t, tz, ty, tx in taps():
        xs = _shifted(x, tz, ty, tx, mode)
        dW[t] = xs.reshape(-1, x.shape[-1]).T @ g.reshape(-1, g.shape[-1])
    return dW, g.reshape(-1, g.shape[-1]).sum(axis=0)


def relu(z):
    return np.maximum(z, 0.0)


def forward(params, x, mode):
    """params: [(W1, b1), (W2, b2), (W3, b3)]; ReLU after the first two
    layers.  Returns the list of activations [x, a1, a2, y]."""
    acts = [x]
    for i, (W, b) in enumerate(params):
        z = conv3d(acts[-1], W, b, mode)
        acts.append(relu(z) if i < len(params) - 1 else z)
    return acts


def backward(params, acts, gy, mode):
    """Gradients of a scalar loss L given gy = dL/dy: [(dW_i, db_i)] and
    dL/dx.  The ReLU derivative is taken as 1 where the activation is > 0."""
    grads = [None] * len(params)
    g = gy
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        grads[i] = conv3d_weight_grad(acts[i], g, mode)
        g = conv3d_transpose(g, W, mode)
        if i > 0:
            g = g * (acts[i] > 0)
    return grads, g


def mse(y, target):
    """L = mean over voxels and channels of (y - target)^2, and dL/dy."""
    d = y - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at step t >= 1;
    returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ restriction --

def restrict_face(u, comp):
    """Fine-to-coarse restriction of MAC component `comp` (faces normal to
    axis comp; arrays (n2, n1, n0), x fastest): the coarse face at coarse
    index I along comp coincides with fine face 2I, and spans the 2 x 2 fine
    faces 2J + {0, 1} along the other axes; its value is their average."""
    ax = 2 - comp                      # numpy axis of grid axis `comp`
    sl = [slice(None)] * 3
    sl[ax] = slice(0, None, 2)
    v = u[tuple(sl)]
    for a in range(3):
        if a != ax:
            s0 = [slice(None)] * 3
            s1 = [slice(None)] * 3
            s0[a] = slice(0, None, 2)
            s1[a] = slice(1, None, 2)
            v = 0.5 * (v[tuple(s0)] + v[tuple(s1)])
    return v


def restrict_cell(p):
    """Cell-centred restriction: the average of the 2 x 2 x 2 fine cells that
    make up a coarse cell."""
    v = p
    for a in range(3):
        s0 = [slice(None)] * 3
        s1 = [slice(None)] * 3
        s0[a] = slice(0, None, 2)
        s1[a] = slice(1, None, 2)
        v = 0.5 * (v[tuple(s0)] + v[tuple(s1)])
    return v
