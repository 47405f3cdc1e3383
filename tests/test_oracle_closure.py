"""Pins of the closure oracle (CPU): brute-force convolution sums, the adjoint
identity, central differences of a small network's loss, Adam's closed form
under a constant gradient, and exact identities of the MAC restriction."""
import itertools

import numpy as np
import pytest

from oracle import closure as oc


def brute_conv(x, W, b, mode):
    """Seven nested loops over the definition (independent of the vectorised
    oracle)."""
    B, D2, D1, D0, Ci = x.shape
    Co = W.shape[2]
    off = oc.OFFSETS[mode]
    if mode == "periodic":
        E = (D2, D1, D0)
    elif mode == "valid":
        E = (D2 - 2, D1 - 2, D0 - 2)
    else:
        E = (D2 + 2, D1 + 2, D0 + 2)
    y = np.zeros((B,) + E + (Co,))
    for bb, k, j, i in itertools.product(range(B), range(E[0]), range(E[1]), range(E[2])):
        acc = b.copy()
        for tz, ty, tx in itertools.product(range(3), repeat=3):
            kk, jj, ii = k + tz + off, j + ty + off, i + tx + off
            if mode == "periodic":
                kk, jj, ii = kk % D2, jj % D1, ii % D0
            elif not (0 <= kk < D2 and 0 <= jj < D1 and 0 <= ii < D0):
                continue
            acc = acc + x[bb, kk, jj, ii, :] @ W[9 * tz + 3 * ty + tx]
        y[bb, k, j, i] = acc
    return y


@pytest.mark.parametrize("mode", ["periodic", "valid", "full"])
def test_conv_matches_brute_force(mode):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 5, 6, 3))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    assert np.allclose(oc.conv3d(x, W, b, mode), brute_conv(x, W, b, mode), rtol=0, atol=1e-12)


def test_conv_identity_and_shift_kernels():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 5, 4, 6, 2))
    W = np.zeros((27, 2, 2))
    W[13] = np.eye(2)                       # centre tap = identity
    assert np.array_equal(oc.conv3d(x, W, np.zeros(2), "periodic"), x)
    W = np.zeros((27, 2, 2))
    W[14] = np.eye(2)                       # tap (1, 1, 2): reads x + 1
    assert np.array_equal(oc.conv3d(x, W, np.zeros(2), "periodic"), np.roll(x, -1, axis=3))


@pytest.mark.parametrize("mode", ["periodic", "valid"])
def test_transpose_is_adjoint(mode):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 6, 5, 7, 3))
    W = rng.standard_normal((27, 3, 4))
    y = oc.conv3d(x, W, np.zeros(4), mode)
    g = rng.standard_normal(y.shape)
    lhs = np.sum(y * g)
    rhs = np.sum(x * oc.conv3d_transpose(g, W, mode))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    if mode == "valid":
        # the transpose of "valid" is the "full" convolution with flipped taps
        # and transposed channel blocks
        Wf = np.stack([W[26 - t].T for t in range(27)])
        assert np.allclose(oc.conv3d_transpose(g, W, mode), oc.conv3d(g, Wf, np.zeros(3), "full"),
                           rtol=0, atol=1e-12)
    else:
        Wf = np.stack([W[26 - t].T for t in range(27)])
        assert np.allclose(oc.conv3d_transpose(g, W, mode),
                           oc.conv3d(g, Wf, np.zeros(3), "periodic"), rtol=0, atol=1e-12)


def small_net(rng, cin=4, hid=5, cout=3):
    return [(rng.standard_normal((27, cin, hid)) * 0.3, rng.standard_normal(hid) * 0.1),
            (rng.standard_normal((27, hid, hid)) * 0.3, rng.standard_normal(hid) * 0.1),
            (rng.standard_normal((27, hid, cout)) * 0.3, rng.standard_normal(cout) * 0.1)]


@pytest.mark.parametrize("mode", ["periodic", "valid"])
def test_gradients_match_central_differences(mode):
    rng = np.random.default_rng(4)
    params = small_net(rng)
    shape = (2, 7, 7, 8, 4) if mode == "valid" else (1, 4, 5, 4, 4)
    x = rng.standard_normal(shape)
    acts = oc.forward(params, x, mode)
    target = rng.standard_normal(acts[-1].shape)

    def loss(ps, xx):
        return oc.mse(oc.forward(ps, xx, mode)[-1], target)[0]

    L, gy = oc.mse(acts[-1], target)
    grads, gx = oc.backward(params, acts, gy, mode)
    h = 1e-5

    def fd(arr, idx):
        # fourth-order central difference: truncation O(h^4), rounding ~eps L / h
        old = arr[idx]
        vals = []
        for k in (2, 1, -1, -2):
            arr[idx] = old + k * h
            vals.append(loss(params, x))
        arr[idx] = old
        return (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)

    for li in range(3):
        for which in (0, 1):
            arr = params[li][which]
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                an = grads[li][which][idx]
                d = fd(arr, idx)
                assert abs(d - an) <= 1e-8 * max(1.0, abs(an)), (li, which, idx, d, an)
    for idx in [tuple(rng.integers(0, s) for s in x.shape) for _ in range(6)]:
        d = fd(x, idx)
        assert abs(d - gx[idx]) <= 1e-8 * max(1.0, abs(gx[idx])), (idx, d, gx[idx])


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the bias-corrected moments are g and g^2 at
    # every step, so each update is -lr g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 1e-2
    for t in range(1, 6):
        new, m, v = oc.adam_step(th, g, m, v, t, lr)
        step = -lr * g / (np.abs(g) + 1e-8)
        assert np.allclose(new - th, step, rtol=1e-12, atol=1e-15)
        th = new


def _mac_div(u, h):
    """Discrete divergence of a 3-D MAC field (periodic), written out here."""
    return sum((np.roll(u[c], -1, axis=2 - c) - u[c]) / h for c in range(3))


def test_restriction_commutes_with_divergence():
    rng = np.random.default_rng(5)
    n = 8
    u = [rng.standard_normal((n, n, n)) for _ in range(3)]
    lhs = _mac_div([oc.restrict_face(u[c], c) for c in range(3)], 2.0 / n)
    rhs = oc.restrict_cell(_mac_div(u, 1.0 / n))
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12)


def test_restriction_of_linear_and_constant_fields():
    n = 8
    h = 1.0 / n
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    # u (faces normal to x) at (i h, (j + 1/2) h, (k + 1/2) h), linear in y and z
    u = 3.0 + 2.0 * (j + 0.5) * h - 1.5 * (k + 0.5) * h
    R = oc.restrict_face(u, 0)
    H = 2 * h
    K, J, I = np.meshgrid(np.arange(n // 2), np.arange(n // 2), np.arange(n // 2), indexing="ij")
    assert np.allclose(R, 3.0 + 2.0 * (J + 0.5) * H - 1.5 * (K + 0.5) * H, rtol=0, atol=1e-14)
    assert np.array_equal(oc.restrict_cell(np.full((n, n, n), 2.5)), np.full((4, 4, 4), 2.5))
