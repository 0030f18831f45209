"""Pins of the FP64 reference network (oracle/cnn.py): convolution against
SciPy's 2D correlation, special kernels, finite-difference gradients of the
whole loss, BF16 rounding on hand-derived values, one Adam step in closed form."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_conv_matches_scipy_correlate():
    g = _rng(1)
    x = g.normal(size=(2, 9, 7, 3))
    w = g.normal(size=(3, 3, 3, 4))
    b = g.normal(size=4)
    out = cnn.conv3x3(x, w, b)
    for n in range(2):
        for co in range(4):
            want = b[co] + sum(correlate2d(x[n, :, :, ci], w[:, :, ci, co], mode="same", boundary="fill")
                               for ci in range(3))
            np.testing.assert_allclose(out[n, :, :, co], want, rtol=1e-12, atol=1e-12)


def test_special_kernels():
    g = _rng(2)
    x = g.normal(size=(1, 6, 5, 4))
    w = np.zeros((3, 3, 4, 4))
    w[1, 1] = np.eye(4)
    np.testing.assert_array_equal(cnn.conv3x3(x, w, np.zeros(4)), x)         # identity
    w = np.zeros((3, 3, 4, 4))
    w[0, 1] = np.eye(4)                                                      # reads (y - 1, x)
    out = cnn.conv3x3(x, w, np.zeros(4))
    np.testing.assert_array_equal(out[:, 1:], x[:, :-1])
    np.testing.assert_array_equal(out[:, 0], 0.0)


def _net_loss(x, ws, bs, mask, logq):
    return cnn.loss(cnn.forward(x, ws, bs)[-1], mask, logq)[0]


def test_finite_difference_gradients():
    """Central differences on ~1% of the weights (and every bias of the last
    layer, and some inputs) against the backward pass: relative error <= 1e-6."""
    g = _rng(3)
    x = g.normal(size=(1, 10, 10, 3))
    ws, bs = cnn.init_params(7)
    bs = [g.normal(scale=0.1, size=b.shape) for b in bs]      # nonzero biases move ReLU kinks off zero
    mask = (g.random((1, 10, 10)) < 0.3).astype(float)
    logq = g.normal(1.0, 0.5, size=(1, 10, 10))
    logq[0, 0, :3] = np.nan                                    # invalid targets are skipped
    acts = cnn.forward(x, ws, bs)
    L, dout = cnn.loss(acts[-1], mask, logq)
    dws, dbs = cnn.backward(acts, ws, dout)
    eps = 1e-4      # the loss is smooth away from ReLU kinks; rounding noise ~1e-16/eps
    worst = 0.0
    for l, w in enumerate(ws):
        flat = w.reshape(-1)
        for k in g.choice(flat.size, size=max(2, flat.size // 100), replace=False):
            old = flat[k]
            flat[k] = old + eps
            lp = _net_loss(x, ws, bs, mask, logq)
            flat[k] = old - eps
            lm = _net_loss(x, ws, bs, mask, logq)
            flat[k] = old
            fd = (lp - lm) / (2 * eps)
            an = dws[l].reshape(-1)[k]
            worst = max(worst, abs(fd - an) / max(abs(fd), abs(an), 1e-8))
    for k in range(bs[-1].size):
        old = bs[-1][k]
        bs[-1][k] = old + eps
        lp = _net_loss(x, ws, bs, mask, logq)
        bs[-1][k] = old - eps
        lm = _net_loss(x, ws, bs, mask, logq)
        bs[-1][k] = old
        fd = (lp - lm) / (2 * eps)
        worst = max(worst, abs(fd - dbs[-1][k]) / max(abs(fd), 1e-8))
    assert worst <= 1e-6, worst


def test_input_gradient_of_one_layer():
    g = _rng(4)
    x = g.normal(size=(2, 5, 6, 3))
    w = g.normal(size=(3, 3, 3, 2))
    b = g.normal(size=2)
    gy = g.normal(size=(2, 5, 6, 2))
    _, db, dx = cnn.conv3x3_backward(x, w, gy)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (1, 4, 5, 2), (0, 2, 3, 1), (1, 0, 5, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = ((cnn.conv3x3(xp, w, b) - cnn.conv3x3(xm, w, b)) * gy).sum() / (2 * eps)
        assert abs(fd - dx[idx]) <= 1e-7 * max(1.0, abs(fd))
    np.testing.assert_allclose(db, gy.sum((0, 1, 2)), rtol=1e-14)


def test_bf16_rounding_values():
    """BF16 keeps 7 fraction bits: 1 + 2^-8 is a tie between 1 (even) and
    1 + 2^-7 (odd) and goes to 1; 1 + 3 2^-8 ties between 1 + 2^-7 (odd) and
    1 + 2^-6 (even); the FP32 rounding first drops 2^-40; 3e38 = 2^127 x
    1.7632.. lies between 225 and 226 steps of 2^120 above 2^127 x 0 and
    rounds to 226 / 128."""
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -40, -2.5, 3.0e38])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1.0, -2.5, 2.0 ** 127 * 226 / 128])
    np.testing.assert_array_equal(cnn.bf16_round(vals), want)


@pytest.mark.parametrize("gval", [0.3, -2.0, 1e-3])
def test_adam_first_step(gval):
    p = np.array([1.0])
    m, v = np.zeros(1), np.zeros(1)
    cnn.adam_step(p, np.array([gval]), m, v, 1, lr=0.01)
    # m_hat = g, v_hat = g^2: the first step moves by lr * g / (|g| + eps)
    assert np.isclose(p[0], 1.0 - 0.01 * gval / (abs(gval) + 1e-8), rtol=0, atol=1e-15)
