"""FP64 reference of the learned refinement proposer (TEST INFRASTRUCTURE ONLY).

The network is an extension beyond the paper: it reads coarse tiles of three
maps the method produces (field-line length, its FLEDGE map of Sect. 3.6, and
the vertical field) and proposes where the refinement of Sect. 3.6 should go.
Written from the definitions of a 3x3 'same' convolution (zero padding),
bias, ReLU, a logistic loss and a squared loss; NHWC arrays in FP64.

Layers: 3 -> 32 -> 32 -> 32 -> 2 channels, ReLU after the first three.
Output channel 0 is the refine-mask logit, channel 1 the predicted log10 Q.
Weights w[l] have shape (3, 3, Ci, Co): tap (dy, dx) multiplies the input at
(y + dy - 1, x + dx - 1).

Nothing here is shared with the HIP library; the only common ground is the
data layout described above.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (3, 32, 32, 32, 2)


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even) after rounding to FP32,
    returned as FP64 (the values the BF16 operands of the GPU path hold)."""
    u = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, w, b):
    """out[n, y, x, :] = b + sum over taps of in[n, y+dy-1, x+dx-1, :] @ w[dy, dx]."""
    n, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(np.asarray(b, np.float64), (n, H, W, w.shape[3])).copy()
    for dy in range(3):
        for dx in range(3):
            out += xp[:, dy:dy + H, dx:dx + W, :] @ w[dy, dx]
    return out


def conv3x3_backward(x, w, dy_out, need_dx=True):
    """Gradients of sum(dy_out * conv3x3(x, w, b)) with respect to w, b and x."""
    n, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros_like(w, dtype=np.float64)
    g = dy_out.reshape(-1, dy_out.shape[3])
    for dy in range(3):
        for dx in range(3):
            dw[dy, dx] = xp[:, dy:dy + H, dx:dx + W, :].reshape(-1, x.shape[3]).T @ g
    db = g.sum(0)
    dx_in = None
    if need_dx:
        dxp = np.zeros_like(xp)
        for dy in range(3):
            for dx in range(3):
                dxp[:, dy:dy + H, dx:dx + W, :] += dy_out @ w[dy, dx].T
        dx_in = dxp[:, 1:-1, 1:-1, :]
    return dw, db, dx_in


def init_params(seed, channels=CHANNELS):
    """He-normal weights (std sqrt(2 / (9 Ci))) and zero biases, seeded."""
    g = np.random.Generator(np.random.PCG64(seed))
    ws, bs = [], []
    for ci, co in zip(channels[:-1], channels[1:]):
        ws.append(g.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(3, 3, ci, co)))
        bs.append(np.zeros(co))
    return ws, bs


def forward(x, ws, bs, round_acts=False):
    """Activations of every layer: acts[0] = x, acts[l] = ReLU(conv) for the
    hidden layers, acts[-1] = the two output channels (no ReLU).  With
    round_acts, inputs and hidden activations are rounded to BF16 where the GPU
    path stores them in BF16."""
    acts = [bf16_round(x) if round_acts else np.asarray(x, np.float64)]
    L = len(ws)
    for l in range(L):
        z = conv3x3(acts[-1], ws[l], bs[l])
        if l < L - 1:
            z = np.maximum(z, 0.0)
            if round_acts:
                z = bf16_round(z)
        acts.append(z)
    return acts


def loss(out, mask, logq, lam=0.1):
    """Mean over pixels of the logistic loss of the mask logit plus lam times
    the mean squared error of log10 Q over pixels with a finite target.
    Returns the loss and its gradient with respect to out."""
    z, qh = out[..., 0], out[..., 1]
    P = z.size
    valid = np.isfinite(logq)
    tq = np.where(valid, logq, 0.0)
    sp = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))          # softplus(z)
    L = (sp - mask * z).sum() / P + lam * (valid * (qh - tq) ** 2).sum() / P
    g = np.empty_like(out)
    g[..., 0] = (1.0 / (1.0 + np.exp(-z)) - mask) / P
    g[..., 1] = 2.0 * lam * valid * (qh - tq) / P
    return L, g


def backward(acts, ws, dout):
    """Gradients of the loss for every layer given dL/d(output): lists dws, dbs,
    following the layers backwards (ReLU passes the gradient where its output
    is positive)."""
    L = len(ws)
    dws, dbs = [None] * L, [None] * L
    g = dout
    for l in range(L - 1, -1, -1):
        dw, db, dx = conv3x3_backward(acts[l], ws[l], g, need_dx=l > 0)
        dws[l], dbs[l] = dw, db
        if l > 0:
            g = dx * (acts[l] > 0.0)
    return dws, dbs


def adam_step(p, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of p in place; t counts from 1."""
    m *= beta1
    m += (1 - beta1) * grad
    v *= beta2
    v += (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)
