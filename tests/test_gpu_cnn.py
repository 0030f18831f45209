"""Learned refinement proposer on the GPU (BF16 matrix-core kernels through the
C-ABI) against the FP64 reference network of oracle/cnn.py.

Each layer is compared on identical BF16 operands (inputs, weights and output
gradients rounded to BF16 on both sides, biases FP32): the FP32-accumulated
GPU results must match the FP64 reference to relative L2 error <= 1e-5 (only
the accumulation order and precision differ).  The whole training step is
checked against the reference gradient more loosely (hidden activations and
gradients are BF16 on the GPU), and a short training run must lower the loss."""
import numpy as np
import pytest

from oracle import cnn as ref

pytestmark = pytest.mark.gpu

CH = (3, 32, 32, 32, 2)


def _rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _setup(seed=11):
    import torch

    from paper_1609_00724_amd import learn
    dev = torch.device("cuda:0")
    g = np.random.Generator(np.random.PCG64(seed))
    ws, _ = ref.init_params(seed)
    bs = [g.normal(scale=0.2, size=co) for co in CH[1:]]
    flat = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(ws, bs)]).astype(np.float32)
    prop = learn.Proposer(torch.from_numpy(flat).to(dev))
    # the reference sees the same values: BF16-rounded weights, FP32 biases
    wr = [ref.bf16_round(w.astype(np.float32)) for w in ws]
    br = [b.astype(np.float32).astype(np.float64) for b in bs]
    return prop, wr, br, g, dev


def _bf16_tensor(a, dev):
    import torch
    return torch.from_numpy(ref.bf16_round(a).astype(np.float32)).to(dev).to(torch.bfloat16).view(torch.int16)


# tile shapes: one 64-pixel column chunk; the narrowest tile (half a chunk);
# three chunks, the middle one with image on both sides and the last half empty
SHAPES = [(2, 64, 64), (3, 32, 32), (1, 32, 160)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_forward(layer, shape):
    import torch

    from paper_1609_00724_amd import learn
    prop, wr, br, g, dev = _setup()
    n, h, w = shape
    if layer == 0:
        x = g.normal(size=(n, h, w, 3)).astype(np.float32)
        xin = torch.from_numpy(x).to(dev)
    else:
        x = np.maximum(g.normal(size=(n, h, w, 32)), 0).astype(np.float32)
        xin = _bf16_tensor(x, dev)
    out = learn.layer_forward(prop, layer, xin).cpu().numpy()
    want = ref.conv3x3(ref.bf16_round(x), wr[layer], br[layer])
    if layer < 3:
        want = np.maximum(want, 0.0)
    err = _rel_l2(out, want)
    print(f"layer {layer} {shape} forward rel L2 {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("shape", [(2, 64, 96)] + SHAPES[1:])
@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_backward(layer, shape):
    import torch

    from paper_1609_00724_amd import learn
    prop, wr, br, g, dev = _setup(12)
    n, h, w = shape
    ci, co = CH[layer], CH[layer + 1]
    if layer == 0:
        x = g.normal(size=(n, h, w, 3)).astype(np.float32)
        xin = torch.from_numpy(x).to(dev)
    else:
        x = g.normal(size=(n, h, w, 32)).astype(np.float32)
        xin = _bf16_tensor(x, dev)
    dy = g.normal(size=(n, h, w, co)).astype(np.float32)
    dw, db, dx = learn.layer_backward(prop, layer, xin, _bf16_tensor(dy, dev))
    rdw, rdb, rdx = ref.conv3x3_backward(ref.bf16_round(x), wr[layer], ref.bf16_round(dy), need_dx=layer > 0)
    e = (_rel_l2(dw.cpu().numpy(), rdw), _rel_l2(db.cpu().numpy(), rdb),
         _rel_l2(dx.cpu().numpy(), rdx) if layer > 0 else 0.0)
    print(f"layer {layer} {shape} backward rel L2 dw {e[0]:.2e} db {e[1]:.2e} dx {e[2]:.2e}")
    assert max(e) <= 1e-5


def _batch(g, n=4, h=64, w=64):
    x = g.normal(size=(n, h, w, 3)).astype(np.float32)
    mask = (g.random((n, h, w)) < 0.3).astype(np.float32)
    logq = g.normal(1.0, 0.5, size=(n, h, w)).astype(np.float32)
    logq[:, :2, :5] = np.nan
    return x, mask, logq


def test_train_step_gradient_and_loss():
    """Loss and full gradient of one step against the FP64 reference on the
    same BF16 weights: the GPU rounds hidden activations and gradients to
    BF16, so the gradient is held to 2e-2 relative L2 per layer, the loss to 1e-3."""
    import torch
    prop, wr, br, g, dev = _setup(13)
    x, mask, logq = _batch(g)
    T = lambda a: torch.from_numpy(a).to(dev)
    loss, grad = prop.train_step(T(x), T(mask), T(logq), lr=1e-3, lam=0.1, want_grad=True)
    torch.cuda.synchronize()
    acts = ref.forward(x, wr, br, round_acts=True)
    L, dout = ref.loss(acts[-1], mask.astype(np.float64), logq.astype(np.float64), lam=0.1)
    dws, dbs = ref.backward(acts, wr, dout)
    gr = grad.cpu().numpy().astype(np.float64)
    o = 0
    for l, (dw, db) in enumerate(zip(dws, dbs)):
        nw = dw.size
        ew, eb = _rel_l2(gr[o:o + nw], dw.ravel()), _rel_l2(gr[o + nw:o + nw + db.size], db)
        print(f"layer {l}: grad rel L2 w {ew:.2e} b {eb:.2e}")
        assert ew <= 2e-2 and eb <= 2e-2
        o += nw + db.size
    assert abs(float(loss) - L) <= 1e-3 * abs(L)


def test_adam_update_matches_oracle():
    """Three training steps through the C-ABI: after each, the FP32 master
    parameters and both Adam moments equal oracle.cnn.adam_step (Kingma & Ba
    2015, FP64) applied to the step's own inputs -- parameters and moments
    before the step, the step's gradient, the step count -- within FP32
    rounding of each operation (a few units in the last place of the terms
    that form each value)."""
    import torch
    prop, wr, br, g, dev = _setup(14)
    x, mask, logq = _batch(g)
    T = lambda a: torch.from_numpy(a).to(dev)   # noqa: E731
    lr = 2e-3
    host = lambda t: t.detach().double().cpu().numpy()   # noqa: E731
    for step in range(3):
        p0, m0, v0 = host(prop.params), host(prop.m), host(prop.v)
        _, grad = prop.train_step(T(x), T(mask), T(logq), lr=lr, lam=0.1, want_grad=True)
        torch.cuda.synchronize()
        gr = host(grad)
        p, m, v = p0.copy(), m0.copy(), v0.copy()
        ref.adam_step(p, gr, m, v, prop.t, lr=lr)
        pg, mg, vg = host(prop.params), host(prop.m), host(prop.v)
        u = np.abs(p - p0)                               # size of the FP64 update
        ulp = 2.0 ** -23
        bm = 4 * ulp * (0.9 * np.abs(m0) + 0.1 * np.abs(gr))     # rounding of m's terms
        bv = 4 * ulp * (0.999 * v0 + 0.001 * gr * gr)            # and of v's
        em = np.abs(mg - m) / (bm + 1e-45)
        ev = np.abs(vg - v) / (bv + 1e-45)
        # p: the rounding of its own operations, plus the rounding of m and v
        # carried through the update lr (m / c1) / (sqrt(v / c2) + eps), whose
        # sensitivities are u / |m| and u / (2 v) (m can be a small difference
        # of its two terms, so its rounding need not be small against m)
        with np.errstate(divide="ignore", invalid="ignore"):
            carried = np.nan_to_num(u * (bm / np.abs(m) + 0.5 * bv / v), nan=0.0, posinf=0.0)
        ep = np.abs(pg - p) / (4 * ulp * (np.abs(p0) + u) + carried + 1e-45)
        print(f"step {prop.t}: max error in units of the bound m {em.max():.3f} v {ev.max():.3f} p {ep.max():.3f}; "
              f"mean |update| {u.mean():.2e}")
        assert em.max() <= 1.0 and ev.max() <= 1.0 and ep.max() <= 1.0
        assert np.count_nonzero(gr) > 0.5 * gr.size and np.median(u[gr != 0]) > 0.5 * lr
        # the step refreshed the prepared weights from the updated parameters:
        # bit for bit what qsq_cnn_prepare makes of them
        refreshed = prop.prep.clone()
        prop.prepare()
        torch.cuda.synchronize()
        assert torch.equal(refreshed, prop.prep)


def test_training_lowers_the_loss():
    """200 Adam steps on a fixed synthetic task (mask = x0 > 0.5 smoothed by
    the 3x3 neighbourhood, log10 Q = 1 + x1): the loss must fall well below
    its start."""
    import torch

    from paper_1609_00724_amd import learn
    dev = torch.device("cuda:0")
    g = np.random.Generator(np.random.PCG64(21))
    prop = learn.Proposer(learn.init_params(3, dev))
    x = g.normal(size=(16, 64, 64, 3)).astype(np.float32)
    mask = (x[..., 0] > 0.5).astype(np.float32)
    logq = (1.0 + x[..., 1]).astype(np.float32)
    xt, mt, qt = (torch.from_numpy(a).to(dev) for a in (x, mask, logq))
    losses = [float(prop.train_step(xt, mt, qt, lr=3e-3, lam=0.5)) for _ in range(200)]
    print(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.25 * losses[0]
    out = prop.forward(xt).cpu().numpy()
    acc = ((out[..., 0] > 0) == (mask > 0.5)).mean()
    assert acc > 0.95
