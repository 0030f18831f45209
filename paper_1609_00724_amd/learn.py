"""Learned refinement proposer: torch-facing wrappers of the libqsq CNN calls
(include/qsq_cnn.h).  Every forward, backward and optimiser step runs in the
library's HIP kernels; torch holds the device buffers.

The network (an extension beyond QSL Squasher) reads coarse 64 x 64 tiles of
three maps -- field-line length, its FLEDGE map and Bz -- and outputs per pixel
a refine-mask logit and a log10 Q estimate."""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _abi as A
from ._abi import check, lib
from .api import _bytes_tensor, _p, _stream

CHANNELS = (3, 32, 32, 32, 2)


def param_offsets():
    """(weight offset, bias offset) of each layer in the FP32 parameter vector."""
    out, o = [], 0
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        out.append((o, o + 9 * ci * co))
        o += 9 * ci * co + co
    assert o == A.CNN_PARAMS
    return out


def init_params(seed: int, device) -> torch.Tensor:
    """He-normal weights (std sqrt(2 / (9 Ci))) and zero biases, seeded."""
    g = torch.Generator().manual_seed(seed)
    p = torch.zeros(A.CNN_PARAMS, dtype=torch.float32)
    for (wo, bo), ci, co in zip(param_offsets(), CHANNELS[:-1], CHANNELS[1:]):
        p[wo:bo] = torch.randn(9 * ci * co, generator=g) * math.sqrt(2.0 / (9 * ci))
    return p.to(device)


class Proposer:
    """FP32 master parameters, Adam state and the prepared BF16 weights."""

    def __init__(self, params: torch.Tensor):
        if params.numel() != A.CNN_PARAMS or params.dtype != torch.float32 or not params.is_cuda:
            raise ValueError(f"params must be {A.CNN_PARAMS} float32 values on the device")
        self.params = params.contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.prep = _bytes_tensor(lib.qsq_cnn_prep_bytes(), params.device)
        self._ws = None
        self.prepare()

    def prepare(self, stream=None):
        check(lib.qsq_cnn_prepare(_p(self.params), _p(self.prep), _stream(stream)))

    def _workspace(self, n, h, w):
        need = lib.qsq_cnn_workspace_bytes(n, h, w)
        if self._ws is None or self._ws.numel() * 8 < need:
            self._ws = _bytes_tensor(need, self.params.device)
        return self._ws

    def workspace(self, n, h, w) -> torch.Tensor:
        """A workspace of its own for forward() on n tiles of h x w (for calls
        that overlap on several streams)."""
        return _bytes_tensor(lib.qsq_cnn_workspace_bytes(n, h, w), self.params.device)

    def forward(self, x: torch.Tensor, stream=None, ws=None) -> torch.Tensor:
        """x: (n, h, w, 3) float32 device tiles -> (n, h, w, 2) logits and log10 Q.
        ws: a workspace from workspace() (default: one shared by the calls
        on this object, which must then not overlap)."""
        x = x.contiguous()
        n, h, w, c = x.shape
        if c != 3 or x.dtype != torch.float32:
            raise ValueError("x must be float32 (n, h, w, 3)")
        out = torch.empty((n, h, w, 2), dtype=torch.float32, device=x.device)
        if ws is None:
            ws = self._workspace(n, h, w)
        elif ws.numel() * 8 < lib.qsq_cnn_workspace_bytes(n, h, w):
            raise ValueError("workspace too small")
        check(lib.qsq_cnn_forward(_p(self.prep), _p(x), n, h, w, _p(out), _p(ws), ws.numel() * 8, _stream(stream)))
        return out

    def train_step(self, x, mask, logq, lr=1e-3, lam=0.1, want_grad=False, stream=None):
        """One Adam step on a batch; returns the loss (device float64 scalar)
        and, if asked, the gradient (params layout)."""
        x, mask, logq = x.contiguous(), mask.contiguous(), logq.contiguous()
        n, h, w, _ = x.shape
        self.t += 1
        ws = self._workspace(n, h, w)
        loss = torch.empty((), dtype=torch.float64, device=x.device)
        grad = torch.empty_like(self.params) if want_grad else None
        check(lib.qsq_cnn_train_step(_p(self.params), _p(self.m), _p(self.v), self.t, float(lr), _p(x), _p(mask),
                                     _p(logq), n, h, w, float(lam), _p(self.prep), _p(grad), _p(loss), _p(ws),
                                     ws.numel() * 8, _stream(stream)))
        return (loss, grad) if want_grad else loss


def layer_forward(prop: Proposer, layer: int, inp: torch.Tensor, stream=None) -> torch.Tensor:
    """One layer on its own: inp float32 (n, h, w, 3) for layer 0, else BF16
    bits as int16 (n, h, w, 32); returns float32 (n, h, w, Co) before rounding."""
    n, h, w, _ = inp.shape
    co = CHANNELS[layer + 1]
    out = torch.empty((n, h, w, co), dtype=torch.float32, device=inp.device)
    check(lib.qsq_cnn_layer_forward(layer, _p(prop.prep), _p(inp.contiguous()), n, h, w, _p(out), _stream(stream)))
    return out


def layer_backward(prop: Proposer, layer: int, inp: torch.Tensor, dy: torch.Tensor, want_dx=True, stream=None):
    """Weight, bias and input gradients of one layer for the output gradient
    dy (BF16 bits as int16, (n, h, w, Co))."""
    n, h, w, _ = inp.shape
    ci, co = CHANNELS[layer], CHANNELS[layer + 1]
    dw = torch.empty(9 * ci * co, dtype=torch.float32, device=inp.device)
    db = torch.empty(co, dtype=torch.float32, device=inp.device)
    dx = torch.empty((n, h, w, ci), dtype=torch.float32, device=inp.device) if (want_dx and layer > 0) else None
    scratch = _bytes_tensor(lib.qsq_cnn_layer_scratch_bytes(n, h, w), inp.device)
    check(lib.qsq_cnn_layer_backward(layer, _p(prop.prep), _p(inp.contiguous()), _p(dy.contiguous()), n, h, w,
                                     _p(dw), _p(db), _p(dx), _p(scratch), scratch.numel() * 8, _stream(stream)))
    return dw, db, dx


def to_bf16_bits(x: torch.Tensor) -> torch.Tensor:
    """Round float32 to BF16 (nearest, ties to even) and return the raw bits as int16."""
    return x.to(torch.bfloat16).view(torch.int16)


def from_bf16_bits(b: torch.Tensor) -> torch.Tensor:
    return b.view(torch.bfloat16).to(torch.float32)


# ---------------------------------------------------------------------------
# features and labels from the maps the tracer makes
# ---------------------------------------------------------------------------

def features(fll_grid: torch.Tensor, fledge: torch.Tensor, bz: torch.Tensor) -> torch.Tensor:
    """(H, W, 3) network input from a coarse map: field-line length / 2,
    log(1 + FLEDGE), and sign(Bz) log(1 + |Bz|) / 3 (all FP32, device)."""
    f0 = torch.nan_to_num(fll_grid.float(), nan=0.0).clamp(0, 16) / 2
    f1 = torch.log1p(torch.nan_to_num(fledge.float(), nan=0.0).clamp(min=0))
    f2 = torch.sign(bz) * torch.log1p(bz.abs()) / 3
    return torch.stack([f0, f1, f2], dim=-1).contiguous()


def refine_labels(keys: torch.Tensor, base_level: int, refine_levels: int, q_base: torch.Tensor):
    """Targets per coarse pixel from a refined map: mask = 1 where the
    FLL-jump rule added samples inside the pixel, logq = log10 of the largest
    Q in the pixel (NaN where not finite)."""
    from .api import hilbert2_d2xy
    side = 1 << base_level
    per = 4 ** refine_levels
    q = torch.div(keys, per, rounding_mode="floor")
    cnt = torch.bincount(q, minlength=side * side)
    x, y = hilbert2_d2xy(base_level, torch.arange(side * side, device=keys.device))
    mask = torch.zeros((side, side), dtype=torch.float32, device=keys.device)
    mask[y.long(), x.long()] = (cnt > 1).float()
    with torch.no_grad():
        logq = torch.log10(q_base.float())
    logq = torch.where(torch.isfinite(logq), logq, torch.full_like(logq, float("nan")))
    return mask, logq


def tiles(img: torch.Tensor, size: int = 64) -> torch.Tensor:
    """Split (H, W, ...) into (H/size * W/size, size, size, ...) tiles, row-major."""
    H, W = img.shape[:2]
    rest = img.shape[2:]
    t = img.reshape(H // size, size, W // size, size, *rest).transpose(1, 2)
    return t.reshape(-1, size, size, *rest).contiguous()


def untile(t: torch.Tensor, H: int, W: int) -> torch.Tensor:
    size = t.shape[1]
    rest = t.shape[3:]
    return t.reshape(H // size, W // size, size, size, *rest).transpose(1, 2).reshape(H, W, *rest)
