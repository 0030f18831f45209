"""Helpers for the GPU parity tests: move inputs to the device, run the HIP path
through its binding, and compare with the oracle element by element."""
import numpy as np


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def gpu_field(b, origin, spacing, storage="f32", mode="paper"):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    bt = [torch.from_numpy(np.ascontiguousarray(c)).to(dev) for c in b]
    return q.field_init(*bt, origin, spacing, storage=storage, mode=mode)


def gpu_trace(field, seeds, **kw):
    import paper_1609_00724_amd as q
    torch, dev = torch_dev()
    s = torch.from_numpy(np.ascontiguousarray(seeds.T)).to(dev)
    out = q.trace(field, s, **kw)
    torch.cuda.synchronize()
    r = {k: v.cpu().numpy() for k, v in out.items()}
    r["fp_fwd"] = r["fp_fwd"].T.copy()
    r["fp_bwd"] = r["fp_bwd"].T.copy()
    return r


def parity(g, o, qmax=1e6):
    """Per-seed errors of the GPU result g against the oracle result o.

    Gate set: both exit faces agree and the oracle's Q < qmax (lines past it
    are counted, not gated).  Returns a dict of arrays and counts.
    """
    same = g["status"] == o["status"]
    qo = o["q_perp"]
    fin = np.isfinite(qo) & np.isfinite(g["q_perp"])
    gate = same & fin & (qo < qmax)
    fp = np.maximum(np.abs(g["fp_fwd"] - o["fp_fwd"]).max(1), np.abs(g["fp_bwd"] - o["fp_bwd"]).max(1))
    fll = np.abs(g["fll"] - o["fll"]) / np.maximum(np.abs(o["fll"]), 1e-300)
    fll[(o["fll"] == 0) & (g["fll"] == 0)] = 0.0
    with np.errstate(invalid="ignore", divide="ignore"):
        lq = np.abs(np.log10(g["q_perp"]) - np.log10(qo)) / np.abs(np.log10(qo))
    return dict(gate=gate, fp=fp, fll=fll, lq=lq, status_mismatch=int((~same).sum()),
                nonfinite_both=int((~np.isfinite(qo) & ~np.isfinite(g["q_perp"])).sum()),
                over_qmax=int((same & fin & (qo >= qmax)).sum()))


def worst(p, o, k=3):
    """The k gated lines with the largest log10 Q error, for failure messages."""
    m = np.nonzero(p["gate"])[0]
    if m.size == 0:
        return ""
    order = m[np.argsort(-np.nan_to_num(p["lq"][m]))[:k]]
    return "; ".join(f"#{i} q={o['q_perp'][i]:.4g} lq={p['lq'][i]:.2e} fll={o['fll'][i]:.4g} "
                     f"st={o['status'][i]:#x}" for i in order)


def summary(p):
    m = p["gate"]
    return (f"gated {m.sum()}/{m.size} status-mismatch {p['status_mismatch']} over-qmax {p['over_qmax']} "
            f"fp max {p['fp'][m].max() if m.any() else 0:.2e} fll max {p['fll'][m].max() if m.any() else 0:.2e} "
            f"lq max {np.nanmax(p['lq'][m]) if m.any() else 0:.2e} lq med {np.nanmedian(p['lq'][m]) if m.any() else 0:.2e}")
