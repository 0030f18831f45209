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
    s = torch.from_numpy(np.ascontiguousarray(seeds)).to(dev)
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


FP_TOL, FLL_TOL, LQ_TOL = 1e-5, 1e-4, 1e-3
# Smallest fraction of gated lines that FP32 stepping may keep inside the
# per-line gates when a test does not measure its own floor: the oracle alone
# keeps 0.988-0.995 of the charge-field lines inside them at tol 1e-5, and
# 0.994-0.997 at tol 1e-4, when its seeds move by 1e-7
# (tests/test_oracle_sensitivity.py); the FP32 tests measure the floor on their
# own seeds with sensitivity_floor().
FP32_MIN_FRAC = 0.98


def perturbed_seeds(seeds, seed, lo=(-1.0, -1.0, 0.0), hi=(1.0, 1.0, 1.0), scale=1e-7):
    """Seeds moved by N(0, scale) in x and y, and in z for interior seeds (a
    seed on the photosphere stays on it), clipped into the box."""
    g = np.random.Generator(np.random.PCG64(seed))
    s = np.array(seeds, dtype=np.float64, copy=True)
    d = g.normal(scale=scale, size=s.shape)
    d[s[:, 2] == lo[2], 2] = 0.0
    return np.clip(s + d, np.array(lo), np.array(hi))


def _in_gates(b, o):
    p = parity(b, o)
    return line_ok(p)[p["gate"]]


def qfp_in_gate(b, o):
    """Lines with two face ends whose q_fp is within the Q gate."""
    m, e = qfp_parity(b, o)
    return np.nan_to_num(e[m], nan=np.inf) <= LQ_TOL


def sensitivity_floor(oracle_mod, fo, seeds, o, kw, draws=3, judge=_in_gates):
    """The oracle's own sensitivity on these seeds: the smallest fraction of
    gated lines that stay inside the per-line gates (or `judge`'s gate) over
    `draws` 1e-7 seed perturbations, less two binomial standard deviations and
    one line.  FP32 stepping perturbs the stage points by about that much, so
    it may move no more lines than this.  Returns (floor, fractions)."""
    fr, n = [], 1
    for k in range(draws):
        b = oracle_mod.trace(fo, perturbed_seeds(seeds, 1000 + k), **kw)
        ok = judge(b, o)
        n = max(int(ok.size), 1)
        fr.append(float(ok.mean()))
    f = min(fr)
    return f - 2.0 * np.sqrt(f * (1.0 - f) / n) - 1.0 / n, fr


def line_ok(p):
    """Per-line gates: footpoints <= 1e-5 domain units, length <= 1e-4 relative,
    relative log10 Q error <= 1e-3."""
    lq = np.nan_to_num(p["lq"], nan=np.inf)
    return (p["fp"] <= FP_TOL) & (p["fll"] <= FLL_TOL) & (lq <= LQ_TOL)


def check_lines(p, o, strict, min_frac=0.998, max_mismatch_frac=0.003):
    """strict (FP64 stepping): every gated line meets the per-line gates.
    Otherwise (FP32 stepping): at least min_frac of the gated lines meet them
    and the median log10 Q error stays <= 1e-5; the rest are counted.  FP32
    stage points differ from FP64 ones by ~1e-7 cell, so a stage that falls on
    the other side of a cell face (where the trilinear gradient jumps) or an
    accept/reject decision at err ~ 1 occasionally sends a line down a
    different, equally valid step sequence."""
    m = p["gate"]
    ok = line_ok(p)
    n_bad = int((~ok[m]).sum())
    msg = (summary(p) + f" | outside per-line gates: {n_bad}/{int(m.sum())} | worst: " + worst(p, o))
    print(msg)
    assert p["status_mismatch"] <= max_mismatch_frac * m.size + (0 if strict else 1), msg
    if strict:
        assert n_bad == 0, msg
    else:
        assert ok[m].mean() >= min_frac, msg
        assert np.nanmedian(p["lq"][m]) <= 1e-5, msg
    return n_bad


def lq_vs(a, ref):
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.abs(np.log10(a) - np.log10(ref)) / np.abs(np.log10(ref))


def check_fp32(p, g, o, ref, min_frac=FP32_MIN_FRAC):
    """FP32 stepping against the FP64 oracle at the same tolerance (o) and
    against the converged FP64 oracle at tolerance 1e-10 (ref).

    FP32 stage arithmetic acts like a ~1e-7 perturbation of the stage points,
    and the discretised method (trilinear gradients jump at cell faces) sends a
    few lines down a different, equally valid step sequence under such
    perturbations (the oracle shows the same lines moving when its own seeds
    move by 1e-7).  So: most lines meet the per-line gates against o, and the
    FP32 error against the converged answer is statistically no larger than the
    FP64 oracle's own error at the same tolerance."""
    m = p["gate"] & np.isfinite(ref["q_perp"]) & (ref["status"] == o["status"])
    ok = line_ok(p)
    e_g = lq_vs(g["q_perp"][m], ref["q_perp"][m])
    e_o = lq_vs(o["q_perp"][m], ref["q_perp"][m])
    msg = (summary(p) + f" | within per-line gates {ok[p['gate']].mean():.4f}"
           f" | vs converged: gpu median {np.nanmedian(e_g):.2e} p90 {np.nanpercentile(e_g, 90):.2e}"
           f" max {np.nanmax(e_g):.2e}; oracle same tol median {np.nanmedian(e_o):.2e}"
           f" p90 {np.nanpercentile(e_o, 90):.2e} max {np.nanmax(e_o):.2e} | worst: " + worst(p, o))
    print(msg)
    assert p["status_mismatch"] <= 0.003 * p["gate"].size + 1, msg
    assert ok[p["gate"]].mean() >= min_frac, msg
    assert np.nanmedian(p["lq"][p["gate"]]) <= 1e-5, msg
    assert np.nanmedian(e_g) <= 1.25 * np.nanmedian(e_o) + 1e-6, msg
    assert np.nanpercentile(e_g, 90) <= 1.5 * np.nanpercentile(e_o, 90) + 1e-6, msg


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


def qfp_parity(g, o, qmax=1e6):
    """Relative log10 error of the exit-face-plane Q (q_fp) per line, on lines
    whose statuses agree, whose two ends are faces (q_fp finite on both sides)
    and whose oracle q_fp < qmax.  Returns (gate mask, errors)."""
    qo, qg = o["q_fp"], g["q_fp"]
    m = (g["status"] == o["status"]) & np.isfinite(qo) & np.isfinite(qg) & (qo < qmax)
    return m, lq_vs(qg, qo)
