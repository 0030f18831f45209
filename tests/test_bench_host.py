"""Host logic of bench.py (no GPU): the one-GPU refusal, the counter summary
and the source-hash gate of the reported HBM traffic."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["requested_gpus"] == 2 and "one GPU" in line["error"]


def _csv(d, rows, counter):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, (name, v) in enumerate(rows):
            w.writerow(dict(Dispatch_Id=k, Kernel_Name=name, Counter_Name=counter, Counter_Value=v))


def test_counter_summary_scales_by_the_copy(tmp_path, monkeypatch):
    """Fetched bytes = FETCH_SIZE KiB x 1024 x (1 GiB / what the copy's FETCH_SIZE
    reads), likewise for writes; every stepping dispatch counts, nothing else."""
    kt = "void qsq::k_trace<float, float, 0, false, false>(qsq::TraceJob)"
    _csv(tmp_path / "f", [(kt, 1000.0), ("other", 5e6), (kt, 3000.0)], "FETCH_SIZE")
    _csv(tmp_path / "w", [(kt, 100.0), ("other", 5e6), (kt, 300.0)], "WRITE_SIZE")
    gib_kib = float(1 << 20)
    _csv(tmp_path / "cf", [("__amd_rocclr_copyBuffer", gib_kib / 2)] * 3, "FETCH_SIZE")
    _csv(tmp_path / "cw", [("__amd_rocclr_copyBuffer", gib_kib)] * 3, "WRITE_SIZE")
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_file", lambda name: str(out) if name == "volume" else "/nonexistent")
    bench.summarize_pmc("volume", str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                        str(tmp_path / "cw"), launch=834)
    t = json.loads(out.read_text())
    assert t["passes"] == 2 and t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert t["write_bytes_per_launch"] == pytest.approx(200.0 * 1024)
    assert t["kernel_sources_sha256"] == bench.kernel_hash()
    assert bench.measured_traffic("volume") == (pytest.approx(t["bytes_per_launch"]), 834)
    assert bench.measured_traffic("map") == (None, None)         # another workload's counters are not used
    # a summary taken on other kernel sources is not reported
    t["kernel_sources_sha256"] = "0" * 64
    out.write_text(json.dumps(t))
    assert bench.measured_traffic("volume") == (None, None)


def test_mismatched_counter_runs_are_rejected(tmp_path, monkeypatch):
    kt = "void qsq::k_trace<float, float, 0, false, false>(qsq::TraceJob)"
    _csv(tmp_path / "f", [(kt, 1.0), (kt, 1.0)], "FETCH_SIZE")
    _csv(tmp_path / "w", [(kt, 1.0)], "WRITE_SIZE")
    _csv(tmp_path / "cf", [("__amd_rocclr_copyBuffer", 1.0)], "FETCH_SIZE")
    _csv(tmp_path / "cw", [("__amd_rocclr_copyBuffer", 1.0)], "WRITE_SIZE")
    monkeypatch.setattr(bench, "traffic_file", lambda name: str(tmp_path / "t.json"))
    with pytest.raises(SystemExit):
        bench.summarize_pmc("volume", str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                            str(tmp_path / "cw"))


def test_tuner_candidates_and_names():
    from paper_1609_00724_amd import _abi as A
    from paper_1609_00724_amd import autotune
    words = autotune.candidates()
    assert len(words) == len(set(words))
    for w in words:
        d = autotune.describe(w)
        assert d["gather"] in ("direct", "lds-cache", "reg-cache", "cell-records")
        if d["gather"] != "direct":              # at most 512 resident lanes per CU
            assert d["lanes_per_cu"] <= 512
    assert autotune.describe(A.launch_word(2, 64, A.GATHER_REGS)) == \
        {"word": 2 | (1 << 4) | (3 << 6), "lanes_per_cu": 512, "workgroup": 64, "gather": "reg-cache",
         "xcd_parts": False}
    assert autotune.describe(A.launch_word(1, 256, A.GATHER_DIRECT, parts=True))["xcd_parts"]
    with pytest.raises(ValueError):
        A.launch_word(2, 96, A.GATHER_REGS)


def test_fixed_error_settings_and_host_info():
    """The sweep covers every tolerance x largest-step pair for CK54 and the
    three Euler step sizes; the host record names the cores and the CPU."""
    ck = bench.sweep_settings(("ck54", "f32"))
    assert len(ck) == len(bench.SWEEP_TOLS) * len(bench.SWEEP_HMAX_CELLS)
    assert {(s.tol, s.hmax_cells) for s in ck} == {(t, c) for t in bench.SWEEP_TOLS for c in bench.SWEEP_HMAX_CELLS}
    eu = bench.sweep_settings(("euler", "f32"))
    assert [s.euler_div for s in eu] == list(bench.SWEEP_EULER_DIVS)
    assert eu[0].oracle_kw(0.5)["h_init"] == pytest.approx(0.1) and eu[0].oracle_kw(0.5)["stepper"] == "euler"
    info = bench.host_info()
    assert info["nproc"] >= 1 and info["cores_allowed"] >= 1
    assert 1 <= bench.host_threads() <= info["cores_allowed"]
    assert bench.FP32_PEAK_TFLOPS == 157.3
    assert bench.FP32_NONPACKED_TFLOPS == pytest.approx(78.6432)


def test_rel_log10_err_masks():
    import numpy as np
    ref = {"q_perp": np.array([10.0, 1e7, np.nan, 100.0]), "status": np.array([1, 1, 1, 2])}
    e = bench.rel_log10_err(np.array([10.0 ** 1.001, 1e7, 5.0, 100.0]), np.array([1, 1, 1, 3]), ref)
    assert e.size == 1 and e[0] == pytest.approx(1e-3)


@pytest.mark.parametrize("dim,r", [(2, 2), (3, 2), (2, 1)])
def test_kept_by_level_follows_the_bisection(dim, r):
    """Levels recovered from keys match a lattice built by bisection: base keys
    q B^r + B^r / 2, then each level the integer midpoints of neighbouring keys
    (the first level also past the last base key)."""
    import numpy as np
    import torch
    levels, blk, nb = dim * r, 1 << (dim * r), 5
    keys = [q * blk + blk // 2 for q in range(nb)]
    level_of = {k: 0 for k in keys}
    for j in range(1, levels + 1):
        cur = sorted(level_of) + ([nb * blk + blk // 2] if j == 1 else [])
        for a, b in zip(cur[:-1], cur[1:]):
            level_of[(a + b) // 2] = j
    ks = np.array(sorted(level_of), np.int64)
    att = np.array([10 * level_of[k] + 1 for k in ks], np.int32)
    rows = bench.kept_by_level(torch.from_numpy(ks), torch.from_numpy(att), levels)
    assert [row["level"] for row in rows] == list(range(levels + 1))
    for row in rows:
        want = [k for k in ks if level_of[k] == row["level"]]
        assert row["lines"] == len(want)
        assert row["attempts"] == len(want) * (10 * row["level"] + 1)
        assert row["max_attempts"] == 10 * row["level"] + 1
