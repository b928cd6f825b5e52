"""Host logic of bench.py: the one-GPU guard, the algorithmic-byte model, and
the rule that a committed counter summary is used only for the kernel sources
it was taken on.  No GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_algorithmic_bytes_per_unit():
    # mixed precision: 128 B per particle update, 36 B per half pair, 40 B per fluid cell
    assert bench.alg_bytes("step", 1000, 3000, 0, 4) == 1000 * 128 + 3000 * 36
    assert bench.alg_bytes("step", 1000, 3000, 0, 8) == 1000 * 156 + 3000 * 60
    assert bench.alg_bytes("fluid", 1000, 0, 500, 4) == 1000 * 64 + 500 * 40
    assert bench.alg_bytes("prologue", 10, 99, 99, 4) == 10 * 128
    assert bench.alg_bytes("rebuild", 10, 20, 0, 4) == 10 * 256 + 20 * 36


@pytest.mark.parametrize("cls", ["step", "fluid"])
def test_traffic_summary_needs_matching_sources(tmp_path, monkeypatch, cls):
    with open(os.path.join(ROOT, "profiles", "%s_c1_pmc.json" % cls)) as f:
        d = json.load(f)
    assert set(d["sources"]) <= set(os.listdir(os.path.join(ROOT, "paper_2211_06142_amd", "csrc")))
    cal = d["calibration"]
    # the calibration buffer is far beyond the 256 MB Infinity Cache, and a copy and
    # a read-only pass give the same fetch factor
    assert cal["buffer_bytes"] >= 1 << 30
    assert cal["fetch_factor_copy"] == pytest.approx(cal["fetch_factor_read"], rel=1e-3)
    per = [k["fetch_kib_median"] * 1024 * cal["fetch_factor_copy"] + k["write_kib_median"] * 1024 * cal["write_factor"]
           for k in d["device_kernels"]]
    assert d["traffic_bytes_per_launch"] == pytest.approx(sum(per))
    # a summary taken on other sources is not used
    prof = tmp_path / "profiles"
    prof.mkdir()
    d2 = dict(d, source_hash="0" * 16)
    (prof / ("%s_c1_pmc.json" % cls)).write_text(json.dumps(d2))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda files=None: "f" * 16)
    assert bench.load_traffic(cls, "c1") is None
    d3 = dict(d, source_hash="f" * 16)
    (prof / ("%s_c1_pmc.json" % cls)).write_text(json.dumps(d3))
    assert bench.load_traffic(cls, "c1") == d["traffic_bytes_per_launch"]


def test_uncompressed_paper_sample_at_full_size_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "f2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode == 2
    assert "--f2-protocol" in p.stderr


def test_ensemble_baseline_in_worker_processes_counts_every_sample():
    import synth
    ws = [synth.c3_crop(s, 120, 0.5) for s in range(3)]
    one = bench.cpu_baseline_ensemble(ws, budget_s=60.0, steps=2, workers=1)
    many = bench.cpu_baseline_ensemble(ws, budget_s=60.0, steps=2, workers=2)
    assert one["cores"] == 1 and many["cores"] == 2
    for b in (one, many):
        assert b["kind"] == "oracle" and b["value"] > 0.0
        assert b["sample"].startswith("3 of 3 samples, 2 steps each")
