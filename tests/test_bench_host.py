"""Host checks of bench.py's contract pieces (no GPU): more than one GPU is
refused with a message, counter records are used only while the kernel
sources hash to what was profiled, and the peaks are the published ones."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_counter_records_follow_the_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"bytes_per_launch": 123, "valu_insts_per_launch": 456, "sources": bench.kernel_sources_hash()}
    (prof / "traffic.json").write_text(json.dumps({"mac|w": rec, "ntt_inv|w": dict(rec, sources="0" * 16)}))
    h = bench.kernel_sources_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: h)
    assert bench.load_traffic("mac", "w") == 123
    assert bench.load_counters("mac", "w")["valu_insts_per_launch"] == 456
    assert bench.load_counters("ntt_inv", "w") is None  # profiled from other sources
    assert bench.load_traffic("mac", "other") is None


def test_peaks():
    assert bench.HBM_PEAK_GBS == 8000.0
    assert abs(bench.VALU_PEAK_GIPS - 614.4) < 1e-9


def test_alu_peak_derivation():
    """The integer-VALU ceiling of the MAC: 256 CUs x 64 lanes x 2.4 GHz, with
    v_mad_u64_u32 at the full rate, four multiply-adds per modmul-add."""
    assert abs(bench.VALU_LANE_OPS_PEAK - 256 * 64 * 2.4e9) < 1
    assert bench.MAD_RATE_FRAC == 1.0
    assert abs(bench.VALU_LANE_OPS_PEAK * bench.MAD_RATE_FRAC / 4 / 1e9 - 9830.4) < 1e-6


def test_oracle_sample_layers_are_bottleneck_layers():
    import synth
    n = len(synth.WORKLOADS["bottleneck_cnn_b16"]["layers"])
    assert bench.ORACLE_SAMPLE_LAYERS and all(0 <= j < n for j in bench.ORACLE_SAMPLE_LAYERS)
