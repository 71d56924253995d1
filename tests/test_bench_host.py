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


def _grids(fwd_ms, mac_ms, inv_ms):
    kavg = {k: {"ms_per_pass": v, "avg_ms_per_launch": v}
            for k, v in (("batch_fwd", fwd_ms), ("batch_mac", mac_ms), ("batch_inv", inv_ms))}
    alg = {"batch_fwd": {"bytes": 1.7e10, "modmuls": 6.94e9},
           "batch_mac": {"bytes": 2.454e11, "modmul_adds": 2.707e11},
           "batch_inv": {"bytes": 3.414e11, "modmuls": 1.387e11}}
    return kavg, alg


def test_headline_roofline_is_the_longest_grid():
    """The headline roofline follows the longest of the three grids: the
    inverse NTT against 21 full-rate VALU instructions per butterfly, or the
    MAC against four multiply-adds per modmul-add; the MAC's HBM line is its
    algorithmic bytes over its duration; traffic comes from the lookup."""
    kavg, alg = _grids(6.0, 84.0, 119.0)
    form = {"grid": 1, "lds": 3}
    seen = []
    roof, mac, hbm, ntt = bench.headline_rooflines(kavg, alg, form, None, lambda k: seen.append(k) or 7)
    assert roof is ntt["batch_inv"] and roof["bound"] == "alu" and roof["traffic"] == 7
    assert abs(roof["peak"] - 256 * 64 * 2.4 / 21) < 0.1  # G butterflies/s
    assert abs(roof["achieved"] - 1.387e11 / 0.119 / 1e9) < 0.1
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert "measured_mix_ceiling" not in roof
    assert mac["kernel"].startswith("batch_mac_grid_kernel") and abs(mac["peak"] - 9830.4) < 1e-6
    assert abs(mac["achieved"] - 2.707e11 / 0.084 / 1e9) < 0.1
    assert abs(hbm["achieved"] - 2.454e11 / 0.084 / 1e9) < 0.1 and hbm["peak"] == 8000.0
    assert sorted(seen) == ["batch_fwd", "batch_inv", "batch_mac"]
    kavg, alg = _grids(6.0, 130.0, 119.0)
    probes = {"mac_mix": {"rate": 5.6e12}, "intt_mix": {"rate": 1.93e12}, "ntt_mix": {"rate": 1.93e12}}
    roof, mac, hbm, ntt = bench.headline_rooflines(kavg, alg, {"grid": 0, "lds": 0}, probes, lambda k: None)
    assert roof is mac and mac["kernel"] == "batch_mac_kernel" and mac["traffic"] is None
    assert abs(mac["measured_mix_ceiling"]["frac"] - mac["achieved"] / 5600.0) < 1e-3
    assert abs(ntt["batch_inv"]["measured_mix_ceiling"]["rate"] - 1930.0) < 1e-6
