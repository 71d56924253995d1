"""Benchmark of the HE convolution hot path on one MI355X.

A step is one pass of the whole hot path -- for every layer solve, forward
NTT of its input ciphertexts, channel-block MAC against NTT-preprocessed
weights, inverse NTT of the results -- over one batch of seeded synthetic
ciphertexts already resident in HBM.  The weights are NTT-preprocessed once
before the timed region (the paper's offline step); its time is reported
separately.

Headline workload: the bottleneck residual CNN (53 convolutions at 224
input) for 16 images, N=8192, three 60-bit primes, all 848 layer solves
resident at once (about 229 GiB), in its batched form (one hipGraph launch
per pass), with the plain per-layer path (one he_conv_layer call per layer
solve) timed beside it on the same buffers.

Prints one JSON line.  `value` = ct x pt MACs per second of the batched
pass; the line also carries layers/s, per-pass p50/p99 of both forms, the
rooflines of the dominant kernel (measured with HIP events on its launch
stream), the CPU oracle timed on a bounded sample of the same workload
(which also checks those layer solves word for word), and the other
workloads as secondary fields.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from synth import Stream  # noqa: E402

METRIC = "HE conv ct×pt MACs/s and layers/s (bit-exact), batched vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0
# The paper's own figures, quoted as context (other hardware, whole-model
# aggregates that include the protocol around the convolutions): they are
# not this bench's metric, so vs_baseline stays null.
PAPER_CONTEXT = {
    "conv_online_all_squeezenet_convs_s": {"gpu": 2.26, "cpu": 3.09,
                                           "source": "Evaluation, Linear Layers (convolution table)"},
    "conv_offline_ntt_preprocessing_s": {"gpu": 0.72, "cpu": 0.76,
                                         "source": "Evaluation, Linear Layers (convolution table)"},
    "e2e_secure_inference_squeezenet_s": {"gpu": 2.8, "cpu": 3.6, "source": "Abstract; Evaluation, E2E Evaluation"},
    "hardware": "NVIDIA RTX A6000 (HE evaluator on GPU) with an Intel Xeon Gold 6338, 16 threads (Evaluation)",
    "model": "SqueezeNet, 37-bit fixed point",
    "note": "context, not the target: the paper times one secure inference end to end (client encryption, "
            "network and 2PC steps included); this bench times the server's HE convolution kernels on "
            "resident ciphertexts (the fire-module CNN field is the closest workload)",
}
VALU_PEAK_GIPS = 256 * 2.4  # G full-rate wave64 VALU instructions/s: one per CU per cycle, 256 CUs at 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9  # full-rate 32-bit lane operations/s: 256 CUs x 64 lanes x 2.4 GHz
MAD_RATE_FRAC = 1.0  # v_mad_u64_u32 issues at the full rate on gfx950 (the probe's mad_u64_u32 field: 0.975)
# VALU instructions of one butterfly in the compiled transforms (the
# probes' butterfly loops: 672 VALU instructions per 32 butterflies, both)
BFLY_VALU_INSTS = {"batch_inv": 21, "batch_fwd": 21}
SCHEDULE_NAMES = {1: "one chain", 2: "two chains", 3: "pipelined in 4 groups", 4: "pipelined in 8 groups"}
# layer solves (image 0) the oracle recomputes in the CPU-baseline leg
ORACLE_SAMPLE_LAYERS = [0, 2, 3, 12, 14, 16, 25, 26, 29, 44, 45, 48]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed batched passes of the headline workload")
    ap.add_argument("--warmup", type=int, default=3, help="untimed batched passes first")
    ap.add_argument("--plain-steps", type=int, default=20, help="timed passes of the plain and per-layer forms")
    ap.add_argument("--kernel-reps", type=int, default=5, help="instrumented passes for the per-grid durations")
    ap.add_argument("--schedule", type=int, default=1, choices=[1, 2, 3, 4],
                    help="schedule of the headline batch (1 one chain, 2 two chains, 3/4 pipelined in 4/8 groups)")
    ap.add_argument("--single-steps", type=int, default=200, help="timed steps of the 64->64 single layer")
    ap.add_argument("--single-warmup", type=int, default=500)
    ap.add_argument("--workload", default="conv64_56x56", choices=["conv4_16x16", "conv64_56x56"],
                    help="workload of the single-layer section")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-headline", action="store_true", help="skip the batch-16 bottleneck CNN (about 230 GiB)")
    ap.add_argument("--no-single", action="store_true", help="skip the single-layer section")
    ap.add_argument("--no-probes", action="store_true", help="skip the integer-VALU rate probes")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched fire-module CNN section")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--no-client", action="store_true", help="skip the client-side encrypt/decrypt section")
    ap.add_argument("--no-rotation", action="store_true", help="skip the ciphertext rotation section")
    ap.add_argument("--no-zp", action="store_true", help="skip the Z_P linear-kernel section")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner runs (single layer and fire-module batch)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-sweep", type=float, nargs="*", default=[1000.0, 2000.0, 4000.0, 8000.0, 16000.0],
                    help="offered rates (req/s) of the open-loop sweep")
    ap.add_argument("--serve-sweep-requests", type=int, default=1500)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM counter scaling)")
    return ap.parse_args()


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_11586_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_counters(kernel: str, workload: str):
    """The committed rocprofv3 counter record of a kernel (HBM bytes per
    launch, VALU instructions per launch), only while the kernel sources
    still hash to what was profiled."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}|{workload}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("sources") != kernel_sources_hash():
        return None
    return rec


def load_traffic(kernel: str, workload: str):
    """HBM traffic per launch from the committed counter record, or None."""
    rec = load_counters(kernel, workload)
    return rec.get("bytes_per_launch") if rec else None


def run_single_layer(torch, heconv, args):
    """One layer solve repeated (he_conv_layer): by default the 3x3 conv
    64->64 on a 56x56 tensor, N=8192, three 60-bit primes, one image (32
    input / 128 output ciphertexts, 2048 ct x pt MACs), with the per-kernel
    breakdown, the MAC's HBM roofline warm and with the caches flushed, the
    autotuner's pick and the oracle's CPU rate on the same layer."""
    cfg = synth.WORKLOADS[args.workload]
    shape = cfg["layers"][0]
    N, L, bits, B = cfg["N"], cfg["L"], cfg["bits"], cfg["batch"]
    ctx = heconv.Context(N, heconv.gen_primes(N, bits, L), 2 ** synth.T_BITS)
    d = ctx.plan(shape, batch=B)
    sz = ctx.sizes(d)
    C, H, W, M, kh, kw, stride, pad = shape
    ct_words = 2 * L * N
    n_in, n_out = B * sz.in_cts, B * sz.out_cts
    macs = B * M * sz.CB * sz.S  # ct x pt MACs per layer solve

    # seeded inputs: ciphertext words uniform mod q_l, integer weights
    seed = cfg["seed"]
    x_host = synth.uniform_mod(Stream(seed, synth.UNIFORM), (n_in * 2, L, N), ctx.q)
    K_host = Stream(seed, synth.WEIGHT).ints(M * C * kh * kw, *cfg["w_range"]).reshape(M, C, kh, kw)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).cuda()
    x_pristine = dev(x_host)
    K_dev = dev(K_host)
    wntt = torch.empty(sz.w_words, dtype=torch.int64, device="cuda")
    d_in = x_pristine.clone()
    d_out = torch.empty(n_out * ct_words, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    # offline: NTT preprocessing of the weights
    ctx.encode_weights(d, K_dev, wntt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ctx.encode_weights(d, K_dev, wntt)
    e1.record()
    torch.cuda.synchronize()
    encode_ms = e0.elapsed_time(e1) / 5

    # correctness sample: one layer on the pristine input, kept for the oracle
    ctx.conv_layer(d, B, d_in, wntt, d_out)
    torch.cuda.synchronize()
    gpu_out = d_out.cpu().numpy().view(np.uint64).copy()

    # timed region: K layer solves (the input buffer is re-transformed each
    # step; the kernels' work does not depend on the values)
    for _ in range(args.single_warmup):
        ctx.conv_layer(d, B, d_in, wntt, d_out)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.single_steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.single_steps):
        ctx.conv_layer(d, B, d_in, wntt, d_out)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.single_steps)])
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.single_steps

    # per-kernel breakdown: the same three launches, events between them
    reps = max(20, args.single_steps // 4)
    ks = {"ntt_fwd": [], "mac": [], "ntt_inv": []}
    for _ in range(reps):
        a, b, c, e = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        a.record(stream)
        ctx.ntt_fwd(d_in, n_in * 2)
        b.record(stream)
        ctx.conv_ntt_mac(d, B, d_in, wntt, d_out)
        c.record(stream)
        ctx.ntt_inv(d_out, n_out * 2)
        e.record(stream)
        ks["ntt_fwd"].append((a, b))
        ks["mac"].append((b, c))
        ks["ntt_inv"].append((c, e))
    torch.cuda.synchronize()
    kavg = {k: float(np.mean([p.elapsed_time(q) for p, q in v])) * 1e3 for k, v in ks.items()}  # us

    # the MAC once more with the device caches cold: 512 MiB of other data
    # are read between launches, more than the 256 MB Infinity Cache, so
    # every weight word comes from HBM (repeated launches above re-read the
    # same 192 MiB of weights, part of which the Infinity Cache can hold).
    # The flush only reads, so it leaves no dirty lines to write back.
    flush = torch.ones(64 << 20, dtype=torch.int64, device="cuda")
    flush.sum()  # one untimed flush and launch first: the clocks after the host sync above
    ctx.conv_ntt_mac(d, B, d_in, wntt, d_out)
    cold = []
    for _ in range(30):
        flush.sum()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.conv_ntt_mac(d, B, d_in, wntt, d_out)
        b.record(stream)
        cold.append((a, b))
    torch.cuda.synchronize()
    cold_us = np.array([p.elapsed_time(q) for p, q in cold]) * 1e3
    mac_cold_us, mac_cold_p50 = float(np.mean(cold_us)), float(np.median(cold_us))
    del flush

    limb_polys_in, limb_polys_out = n_in * 2 * L, n_out * 2 * L
    kbytes = {  # algorithmic bytes per launch
        "ntt_fwd": limb_polys_in * 16 * N,
        "mac": (sz.w_words + (n_in + n_out) * ct_words) * 8,
        "ntt_inv": limb_polys_out * 16 * N,
    }
    logN = N.bit_length() - 1
    kmodmul = {"ntt_fwd": limb_polys_in * (N // 2) * logN, "mac": macs * ct_words,
               "ntt_inv": limb_polys_out * (N // 2) * logN}
    kernels = {k: {"avg_us": round(kavg[k], 3), "alg_bytes": kbytes[k], "modmuls": kmodmul[k],
                   "GBps": round(kbytes[k] / (kavg[k] * 1e-6) / 1e9, 1),
                   "Gmodmul_per_s": round(kmodmul[k] / (kavg[k] * 1e-6) / 1e9, 1)} for k in ks}
    dom = max(kavg, key=kavg.get)
    wl_name = cfg["name"]
    achieved = kbytes[dom] / (kavg[dom] * 1e-6) / 1e9
    traffic = load_traffic(dom, wl_name)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    # integer-VALU side: wave64 VALU instructions per launch from the SQ
    # counters of the committed profile, over this run's live average
    # duration, against one full-rate wave64 VALU instruction per CU per
    # cycle (256 CUs x 2.4 GHz).  The clock under a long integer load runs
    # below 2.4 GHz, so the VALU's busy fraction of the cycles actually run
    # is higher than this.
    for k in ks:
        rec = load_counters(k, wl_name)
        if rec and rec.get("valu_insts_per_launch"):
            rate = rec["valu_insts_per_launch"] / (kavg[k] * 1e-6) / 1e9
            kernels[k]["valu"] = {"insts_per_launch": rec["valu_insts_per_launch"],
                                  "achieved": round(rate, 1), "peak": VALU_PEAK_GIPS, "unit": "G wave64 instr/s",
                                  "issue_frac": round(rate / VALU_PEAK_GIPS, 3)}
    valu_k = "ntt_inv"
    roofline_valu = None
    if "valu" in kernels[valu_k]:
        v = kernels[valu_k]["valu"]
        roofline_valu = {"bound": "alu", "kernel": valu_k, "achieved": v["achieved"], "peak": VALU_PEAK_GIPS,
                         "unit": v["unit"], "frac": v["issue_frac"],
                         "note": "each VALU instruction counted once, against 2.4 GHz; the clock under "
                                 "sustained integer load is lower, so the busy fraction is higher"}

    # the autotuner on the same layer, after the timed region: it starts from
    # the context's defaults (which time the headline above) and reports its
    # pick; the output under the pick is checked word for word
    autotuned = None
    if not args.no_autotune:
        from paper_2506_11586_amd import autotune
        tr = autotune.tune_layer(torch, ctx, d, B, d_in, wntt, d_out, reps=20, warm_s=0.05, apply=False)
        default_tuning = ctx.get_tuning().as_dict()
        ctx.set_tuning(**tr.tuning)
        d_in.copy_(x_pristine)
        ctx.conv_layer(d, B, d_in, wntt, d_out)
        torch.cuda.synchronize()
        same = bool(np.array_equal(d_out.cpu().numpy().view(np.uint64), gpu_out))
        ctx.set_tuning(**default_tuning)
        autotuned = {"tuning": {k: v for k, v in tr.tuning.items() if default_tuning[k] != v},
                     "default_ms": tr.default_ms, "tuned_ms": tr.ms, "candidates_timed": len(tr.evaluations),
                     "output_equals_default": same,
                     "note": "median of 20 launches per candidate; coordinate descent from the defaults"}

    res = {
        "workload": wl_name, "steps": args.single_steps, "warmup": args.single_warmup,
        "value": macs / (ms_per_step * 1e-3), "unit": "ct×pt MACs/s", "ms_per_step": ms_per_step,
        "config": {"conv": dict(C=C, H=H, W=W, M=M, k=kh, stride=stride, pad=pad),
                   "N": N, "L": L, "q_bits": bits, "t": f"2^{synth.T_BITS}", "batch": B,
                   "packing": dict(Cw=d.Cw, Hw=d.Hw, Ww=d.Ww, CB=sz.CB, S=sz.S),
                   "in_cts": n_in, "out_cts": n_out, "ctpt_macs_per_layer": macs, "path": "plain per-layer"},
        "layers_per_s": 1e3 / ms_per_step * B,
        "p50_ms": float(np.percentile(per_step, 50)), "p99_ms": float(np.percentile(per_step, 99)),
        "wall_s": wall,
        "offline_encode_ms": encode_ms,
        "kernels": kernels,
        "mac_cold_cache": {"avg_us": round(mac_cold_us, 3), "p50_us": round(mac_cold_p50, 3),
                           "min_us": round(float(cold_us.min()), 3), "max_us": round(float(cold_us.max()), 3),
                           "GBps": round(kbytes["mac"] / (mac_cold_us * 1e-6) / 1e9, 1),
                           "frac": round(kbytes["mac"] / (mac_cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                           "p50_GBps": round(kbytes["mac"] / (mac_cold_p50 * 1e-6) / 1e9, 1),
                           "note": "30 launches after one untimed one, 512 MiB read before each (Infinity Cache 256 MB); "
                                   "GBps and frac from the mean"},
        "roofline": roofline,
    }
    if roofline_valu is not None:
        res["roofline_valu"] = roofline_valu
    if autotuned is not None:
        res["autotuned"] = autotuned
    if not args.no_cpu_baseline:
        res["cpu_baseline"], res["bit_exact"] = cpu_baseline(args, cfg, ctx, d, sz, x_host, K_host, gpu_out)
    ctx.close()
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the HE convolution path runs on a single MI355X here "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2506_11586_amd import heconv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    probes = None if args.no_probes else run_probes(torch, heconv)
    result, pending = {}, None
    if not args.no_headline:
        result, pending = run_bottleneck_main(torch, heconv, args, probes)
        torch.cuda.empty_cache()
    if probes is not None:
        result["valu_probes"] = probes
    result["paper_context"] = PAPER_CONTEXT
    if not args.no_single:
        result["single_layer"] = run_single_layer(torch, heconv, args)
    if not args.no_batched:
        result["batched"] = run_batched(torch, heconv, tune=not args.no_autotune, cpu_args=args)
        result["batched_polyphase"] = run_batched(torch, heconv, polyphase=True)
        result["stem_polyphase_b16"] = run_stem_polyphase(torch, heconv)
    if not args.no_serving:
        result["serving"] = run_serving(torch, heconv, args)
    if not args.no_client:
        result["client"] = run_client(torch, heconv)
    if not args.no_rotation:
        result["rotation"] = run_rotation(torch, heconv)
    if not args.no_zp:
        result["zp_fc"] = run_zp(torch, heconv)
    if args.copy_probe:
        src = torch.ones(32 << 20, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_probe_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}
    if pending is not None and not args.no_cpu_baseline:
        result["cpu_baseline"], chk = cpu_baseline_bottleneck(args, pending)
        result["oracle_checked_layer_solves"] = chk
        result["bit_exact"] = bool(result["batched_equals_plain_all_words"] and chk["words_equal"])
    print(json.dumps(result), flush=True)


def _timed(torch, fn, reps, warm=2, warm_s=0.1):
    """Average ms of fn over reps calls, after at least `warm` calls and
    warm_s seconds of calls: the GPU raises its clocks only under sustained
    load, and a few milliseconds of warm-up time it while still ramping."""
    t0, k = time.perf_counter(), 0
    while k < warm or time.perf_counter() - t0 < warm_s:
        fn()
        torch.cuda.synchronize()
        k += 1
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def run_batched(torch, heconv, polyphase=False, tune=False, cpu_args=None):
    """Fire-module CNN (26 convs at 224 input, B=1, N=8192, L=3): the 26 layer
    solves one after another through he_conv_layer (plain) vs one batch (two
    chains of three grids, one hipGraph launch).  Outputs compared word for
    word.  With polyphase, every strided layer for which the planner's
    objective prefers it (here the first layer) runs as its polyphase
    stride-1 layer (the same outputs, fewer output ciphertexts)."""
    cfg = synth.WORKLOADS["fire_cnn"]
    N, L, bits = cfg["N"], cfg["L"], cfg["bits"]
    ctx = heconv.Context(N, heconv.gen_primes(N, bits, L), 2 ** synth.T_BITS)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).cuda()
    jobs, pristine, macs, out_cts, mac_bytes = [], [], 0, 0, 0
    host = []  # per layer: the input words and kernel the oracle leg takes
    for i, shape in enumerate(cfg["layers"]):
        C, H, W, M, kh, kw, stride, pad = shape
        K = Stream(cfg["seed"] * 1000 + i, synth.WEIGHT).ints(M * C * kh * kw, *cfg["w_range"])
        Kd = dev(K)
        if polyphase and heconv.polyphase_advised(N, L, shape, 1):
            shape = heconv.polyphase_shape(shape)
            Kp = torch.empty(shape[3] * shape[0] * shape[4] * shape[5], dtype=torch.int64, device="cuda")
            heconv.polyphase_weights((C, H, W, M, kh, kw, stride, pad), Kd, Kp)
            Kd = Kp
            C, H, W, M, kh, kw, stride, pad = shape
        d = ctx.plan(shape)
        s = ctx.sizes(d)
        wntt = torch.empty(s.w_words, dtype=torch.int64, device="cuda")
        ctx.encode_weights(d, Kd, wntt)
        out_cts += s.out_cts
        mac_bytes += s.w_words * 8 + (s.in_cts + s.out_cts) * 2 * L * N * 8
        x = synth.uniform_mod(Stream(cfg["seed"] * 1000 + i, synth.UNIFORM), (s.in_cts * 2, L, N), ctx.q)
        pristine.append(dev(x))
        if not polyphase:
            host.append((x, K.reshape(M, C, kh, kw), (d.Cw, d.Hw, d.Ww)))
        jobs.append((d, 1, pristine[-1].clone(), wntt, torch.empty(s.out_cts * 2 * L * N, dtype=torch.int64,
                                                                         device="cuda")))
        macs += M * s.CB * s.S
    plain_out = [torch.empty_like(j[4]) for j in jobs]
    # correctness: batch outputs == plain outputs on the same inputs
    for j, p, o in zip(jobs, pristine, plain_out):
        ctx.conv_layer(j[0], 1, p.clone(), j[3], o)
    b = heconv.Batch(ctx, jobs, schedule=heconv.SCHED_TWO_CHAINS)
    b.launch(graph=True)
    b.status()
    exact = all(torch.equal(j[4], o) for j, o in zip(jobs, plain_out))

    def plain():
        for j in jobs:
            ctx.conv_layer(j[0], 1, j[2], j[3], j[4])

    stream = torch.cuda.current_stream()
    st_plain = _passes(torch, plain, 40, 2, stream)
    st_batch = _passes(torch, lambda: b.launch(graph=True), 40, 2, stream)
    t_plain, t_batch = st_plain["mean_ms"], st_batch["mean_ms"]
    n = len(jobs)
    fixed_mac_form = b.mac_form
    b.close()
    # per-grid durations of the same jobs as one chain (HIP events around
    # each grid, eager): the MAC grid's algorithmic bytes over its duration
    b1 = heconv.Batch(ctx, jobs, schedule=heconv.SCHED_ONE_CHAIN)
    g1 = [b1.launch_timed(stream)[0] for _ in range(4)][1:]
    b1.close()
    fwd_ms, mac_ms, inv_ms = (float(np.mean([r[p] for r in g1])) for p in range(3))
    one_chain = {"fwd_ms": round(fwd_ms, 4), "mac_ms": round(mac_ms, 4), "inv_ms": round(inv_ms, 4),
                 "mac_alg_bytes": mac_bytes, "mac_GBps": round(mac_bytes / (mac_ms * 1e-3) / 1e9, 1),
                 "mac_hbm_frac": round(mac_bytes / (mac_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "note": "the 26 jobs as one chain, eager, HIP events around each grid (mean of 3)"}
    tuned = None
    if tune:
        # the autotuner over schedule x MAC tile x NTT grouping, then the
        # picked batch timed as above and checked against the plain outputs
        from paper_2506_11586_amd import autotune
        tr = autotune.tune_batch(torch, ctx, jobs, reps=5, warm_s=0.05)
        for j, p in zip(jobs, pristine):
            j[2].copy_(p)
        bt = heconv.Batch(ctx, jobs, schedule=tr.schedule)
        bt.launch(graph=True)
        bt.status()
        same = all(torch.equal(j[4], o) for j, o in zip(jobs, plain_out))
        st_tuned = _passes(torch, lambda: bt.launch(graph=True), 40, 2, stream)
        t_tuned = st_tuned["mean_ms"]
        tuned_mac_form = bt.mac_form
        bt.close()
        tuned = {"schedule": SCHEDULE_NAMES[tr.schedule], "mac_form": tuned_mac_form,
                 "tuning": {k: tr.tuning[k] for k in ("mac_mt", "mac_rt", "mac_lds", "mac_tiles", "mac_grid", "ntt_loge_small", "ntt_loge_large")},
                 "batched_ms": t_tuned, "batched_layers_per_s": n / t_tuned * 1e3,
                 "batched_p50_ms": st_tuned["p50_ms"], "batched_p99_ms": st_tuned["p99_ms"],
                 "candidates_timed": len(tr.evaluations), "bit_exact_vs_plain": bool(same)}
    cpu = None
    if cpu_args is not None and not cpu_args.no_cpu_baseline and not polyphase:
        cpu = cpu_baseline_fire(cpu_args, cfg, ctx.q, host, plain_out)
    del plain_out
    ctx.close()
    if polyphase:
        return {"workload": cfg["name"] + ", strided layers in polyphase form where the planner prefers it",
                "out_cts_per_pass": out_cts,
                "ctpt_macs_per_pass": macs, "plain_ms": t_plain, "batched_ms": t_batch,
                "plain_layers_per_s": n / t_plain * 1e3, "batched_layers_per_s": n / t_batch * 1e3,
                "bit_exact_vs_plain": bool(exact)}
    # the batched form is the autotuner's pick when it ran (schedule, MAC
    # tile and NTT grouping chosen by measurement), else the fixed form
    fixed = {"batched_ms": t_batch, "batched_layers_per_s": n / t_batch * 1e3,
             "batched_p50_ms": st_batch["p50_ms"], "batched_p99_ms": st_batch["p99_ms"],
             "form": "two chains of three grids, tiles by shape, one hipGraph", "mac_form": fixed_mac_form,
             "bit_exact_vs_plain": bool(exact)}
    if tuned is not None:
        mt, rt = tuned["tuning"]["mac_mt"], tuned["tuning"]["mac_rt"]
        tile = "by shape" if mt == 0 else f"{mt}x{rt}"
        p50, p99 = tuned["batched_p50_ms"], tuned["batched_p99_ms"]
        t_b, ok, form = tuned["batched_ms"], tuned["bit_exact_vs_plain"] and exact, (
            f"autotuned: {tuned['schedule']} of three grids (forward NTTs, MAC tiles {tile}, inverse NTTs), "
            "one hipGraph")
    else:
        p50, p99 = st_batch["p50_ms"], st_batch["p99_ms"]
        t_b, ok, form = t_batch, exact, fixed["form"]
    return {"workload": cfg["name"], "layers": n, "ctpt_macs_per_pass": macs, "out_cts_per_pass": out_cts,
            "plain_ms": t_plain, "batched_ms": t_b,
            "plain_p50_ms": st_plain["p50_ms"], "plain_p99_ms": st_plain["p99_ms"],
            "batched_p50_ms": p50, "batched_p99_ms": p99, "passes_timed": 40,
            "plain_layers_per_s": n / t_plain * 1e3, "batched_layers_per_s": n / t_b * 1e3,
            "plain_ctpt_macs_per_s": macs / t_plain * 1e3, "batched_ctpt_macs_per_s": macs / t_b * 1e3,
            "speedup": t_plain / t_b, "bit_exact_vs_plain": bool(ok), "batched_form": form,
            "one_chain_grids": one_chain, "fixed_form": fixed, **({"autotuned": tuned} if tuned is not None else {}),
            **({"cpu_baseline": cpu[0], "oracle_checked_layer_solves": cpu[1]} if cpu is not None else {})}


def run_stem_polyphase(torch, heconv):
    """The bottleneck CNN's stem (7x7 stride 2, 3 -> 64 at 224, batch 16) as
    he_conv_layer on the strided layer (stride 1 + subsample) vs on its
    polyphase stride-1 layer (12 phase channels, 4x4 kernel); inputs uniform
    mod q_l (the kernels' work does not depend on the values)."""
    cfg = synth.WORKLOADS["bottleneck_cnn_b16"]
    N, L, bits, B = cfg["N"], cfg["L"], cfg["bits"], cfg["batch"]
    ctx = heconv.Context(N, heconv.gen_primes(N, bits, L), 2 ** synth.T_BITS)
    shape = cfg["layers"][0]
    assert shape[6] == 2 and shape[4] == 7
    gen = torch.Generator(device="cuda")
    gen.manual_seed(17)
    qx = torch.tensor(ctx.q, dtype=torch.int64, device="cuda").view(1, L, 1)
    res = {"workload": f"stem {shape}, batch {B}"}
    for form in ("strided", "polyphase"):
        lshape = heconv.polyphase_shape(shape) if form == "polyphase" else shape
        d = ctx.plan(lshape, batch=B)
        s = ctx.sizes(d)
        C, H, W, M, kh, kw = lshape[:6]
        K = torch.randint(-2 ** 12, 2 ** 12, (M * C * kh * kw,), generator=gen, dtype=torch.int64, device="cuda")
        wntt = torch.empty(s.w_words, dtype=torch.int64, device="cuda")
        ctx.encode_weights(d, K, wntt)
        x = (torch.randint(0, 2 ** 62, (B * s.in_cts * 2, L, N), generator=gen, dtype=torch.int64,
                           device="cuda") % qx).reshape(-1)
        out = torch.empty(B * s.out_cts * 2 * L * N, dtype=torch.int64, device="cuda")
        ms = _timed(torch, lambda: ctx.conv_layer(d, B, x, wntt, out), 5)
        res[form] = {"ms": ms, "in_cts_per_image": s.in_cts, "out_cts_per_image": s.out_cts,
                     "packing": [d.Cw, d.Hw, d.Ww]}
        del x, out, wntt
    res["speedup"] = res["strided"]["ms"] / res["polyphase"]["ms"]
    ctx.close()
    return res


def run_probes(torch, heconv):
    """Integer-VALU rates measured by the library's probes (heconv_probe.h):
    the v_mad_u64_u32 / v_mul_hi_u32 / v_mul_lo_u32 / v_add_u32 lane rates
    and the ceilings of the MAC's and the transforms' own instruction mixes
    (operands in registers, no memory traffic).  Best of three runs each."""
    ctx = heconv.Context(8192, heconv.gen_primes(8192, 60, 3))
    spec = [("mad_u64_u32", heconv.PROBE_MAD_U64_U32, 3000, "lane ops/s"),
            ("mul_hi_u32", heconv.PROBE_MUL_HI_U32, 3000, "lane ops/s"),
            ("mul_lo_u32", heconv.PROBE_MUL_LO_U32, 3000, "lane ops/s"),
            ("add_u32", heconv.PROBE_ADD_U32, 3000, "lane ops/s"),
            ("mac_mix", heconv.PROBE_MAC_MIX, 300, "modmul-adds/s (6x4 tile, three accumulators, carry per 8 blocks)"),
            ("intt_mix", heconv.PROBE_INTT_MIX, 900, "butterflies/s"),
            ("ntt_mix", heconv.PROBE_NTT_MIX, 900, "butterflies/s")]
    out = {}
    for name, which, iters, unit in spec:
        out[name] = {"rate": max(ctx.probe_valu(which, iters) for _ in range(3)), "unit": unit}
    full = VALU_LANE_OPS_PEAK
    for k in ("mad_u64_u32", "mul_hi_u32", "mul_lo_u32", "add_u32"):
        out[k]["frac_of_full_rate"] = round(out[k]["rate"] / full, 3)
    ctx.close()
    return out


def run_bottleneck_main(torch, heconv, args, probes):
    """The headline: the bottleneck residual CNN (53 convs at 224 input, 16
    images, N=8192, L=3 60-bit primes), every layer solve of all 16 images
    resident at once (NTT-form weights about 62 GiB, inputs 8 GiB, outputs
    about 159 GiB).

      batched:  the 53 layer jobs of 16 images each in one batch, replayed as
                one hipGraph launch per pass (the step of this bench);
      plain:    the plain per-layer path, one he_conv_layer call per layer
                solve (one image, one layer): 848 calls per pass;
      per-layer x16: one he_conv_layer call of 16 images per layer.

    All three use the same packing (planned for 16 images) and the same
    ciphertexts.  Batched and plain outputs are compared word for word on
    the device for every layer; the oracle checks sampled layer solves in
    the CPU-baseline leg.  Input words are drawn on the device (torch's
    seeded generator, uniform mod q_l)."""
    cfg = synth.WORKLOADS["bottleneck_cnn_b16"]
    N, L, bits, B = cfg["N"], cfg["L"], cfg["bits"], cfg["batch"]
    ctx = heconv.Context(N, heconv.gen_primes(N, bits, L), 2 ** synth.T_BITS)
    qd = torch.tensor(ctx.q, dtype=torch.int64, device="cuda").view(1, L, 1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).cuda()
    ct_words = 2 * L * N
    descs, sizes, Ks, wntts, ins, outs = [], [], [], [], [], []
    macs = 0
    t_enc = 0.0
    for i, shape in enumerate(cfg["layers"]):
        C, H, W, M, kh, kw, stride, pad = shape
        d = ctx.plan(shape, batch=B)
        s = ctx.sizes(d)
        K = Stream(cfg["seed"] * 1000 + i, synth.WEIGHT).ints(M * C * kh * kw, *cfg["w_range"]).reshape(M, C, kh, kw)
        w = torch.empty(s.w_words, dtype=torch.int64, device="cuda")
        Kd = dev(K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.encode_weights(d, Kd, w)
        torch.cuda.synchronize()
        t_enc += time.perf_counter() - t0
        del Kd
        descs.append(d), sizes.append(s), Ks.append(K), wntts.append(w)
        ins.append(torch.empty(B * s.in_cts * ct_words, dtype=torch.int64, device="cuda"))
        outs.append(torch.empty(B * s.out_cts * ct_words, dtype=torch.int64, device="cuda"))
        macs += B * M * s.CB * s.S
    n_solves = len(descs) * B
    gen = torch.Generator(device="cuda")

    def fill_input(j):
        gen.manual_seed(4000 + j)
        v = ins[j].view(-1, L, N)
        for r0 in range(0, v.shape[0], 4096):
            r1 = min(v.shape[0], r0 + 4096)
            v[r0:r1] = torch.randint(0, 2 ** 62, (r1 - r0, L, N), generator=gen, device="cuda") % qd

    for j in range(len(ins)):
        fill_input(j)
    # layer solves the oracle checks in the CPU-baseline leg: image 0 of
    # these layers, input read back before the first pass
    sample_layers = [j for j in ORACLE_SAMPLE_LAYERS if j < len(descs)]
    samples = {j: ins[j][:sizes[j].in_cts * ct_words].cpu().numpy().view(np.uint64).copy() for j in sample_layers}

    sched = heconv.SCHED_ONE_CHAIN if args.schedule == 1 else heconv.SCHED_TWO_CHAINS
    jobs = [(d, B, x, w, o) for d, x, w, o in zip(descs, ins, wntts, outs)]
    bt = heconv.Batch(ctx, jobs, schedule=sched)
    bt.launch(graph=True)
    bt.status()
    sample_out = {j: outs[j][:sizes[j].out_cts * ct_words].cpu().numpy().view(np.uint64).copy()
                  for j in sample_layers}

    # every output word of the batched pass against the plain per-layer path
    # (one he_conv_layer call per image), layer by layer into a scratch buffer
    scratch = torch.empty(max(o.numel() for o in outs), dtype=torch.int64, device="cuda")
    equal_layers = 0
    for j, (d, s) in enumerate(zip(descs, sizes)):
        fill_input(j)
        iw, ow = s.in_cts * ct_words, s.out_cts * ct_words
        for b in range(B):
            ctx.conv_layer(d, 1, ins[j][b * iw:(b + 1) * iw], wntts[j], scratch[b * ow:(b + 1) * ow])
        equal_layers += bool(torch.equal(scratch[:B * ow], outs[j]))
    del scratch
    torch.cuda.synchronize()

    def plain_pass():
        for d, s, x, w, o in zip(descs, sizes, ins, wntts, outs):
            iw, ow = s.in_cts * ct_words, s.out_cts * ct_words
            for b in range(B):
                ctx.conv_layer(d, 1, x[b * iw:(b + 1) * iw], w, o[b * ow:(b + 1) * ow])

    def per_layer_pass():
        for d, x, w, o in zip(descs, ins, wntts, outs):
            ctx.conv_layer(d, B, x, w, o)

    stream = torch.cuda.current_stream()
    batched = _passes(torch, lambda: bt.launch(graph=True), args.steps, args.warmup, stream)
    plain = _passes(torch, plain_pass, args.plain_steps, 1, stream)
    per_layer = _passes(torch, per_layer_pass, args.plain_steps, 1, stream)

    # per-grid durations: instrumented eager passes of the same batch (the
    # same kernels as the graph), HIP events around every grid on its stream
    grid_ms = [bt.launch_timed(stream) for _ in range(args.kernel_reps)]
    n_ch = bt.n_chains
    # grids of each kind per pass: one per chain, or one per group when pipelined
    launches = {1: 1, 2: n_ch, 3: min(len(descs), 4), 4: min(len(descs), 8)}[args.schedule]
    kavg = {}
    for p, name in enumerate(("batch_fwd", "batch_mac", "batch_inv")):
        per_pass = float(np.mean([sum(grid_ms[r][c][p] for c in range(n_ch)) for r in range(len(grid_ms))]))
        kavg[name] = {"avg_ms_per_launch": per_pass / launches, "launches_per_pass": launches,
                      "ms_per_pass": per_pass}
    in_cts = sum(B * s.in_cts for s in sizes)
    out_cts = sum(B * s.out_cts for s in sizes)
    logN = N.bit_length() - 1
    w_bytes = sum(s.w_words * 8 for s in sizes)
    alg = {"batch_fwd": {"bytes": in_cts * 2 * L * 16 * N, "modmuls": in_cts * 2 * L * (N // 2) * logN},
           "batch_mac": {"bytes": w_bytes + (in_cts + out_cts) * ct_words * 8, "modmul_adds": macs * ct_words},
           "batch_inv": {"bytes": out_cts * 2 * L * 16 * N, "modmuls": out_cts * 2 * L * (N // 2) * logN}}
    for k in kavg:
        t = kavg[k]["ms_per_pass"] * 1e-3
        kavg[k]["alg"] = alg[k]
        kavg[k]["GBps"] = round(alg[k]["bytes"] / t / 1e9, 1)
    roofline, roofline_mac, roofline_hbm, ntt_roof = headline_rooflines(
        kavg, alg, bt.mac_form, probes, lambda k: load_traffic(k, cfg["name"]))
    resident = sum(t.numel() * 8 for t in wntts + ins + outs) / 2 ** 30
    res = {
        "metric": METRIC,
        "value": macs / (batched["mean_ms"] * 1e-3),
        "unit": "ct×pt MACs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": batched["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": cfg["name"], "N": N, "L": L, "q_bits": bits, "t": f"2^{synth.T_BITS}", "batch": B,
                   "layers": len(descs), "layer_solves_per_step": n_solves, "ctpt_macs_per_step": macs,
                   "in_cts_per_step": in_cts, "out_cts_per_step": out_cts, "resident_GiB": round(resident, 1),
                   "path": f"batched: {len(descs)} layer jobs x {B} images, "
                           f"{SCHEDULE_NAMES[args.schedule]} of three grids, one hipGraph launch",
                   "mac_form": bt.mac_form},
        "layers_per_s": n_solves / (batched["mean_ms"] * 1e-3),
        "p50_ms": batched["p50_ms"], "p99_ms": batched["p99_ms"],
        "plain": {"path": "plain per-layer: one he_conv_layer call per layer solve (one image)",
                  "calls_per_pass": n_solves, **plain,
                  "layers_per_s": n_solves / (plain["mean_ms"] * 1e-3),
                  "ctpt_macs_per_s": macs / (plain["mean_ms"] * 1e-3)},
        "per_layer_x16": {"path": "one he_conv_layer call of 16 images per layer", "calls_per_pass": len(descs),
                          **per_layer, "layers_per_s": n_solves / (per_layer["mean_ms"] * 1e-3),
                          "ctpt_macs_per_s": macs / (per_layer["mean_ms"] * 1e-3)},
        "batched_vs_plain": plain["mean_ms"] / batched["mean_ms"],
        "batched_vs_per_layer_x16": per_layer["mean_ms"] / batched["mean_ms"],
        "batched_equals_plain_all_words": equal_layers == len(descs),
        "layers_compared_all_words": equal_layers,
        "kernels": kavg,
        "roofline": roofline,
        "roofline_mac": roofline_mac,
        "roofline_hbm": roofline_hbm,
        "roofline_ntt_inv": ntt_roof["batch_inv"],
        "roofline_ntt_fwd": ntt_roof["batch_fwd"],
        "offline_encode_ms": t_enc * 1e3,
    }
    pending = {"q": list(ctx.q), "samples": {j: (samples[j], sample_out[j], Ks[j], (descs[j].Cw, descs[j].Hw,
                                                                                      descs[j].Ww))
                                             for j in sample_layers}}
    bt.close()
    del ins, outs, wntts, jobs
    ctx.close()
    return res, pending


def headline_rooflines(kavg, alg, form, probes, traffic):
    """The bottleneck batch's rooflines from its per-grid durations (kavg:
    ms_per_pass and avg_ms_per_launch per grid), algorithmic work (alg), the
    batch's MAC form, the VALU probes (or None) and a traffic lookup by grid
    name.  Returns (roofline, roofline_mac, roofline_hbm, {grid: roofline})
    for the transforms; roofline is the longest grid's."""
    mac_kernel = ("batch_mac_grid_kernel (streamed MAC, 2x2 wave grid)" if form["grid"] else
                  "batch_mac_stream_kernel (streamed MAC)" if form["lds"] >= 2 else "batch_mac_kernel")
    # the MAC at 16 images is bound by integer multiply-adds: each modmul-add
    # is four v_mad_u64_u32 of 30-bit halves, so the ceiling is the chip's
    # v_mad_u64_u32 rate / 4 (256 CUs x 64 lanes x 2.4 GHz; the probe
    # measures that instruction at the full rate)
    mac_t = kavg["batch_mac"]["ms_per_pass"] * 1e-3
    achieved = alg["batch_mac"]["modmul_adds"] / mac_t / 1e9
    peak = VALU_LANE_OPS_PEAK * MAD_RATE_FRAC / 4 / 1e9
    mac_gbps = alg["batch_mac"]["bytes"] / mac_t / 1e9
    roofline_mac = {"bound": "alu", "kernel": mac_kernel, "achieved": round(achieved, 1),
                    "peak": round(peak, 1), "unit": "G modmul-adds/s", "frac": round(achieved / peak, 4),
                    "traffic": traffic("batch_mac"),
                    "peak_derivation": "256 CUs x 64 lanes x 2.4 GHz (v_mad_u64_u32 issues at the full rate) / 4 "
                                       "multiply-adds per modmul-add",
                    "avg_launch_ms": round(kavg["batch_mac"]["avg_ms_per_launch"], 4)}
    if probes:
        mix = probes["mac_mix"]["rate"] / 1e9
        roofline_mac["measured_mix_ceiling"] = {
            "rate": round(mix, 1), "frac": round(achieved / mix, 4),
            "note": "the streamed MAC's channel-block step and carry on registers (6x4 tile, 8-block chunks)"}
    roofline_hbm = {"bound": "hbm", "kernel": mac_kernel, "achieved": round(mac_gbps, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(mac_gbps / HBM_PEAK_GBS, 4)}
    # the transforms are bound by integer VALU issue: the peak is the chip's
    # full-rate lane operations over the VALU instructions of one butterfly
    # as compiled (21 in either direction)
    ntt_roof = {}
    for k, kname, mix_key in (("batch_inv", "batch_inv_kernel (inverse NTTs)", "intt_mix"),
                              ("batch_fwd", "batch_fwd_kernel (forward NTTs)", "ntt_mix")):
        t = kavg[k]["ms_per_pass"] * 1e-3
        bfly = alg[k]["modmuls"] / t / 1e9
        peak_b = VALU_LANE_OPS_PEAK / BFLY_VALU_INSTS[k] / 1e9
        r = {"bound": "alu", "kernel": kname, "achieved": round(bfly, 1), "peak": round(peak_b, 1),
             "unit": "G butterflies/s", "frac": round(bfly / peak_b, 4), "traffic": traffic(k),
             "peak_derivation": f"256 CUs x 64 lanes x 2.4 GHz / {BFLY_VALU_INSTS[k]} VALU instructions per "
                                "butterfly (compiled)",
             "avg_launch_ms": round(kavg[k]["avg_ms_per_launch"], 4)}
        if probes:
            ceil = probes[mix_key]["rate"] / 1e9
            r["measured_mix_ceiling"] = {"rate": round(ceil, 1), "frac": round(bfly / ceil, 4),
                                         "note": "the butterfly's own instruction mix on registers (he_probe_valu)"}
        ntt_roof[k] = r
    # the headline roofline is the dominant grid's: the longest of the three
    dom = max(kavg, key=lambda k: kavg[k]["ms_per_pass"])
    roofline = roofline_mac if dom == "batch_mac" else ntt_roof[dom]
    return roofline, roofline_mac, roofline_hbm, ntt_roof


def _passes(torch, fn, k, warm, stream):
    """k timed calls of fn (one pass each) after `warm` calls and at least
    0.2 s of warm-up; HIP events between passes on `stream`.  Returns mean,
    p50 and p99 in ms."""
    t0, n = time.perf_counter(), 0
    while n < warm or time.perf_counter() - t0 < 0.2:
        fn()
        torch.cuda.synchronize()
        n += 1
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
    ev[0].record(stream)
    for i in range(k):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(k)])
    return {"passes_timed": k, "mean_ms": float(ev[0].elapsed_time(ev[-1]) / k),
            "p50_ms": float(np.percentile(per, 50)), "p99_ms": float(np.percentile(per, 99))}


def cpu_baseline_fire(args, cfg, q, host, gpu_out):
    """The CPU oracle (as it stands) on the fire-module CNN: its layers in
    order through the oracle's textbook NTT flow (forward NTT, MAC, inverse
    NTT; OpenMP over limb polynomials) on the same input words and kernels
    as the GPU pass, until about --cpu-seconds (the whole pass takes about
    one second), scaled to ct x pt MACs/s; every word of each layer solve is
    compared with the GPU's output."""
    import oracle

    prm = oracle.Params(cfg["N"], cfg["L"], cfg["bits"], 2 ** synth.T_BITS)
    assert prm.q == list(q)
    spent, macs, done, exact = 0.0, 0, 0, True
    for j, (x, K, (Cw, Hw, Ww)) in enumerate(host):
        cv = oracle.Conv(*cfg["layers"][j])
        g = oracle.geometry(cv, Cw, Hw, Ww)
        w_ntt = oracle.encode_weights(K, cv, g, prm)
        t0 = time.perf_counter()
        want = oracle.conv_layer_ntt(x.reshape(1, g.CB, g.S, 2, prm.L, prm.N), w_ntt, 1, g, cv.M, prm)
        spent += time.perf_counter() - t0
        macs += cv.M * g.CB * g.S
        got = gpu_out[j].cpu().numpy().view(np.uint64)
        exact &= bool(np.array_equal(got, want.reshape(-1)))
        done += 1
        del want, got, w_ntt
        if spent > args.cpu_seconds:
            break
    return ({"value": macs / spent, "unit": "ct×pt MACs/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": f"layers 0-{done - 1} of the fire-module CNN ({macs} ct x pt MACs, one image) through the "
                       f"oracle's textbook NTT flow (forward NTT, MAC, inverse NTT; OpenMP over limb "
                       f"polynomials), {spent:.1f} s; weight preprocessing not included"},
            {"layer_solves": done, "words_equal": exact})


def cpu_baseline_bottleneck(args, pending):
    """The CPU oracle (as it stands) on a bounded sample of the headline
    workload: image 0 of the layers in ORACLE_SAMPLE_LAYERS through the
    oracle's textbook NTT flow (forward NTT, MAC, inverse NTT; OpenMP over
    limb polynomials), one layer after another until about --cpu-seconds,
    scaled to ct x pt MACs/s.  Every word of each computed layer solve is
    compared with the GPU's batched output."""
    import oracle

    cfg = synth.WORKLOADS["bottleneck_cnn_b16"]
    prm = oracle.Params(cfg["N"], cfg["L"], cfg["bits"], 2 ** synth.T_BITS)
    assert prm.q == pending["q"]
    spent, macs, done, exact = 0.0, 0, [], True
    for j, (x, y, K, (Cw, Hw, Ww)) in pending["samples"].items():
        cv = oracle.Conv(*cfg["layers"][j])
        g = oracle.geometry(cv, Cw, Hw, Ww)
        w_ntt = oracle.encode_weights(K, cv, g, prm)
        t0 = time.perf_counter()
        want = oracle.conv_layer_ntt(x.reshape(1, g.CB, g.S, 2, prm.L, prm.N), w_ntt, 1, g, cv.M, prm)
        spent += time.perf_counter() - t0
        macs += cv.M * g.CB * g.S
        exact &= bool(np.array_equal(y.reshape(want.shape), want))
        done.append(int(j))
        if spent > args.cpu_seconds:
            break
    cores = oracle.num_threads()
    return ({"value": macs / spent, "unit": "ct×pt MACs/s", "cores": cores, "kind": "oracle",
             "sample": f"image 0 of layers {done} of the bottleneck CNN ({macs} ct x pt MACs) through the "
                       f"oracle's textbook NTT flow (forward NTT, MAC, inverse NTT; OpenMP over limb "
                       f"polynomials), {spent:.1f} s; weight preprocessing not included"},
            {"layer_solves": len(done), "words_equal": exact})


def run_client(torch, heconv):
    """Client-side encryption and decryption on the GPU (load generation):
    256 ciphertexts at N=8192, L=3 (eight times the 64->64 layer's input),
    messages uniform in [0, t), ternary key, small errors; every decrypted
    coefficient must equal its message."""
    cfg = synth.WORKLOADS["conv64_56x56"]
    N, L, bits = cfg["N"], cfg["L"], cfg["bits"]
    t = 2 ** synth.T_BITS
    ctx = heconv.Context(N, heconv.gen_primes(N, bits, L), t)
    n = 256
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    q = torch.tensor(ctx.q, dtype=torch.int64, device="cuda").view(1, L, 1)
    sk = torch.randint(-1, 2, (N,), dtype=torch.int64, generator=gen, device="cuda")
    msgs = torch.randint(0, t, (n, N), dtype=torch.int64, generator=gen, device="cuda")
    a = torch.randint(0, 2 ** 62, (n, L, N), dtype=torch.int64, generator=gen, device="cuda") % q
    err = torch.randint(-21, 22, (n, N), dtype=torch.int64, generator=gen, device="cuda")
    skn = torch.empty(L * N, dtype=torch.int64, device="cuda")
    ct = torch.empty(n * 2 * L * N, dtype=torch.int64, device="cuda")
    work = torch.empty(n * L * N, dtype=torch.int64, device="cuda")
    out = torch.empty(n * N, dtype=torch.int64, device="cuda")
    ctx.key_encode(sk, skn)
    ctx.encrypt(n, msgs, a, err, skn, ct, work)
    ctx.decrypt(n, ct, skn, out, work)
    want = torch.where(msgs >= t // 2, msgs - t, msgs).reshape(-1)
    exact = bool(torch.equal(out, want))
    t_enc = _timed(torch, lambda: ctx.encrypt(n, msgs, a, err, skn, ct, work), 20)
    t_dec = _timed(torch, lambda: ctx.decrypt(n, ct, skn, out, work), 20)
    ctx.close()
    return {"workload": f"{n} ciphertexts, N={N}, L={L}", "encrypt_ms": t_enc, "decrypt_ms": t_dec,
            "encrypt_cts_per_s": n / t_enc * 1e3, "decrypt_cts_per_s": n / t_dec * 1e3,
            "roundtrip_exact": exact}


def rotation_alg_bytes(N: int, L: int) -> int:
    """HBM bytes one ciphertext's rotation must move through the five steps
    (L ciphertext limbs, L+1 extended): digits written and transformed in
    place, products summed into two polynomials, transformed back, divided
    by P; the key (read once per launch) is not counted."""
    w = 8 * N
    modup = L * w + L * (L + 1) * w
    ntt_fwd = 2 * L * (L + 1) * w
    inner = L * (L + 1) * w + 2 * (L + 1) * w
    ntt_inv = 2 * 2 * (L + 1) * w
    moddown = 2 * (L + 1) * w + L * w + 2 * L * w
    return modup + ntt_fwd + inner + ntt_inv + moddown


def run_rotation(torch, heconv):
    """Ciphertext rotation for the Z_P variant: 256 ciphertexts at N=8192,
    L=3 (60-bit primes) with a 60-bit special prime, g = 5, one he_rotate
    call; the key made on the GPU; every ciphertext decrypts to m(X^g)."""
    cfg = synth.WORKLOADS["conv64_56x56"]
    N, L, bits = cfg["N"], cfg["L"], cfg["bits"]
    t = 2 ** synth.T_BITS
    primes = heconv.gen_primes(N, bits, L + 1)
    base, ext = heconv.Context(N, primes[:L], t), heconv.Context(N, primes, t)
    n, g = 256, 5
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    dev = dict(dtype=torch.int64, device="cuda")
    qx = torch.tensor(primes, **dev).view(1, L + 1, 1)
    sk = torch.randint(-1, 2, (N,), generator=gen, **dev)
    ka = torch.randint(0, 2 ** 62, (L, L + 1, N), generator=gen, **dev) % qx
    ke = torch.randint(-21, 22, (L, N), generator=gen, **dev)
    ksk = torch.empty(L * 2 * (L + 1) * N, **dev)
    ext.galois_key(g, sk, ka.reshape(-1), ke.reshape(-1), ksk, torch.empty(ext.galois_key_work_words(), **dev))
    skn = torch.empty(L * N, **dev)
    base.key_encode(sk, skn)
    msgs = torch.randint(0, t, (n, N), generator=gen, **dev)
    a = torch.randint(0, 2 ** 62, (n, L, N), generator=gen, **dev) % qx[:, :L]
    err = torch.randint(-21, 22, (n, N), generator=gen, **dev)
    ct = torch.empty(n * 2 * L * N, **dev)
    base.encrypt(n, msgs, a, err, skn, ct, torch.empty(n * L * N, **dev))
    out = torch.empty_like(ct)
    work = torch.empty(ext.keyswitch_work_words(n), **dev)
    ext.rotate(g, n, ct, ksk, out, work)
    dec = torch.empty(n * N, **dev)
    base.decrypt(n, out, skn, dec, torch.empty(n * L * N, **dev))
    ginv = pow(g, -1, 2 * N)
    k = (torch.arange(N, **dev) * ginv) % (2 * N)
    neg = k >= N
    want = msgs[:, torch.where(neg, k - N, k)]
    want = torch.where(neg, (t - want) % t, want)
    want = torch.where(want >= t // 2, want - t, want).reshape(-1)
    exact = bool(torch.equal(dec, want))
    ms = _timed(torch, lambda: ext.rotate(g, n, ct, ksk, out, work), 20)
    alg = rotation_alg_bytes(N, L) * n
    base.close()
    ext.close()
    return {"workload": f"{n} ciphertexts, N={N}, L={L} + one special prime, g={g}", "ms": ms,
            "rotations_per_s": n / ms * 1e3, "alg_bytes": alg, "GBps": alg / (ms * 1e-3) / 1e9,
            "decrypts_to_automorphism": exact}


def run_zp(torch, heconv):
    """The Z_P variant's linear kernel on a fully connected layer of
    ResNet-50's classifier shape, 2048 -> 1000, at 16 and at 64 images per
    call (square diagonal layout, the same as batched chains, and the
    generalized diagonals of a matrix with fewer rows than columns with
    one rotate-and-add): N=8192, L=3 (60-bit) plus a 60-bit special prime, t the largest
    37-bit prime = 1 mod 2N; 2048 diagonals, so 2048 iterations (2047
    rotations of every ciphertext).  Inputs and weights are uniform mod t;
    the first images of each batch are decrypted and decoded on the GPU and
    checked against W x mod t."""
    cfg = synth.WORKLOADS["conv64_56x56"]
    N, L, bits = cfg["N"], cfg["L"], cfg["bits"]
    rows, cols, g = 1000, 2048, 5
    n = cols
    t = heconv.gen_primes(N, 37, 1)[0]  # the largest prime = 1 mod 2N below 2^37
    primes = heconv.gen_primes(N, bits, L + 1)
    base, ext, tctx = heconv.Context(N, primes[:L], t), heconv.Context(N, primes, t), heconv.Context(N, [t])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13)
    dev = dict(dtype=torch.int64, device="cuda")
    qx = torch.tensor(primes, **dev).view(1, L + 1, 1)
    sk = torch.randint(-1, 2, (N,), generator=gen, **dev)
    ka = torch.randint(0, 2 ** 62, (L, L + 1, N), generator=gen, **dev) % qx
    ke = torch.randint(-21, 22, (L, N), generator=gen, **dev)
    ksk = torch.empty(L * 2 * (L + 1) * N, **dev)
    ext.galois_key(g, sk, ka.reshape(-1), ke.reshape(-1), ksk, torch.empty(ext.galois_key_work_words(), **dev))
    skn = torch.empty(L * N, **dev)
    base.key_encode(sk, skn)
    # weights: diagonals -> slots -> plaintexts -> scaled NTT form (offline)
    W = torch.randint(0, t, (rows, cols), generator=gen, **dev)
    slots = torch.empty(n * N, **dev)
    tctx.zp_diagonals(W.reshape(-1), rows, cols, n, slots)
    coeffs = torch.empty(n * N, **dev)
    tctx.simd_encode(n, slots, coeffs)
    w = torch.empty(n * L * N, **dev)
    ext.zp_encode_plain(n, coeffs, w)
    del slots, coeffs
    # the same matrix as 1024 generalized diagonals of period 2048 (rows
    # padded to 1024 < 2048 columns) and the Galois element of the fold
    n_rect = 1024
    slots = torch.empty(n_rect * N, **dev)
    tctx.zp_diagonals_rect(W.reshape(-1), rows, cols, n_rect, cols, slots)
    coeffs = torch.empty(n_rect * N, **dev)
    tctx.simd_encode(n_rect, slots, coeffs)
    w_rect = torch.empty(n_rect * L * N, **dev)
    ext.zp_encode_plain(n_rect, coeffs, w_rect)
    del slots, coeffs
    g_fold = pow(g, n_rect, 2 * N)
    Wh = W.cpu().numpy().astype(object)
    keys2 = {}
    res = {"workload": f"FC {cols}->{rows}, N={N}, L={L} + one special prime, t={t} (37-bit prime), "
                       f"{n} diagonals", "by_batch": {}}
    for B, checked in ((16, 4), (64, 2)):
        # inputs: x repeated with period 2048 in both slot rows, encoded, encrypted
        x = torch.randint(0, t, (B, cols), generator=gen, **dev)
        xc = torch.empty(B * N, **dev)
        tctx.simd_encode(B, x.repeat(1, N // cols).contiguous().reshape(-1), xc)
        a = torch.randint(0, 2 ** 62, (B, L, N), generator=gen, **dev) % qx[:, :L]
        err = torch.randint(-21, 22, (B, N), generator=gen, **dev)
        ct = torch.empty(B * 2 * L * N, **dev)
        base.encrypt(B, xc, a, err, skn, ct, torch.empty(B * L * N, **dev))
        base.ntt_fwd(ct, 2 * B)
        out = torch.empty_like(ct)
        work = torch.empty(ext.zp_work_words(B), **dev)
        ext.zp_matvec(g, B, ct, w, n, ksk, out, work)
        dec = torch.empty(B * N, **dev)
        base.decrypt(B, out, skn, dec, torch.empty(B * L * N, **dev))
        ys = torch.empty(B * N, **dev)
        tctx.simd_decode(B, dec, ys, torch.empty(B * N, **dev))
        ys = ys.view(B, N)[:, :rows].cpu().numpy()
        xh = x.cpu().numpy().astype(object)
        exact = all(np.array_equal(ys[b].astype(object), (Wh @ xh[b]) % t) for b in range(checked))
        ms = _timed(torch, lambda: ext.zp_matvec(g, B, ct, w, n, ksk, out, work), 3)
        res["by_batch"][str(B)] = {"ms": ms, "fc_layers_per_s": B / ms * 1e3,
                                   "zp_macs_per_s": B * rows * cols / (ms * 1e-3),
                                   "ct_iterations_per_s": B * n / (ms * 1e-3),
                                   "us_per_iteration": ms * 1e3 / n, "decrypts_to_Wx": exact,
                                   "images_checked": checked}
        del work
        # the same kernel as G chains batched together, combined by G - 1
        # rotations of n/G slots (a second Galois key)
        grouped = {}
        for G in ((4, 8, 16) if B == 16 else (4,)):
            g2 = pow(g, n // G, 2 * N)
            if g2 not in keys2:
                k2 = torch.empty_like(ksk)
                ext.galois_key(g2, sk, ka.reshape(-1), ke.reshape(-1), k2,
                               torch.empty(ext.galois_key_work_words(), **dev))
                keys2[g2] = k2
            workg = torch.empty(ext.zp_grouped_work_words(B, G), **dev)
            run = lambda: ext.zp_matvec_grouped(g, B, ct, w, n, G, ksk, g2, keys2[g2], out, workg)
            run()
            base.decrypt(B, out, skn, dec, torch.empty(B * L * N, **dev))
            ys2 = torch.empty(B * N, **dev)
            tctx.simd_decode(B, dec, ys2, torch.empty(B * N, **dev))
            yg = ys2.view(B, N)[:, :rows].cpu().numpy()
            ok = all(np.array_equal(yg[b].astype(object), (Wh @ xh[b]) % t) for b in range(checked))
            msg = _timed(torch, run, 3)
            grouped[str(G)] = {"ms": msg, "fc_layers_per_s": B / msg * 1e3,
                               "zp_macs_per_s": B * rows * cols / (msg * 1e-3), "dependent_steps": n // G + G - 1,
                               "decrypts_to_Wx": ok}
            del workg
        res["by_batch"][str(B)]["grouped"] = grouped
        # fewer rows than columns: 1024 generalized diagonals (period 2048),
        # then one rotate-and-add by 1024 slots
        rect = {}
        z = torch.empty_like(ct)
        workf = torch.empty(ext.keyswitch_work_words(B), **dev)
        for G in ((1, 8) if B == 16 else (1, 2)):
            g2 = pow(g, n_rect // G, 2 * N) if G > 1 else 1
            for gg in ([g2] if G > 1 else []) + [g_fold]:
                if gg not in keys2:
                    k2 = torch.empty_like(ksk)
                    ext.galois_key(gg, sk, ka.reshape(-1), ke.reshape(-1), k2,
                                   torch.empty(ext.galois_key_work_words(), **dev))
                    keys2[gg] = k2
            workg = torch.empty(ext.zp_grouped_work_words(B, G), **dev)

            def run_rect():
                if G == 1:
                    ext.zp_matvec(g, B, ct, w_rect, n_rect, ksk, z, workg)
                else:
                    ext.zp_matvec_grouped(g, B, ct, w_rect, n_rect, G, ksk, g2, keys2[g2], z, workg)
                ext.zp_fold(g_fold, B, z, keys2[g_fold], out, workf)

            run_rect()
            base.decrypt(B, out, skn, dec, torch.empty(B * L * N, **dev))
            ys3 = torch.empty(B * N, **dev)
            tctx.simd_decode(B, dec, ys3, torch.empty(B * N, **dev))
            yr = ys3.view(B, N)[:, :rows].cpu().numpy()
            ok = all(np.array_equal(yr[b].astype(object), (Wh @ xh[b]) % t) for b in range(checked))
            msr = _timed(torch, run_rect, 3)
            rect[str(G)] = {"ms": msr, "fc_layers_per_s": B / msr * 1e3,
                            "zp_macs_per_s": B * rows * cols / (msr * 1e-3),
                            "dependent_steps": n_rect // G + G - 1 + 1, "decrypts_to_Wx": ok}
            del workg
        res["by_batch"][str(B)]["rectangular"] = rect
        del ct, out, z, workf
    for c in (base, ext, tctx):
        c.close()
    return res


def run_serving(torch, heconv, args):
    """Open-loop Poisson arrivals over the 28 single-layer shapes of the three
    workloads above (the small layer keeps N=4096, L=2), weights resident,
    HBM budget 200 GB, four streams, queued requests of one layer merged
    into one launch; then the same requests closed-loop (saturation), served
    vs the plain path (one request per launch, one stream) and vs four
    streams without merging; an open-loop sweep of offered rates across the
    plain capacity, served and plain, with p50/p99; then closed-loop in
    protocol mode (each request also folds in the server's input share and
    returns masked, extracted outputs)."""
    from paper_2506_11586_amd import serving

    shapes = [("conv4_16x16", synth.WORKLOADS["conv4_16x16"]["layers"][0]),
              ("conv64_56x56", synth.WORKLOADS["conv64_56x56"]["layers"][0])] + \
             [("fire_cnn", s) for s in synth.WORKLOADS["fire_cnn"]["layers"]]
    ctxs, layers = {}, []
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).cuda()
    for i, (c, shape) in enumerate(shapes):
        cfg = synth.WORKLOADS[c]
        key = (cfg["N"], cfg["L"], cfg["bits"])
        if key not in ctxs:
            ctxs[key] = heconv.Context(cfg["N"], heconv.gen_primes(cfg["N"], cfg["bits"], cfg["L"]))
        ctx = ctxs[key]
        C, H, W, M, kh, kw, stride, pad = shape
        K = Stream(5000 + i, synth.WEIGHT).ints(M * C * kh * kw, *cfg["w_range"])
        layers.append(serving.make_layer(ctx, shape, dev(K)))
    # a pool of two distinct seeded inputs per layer, reused round-robin
    pool = []
    for i, lay in enumerate(layers):
        rows = lay.in_words // lay.ctx.N
        pool.append([torch.from_numpy(synth.uniform_mod(Stream(6000 + 2 * i + v, synth.UNIFORM),
                                                        (rows // lay.ctx.L, lay.ctx.L, lay.ctx.N),
                                                        lay.ctx.q).view(np.int64).ravel().copy()).pin_memory()
                     for v in range(2)])
    n = args.serve_requests
    mix = Stream(5, synth.MIX).below(n, len(layers)).astype(int)
    times = serving.poisson_arrivals(args.serve_rate, n, Stream(5, synth.ARRIVAL).uniform_f64(n))

    def requests():
        return [serving.Request(i, int(mix[i]), float(times[i]), pool[mix[i]][i % 2]) for i in range(n)]

    def requests_at(rate, k, seed):
        mx = Stream(seed, synth.MIX).below(k, len(layers)).astype(int)
        ts = serving.poisson_arrivals(rate, k, Stream(seed, synth.ARRIVAL).uniform_f64(k))
        return [serving.Request(i, int(mx[i]), float(ts[i]), pool[mx[i]][i % 2]) for i in range(k)]

    def summary(st, macs_of=None):
        d = {"layers_per_s": st.layers_per_s, "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms,
             "max_inflight": st.max_inflight, "launches": st.launches, "mean_batch": round(st.mean_batch, 3),
             "wall_s": st.wall_s}
        return d

    server = serving.Server(layers, n_streams=4, hbm_budget=200e9)
    server.run(requests()[:64], closed_loop=True)  # warm-up: launch buffers, code paths
    op = server.run(requests())
    cl = server.run(requests(), closed_loop=True)
    # plain: one request per launch on one stream (the plain per-layer path)
    one = serving.Server(layers, n_streams=1, hbm_budget=200e9, max_batch=1)
    one.run(requests()[:32], closed_loop=True)
    seq = one.run(requests(), closed_loop=True)
    # served without merging (four streams, one request per launch)
    nomerge = serving.Server(layers, n_streams=4, hbm_budget=200e9, max_batch=1)
    nomerge.run(requests()[:32], closed_loop=True)
    ncl = nomerge.run(requests(), closed_loop=True)
    # open-loop arrival-rate sweep across the plain capacity
    sweep = []
    for k, rate in enumerate(args.serve_sweep):
        reqs = requests_at(rate, args.serve_sweep_requests, 50 + k)
        st = server.run(reqs)
        pl = one.run(requests_at(rate, args.serve_sweep_requests, 50 + k))
        sweep.append({"offered_per_s": rate, "served": summary(st), "plain_one_stream": summary(pl)})
    # protocol mode: a seeded share and mask per layer, reused by its requests
    shares = [torch.from_numpy(Stream(7000 + i, synth.SHARE).below(lay.share_words, 2 ** synth.T_BITS)
                               .astype(np.int64)).pin_memory() for i, lay in enumerate(layers)]
    masks = [torch.from_numpy(Stream(7000 + i, synth.MASK).below(lay.mask_words, 2 ** synth.T_BITS)
                              .astype(np.int64)).pin_memory() for i, lay in enumerate(layers)]

    def proto_requests():
        rs = requests()
        for r in rs:
            r.host_share, r.host_mask = shares[r.layer], masks[r.layer]
        return rs

    proto = serving.Server(layers, n_streams=4, hbm_budget=200e9, protocol=True)
    proto.run(proto_requests()[:64], closed_loop=True)
    pcl = proto.run(proto_requests(), closed_loop=True)
    macs = {i: lay.desc.M * lay.sizes.CB * lay.sizes.S for i, lay in enumerate(layers)}
    tot_macs = sum(macs[int(m)] for m in mix)
    out = {"workload": f"Poisson {args.serve_rate:g} req/s, {n} single-layer requests over {len(layers)} shapes",
           "form": "continuous batching: queued requests of one layer merged into one he_conv_layer launch "
                   "(up to 16 images), four streams",
           "open_loop": summary(op),
           "closed_loop_served": dict(summary(cl), ctpt_macs_per_s=tot_macs / cl.wall_s),
           "closed_loop_plain_one_stream": dict(summary(seq), ctpt_macs_per_s=tot_macs / seq.wall_s),
           "closed_loop_four_streams_no_merging": summary(ncl),
           "served_vs_plain": cl.layers_per_s / seq.layers_per_s,
           "sweep": sweep,
           "closed_loop_protocol": dict(summary(pcl), ctpt_macs_per_s=tot_macs / pcl.wall_s,
                                        steps="share folded in, layer, masked extraction (Sec. 7)"),
           "hbm_budget_GB": 200, "resident_weights_GB": server.resident / 1e9,
           "latency": "arrival -> device completion (H2D copy of the input included; results stay in HBM)"}
    for c in ctxs.values():
        c.close()
    return out


def cpu_baseline(args, cfg, ctx, d, sz, x_host, K_host, gpu_out):
    """The CPU oracle (as it stands) on the same seeded input: its textbook
    NTT flow for the whole layer, repeated until about --cpu-seconds of CPU
    time, scaled to ct x pt MACs/s.  Its first result is also compared word
    for word with the GPU output."""
    import oracle

    prm = oracle.Params(cfg["N"], cfg["L"], cfg["bits"], 2 ** synth.T_BITS)
    assert prm.q == ctx.q and prm.psi == ctx.psi
    cv = oracle.Conv(*cfg["layers"][0])
    g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
    B = cfg["batch"]
    x = x_host.reshape(B, g.CB, g.S, 2, prm.L, prm.N)
    t0 = time.perf_counter()
    w_ntt = oracle.encode_weights(K_host, cv, g, prm)
    enc_s = time.perf_counter() - t0
    reps, spent, want = 0, 0.0, None
    while spent < args.cpu_seconds or reps == 0:
        t0 = time.perf_counter()
        out = oracle.conv_layer_ntt(x, w_ntt, B, g, cv.M, prm)
        spent += time.perf_counter() - t0
        reps += 1
        if want is None:
            want = out
        if spent > 0 and spent / reps * (reps + 1) > 3 * args.cpu_seconds:
            break
    macs = B * cv.M * g.CB * g.S
    bit_exact = bool(np.array_equal(gpu_out.reshape(want.shape), want))
    cores = oracle.num_threads()
    # the same flow on one core, one layer solve
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.conv_layer_ntt(x, w_ntt, B, g, cv.M, prm)
    one_core = macs / (time.perf_counter() - t0)
    oracle.set_threads(cores)
    # the layer by definition (schoolbook negacyclic products, all cores) on
    # the small 4->4 layer at N=4096
    c1 = synth.WORKLOADS["conv4_16x16"]
    p1 = oracle.Params(c1["N"], c1["L"], c1["bits"], 2 ** synth.T_BITS)
    cv1 = oracle.Conv(*c1["layers"][0])
    g1 = oracle.plan_conv(cv1, p1.N, p1.L)
    x1 = synth.uniform_mod(Stream(c1["seed"], synth.UNIFORM), (1, g1.CB, g1.S, 2, p1.L, p1.N), p1.q)
    K1 = Stream(c1["seed"], synth.WEIGHT).ints(cv1.M * cv1.C * 9, *c1["w_range"]).reshape(cv1.M, cv1.C, 3, 3)
    t0 = time.perf_counter()
    oracle.conv_layer_def(x1, oracle.pack_weights(K1, cv1, g1, p1), 1, g1, cv1.M, p1)
    def_rate = cv1.M * g1.CB * g1.S / (time.perf_counter() - t0)
    return ({"value": macs * reps / spent, "unit": "ct×pt MACs/s", "cores": cores,
             "kind": "oracle",
             "sample": f"{reps} full layer solve(s) of the same workload through the oracle's textbook "
                       f"NTT flow (forward NTT, MAC, inverse NTT; OpenMP over limb polynomials), "
                       f"{spent:.1f} s; weight preprocessing {enc_s:.2f} s not included",
             "value_one_core": one_core,
             "value_by_definition_small_layer": def_rate,
             "by_definition_sample": "one 4->4 3x3 16x16 layer solve at N=4096, L=2 by schoolbook negacyclic "
                                     "products (O(N^2) per ct x pt product), all cores"},
            bit_exact)


if __name__ == "__main__":
    main()
