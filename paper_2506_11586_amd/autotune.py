"""Measured autotuner for a context's launch shapes (he_tuning) and for the
batch executor's.

What it picks:
- the NTT's stage grouping: 2^loge coefficients per thread, i.e. loge
  butterfly stages per register pass and one LDS exchange per pass; chosen
  separately for small and large calls;
- the MAC's register tile: output channels x ciphertext rows per thread;
- whether the MAC stages its operands in LDS, and how many blocks ahead;
- the output-channel MAC/iNTT pipeline of a one-image layer;
- the two-grid forward and inverse NTTs for small calls;
- the MAC and inverse NTT as one fused kernel or two (one launch fewer on
  small layers);
- double-precision transforms where every prime is below 2^50 (the switch
  is ignored otherwise);
- for a batch: the schedule (one or two chains, or the pipeline of 4 or 8
  groups) and the MAC tile.

A tuning changes only launch shapes, never a result word, so the tuner can
time candidates on whatever the buffers hold.  A layer clobbers its input
(the forward NTT is in place), and the timing does not depend on the data.

Search: greedy coordinate descent from the context's current tuning.  Each
knob in turn takes every candidate value while the others are held, and the
fastest value stays if it beats the current best by more than `min_gain`
(1% by default: smaller differences are within the run-to-run spread of
the timings, and the starting tuning should not drift on noise); `sweeps`
passes over the knobs.  A candidate's time is
the median over `reps` launches, each bracketed by HIP events on the
launching stream, after `warm_s` seconds of warm-up launches: the GPU
raises its clocks only under sustained load.

Cache: the best tuning per key (device name, N, L, primes, layer shape,
packing, batch) in memory, and in a JSON file when a path is given, so a
server tunes each shape once.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
import time
from dataclasses import dataclass, field

from . import heconv

# Candidate values per knob.  A knob is a name and a list of values; each
# value is a dict of he_tuning fields.
MAC_TILES = ((0, 0), (4, 4), (4, 2), (2, 4), (8, 2), (2, 8), (8, 1), (1, 8), (2, 2))


def layer_space(N: int) -> list[tuple[str, list[dict]]]:
    """Knobs of a single layer solve (he_conv_layer) at ring degree N."""
    loges = (3, 4) if N <= 8192 else (4,)  # 2^3 per thread needs N/8 <= 1024 threads
    return [
        ("ntt_loge_small", [{"ntt_loge_small": v} for v in loges]),
        ("ntt_loge_large", [{"ntt_loge_large": v} for v in loges]),
        ("mac", [{"mac_mt": a, "mac_rt": b} for a, b in MAC_TILES]),
        ("mac_lds", [{"mac_lds": v} for v in (0, 2, 3, 4)]),
        ("layer_split", [{"layer_split": v} for v in (1, 2, 4)]),
        ("ntt_split_below", [{"ntt_split_below": v} for v in (0, 96, 160, 224, 320)]),
        ("ntt_inv_split_below", [{"ntt_inv_split_below": v} for v in (0, 64, 128, 192)]),
        ("layer_fused", [{"layer_fused": v} for v in (0, 1)]),
        ("ntt_fp64", [{"ntt_fp64": v} for v in (0, 1)]),
    ]


def batch_space(N: int) -> list[tuple[str, list[dict]]]:
    """Knobs of a batch: the MAC tile ((0, 0) lets the executor pick by
    shape; the others force that tile where the chosen kernel has it), the
    LDS stages, the streamed MAC's tiles per workgroup and 2x2 wave grid,
    and the NTT grouping; the schedule is a separate argument of Batch and
    is searched by tune_batch."""
    loges = (3, 4) if N <= 8192 else (4,)
    return [
        ("mac", [{"mac_mt": a, "mac_rt": b} for a, b in ((0, 0), (2, 2), (4, 4), (4, 2), (2, 4), (6, 4))]),
        ("mac_lds", [{"mac_lds": v} for v in (0, 2, 3, 4)]),
        ("mac_grid", [{"mac_grid": v} for v in (0, 1)]),
        ("mac_tiles", [{"mac_tiles": v} for v in (0, 1, 2, 8)]),
        ("ntt_loge_small", [{"ntt_loge_small": v} for v in loges]),
        ("ntt_loge_large", [{"ntt_loge_large": v} for v in loges]),
    ]


def coordinate_descent(space, start: dict, cost, sweeps: int = 1, min_gain: float = 0.0):
    """Greedy search: returns (best tuning dict, its cost, every evaluation
    as a list of (tuning dict, cost)).  `cost(tuning)` is called with a
    complete tuning dict.  A candidate replaces the best only if its cost is
    below best * (1 - min_gain), so the result costs at most
    min(evaluated) / (1 - min_gain); equal costs keep the earlier value."""
    best = dict(start)
    seen: dict[tuple, float] = {}
    trail = []

    def evaluate(t):
        key = tuple(sorted(t.items()))
        if key not in seen:
            seen[key] = float(cost(dict(t)))
            trail.append((dict(t), seen[key]))
        return seen[key]

    best_cost = evaluate(best)
    for _ in range(max(1, sweeps)):
        changed = False
        for _name, values in space:
            for v in values:
                cand = dict(best)
                cand.update(v)
                c = evaluate(cand)
                if c < best_cost * (1.0 - min_gain):
                    best, best_cost, changed = cand, c, True
        if not changed:
            break
    return best, best_cost, trail


def median_ms(torch, fn, reps: int = 20, warm_s: float = 0.05, stream=None) -> float:
    """Median duration in ms of fn() over `reps` calls on `stream` (torch's
    current stream by default), each between two HIP events, after warm-up
    calls for at least warm_s seconds."""
    st = stream if stream is not None else torch.cuda.current_stream()
    t0 = time.perf_counter()
    k = 0
    while k < 2 or time.perf_counter() - t0 < warm_s:
        fn()
        torch.cuda.synchronize()
        k += 1
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in ev)


@dataclass
class TuneCache:
    """Best tunings by key; persisted as JSON when `path` is set."""
    path: str | None = None
    entries: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.path and os.path.exists(self.path):
            with open(self.path) as f:
                data = json.load(f)
            if not isinstance(data, dict):
                raise ValueError(f"{self.path}: not a tuning cache")
            self.entries = data

    def get(self, key: str):
        e = self.entries.get(key)
        return dict(e["tuning"]) if e else None

    def put(self, key: str, tuning: dict, ms: float, default_ms: float):
        self.entries[key] = {"tuning": dict(tuning), "ms": ms, "default_ms": default_ms}
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _ctx_key(ctx) -> str:
    h = hashlib.sha256(",".join(str(q) for q in ctx.q).encode()).hexdigest()[:12]
    return f"N{ctx.N}_L{ctx.L}_q{h}"


def layer_key(device_name: str, ctx, d, B: int) -> str:
    """Cache key of one layer solve: device, ring, primes, shape, packing, B."""
    s = d.shape()
    return (f"{device_name}|{_ctx_key(ctx)}|layer|C{s[0]}H{s[1]}W{s[2]}M{s[3]}k{s[4]}x{s[5]}"
            f"s{s[6]}p{s[7]}|pk{d.Cw}x{d.Hw}x{d.Ww}|B{B}")


def batch_key(device_name: str, ctx, jobs) -> str:
    """Cache key of a batch: device, ring, primes and every job's shape,
    packing and B, in order."""
    parts = []
    for d, B, *_ in jobs:
        s = d.shape()
        parts.append(f"{'x'.join(str(v) for v in s)}:{d.Cw}x{d.Hw}x{d.Ww}:{B}")
    h = hashlib.sha256(";".join(parts).encode()).hexdigest()[:16]
    return f"{device_name}|{_ctx_key(ctx)}|batch|{len(jobs)}jobs|{h}"


@dataclass
class TuneResult:
    tuning: dict          # the chosen he_tuning fields (complete)
    ms: float             # its median time
    default_ms: float     # the starting tuning's median time
    evaluations: list     # (tuning dict, ms) in the order they were timed
    cached: bool = False
    schedule: int | None = None  # batches only


def tune_layer(torch, ctx, d, B: int, in_dev, wntt_dev, out_dev, cache: TuneCache | None = None,
               reps: int = 20, warm_s: float = 0.05, sweeps: int = 1, apply: bool = True,
               min_gain: float = 0.01) -> TuneResult:
    """Tune he_conv_layer for (d, B) on the given device buffers.  The
    input buffer is clobbered.  With apply the context keeps the best
    tuning, else its tuning is restored."""
    start = ctx.get_tuning().as_dict()
    key = layer_key(torch.cuda.get_device_name(), ctx, d, B)
    if cache is not None:
        hit = cache.get(key)
        if hit is not None:
            ctx.set_tuning(**hit)
            ms = median_ms(torch, lambda: ctx.conv_layer(d, B, in_dev, wntt_dev, out_dev), reps, warm_s)
            if not apply:
                ctx.set_tuning(**start)
            return TuneResult(hit, ms, float("nan"), [(hit, ms)], cached=True)

    def cost(t):
        try:
            ctx.set_tuning(**t)
            return median_ms(torch, lambda: ctx.conv_layer(d, B, in_dev, wntt_dev, out_dev), reps, warm_s)
        except heconv.HeError:  # a value the library rejects for this shape
            return float("inf")

    best, best_ms, trail = coordinate_descent(layer_space(ctx.N), start, cost, sweeps, min_gain)
    ctx.set_tuning(**(best if apply else start))
    if cache is not None:
        cache.put(key, best, best_ms, trail[0][1])
    return TuneResult(best, best_ms, trail[0][1], trail)


def tune_batch(torch, ctx, jobs, cache: TuneCache | None = None, schedules=None, reps: int = 10,
               warm_s: float = 0.1, apply: bool = True, min_gain: float = 0.01) -> TuneResult:
    """Tune a batch of layer solves (the jobs list of heconv.Batch): every
    schedule in `schedules` (default: one and two chains) crossed with a
    coordinate descent over batch_space.  Each candidate builds its own
    Batch (the MAC tile is fixed when a batch is built) and times graph
    launches.  Returns the best tuning and schedule; with apply the context
    keeps the tuning."""
    start = ctx.get_tuning().as_dict()
    key = batch_key(torch.cuda.get_device_name(), ctx, jobs)
    if schedules is None:
        schedules = (heconv.SCHED_ONE_CHAIN, heconv.SCHED_TWO_CHAINS, heconv.SCHED_PIPELINED_4,
                     heconv.SCHED_PIPELINED_8)
    if cache is not None:
        hit = cache.get(key)
        if hit is not None:
            sched = hit.pop("schedule")
            ctx.set_tuning(**hit)
            if not apply:
                ctx.set_tuning(**start)
            e = cache.entries[key]
            return TuneResult(hit, e["ms"], e["default_ms"], [], cached=True, schedule=sched)

    def timed(t, sched):
        try:
            ctx.set_tuning(**t)
            b = heconv.Batch(ctx, jobs, schedule=sched)
        except heconv.HeError:  # a value the library rejects for these jobs
            return float("inf")
        try:
            return median_ms(torch, lambda: b.launch(graph=True), reps, warm_s)
        finally:
            b.close()

    best = None
    trail_all = []
    for sched in schedules:
        t, ms, trail = coordinate_descent(batch_space(ctx.N), start, lambda t: timed(t, sched), 1, min_gain)
        trail_all += [(dict(tt, schedule=sched), m) for tt, m in trail]
        if best is None or ms < best[1] * (1.0 - min_gain):
            best = (t, ms, sched)
    t, ms, sched = best
    ctx.set_tuning(**(t if apply else start))
    default_ms = trail_all[0][1]
    if cache is not None:
        cache.put(key, dict(t, schedule=sched), ms, default_ms)
    return TuneResult(t, ms, default_ms, trail_all, schedule=sched)
