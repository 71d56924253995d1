"""Request server for single-layer HE convolutions: continuous batching over
a pool of HIP streams with weights resident in HBM.

Each request is one layer solve (one image) of a resident layer: its input
ciphertexts arrive in host memory and the layer's NTT -> MAC -> iNTT runs on
the device.  In protocol mode (the server's whole step for a linear layer
in the online protocol, Sec. 7) a request also brings the server's input
share and output mask: the share is folded into the input ciphertexts
before the layer, and the output is masked and reduced to the coefficients
that hold results (he_add_share, he_conv_layer, he_mask_extract).

Continuous batching.  Whenever a stream is free, the dispatcher takes the
oldest waiting request and every other waiting request of the same layer
(up to `max_batch`), copies their inputs into consecutive image slots of a
launch buffer of that layer, and runs them as ONE he_conv_layer call of b
images: the layer's weights are read once for all of them, which is where
serving many requests beats one call per request.  Requests that arrive
while others are on the GPU join the next launch of their layer.  Launch
buffers are allocated on first use, then reused (a launch allocates
nothing); their memory counts against the HBM budget together with the
resident weights, and admission waits while the budget is used up.  The
packing of each layer is planned for one image; a launch of b images uses
the same descriptor, so each request's output words do not depend on what
it was batched with.  Latency is arrival -> device completion, measured on
the GPU timeline with events.

All device work is the C library's; this module is scheduling only.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import heconv


@dataclass
class Layer:
    """A resident layer: its context, descriptor, sizes and NTT-form weights."""

    ctx: heconv.Context
    shape: tuple
    desc: heconv.ConvDesc
    sizes: heconv.Sizes
    wntt: object  # device tensor
    in_words: int
    out_words: int
    share_words: int = 0  # C*H*W: the server's input share (protocol mode)
    mask_words: int = 0   # M*Ho*Wo: the server's output share
    y_words: int = 0      # M*L*Ho*Wo: the extracted, masked outputs


@dataclass(eq=False)
class Request:
    rid: int
    layer: int
    t_arrival: float  # seconds from the start of the run
    host_in: object   # pinned host tensor with the request's input words
    t_done: float = math.nan
    result: object = None      # keep_outputs: device tensor with the output (protocol mode: extracted words)
    batch: int = 0             # images in the launch that served it
    host_share: object = None  # protocol mode: pinned int64 share [C*H*W]
    host_mask: object = None   # protocol mode: pinned int64 mask [M*Ho*Wo]


@dataclass
class Stats:
    n: int
    wall_s: float
    layers_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_inflight: int
    launches: int = 0
    mean_batch: float = 1.0
    latencies_ms: list = field(default_factory=list)


def single_stream_tunings(ctxs) -> list:
    """Set layer_split = 1 on every context that is not already so, and
    return those contexts.  A split layer runs its inverse NTTs on the
    context's one internal stream with shared events, so calls from several
    streams would wait on and race with each other's transforms."""
    changed = []
    for c in ctxs:
        if c.get_tuning().layer_split != 1:
            c.set_tuning(layer_split=1)
            changed.append(c)
    return changed


class Server:
    """Resident layers + launch buffers per layer + a stream pool."""

    def __init__(self, layers: list[Layer], n_streams: int = 4, hbm_budget: float = 200e9, protocol: bool = False,
                 max_batch: int = 16):
        import torch
        self.torch = torch
        self.protocol = protocol
        self.layers = layers
        self.max_batch = max(1, int(max_batch))
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]  # default priority
        self.budget = float(hbm_budget)
        self.resident = sum(l.wntt.numel() * 8 for l in layers)
        if self.resident > self.budget:
            raise MemoryError(f"weights ({self.resident / 1e9:.1f} GB) exceed the HBM budget")
        self.used = self.resident
        self.free_bufs = {i: [] for i in range(len(layers))}
        single_stream_tunings({id(l.ctx): l.ctx for l in layers}.values())

    # -- launch buffers: max_batch image slots of one layer ------------------
    def _slot_words(self, L: Layer) -> list[int]:
        w = [L.in_words, L.out_words]
        if self.protocol:
            w += [L.share_words, L.mask_words, L.y_words]
        return w

    def _buf_bytes(self, li: int) -> int:
        return sum(self._slot_words(self.layers[li])) * 8 * self.max_batch

    def _buffer(self, li: int):
        """A launch buffer of layer li (one tensor per slot kind, max_batch
        images each) from the pool, or a new one if the budget allows; None
        when it does not."""
        if self.free_bufs[li]:
            return self.free_bufs[li].pop()
        need = self._buf_bytes(li)
        # idle buffers of other layers give their memory back first
        for lj, pool in self.free_bufs.items():
            while pool and self.used + need > self.budget:
                pool.pop()
                self.used -= self._buf_bytes(lj)
        if self.used + need > self.budget:
            return None
        self.used += need
        t = self.torch
        return tuple(t.empty(w * self.max_batch, dtype=t.int64, device="cuda")
                     for w in self._slot_words(self.layers[li]))

    def _release(self, li: int, buf):
        self.free_bufs[li].append(buf)

    # -- one launch of b requests of one layer on one stream -----------------
    def _launch(self, li: int, reqs: list[Request], buf, stream, keep: bool):
        t = self.torch
        L = self.layers[li]
        b = len(reqs)
        iw, ow = L.in_words, L.out_words
        with t.cuda.stream(stream):
            for i, r in enumerate(reqs):
                buf[0][i * iw:(i + 1) * iw].copy_(r.host_in, non_blocking=True)
                if self.protocol:
                    buf[2][i * L.share_words:(i + 1) * L.share_words].copy_(r.host_share, non_blocking=True)
                    buf[3][i * L.mask_words:(i + 1) * L.mask_words].copy_(r.host_mask, non_blocking=True)
            if self.protocol:
                L.ctx.add_share(L.desc, b, buf[0], buf[2], stream=stream)
            L.ctx.conv_layer(L.desc, b, buf[0], L.wntt, buf[1], stream=stream)
            if self.protocol:
                L.ctx.mask_extract(L.desc, b, buf[1], buf[3], None, buf[4], stream=stream)
            if keep:  # each request keeps its own copy of its result (before the buffer is free again)
                src, w = (buf[4], L.y_words) if self.protocol else (buf[1], ow)
                for i, r in enumerate(reqs):
                    r.result = src[i * w:(i + 1) * w].clone()
            ev = t.cuda.Event(enable_timing=True)
            ev.record(stream)
        for r in reqs:
            r.batch = b
        return ev

    def run(self, requests: list[Request], closed_loop: bool = False, keep_outputs: bool = False) -> Stats:
        """Serve `requests`.  Open loop: a request becomes available at its
        arrival time.  Closed loop: all are available at once (saturation).
        keep_outputs: each request gets r.result, a device tensor with its
        output words (in protocol mode the extracted outputs)."""
        t = self.torch
        t.cuda.synchronize()
        start_ev = t.cuda.Event(enable_timing=True)
        start_ev.record(t.cuda.current_stream())
        t.cuda.synchronize()
        t0 = time.perf_counter()
        arrivals = deque(sorted(requests, key=lambda r: r.t_arrival))
        if closed_loop:
            for r in arrivals:
                r.t_arrival = 0.0
        waiting = deque()                       # arrival order
        free = list(range(len(self.streams)))
        inflight = []  # (stream index, event, layer, buffer, requests)
        max_inflight = n_done = launches = 0
        while n_done < len(requests):
            now = time.perf_counter() - t0
            while arrivals and arrivals[0].t_arrival <= now:
                waiting.append(arrivals.popleft())
            # completions free their stream and their buffer
            still = []
            for si, ev, li, buf, rs in inflight:
                if ev.query():
                    done_t = start_ev.elapsed_time(ev) / 1e3
                    for r in rs:
                        r.t_done = done_t
                    self._release(li, buf)
                    free.append(si)
                    n_done += len(rs)
                else:
                    still.append((si, ev, li, buf, rs))
            inflight = still
            # launches: the oldest waiting request's layer, with every other
            # waiting request of that layer, onto any free stream
            while free and waiting:
                li = waiting[0].layer
                buf = self._buffer(li)
                if buf is None:
                    if not inflight:
                        raise MemoryError(f"layer {li} needs more HBM than the budget leaves for launch buffers")
                    break
                group, rest = [], deque()
                for r in waiting:
                    (group if r.layer == li and len(group) < self.max_batch else rest).append(r)
                waiting = rest
                si = free.pop()
                inflight.append((si, self._launch(li, group, buf, self.streams[si], keep_outputs), li, buf, group))
                launches += 1
                max_inflight = max(max_inflight, len(inflight))
            if inflight and not (free and waiting):
                time.sleep(20e-6)
            elif not inflight and not waiting and arrivals:
                time.sleep(max(0.0, min(1e-3, arrivals[0].t_arrival - (time.perf_counter() - t0))))
        t.cuda.synchronize()
        wall = max(r.t_done for r in requests) - min(r.t_arrival for r in requests)
        lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in requests])
        return Stats(n=len(requests), wall_s=wall, layers_per_s=len(requests) / wall,
                     p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                     mean_ms=float(lat.mean()), max_inflight=max_inflight, launches=launches,
                     mean_batch=len(requests) / max(1, launches), latencies_ms=lat.tolist())


def make_layer(ctx: heconv.Context, shape, w_dev) -> Layer:
    """Plan a layer for one image and NTT-preprocess its weights (resident)."""
    import torch
    d = ctx.plan(shape, batch=1)
    s = ctx.sizes(d)
    wntt = torch.empty(s.w_words, dtype=torch.int64, device="cuda")
    ctx.encode_weights(d, w_dev, wntt)
    ct = 2 * ctx.L * ctx.N
    ho, wo = ctx.out_hw(d)
    return Layer(ctx, tuple(shape), d, s, wntt, s.in_cts * ct, s.out_cts * ct,
                 share_words=d.C * d.H * d.W, mask_words=d.M * ho * wo, y_words=d.M * ctx.L * ho * wo)


def poisson_arrivals(rate: float, n: int, u: np.ndarray) -> np.ndarray:
    """Arrival times of an open-loop Poisson process of `rate` per second
    from n uniforms in [0, 1) (inverse-CDF exponential gaps)."""
    gaps = -np.log1p(-u[:n]) / rate
    return np.cumsum(gaps)
