"""Request server for single-layer HE convolutions: continuous batching over
a pool of HIP streams with weights resident in HBM.

Each request is one layer solve (one image) of a resident layer: its input
ciphertexts arrive in host memory, are copied into a device slot, and the
layer's NTT -> MAC -> iNTT runs on the device; results stay resident in the
request's output slot.  In protocol mode (the server's whole step for a
linear layer in the online protocol, Sec. 7) a request also brings the
server's input share and output mask: the share is folded into the input
ciphertexts before the layer, and the output is masked and reduced to the
coefficients that hold results (he_add_share, he_conv_layer,
he_mask_extract).  The dispatcher admits requests as they arrive, as
long as the HBM budget allows their slots, and puts them on any free
stream, so requests that arrive while others are on the GPU run alongside
them.  Latency is arrival -> device completion, measured on the GPU timeline with
events.  Each request runs as one he_conv_layer call (which allocates
nothing) on its stream; grouping queued requests into one he_batch would
allocate and free device memory per group, and a device free synchronises
every stream, so the server does not group.

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
    slot: tuple = None
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
    latencies_ms: list = field(default_factory=list)


class Server:
    """Resident layers + slot pools + a stream pool."""

    def __init__(self, layers: list[Layer], n_streams: int = 4, hbm_budget: float = 200e9, protocol: bool = False):
        import torch
        self.torch = torch
        self.protocol = protocol
        self.layers = layers
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]  # default priority
        self.budget = float(hbm_budget)
        self.resident = sum(l.wntt.numel() * 8 for l in layers)
        if self.resident > self.budget:
            raise MemoryError(f"weights ({self.resident / 1e9:.1f} GB) exceed the HBM budget")
        self.used = self.resident
        self.free_slots = {i: [] for i in range(len(layers))}

    # -- slots ---------------------------------------------------------------
    def _slot_words(self, L: Layer) -> list[int]:
        w = [L.in_words, L.out_words]
        if self.protocol:
            w += [L.share_words, L.mask_words, L.y_words]
        return w

    def _slot(self, li: int):
        """(d_in, d_out[, d_share, d_mask, d_y]) for layer li from the pool,
        or a new set if the budget allows; None when it does not."""
        if self.free_slots[li]:
            return self.free_slots[li].pop()
        L = self.layers[li]
        need = sum(self._slot_words(L)) * 8
        # idle slots of other layers give their memory back first
        for lj, pool in self.free_slots.items():
            while pool and self.used + need > self.budget:
                pool.pop()
                self.used -= sum(self._slot_words(self.layers[lj])) * 8
        if self.used + need > self.budget:
            return None
        self.used += need
        t = self.torch
        return tuple(t.empty(w, dtype=t.int64, device="cuda") for w in self._slot_words(L))

    def _release(self, li: int, slot):
        self.free_slots[li].append(slot)

    # -- one request on one stream -------------------------------------------
    def _launch(self, r: Request, stream):
        t = self.torch
        L = self.layers[r.layer]
        with t.cuda.stream(stream):
            r.slot[0].copy_(r.host_in, non_blocking=True)
            if self.protocol:
                r.slot[2].copy_(r.host_share, non_blocking=True)
                r.slot[3].copy_(r.host_mask, non_blocking=True)
                L.ctx.add_share(L.desc, 1, r.slot[0], r.slot[2], stream=stream)
            L.ctx.conv_layer(L.desc, 1, r.slot[0], L.wntt, r.slot[1], stream=stream)
            if self.protocol:
                L.ctx.mask_extract(L.desc, 1, r.slot[1], r.slot[3], None, r.slot[4], stream=stream)
            ev = t.cuda.Event(enable_timing=True)
            ev.record(stream)
        return ev

    def run(self, requests: list[Request], closed_loop: bool = False, keep_outputs: bool = False) -> Stats:
        """Serve `requests`.  Open loop: a request becomes available at its
        arrival time.  Closed loop: all are available at once (saturation).
        keep_outputs: completed requests keep their slot (r.slot[1] holds the
        result after the run, and in protocol mode r.slot[4] the extracted
        outputs) instead of returning it to the pool."""
        t = self.torch
        t.cuda.synchronize()
        start_ev = t.cuda.Event(enable_timing=True)
        start_ev.record(t.cuda.current_stream())
        t.cuda.synchronize()
        t0 = time.perf_counter()
        pending = deque()
        arrivals = deque(sorted(requests, key=lambda r: r.t_arrival))
        if closed_loop:
            for r in arrivals:
                r.t_arrival = 0.0
        free = list(range(len(self.streams)))
        inflight = []  # (stream index, event, request)
        max_inflight = 0
        n_done = 0
        while n_done < len(requests):
            now = time.perf_counter() - t0
            while arrivals and arrivals[0].t_arrival <= now:
                pending.append(arrivals.popleft())
            # completions free their stream and their slot
            still = []
            for si, ev, r in inflight:
                if ev.query():
                    r.t_done = start_ev.elapsed_time(ev) / 1e3
                    if not keep_outputs:
                        self._release(r.layer, r.slot)
                        r.slot = None
                    free.append(si)
                    n_done += 1
                else:
                    still.append((si, ev, r))
            inflight = still
            # admissions: FIFO, onto any free stream, while the budget allows
            while free and pending:
                r = pending[0]
                slot = self._slot(r.layer)
                if slot is None:
                    if not inflight:
                        raise MemoryError(f"request {r.rid} needs more HBM than the budget leaves for slots")
                    break
                pending.popleft()
                r.slot = slot
                si = free.pop()
                inflight.append((si, self._launch(r, self.streams[si]), r))
                max_inflight = max(max_inflight, len(inflight))
            if inflight and not (free and pending):
                time.sleep(20e-6)
            elif not inflight and not pending and arrivals:
                time.sleep(max(0.0, min(1e-3, arrivals[0].t_arrival - (time.perf_counter() - t0))))
        t.cuda.synchronize()
        wall = max(r.t_done for r in requests) - min(r.t_arrival for r in requests)
        lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in requests])
        return Stats(n=len(requests), wall_s=wall, layers_per_s=len(requests) / wall,
                     p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                     mean_ms=float(lat.mean()), max_inflight=max_inflight, latencies_ms=lat.tolist())


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
