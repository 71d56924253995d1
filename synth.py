"""Seeded synthetic input generators.

This module is the only code that the product path and the CPU oracle both
use.  It holds no arithmetic of the method: it only turns a (seed, purpose)
pair into reproducible random integers.  Random numbers that encryption draws
(the secret key, the uniform `a` polynomials, the error) are made here and
passed to the oracle as inputs.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  It is counter based: output k of a stream
with start state s0 is mix(s0 + (k + 1) * GAMMA), so whole arrays are made at
once with wrapping uint64 arithmetic.  One stream per (workload seed, purpose);
the start state is (seed << 8) | purpose.

Purposes: 1 secret key, 2 uniform a-polynomials / ciphertext words,
3 errors, 4 inputs (activations), 5 weights, 6 arrival times, 7 request mix.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

KEY, UNIFORM, ERROR, INPUT, WEIGHT, ARRIVAL, MIX = 1, 2, 3, 4, 5, 6, 7
SHARE, MASK, FLOOD = 8, 9, 10  # server input share, server output share (mask), smudging noise


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


class Stream:
    """One SplitMix64 stream; draws continue where the previous draw ended."""

    def __init__(self, seed: int, purpose: int):
        self.state = np.uint64(((int(seed) << 8) | int(purpose)) & 0xFFFFFFFFFFFFFFFF)
        self.count = 0

    def words(self, n: int) -> np.ndarray:
        """n raw 64-bit outputs."""
        k = np.arange(self.count + 1, self.count + 1 + n, dtype=np.uint64)
        self.count += n
        with np.errstate(over="ignore"):
            return _mix(self.state + k * GAMMA)

    def below(self, n: int, bound: int) -> np.ndarray:
        """n values uniform in [0, bound), 1 <= bound <= 2^64, by rejection on
        the top bits: a word's top bit_length(bound-1) bits are kept and
        values >= bound are discarded."""
        bound = int(bound)
        if bound == 1:
            return np.zeros(n, dtype=np.uint64)
        bits = (bound - 1).bit_length()
        out = np.empty(0, dtype=np.uint64)
        while out.size < n:
            need = n - out.size
            w = self.words(need + need // 2 + 16) >> np.uint64(64 - bits)
            if bound < (1 << 64):
                w = w[w < np.uint64(bound)]
            out = np.concatenate([out, w])
        return out[:n]

    def ints(self, n: int, lo: int, hi: int) -> np.ndarray:
        """n signed integers uniform in [lo, hi) as int64."""
        return (self.below(n, hi - lo).astype(np.int64) + np.int64(lo))

    def ternary(self, n: int) -> np.ndarray:
        """n values uniform in {-1, 0, 1} (int64)."""
        return self.below(n, 3).astype(np.int64) - 1

    def cbd(self, n: int, eta: int) -> np.ndarray:
        """n samples of the centred binomial distribution with parameter eta
        (variance eta/2): popcount of eta bits minus popcount of the next eta
        bits of one word.  Needs 2*eta <= 64."""
        assert 2 * eta <= 64
        w = self.words(n)
        mask = np.uint64((1 << eta) - 1)
        lo = w & mask
        hi = (w >> np.uint64(eta)) & mask
        return _popcount(lo) - _popcount(hi)

    def uniform_f64(self, n: int) -> np.ndarray:
        """n doubles uniform in [0, 1) from the top 53 bits."""
        return (self.words(n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def _popcount(x: np.ndarray) -> np.ndarray:
    return np.bitwise_count(x.astype(np.uint64)).astype(np.int64)


def uniform_mod(stream: Stream, shape, moduli) -> np.ndarray:
    """Array of `shape` whose axis -2 runs over RNS limbs: entry [..., l, k] is
    uniform in [0, moduli[l]).  shape[-2] must equal len(moduli)."""
    shape = tuple(int(s) for s in shape)
    L = shape[-2]
    assert L == len(moduli)
    out = np.empty(shape, dtype=np.uint64)
    lead = int(np.prod(shape[:-2])) if len(shape) > 2 else 1
    view = out.reshape(lead, L, shape[-1])
    for i in range(lead):
        for l in range(L):
            view[i, l] = stream.below(shape[-1], int(moduli[l]))
    return out


# --------------------------------------------------------------------------
# Workload recipes: layer shapes, HE parameter sizes, value ranges and seeds.
# Pure data; each consumer derives its own parameters from (N, L, bits, t).
# --------------------------------------------------------------------------
T_BITS = 37  # plaintext modulus t = 2^37 (37-bit fixed point)


def conv(C, H, W, M, k, stride=1, pad=0):
    """Layer shape tuple (C, H, W, M, kh, kw, stride, pad)."""
    return (C, H, W, M, k, k, stride, pad)


def fire_cnn_layers():
    """Fire-module CNN at 3x224x224 (26 convolutions).  conv1 3x3/2 pad 1;
    the 3x3/2 max-pools between stages (not computed here) take the spatial
    size 112 -> 55 -> 27 -> 13."""
    L = [conv(3, 224, 224, 64, 3, 2, 1)]
    fires = [  # (input channels, spatial, squeeze, expand)
        (64, 55, 16, 64), (128, 55, 16, 64), (128, 27, 32, 128), (256, 27, 32, 128),
        (256, 13, 48, 192), (384, 13, 48, 192), (384, 13, 64, 256), (512, 13, 64, 256)]
    for cin, hw, sq, ex in fires:
        L.append(conv(cin, hw, hw, sq, 1))
        L.append(conv(sq, hw, hw, ex, 1))
        L.append(conv(sq, hw, hw, ex, 3, 1, 1))
    L.append(conv(512, 13, 13, 1000, 1))
    return L


def bottleneck_cnn_layers():
    """Bottleneck residual CNN at 3x224x224 (53 convolutions): stem 7x7/2
    pad 3, max-pool to 56, stages of 3/4/6/3 blocks of widths 64/128/256/512
    with expansion 4, stride 2 on the 3x3 of the first block of stages 2-4,
    and a 1x1 projection shortcut on each stage's first block."""
    L = [conv(3, 224, 224, 64, 7, 2, 3)]
    cin, hw = 64, 56
    for si, (blocks, width) in enumerate([(3, 64), (4, 128), (6, 256), (3, 512)]):
        for b in range(blocks):
            s = 2 if (b == 0 and si > 0) else 1
            L.append(conv(cin, hw, hw, width, 1))
            L.append(conv(width, hw, hw, width, 3, s, 1))
            ho = (hw + 2 - 3) // s + 1
            L.append(conv(width, ho, ho, 4 * width, 1))
            if b == 0:
                L.append(conv(cin, hw, hw, 4 * width, 1, s, 0))
            cin, hw = 4 * width, ho
    return L


WORKLOADS = {
    "conv4_16x16": dict(name="single 3x3 conv 4->4 @16x16, N=4096, L=2x50-bit", layers=[conv(4, 16, 16, 4, 3, 1, 1)],
            N=4096, L=2, bits=50, batch=1, x_range=(-2 ** 7, 2 ** 7), w_range=(-2 ** 7, 2 ** 7), seed=1),
    "conv64_56x56": dict(name="3x3 conv 64->64 @56x56, N=8192, L=3x60-bit", layers=[conv(64, 56, 56, 64, 3, 1, 1)],
            N=8192, L=3, bits=60, batch=1, x_range=(-2 ** 12, 2 ** 12), w_range=(-2 ** 8, 2 ** 8), seed=2),
    "fire_cnn": dict(name="fire-module CNN, 26 convs @224, B=1", layers=fire_cnn_layers(),
            N=8192, L=3, bits=60, batch=1, x_range=(0, 2 ** 37), w_range=(-2 ** 12, 2 ** 12), seed=3),
    "bottleneck_cnn_b16": dict(name="bottleneck residual CNN, 53 convs @224, B=16", layers=bottleneck_cnn_layers(),
            N=8192, L=3, bits=60, batch=16, x_range=(0, 2 ** 37), w_range=(-2 ** 12, 2 ** 12), seed=4),
}
