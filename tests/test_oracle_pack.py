"""Pins for the packing (coefficient encoding of a conv into ring products)
and the planner.

The paper only says messages are placed in the coefficients so that a
polynomial product computes the dot products (Sec. 2.3, Cheetah paragraph;
Sec. 6.1).  The layout used is the library's reading; it is pinned here by
brute force: packed ring products, extracted, equal the plaintext integer
convolution for strides 1/2, pads 0/1/2/3, kernels 1/3/5/7 and several
tilings, and the plaintext convolution is itself pinned to scipy."""
import numpy as np
import pytest
import scipy.signal

import oracle
from oracle import Conv
from synth import Stream


def test_plain_conv_matches_scipy():
    rng = Stream(11, 4)
    x = rng.ints(3 * 9 * 8, -50, 50).reshape(3, 9, 8)
    K = rng.ints(2 * 3 * 3 * 3, -9, 9).reshape(2, 3, 3, 3)
    for stride, pad in [(1, 0), (1, 1), (2, 1), (2, 0), (3, 2)]:
        y = oracle.plain_conv(x, K, stride, pad)
        xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad)))
        for m in range(2):
            full = sum(scipy.signal.correlate2d(xp[c], K[m, c], mode="valid") for c in range(3))
            assert np.array_equal(y[m], full[::stride, ::stride]), (stride, pad)


def ring_conv(x, K, cv, g, q, N):
    """Packed product over Z_q[X]/(X^N+1) with small values, extracted and
    centred: sum_cb pack_in[cb][s] * pack_w[m][cb], slots O + i*Ww + j."""
    prm = oracle.Params(N, 1, 50, 2 ** 37, q=[q], psi=[oracle.find_psi(q, N)])
    pin = oracle.pack_input(x, cv, g, 2 ** 60, N).astype(np.uint64)  # small signed values: mod 2^60
    pin = np.where(pin >= 2 ** 59, pin.astype(object) - 2 ** 60 + q, pin.astype(object)).astype(np.uint64)
    wc = oracle.pack_weights(K, cv, g, prm)  # [M][CB][1][N]
    ct = np.stack([pin, pin], axis=2)[None, :, :, :, None, :]  # [1][CB][S][2][1][N]
    out = oracle.conv_layer_def(np.ascontiguousarray(ct), wc, 1, g, cv.M, prm)  # [1][M][S][2][1][N]
    assert np.array_equal(out[0, :, :, 0], out[0, :, :, 1])
    slots = oracle.output_slots(g)
    vals = out[0, :, :, 0, 0][:, :, slots].astype(object)
    vals = np.where(vals > q // 2, vals - q, vals).astype(np.int64)
    return oracle.assemble_output(vals, cv, g)


SHAPES = [
    Conv(2, 5, 5, 3, 3, 3, 1, 1),
    Conv(3, 7, 6, 2, 3, 3, 2, 1),
    Conv(3, 6, 7, 2, 3, 3, 1, 0),
    Conv(4, 6, 6, 2, 1, 1, 2, 0),
    Conv(5, 5, 5, 3, 1, 1, 1, 0),
    Conv(3, 9, 9, 2, 5, 5, 2, 2),
    Conv(2, 11, 11, 2, 7, 7, 2, 3),
    Conv(3, 7, 7, 2, 1, 1, 3, 0),
]


@pytest.mark.parametrize("cv", SHAPES, ids=str)
def test_packed_ring_product_equals_conv(cv):
    N = 256
    q = oracle.find_primes(N, 50, 1)[0]
    rng = Stream(cv.C * 100 + cv.H, 4)
    x = rng.ints(cv.C * cv.H * cv.W, -20, 20).reshape(cv.C, cv.H, cv.W)
    K = rng.ints(cv.M * cv.C * cv.kh * cv.kw, -6, 6).reshape(cv.M, cv.C, cv.kh, cv.kw)
    want = oracle.plain_conv(x, K, cv.stride, cv.pad)
    g = oracle.plan_conv(cv, N, 1)
    assert g.Cw * g.Hw * g.Ww <= N
    assert np.array_equal(ring_conv(x, K, cv, g, q, N), want)
    # forced small tiles and channel blocks: ragged edges, several tiles and blocks
    g0 = oracle.geometry(cv, 1, cv.kh, cv.kw)
    for Cw, Hw, Ww in [(1, cv.kh + 1, cv.kw + 2), (2, cv.kh + 2, cv.kw), (min(cv.C, 3), cv.kh + 3, cv.kw + 1)]:
        Hw, Ww = min(Hw, g0.He), min(Ww, g0.We)
        if Cw * Hw * Ww > N:
            continue
        g = oracle.geometry(cv, Cw, Hw, Ww)
        assert np.array_equal(ring_conv(x, K, cv, g, q, N), want), (Cw, Hw, Ww)


def test_delta_kernel_and_scalar():
    """A centred delta kernel returns the input; a 1x1 kernel with Cw = 1 is
    a scalar multiple per channel."""
    N = 256
    q = oracle.find_primes(N, 50, 1)[0]
    cv = Conv(2, 6, 6, 2, 3, 3, 1, 1)
    x = Stream(5, 4).ints(2 * 36, -30, 30).reshape(2, 6, 6)
    K = np.zeros((2, 2, 3, 3), dtype=np.int64)
    K[0, 0, 1, 1] = 1
    K[1, 1, 1, 1] = 1
    g = oracle.plan_conv(cv, N, 1)
    assert np.array_equal(ring_conv(x, K, cv, g, q, N), x)
    cv1 = Conv(2, 6, 6, 2, 1, 1, 1, 0)
    K1 = np.array([[[[3]], [[0]]], [[[0]], [[-2]]]], dtype=np.int64)
    g1 = oracle.geometry(cv1, 1, 6, 6)
    y = ring_conv(x, K1, cv1, g1, q, N)
    assert np.array_equal(y[0], 3 * x[0]) and np.array_equal(y[1], -2 * x[1])


def test_planner_choices():
    """The bytes-objective planner on the two single-layer workloads.
    4->4 3x3 @16x16 pad 1, N=4096: one 18x18 window of all 4 channels fits
    (4*324 <= 4096): Cw=4, 18x18, CB=S=1.
    64->64 3x3 @56x56 pad 1, N=8192, L=3: cost/(L*N*8) = M*CB + 6*S*(CB+M);
    Cw=4 (CB=16) with two 58-row tiles costs 1024 + 12*80 = 1984, below
    Cw=2 (2624), Cw=5 (2218) and Cw=8 (2240); among the Cw=4, S=2 windows
    the largest height 58 wins, then the largest width with 4*58*Ww <= 8192,
    Ww=35."""
    g = oracle.plan_conv(Conv(4, 16, 16, 4, 3, 3, 1, 1), 4096, 2)
    assert (g.Cw, g.Hw, g.Ww, g.CB, g.S) == (4, 18, 18, 1, 1)
    g = oracle.plan_conv(Conv(64, 56, 56, 64, 3, 3, 1, 1), 8192, 3)
    assert (g.Cw, g.Hw, g.Ww, g.CB, g.S, g.bh, g.bw) == (4, 58, 35, 16, 2, 56, 33)
    byts, _ = oracle.layer_cost(Conv(64, 56, 56, 64, 3, 3, 1, 1), g, 8192, 3, 1)
    assert byts == 1984 * 3 * 8192 * 8


def test_output_slots_do_not_wrap():
    """Every output slot index is below N and at or above O, and the largest
    product index that wraps lands below O (Cw*Hw*Ww <= N)."""
    cv = Conv(64, 56, 56, 64, 3, 3, 1, 1)
    g = oracle.plan_conv(cv, 8192, 3)
    s = oracle.output_slots(g)
    assert s.min() == g.O and s.max() < 8192
    max_in = g.Cw * g.Hw * g.Ww - 1
    assert max_in + g.O - 8192 < g.O


def test_weight_lift_of_int64_extremes():
    """The signed lift of every kernel value into [0, q_l) is the integer
    residue v mod q_l, including the int64 extremes and values above q_l;
    each value lands at coefficient O - cc*Hw*Ww - i*Ww - j of its block."""
    prm = oracle.Params(8192, 3, 60, 2 ** 37)
    cv = Conv(3, 4, 4, 2, 2, 2, 1, 0)
    g = oracle.geometry(cv, 2, 4, 4)
    vals = [-2 ** 63, 2 ** 63 - 1, -1, 0, prm.q[0], prm.q[1] + 5, -prm.q[2] - 7, 12345, -2 ** 12, 2 ** 12 - 1]
    K = np.array([vals[k % len(vals)] for k in range(2 * 3 * 2 * 2)], dtype=np.int64).reshape(2, 3, 2, 2)
    wc = oracle.pack_weights(K, cv, g, prm)
    seen = np.zeros(wc.shape, dtype=bool)
    for m in range(2):
        for c in range(3):
            cb, cc = divmod(c, g.Cw)
            for i in range(2):
                for j in range(2):
                    idx = g.O - cc * 16 - i * 4 - j
                    for l, q in enumerate(prm.q):
                        assert int(wc[m, cb, l, idx]) == int(K[m, c, i, j]) % q
                        seen[m, cb, l, idx] = True
    assert not wc[~seen].any()
