"""Pins for the oracle's protocol steps either side of the layer (Sec. 7:
the server adds its share of the input to the client's ciphertexts, runs the
linear layer, masks the result; Sec. 6.2: only the output coefficients are
extracted).

The pins use the protocol's own invariants, computed through decryption and
the plaintext integer convolution, not through the functions under test:
  - the ciphertext with the server's share added decrypts to the packing of
    (client share + server share) mod t;
  - client output share + server output share = conv(x) mod t, for every
    stride / 1x1-subsampling case of the packing;
  - a smudging term of +delta (or -delta) moves the client's output by
    exactly +1 (or -1);
  - extraction reads the same positions as the output assembly."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests import workload as wl

T = 2 ** synth.T_BITS


def _shares(seed, shape, t):
    """Two additive shares of a random tensor, each uniform in [0, t)."""
    xc = Stream(seed, synth.INPUT).below(int(np.prod(shape)), t).astype(np.int64).reshape(shape)
    xs = Stream(seed, synth.SHARE).below(int(np.prod(shape)), t).astype(np.int64).reshape(shape)
    return xc, xs


def test_add_share_decrypts_to_sum(prm4096):
    p = prm4096
    cv = oracle.Conv(4, 16, 16, 4, 3, 3, 1, 1)
    g = oracle.plan_conv(cv, p.N, p.L)
    sk = wl.secret_key(21, p.N)
    xc, xs = _shares(21, (cv.C, cv.H, cv.W), p.t)
    ct = wl.encrypt_input(xc, cv, g, p, 21, sk)
    ct2 = oracle.add_share(ct, xs, cv, g, p)
    assert np.array_equal(ct2[:, :, 0], ct[:, :, 0])  # a untouched
    dec = oracle.bfv_decrypt(ct2.reshape(-1, 2, p.L, p.N), sk, p).reshape(g.CB, g.S, p.N)
    want = oracle.centre_mod(oracle.pack_input(xc, cv, g, p.t, p.N).astype(object) +
                             oracle.pack_input(xs, cv, g, p.t, p.N).astype(object), p.t)
    assert np.array_equal(dec, want)


def test_add_share_zero_is_identity(prm4096):
    p = prm4096
    cv = oracle.Conv(3, 9, 11, 2, 3, 3, 1, 1)
    g = oracle.plan_conv(cv, p.N, p.L)
    ct = synth.uniform_mod(Stream(22, synth.UNIFORM), (g.CB, g.S, 2, p.L, p.N), p.q)
    assert np.array_equal(oracle.add_share(ct, np.zeros((3, 9, 11), np.int64), cv, g, p), ct)
    # a share of t is the zero share too (values are taken mod t)
    assert np.array_equal(oracle.add_share(ct, np.full((3, 9, 11), p.t, np.int64), cv, g, p), ct)


# (C, H, W, M, k, stride, pad): stride 1, strided 3x3 (stride-1 result
# subsampled), strided 1x1 (input subsampled first), 5x5, no padding
PROTO_SHAPES = [(4, 16, 16, 4, 3, 1, 1), (3, 15, 13, 5, 3, 2, 1), (6, 14, 14, 3, 1, 2, 0), (2, 12, 12, 2, 5, 1, 2),
                (5, 10, 9, 3, 3, 1, 0)]


@pytest.mark.parametrize("shape", PROTO_SHAPES)
def test_shares_reconstruct_the_convolution(shape, prm4096):
    """Client encrypts its share, server adds its share, runs the layer
    (by definition), masks with R and extracts; the client's decryption plus
    R equals the plaintext conv of the full input, mod t."""
    p = prm4096
    C, H, W, M, k, stride, pad = shape
    cv = oracle.Conv(C, H, W, M, k, k, stride, pad)
    g = oracle.plan_conv(cv, p.N, p.L)
    sk = wl.secret_key(23, p.N)
    xc, xs = _shares(23, (C, H, W), p.t)
    K = Stream(23, synth.WEIGHT).ints(M * C * k * k, -2 ** 7, 2 ** 7).reshape(M, C, k, k)
    ct = oracle.add_share(wl.encrypt_input(xc, cv, g, p, 23, sk), xs, cv, g, p)
    out = oracle.conv_layer_def(ct[None], oracle.pack_weights(K, cv, g, p), 1, g, M, p)[0]
    R = Stream(23, synth.MASK).below(M * g.Ho * g.Wo, p.t).astype(np.int64).reshape(M, g.Ho, g.Wo)
    y = oracle.mask_extract(out, R, None, cv, g, p)
    assert y.shape == (M, p.L, g.Ho, g.Wo)
    client = oracle.decrypt_extracted(out[:, :, 0], y, sk, cv, g, p)
    want = oracle.plain_conv(xc + xs, K, stride, pad)
    assert want.shape == client.shape
    assert np.array_equal(np.mod(client.astype(object) + R, p.t), np.mod(want, p.t).astype(object))


def test_extract_without_mask_equals_output_decryption(prm4096):
    p = prm4096
    cfg = synth.WORKLOADS["conv4_16x16"]
    cv = wl.conv_of(cfg["layers"][0])
    g = oracle.plan_conv(cv, p.N, p.L)
    x, K = wl.draw_layer(cfg, cfg["layers"][0])
    sk = wl.secret_key(24, p.N)
    ct = wl.encrypt_input(x, cv, g, p, 24, sk)
    out = oracle.conv_layer_ntt(ct[None], oracle.encode_weights(K, cv, g, p), 1, g, cv.M, p)[0]
    y = oracle.mask_extract(out, np.zeros((cv.M, g.Ho, g.Wo), np.int64), None, cv, g, p)
    assert np.array_equal(oracle.decrypt_extracted(out[:, :, 0], y, sk, cv, g, p), wl.decrypt_output(out, cv, g, p, sk))
    assert np.array_equal(wl.decrypt_output(out, cv, g, p, sk), oracle.plain_conv(x, K, 1, 1))


def test_smudging_term_sign_and_position():
    """With 40-bit primes delta fits an int64: a smudging term of +delta at one
    output moves that output (and only it) by +1, -delta by -1."""
    p = oracle.Params(4096, 2, 40, T)
    assert p.delta < 2 ** 62
    cv = oracle.Conv(2, 8, 8, 2, 3, 3, 1, 1)
    g = oracle.plan_conv(cv, p.N, p.L)
    sk = wl.secret_key(25, p.N)
    x = Stream(25, synth.INPUT).ints(2 * 64, -50, 50).reshape(2, 8, 8)
    K = Stream(25, synth.WEIGHT).ints(2 * 2 * 9, -9, 9).reshape(2, 2, 3, 3)
    out = oracle.conv_layer_def(wl.encrypt_input(x, cv, g, p, 25, sk)[None], oracle.pack_weights(K, cv, g, p), 1, g,
                                2, p)[0]
    R = np.zeros((2, g.Ho, g.Wo), np.int64)
    base = oracle.decrypt_extracted(out[:, :, 0], oracle.mask_extract(out, R, None, cv, g, p), sk, cv, g, p)
    assert np.array_equal(base, oracle.plain_conv(x, K, 1, 1))
    for sign in (1, -1):
        e = np.zeros_like(R)
        e[1, 3, 5] = sign * p.delta
        got = oracle.decrypt_extracted(out[:, :, 0], oracle.mask_extract(out, R, e, cv, g, p), sk, cv, g, p)
        d = got - base
        assert d[1, 3, 5] == sign and np.count_nonzero(d) == 1


@pytest.mark.parametrize("shape", PROTO_SHAPES)
def test_output_coeffs_match_assembly(shape, prm4096):
    C, H, W, M, k, stride, pad = shape
    cv = oracle.Conv(C, H, W, M, k, k, stride, pad)
    g = oracle.plan_conv(cv, prm4096.N, prm4096.L)
    slots = oracle.output_slots(g)
    ids = (np.arange(g.S)[:, None] * prm4096.N + slots[None, :])[None]  # [1][S][bh*bw]: s*N + coefficient
    full = oracle.assemble_output(ids, cv, g)[0]
    s, kk = oracle.output_coeffs(cv, g)
    assert np.array_equal(full, s * prm4096.N + kk)
