"""Pins for the oracle's BFV client side and whole-layer references (App. C;
Sec. 6.2).

Dec(Enc(m)) = m; the layer through the paper's flow (NTT, MAC in the NTT
domain, inverse NTT) equals the layer by definition (schoolbook products)
word for word; decrypting the layer's output slots gives the plaintext
integer convolution; the RNS/CRT flow agrees with a single-modulus big-integer
mirror; noise stays below delta/2."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mirror
from synth import Stream
from tests import workload as wl


@pytest.mark.parametrize("which", ["4096", "8192"])
def test_encrypt_decrypt_roundtrip(which, prm4096, prm8192):
    p = prm4096 if which == "4096" else prm8192
    sk = wl.secret_key(9, p.N)
    msgs = Stream(9, synth.INPUT).below(2 * p.N, p.t).reshape(2, p.N)
    modes = [oracle.MODE_FAST, oracle.MODE_DEF] if which == "4096" else [oracle.MODE_FAST]
    cts = [wl.encrypt_polys(msgs, p, 9, sk, mode=m) for m in modes]
    for ct in cts[1:]:
        assert np.array_equal(ct, cts[0])  # a*sk by schoolbook == via NTT
    dec, bits = oracle.bfv_decrypt(cts[0], sk, p, with_noise=True)
    want = np.where(msgs >= p.t // 2, msgs.astype(np.int64) - p.t, msgs.astype(np.int64))
    assert np.array_equal(dec, want)
    assert bits <= 8  # fresh noise: centred binomial, |e| <= 21


def test_cfg1_layer_end_to_end(prm4096):
    """4->4 3x3 conv @16x16: encrypt, layer by the NTT flow and by the
    definition, decrypt; equals the exact integer convolution (|y| < t/2)."""
    cfg = synth.WORKLOADS["conv4_16x16"]
    p = prm4096
    cv = wl.conv_of(cfg["layers"][0])
    g = oracle.plan_conv(cv, p.N, p.L)
    x, K = wl.draw_layer(cfg, cfg["layers"][0])
    sk = wl.secret_key(cfg["seed"], p.N)
    ct = wl.encrypt_input(x, cv, g, p, cfg["seed"], sk)[None]  # [1][CB][S][2][L][N]
    wc = oracle.pack_weights(K, cv, g, p)
    w_ntt = oracle.ntt(wc, p)
    assert np.array_equal(w_ntt, oracle.encode_weights(K, cv, g, p, oracle.MODE_DEF))
    out_fast = oracle.conv_layer_ntt(ct, w_ntt, 1, g, cv.M, p)
    out_def = oracle.conv_layer_def(ct, wc, 1, g, cv.M, p)
    assert np.array_equal(out_fast, out_def)
    for (m, s, c, l, k) in [(0, 0, 0, 0, 0), (3, 0, 1, 1, 4095), (2, 0, 1, 0, g.O)]:
        assert oracle.conv_layer_coeff(ct, wc, g, p, 0, m, s, c, l, k) == int(out_def[0, m, s, c, l, k])
    y, bits = wl.decrypt_output(out_fast[0], cv, g, p, sk, with_noise=True)
    want = oracle.plain_conv(x, K, cv.stride, cv.pad)
    assert np.abs(want).max() < p.t // 2
    assert np.array_equal(y, want)
    assert bits < p.delta.bit_length() - 1


def test_rns_flow_matches_bigint_mirror():
    """N = 64, L = 2: the RNS oracle (per-limb products, CRT at decryption)
    and the mirror over the single modulus Q give the same phase and the same
    decrypted conv."""
    N = 64
    p = oracle.Params(N, 2, 50, 2 ** 37)
    cv = oracle.Conv(1, 4, 4, 2, 3, 3, 1, 1)
    g = oracle.plan_conv(cv, N, 2)
    assert g.CB == 1 and g.S == 1
    x = Stream(3, 4).ints(16, -100, 100).reshape(1, 4, 4)
    K = Stream(3, 5).ints(18, -100, 100).reshape(2, 1, 3, 3)
    sk = wl.secret_key(3, N)
    pin = oracle.pack_input(x, cv, g, p.t, N).reshape(1, N)
    a = synth.uniform_mod(Stream(3, synth.UNIFORM), (1, 2, N), p.q)
    e = Stream(3, synth.ERROR).cbd(N, wl.ETA).reshape(1, N)
    ct = oracle.bfv_encrypt(pin, sk, a, e, p)
    wc = oracle.pack_weights(K, cv, g, p)
    out = oracle.conv_layer_ntt(ct.reshape(1, 1, 1, 2, 2, N), oracle.ntt(wc, p), 1, g, cv.M, p)
    # mirror over Q
    a_big = [int(v) for v in oracle.crt(np.moveaxis(a[0], 0, 1), p)]
    ct_big = mirror.bfv_encrypt([int(v) for v in pin[0]], [int(v) for v in sk], a_big, [int(v) for v in e[0]],
                                p.Q, p.t)
    for m in range(cv.M):
        wpoly = [0] * N
        for c in range(1):
            for i in range(3):
                for j in range(3):
                    wpoly[g.O - i * g.Ww - j] = int(K[m, c, i, j])
        prod = mirror.ct_mul_plain(ct_big, wpoly, p.Q)
        for comp in range(2):
            rns = oracle.crt(np.moveaxis(out[0, m, 0, comp], 0, 1), p)
            assert [int(v) for v in rns] == prod[comp]
        dec_m = mirror.bfv_decrypt(prod, [int(v) for v in sk], p.Q, p.t)
        dec_o = oracle.bfv_decrypt(out[0, m, 0][None], sk, p)[0]
        assert [int(v) for v in dec_o] == dec_m
    y = wl.decrypt_output(out[0], cv, g, p, sk)
    assert np.array_equal(y, oracle.plain_conv(x, K, 1, 1))


@pytest.mark.slow
def test_cfg2_layer_decrypts_to_conv(prm8192):
    """64->64 3x3 @56x56, N=8192, L=3: oracle NTT flow, decrypted, equals the
    exact integer convolution; sampled words equal the definition."""
    cfg = synth.WORKLOADS["conv64_56x56"]
    p = prm8192
    shape = cfg["layers"][0]
    cv = wl.conv_of(shape)
    g = oracle.plan_conv(cv, p.N, p.L)
    x, K = wl.draw_layer(cfg, shape)
    sk = wl.secret_key(cfg["seed"], p.N)
    ct = wl.encrypt_input(x, cv, g, p, cfg["seed"], sk)[None]
    wc = oracle.pack_weights(K, cv, g, p)
    out = oracle.conv_layer_ntt(ct, oracle.ntt(wc, p), 1, g, cv.M, p)
    rng = Stream(77, 7)
    for _ in range(6):
        m, s, c, l, k = (int(rng.below(1, v)[0]) for v in (cv.M, g.S, 2, p.L, p.N))
        assert oracle.conv_layer_coeff(ct, wc, g, p, 0, m, s, c, l, k) == int(out[0, m, s, c, l, k])
    y, bits = wl.decrypt_output(out[0], cv, g, p, sk, with_noise=True)
    want = oracle.plain_conv(x, K, 1, 1)
    assert np.abs(want).max() < p.t // 2
    assert np.array_equal(y, want)
    assert bits < 100


def test_odd_plaintext_modulus_centres_symmetrically(prm4096):
    """For an odd t the centred range [-t/2, t/2) is -(t-1)/2 .. (t-1)/2:
    (t-1)/2 stays positive and (t+1)/2 becomes -(t-1)/2, through decryption
    and through centre_mod alike (t = 7 written out)."""
    assert list(oracle.centre_mod(np.arange(7), 7)) == [0, 1, 2, 3, -3, -2, -1]
    assert list(oracle.centre_mod(np.arange(8), 8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    N = prm4096.N
    t = oracle.find_primes(N, 37, 1)[0]  # a prime plaintext modulus, t = 1 mod 2N
    p = oracle.Params(N, prm4096.L, prm4096.bits, t, q=prm4096.q)
    sk = wl.secret_key(10, N)
    msgs = Stream(10, synth.INPUT).below(N, t).reshape(1, N)
    msgs[0, :4] = [(t - 1) // 2, (t + 1) // 2, 0, t - 1]
    dec = oracle.bfv_decrypt(wl.encrypt_polys(msgs, p, 10, sk), sk, p)
    assert list(dec[0, :4]) == [(t - 1) // 2, -(t - 1) // 2, 0, -1]
    m = msgs.astype(object)
    assert np.array_equal(dec, np.where(2 * m >= t, m - t, m).astype(np.int64))
