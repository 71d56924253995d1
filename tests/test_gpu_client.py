"""GPU parity of the client-side BFV steps (App. C): key transform,
encryption word for word against the oracle's encryption, and decryption
against the oracle's exact big-integer CRT decoding -- on fresh
encryptions, on layer outputs (grown noise), and on arbitrary words."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests import workload as wl
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built

pytestmark = pytest.mark.gpu
_cache = {}

PARAMS = [(4096, 2, 50), (8192, 3, 60), (2048, 4, 40), (16384, 2, 60)]


def ctx_and_prm(N, L, bits, t=2 ** 37):
    key = (N, L, bits, t)
    if key not in _cache:
        require_gpu()
        ensure_built()
        from paper_2506_11586_amd import heconv
        _cache[key] = (heconv.Context(N, heconv.gen_primes(N, bits, L), t), oracle.Params(N, L, bits, t))
    return _cache[key]


def key_ntt(ctx, prm, sk):
    d = empty_words(prm.L * prm.N)
    ctx.key_encode(to_dev(np.asarray(sk, dtype=np.int64)), d)
    return d


@pytest.mark.parametrize("N,L,bits", PARAMS)
def test_key_encode_matches_oracle(N, L, bits):
    ctx, prm = ctx_and_prm(N, L, bits)
    sk = wl.secret_key(61, N)
    lifted = np.array([[s % q for s in sk.tolist()] for q in prm.q], dtype=np.uint64)
    assert np.array_equal(to_host(key_ntt(ctx, prm, sk)).reshape(L, N), oracle.ntt(lifted, prm))


@pytest.mark.parametrize("N,L,bits", PARAMS)
def test_encrypt_matches_oracle_and_decrypts(N, L, bits):
    ctx, prm = ctx_and_prm(N, L, bits)
    n = 3
    sk = wl.secret_key(62, N)
    msgs = Stream(62, synth.INPUT).below(n * N, prm.t).reshape(n, N)
    a = synth.uniform_mod(Stream(62, synth.UNIFORM), (n, L, N), prm.q)
    e = Stream(62, synth.ERROR).cbd(n * N, wl.ETA).reshape(n, N)
    want = oracle.bfv_encrypt(msgs, sk, a, e, prm)
    skn = key_ntt(ctx, prm, sk)
    ct = empty_words(n * 2 * L * N)
    work = empty_words(n * L * N)
    ctx.encrypt(n, to_dev(msgs.astype(np.int64)), to_dev(a), to_dev(e), skn, ct, work)
    got = to_host(ct).reshape(want.shape)
    assert np.array_equal(got, want)
    out = empty_words(n * N)
    ctx.decrypt(n, ct, skn, out, work)
    dec = out.cpu().numpy().reshape(n, N)
    assert np.array_equal(dec, oracle.centre_mod(msgs.astype(object), prm.t).astype(np.int64))
    assert np.array_equal(dec, oracle.bfv_decrypt(want, sk, prm))


def test_encrypt_reduces_messages_mod_t():
    ctx, prm = ctx_and_prm(4096, 2, 50)
    N, L = prm.N, prm.L
    sk = wl.secret_key(63, N)
    raw = Stream(63, synth.INPUT).words(N).view(np.int64).reshape(1, N)  # any int64, negative included
    a = synth.uniform_mod(Stream(63, synth.UNIFORM), (1, L, N), prm.q)
    e = Stream(63, synth.ERROR).cbd(N, wl.ETA).reshape(1, N)
    want = oracle.bfv_encrypt(np.mod(raw, prm.t).astype(np.uint64), sk, a, e, prm)
    skn = key_ntt(ctx, prm, sk)
    ct, work = empty_words(2 * L * N), empty_words(L * N)
    ctx.encrypt(1, to_dev(raw), to_dev(a), to_dev(e), skn, ct, work)
    assert np.array_equal(to_host(ct).reshape(want.shape), want)


@pytest.mark.parametrize("cfg_id", ["conv4_16x16", "conv64_56x56"])
def test_decrypt_layer_output_matches_oracle(cfg_id):
    """Layer outputs carry grown noise; every coefficient decrypts as the
    oracle's exact decoding does, and the output slots give the conv."""
    cfg = synth.WORKLOADS[cfg_id]
    shape = cfg["layers"][0]
    ctx, prm = ctx_and_prm(cfg["N"], cfg["L"], cfg["bits"])
    cv = wl.conv_of(shape)
    d = ctx.plan(shape)
    g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
    x, K = wl.draw_layer(cfg, shape)
    sk = wl.secret_key(cfg["seed"], prm.N)
    ct = wl.encrypt_input(x, cv, g, prm, cfg["seed"], sk)
    s = ctx.sizes(d)
    wntt = empty_words(s.w_words)
    ctx.encode_weights(d, to_dev(K), wntt)
    out = empty_words(s.out_cts * 2 * prm.L * prm.N)
    ctx.conv_layer(d, 1, to_dev(ct), wntt, out)
    n = s.out_cts
    skn = key_ntt(ctx, prm, sk)
    msgs, work = empty_words(n * prm.N), empty_words(n * prm.L * prm.N)
    ctx.decrypt(n, out, skn, msgs, work)
    dec = msgs.cpu().numpy().reshape(n, prm.N)
    host = to_host(out).reshape(n, 2, prm.L, prm.N)
    rows = range(n) if n <= 8 else Stream(64, synth.MIX).below(8, n).tolist()
    for r in rows:
        assert np.array_equal(dec[r], oracle.bfv_decrypt(host[r:r + 1], sk, prm)[0]), r
    y = oracle.assemble_output(dec.reshape(cv.M, g.S, prm.N)[:, :, oracle.output_slots(g)], cv, g)
    assert np.array_equal(y, oracle.plain_conv(x, K, 1, 1))


def test_decrypt_arbitrary_words_matches_exact_rounding():
    """Uniform words (no noise bound): the fixed-point decode still equals
    the exact rounding (a flip needs t*V/Q within 2^-68 of a half-integer)."""
    ctx, prm = ctx_and_prm(8192, 3, 60)
    n = 2
    ct = synth.uniform_mod(Stream(65, synth.UNIFORM), (n, 2, prm.L, prm.N), prm.q)
    sk = wl.secret_key(65, prm.N)
    skn = key_ntt(ctx, prm, sk)
    msgs, work = empty_words(n * prm.N), empty_words(n * prm.L * prm.N)
    ctx.decrypt(n, to_dev(ct), skn, msgs, work)
    assert np.array_equal(msgs.cpu().numpy().reshape(n, prm.N), oracle.bfv_decrypt(ct, sk, prm))


@pytest.mark.parametrize("N,L,bits", [(4096, 2, 50), (8192, 3, 60)])
@pytest.mark.parametrize("t", ["prime", 3])
def test_odd_plaintext_modulus_roundtrip(N, L, bits, t):
    """An odd t (the Z_P variant's prime, t = 1 mod 2N, or t = 3): encryption
    word for word against the oracle; decryption of those encryptions and of
    arbitrary words against the oracle's exact decoding, centred into
    -(t-1)/2 .. (t-1)/2."""
    if t == "prime":
        t = oracle.find_primes(N, 37, 1)[0]
    ctx, prm = ctx_and_prm(N, L, bits, t)
    n = 2
    sk = wl.secret_key(66, N)
    msgs = Stream(66, synth.INPUT).below(n * N, t).reshape(n, N)
    msgs[0, :2] = [(t - 1) // 2, (t + 1) // 2]
    a = synth.uniform_mod(Stream(66, synth.UNIFORM), (n, L, N), prm.q)
    e = Stream(66, synth.ERROR).cbd(n * N, wl.ETA).reshape(n, N)
    want = oracle.bfv_encrypt(msgs, sk, a, e, prm)
    skn = key_ntt(ctx, prm, sk)
    ct, work = empty_words(n * 2 * L * N), empty_words(n * L * N)
    ctx.encrypt(n, to_dev(msgs.astype(np.int64)), to_dev(a), to_dev(e), skn, ct, work)
    assert np.array_equal(to_host(ct).reshape(want.shape), want)
    out = empty_words(n * N)
    ctx.decrypt(n, ct, skn, out, work)
    dec = out.cpu().numpy().reshape(n, N)
    assert np.array_equal(dec, oracle.centre_mod(msgs.astype(object), t))
    assert list(dec[0, :2]) == [(t - 1) // 2, -((t - 1) // 2)]
    rand = synth.uniform_mod(Stream(67, synth.UNIFORM), (n, 2, L, N), prm.q)
    ctx.decrypt(n, to_dev(rand), skn, out, work)
    assert np.array_equal(out.cpu().numpy().reshape(n, N), oracle.bfv_decrypt(rand, sk, prm))


def test_client_errors():
    from paper_2506_11586_amd import heconv
    ctx1, _ = ctx_and_prm(4096, 2, 50, t=1)  # t = 1: delta = Q, no usable plaintext space
    L = heconv.lib()
    assert L.he_decrypt(ctx1.handle, 1, None, None, None, None, None) == heconv.HE_EPARAM
    assert L.he_encrypt(ctx1.handle, 1, None, None, None, None, None, None, None) == heconv.HE_EPARAM
    ctx, _ = ctx_and_prm(4096, 2, 50)
    assert L.he_encrypt(ctx.handle, 1, None, None, None, None, None, None, None) == heconv.HE_EINVAL
    assert L.he_decrypt(ctx.handle, 0, None, None, None, None, None) == heconv.HE_OK
    assert L.he_key_encode(ctx.handle, None, None, None) == heconv.HE_EINVAL
