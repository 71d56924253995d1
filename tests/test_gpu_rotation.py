"""GPU parity of ciphertext rotation for the Z_P variant (Sec. 2, Sec. 6.1):
the Galois automorphism, hybrid key switching with a special prime and the
fused rotation, word for word against the oracle's automorphism,
key_switch and rotate, plus decryption of rotated encryptions (the
library's own decryption) to m(X^g)."""
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

PARAMS = [(4096, 2, 50), (8192, 3, 60)]


def contexts(N, L, bits):
    """(base context over q_0..q_{L-1}, extended context with P last, base
    Params, P)."""
    key = (N, L, bits)
    if key not in _cache:
        require_gpu()
        ensure_built()
        from paper_2506_11586_amd import heconv
        primes = oracle.find_primes(N, bits, L + 1)
        prm = oracle.Params(N, L, bits, 2 ** synth.T_BITS, q=primes[:L])
        _cache[key] = (heconv.Context(N, primes[:L]), heconv.Context(N, primes), prm, primes[L])
    return _cache[key]


def make_key(prm, P, sk, g, seed):
    ext = oracle.ext_params(prm, P)
    a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (prm.L, prm.L + 1, prm.N), ext.q)
    e = Stream(seed, synth.ERROR).cbd(prm.L * prm.N, wl.ETA).reshape(prm.L, prm.N)
    return oracle.galois_key(sk, g, a, e, prm, P)


def key_to_dev(ext_ctx, prm, ksk):
    d = to_dev(ksk)
    ext_ctx.ntt_fwd(d, 2 * prm.L)
    return d


@pytest.mark.parametrize("N,L,bits", PARAMS)
@pytest.mark.parametrize("g", [1, 3, 5, 25, "2N-1", "2N-3"])
def test_automorph_matches_oracle(N, L, bits, g):
    base, _, prm, _ = contexts(N, L, bits)
    g = {"2N-1": 2 * N - 1, "2N-3": 2 * N - 3}.get(g, g)
    n = 3
    x = synth.uniform_mod(Stream(70 + N, synth.UNIFORM), (n, L, N), prm.q)
    x[0, 0, :4] = 0  # zero coefficients stay zero under negation
    out = empty_words(n * L * N)
    base.automorph(g, n, to_dev(x), out)
    assert np.array_equal(to_host(out).reshape(n, L, N), oracle.automorphism(x, g, prm.q))


@pytest.mark.parametrize("fused", [1, 2, 0])
@pytest.mark.parametrize("N,L,bits", PARAMS)
def test_keyswitch_matches_oracle(N, L, bits, fused):
    """Arbitrary words as the ciphertext (every digit value range): the
    output equals the oracle's exact CRT key switching word for word, with
    the digit steps fused into one kernel and as separate steps."""
    _, ext, prm, P = contexts(N, L, bits)
    ext.set_tuning(ks_fused=fused)
    n = 2 if N == 4096 else 1
    sk = wl.secret_key(71, N)
    ksk = make_key(prm, P, sk, 5, 72)
    ct = synth.uniform_mod(Stream(73, synth.UNIFORM), (n, 2, L, N), prm.q)
    ct[0, 0, :, :3] = np.array(prm.q, dtype=np.uint64)[:, None] - 1  # largest digits
    want = oracle.key_switch(ct, ksk, prm, P)
    dk = key_to_dev(ext, prm, ksk)
    out = empty_words(ct.size)
    work = empty_words(ext.keyswitch_work_words(n))
    ext.keyswitch(n, to_dev(ct), dk, out, work)
    assert np.array_equal(to_host(out).reshape(want.shape), want)
    # in place: d_out aliasing d_ct gives the same words
    dct = to_dev(ct)
    ext.keyswitch(n, dct, dk, dct, work)
    assert np.array_equal(to_host(dct).reshape(want.shape), want)


@pytest.mark.parametrize("fused", [1, 2, 0])
@pytest.mark.parametrize("N,L,bits", PARAMS)
def test_rotate_matches_oracle_and_decrypts(N, L, bits, fused):
    base, ext, prm, P = contexts(N, L, bits)
    ext.set_tuning(ks_fused=fused)
    g = 3
    n = 2 if N == 4096 else 1
    sk = wl.secret_key(74, N)
    ksk = make_key(prm, P, sk, g, 75)
    msgs = Stream(76, synth.INPUT).below(n * N, prm.t).reshape(n, N)
    ct = wl.encrypt_polys(msgs, prm, 76, sk)
    want = oracle.rotate(ct, g, ksk, prm, P)
    dk = key_to_dev(ext, prm, ksk)
    out = empty_words(ct.size)
    work = empty_words(ext.keyswitch_work_words(n))
    ext.rotate(g, n, to_dev(ct), dk, out, work)
    got = to_host(out).reshape(want.shape)
    assert np.array_equal(got, want)
    # the library's decryption of the rotated ciphertexts gives m(X^g)
    skn = empty_words(L * N)
    base.key_encode(to_dev(np.asarray(sk, dtype=np.int64)), skn)
    dec = empty_words(n * N)
    base.decrypt(n, out, skn, dec, empty_words(n * L * N))
    m_rot = oracle.automorphism(msgs.astype(np.uint64)[:, None, :], g, [prm.t])[:, 0, :]
    assert np.array_equal(dec.cpu().numpy().reshape(n, N), oracle.centre_mod(m_rot.astype(object), prm.t).astype(np.int64))


@pytest.mark.parametrize("N,L,bits", PARAMS)
def test_galois_key_matches_oracle_and_rotates(N, L, bits):
    """The library's key generation equals the oracle's key in NTT form word
    for word, and a rotation with it decrypts to m(X^g)."""
    base, ext, prm, P = contexts(N, L, bits)
    g, seed = 2 * N - 3, 90
    eprm = oracle.ext_params(prm, P)
    sk = wl.secret_key(seed, N)
    a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (L, L + 1, N), eprm.q)
    e = Stream(seed, synth.ERROR).cbd(L * N, wl.ETA).reshape(L, N)
    want = oracle.ntt(oracle.galois_key(sk, g, a, e, prm, P), eprm)
    dk = empty_words(L * 2 * (L + 1) * N)
    ext.galois_key(g, to_dev(np.asarray(sk, dtype=np.int64)), to_dev(a), to_dev(e.astype(np.int64)), dk,
                   empty_words(ext.galois_key_work_words()))
    assert np.array_equal(to_host(dk).reshape(want.shape), want)
    n = 2
    msgs = Stream(seed + 1, synth.INPUT).below(n * N, prm.t).reshape(n, N)
    ct = wl.encrypt_polys(msgs, prm, seed + 1, sk)
    out = empty_words(ct.size)
    ext.rotate(g, n, to_dev(ct), dk, out, empty_words(ext.keyswitch_work_words(n)))
    skn = empty_words(L * N)
    base.key_encode(to_dev(np.asarray(sk, dtype=np.int64)), skn)
    dec = empty_words(n * N)
    base.decrypt(n, out, skn, dec, empty_words(n * L * N))
    m_rot = oracle.automorphism(msgs.astype(np.uint64)[:, None, :], g, [prm.t])[:, 0, :]
    assert np.array_equal(dec.cpu().numpy().reshape(n, N), oracle.centre_mod(m_rot.astype(object), prm.t).astype(np.int64))


@pytest.mark.parametrize("fused", [1, 2, 0])
def test_rotate_equals_automorph_then_keyswitch(fused):
    """The rotation equals the two library steps run one after the other,
    for several g (N=4096, L=2), with 4 and with 13 ciphertexts (a partial
    group of eight in the fused kernel's XCD mapping)."""
    base, ext, prm, P = contexts(4096, 2, 50)
    ext.set_tuning(ks_fused=fused)
    N, L = prm.N, prm.L
    sk = wl.secret_key(77, N)
    ksk = to_dev(make_key(prm, P, sk, 7, 78))  # any key: both paths use the same words
    ext.ntt_fwd(ksk, 2 * L)
    for n, g in ((4, 3), (4, 7), (4, 2 * N - 1), (4, 1), (13, 3), (13, 1)):
        ct = synth.uniform_mod(Stream(79 + n, synth.UNIFORM), (n, 2, L, N), prm.q)
        work = empty_words(ext.keyswitch_work_words(n))
        one = empty_words(ct.size)
        ext.rotate(g, n, to_dev(ct), ksk, one, work)
        rot = empty_words(ct.size)
        base.automorph(g, 2 * n, to_dev(ct), rot)
        two = empty_words(ct.size)
        ext.keyswitch(n, rot, ksk, two, work)
        assert np.array_equal(to_host(one), to_host(two)), (n, g)


def test_rotate_full_size_batch():
    """N=8192, L=3 (60-bit q's and P), 64 ciphertexts in one call, the
    launch shape the bench times: every ciphertext decrypts to m(X^g) with
    the library's decryption, one sampled ciphertext equals the oracle word
    for word, and each ciphertext's result does not depend on the batch;
    the unfused steps give the same words."""
    base, ext, prm, P = contexts(8192, 3, 60)
    ext.set_tuning(ks_fused=1)
    N, L, n, g = prm.N, prm.L, 64, 5
    sk = wl.secret_key(80, N)
    ksk = make_key(prm, P, sk, g, 81)
    dk = key_to_dev(ext, prm, ksk)
    skn = empty_words(L * N)
    base.key_encode(to_dev(np.asarray(sk, dtype=np.int64)), skn)
    msgs = Stream(82, synth.INPUT).below(n * N, prm.t).reshape(n, N)
    a = synth.uniform_mod(Stream(82, synth.UNIFORM), (n, L, N), prm.q)
    e = Stream(82, synth.ERROR).cbd(n * N, wl.ETA).reshape(n, N)
    ct = empty_words(n * 2 * L * N)
    base.encrypt(n, to_dev(msgs.astype(np.int64)), to_dev(a), to_dev(e), skn, ct, empty_words(n * L * N))
    out = empty_words(ct.numel())
    work = empty_words(ext.keyswitch_work_words(n))
    ext.rotate(g, n, ct, dk, out, work)
    dec = empty_words(n * N)
    base.decrypt(n, out, skn, dec, empty_words(n * L * N))
    m_rot = oracle.automorphism(msgs.astype(np.uint64)[:, None, :], g, [prm.t])[:, 0, :]
    assert np.array_equal(dec.cpu().numpy().reshape(n, N), oracle.centre_mod(m_rot.astype(object), prm.t).astype(np.int64))
    i = int(Stream(83, synth.MIX).below(1, n)[0])
    cts = to_host(ct).reshape(n, 2, L, N)
    got = to_host(out).reshape(n, 2, L, N)
    assert np.array_equal(got[i:i + 1], oracle.rotate(cts[i:i + 1], g, ksk, prm, P))
    one = empty_words(2 * L * N)
    ext.rotate(g, 1, to_dev(cts[i:i + 1]), dk, one, work)
    assert np.array_equal(to_host(one).reshape(1, 2, L, N), got[i:i + 1])
    for mode in (2, 0):
        ext.set_tuning(ks_fused=mode)
        other = empty_words(ct.numel())
        ext.rotate(g, n, ct, dk, other, work)
        assert bool(torch_equal(other, out)), mode
    ext.set_tuning(ks_fused=1)


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def test_rotation_argument_errors_and_empty():
    from paper_2506_11586_amd import heconv
    base, ext, prm, P = contexts(4096, 2, 50)
    N, L = prm.N, prm.L
    x = empty_words(2 * L * N)
    y = empty_words(2 * L * N)
    work = empty_words(ext.keyswitch_work_words(1))
    ksk = empty_words(L * 2 * (L + 1) * N)
    for g in (0, 2, 2 * N, 2 * N + 1):
        with pytest.raises(heconv.HeError) as e:
            base.automorph(g, 1, x, y)
        assert e.value.status == heconv.HE_EINVAL
        with pytest.raises(heconv.HeError) as e:
            ext.galois_key(g, x, ksk, x, ksk, empty_words(ext.galois_key_work_words()))
        assert e.value.status == heconv.HE_EINVAL
        with pytest.raises(heconv.HeError) as e:
            ext.rotate(g, 1, x, ksk, y, work)
        assert e.value.status == heconv.HE_EINVAL
    with pytest.raises(heconv.HeError) as e:
        base.automorph(3, 1, x, x)
    assert e.value.status == heconv.HE_EINVAL
    with pytest.raises(heconv.HeError) as e:
        ext.rotate(3, 1, x, ksk, x, work)
    assert e.value.status == heconv.HE_EINVAL
    one = heconv.Context(N, [prm.q[0]])  # no special prime
    with pytest.raises(heconv.HeError) as e:
        one.keyswitch_work_words(1)
    assert e.value.status == heconv.HE_EPARAM
    one.close()
    # n = 0 leaves the output untouched
    y.fill_(-1)
    base.automorph(3, 0, x, y)
    ext.keyswitch(0, x, ksk, y, work)
    ext.rotate(3, 0, x, ksk, y, work)
    assert bool((y == -1).all())


@pytest.mark.parametrize("N,L,bits", [(2048, 7, 40), (1024, 2, 30), (16384, 2, 60)])
def test_rotate_edge_rings_match_oracle(N, L, bits):
    """The largest digit count (7 ciphertext primes plus P: 7 products and
    their 128-bit sums), the smallest ring, and N=2^14 (where every mode
    runs the separate steps): rotation word for word against the oracle."""
    base, ext, prm, P = contexts(N, L, bits)
    g = 2 * N - 3
    sk = wl.secret_key(120, N)
    ksk = make_key(prm, P, sk, g, 121)
    ct = synth.uniform_mod(Stream(122, synth.UNIFORM), (1, 2, L, N), prm.q)
    ct[0, 0, :, :2] = np.array(prm.q, dtype=np.uint64)[:, None] - 1
    want = oracle.rotate(ct, g, ksk, prm, P)
    dk = key_to_dev(ext, prm, ksk)
    work = empty_words(ext.keyswitch_work_words(1))
    for mode in (1, 2, 0):
        ext.set_tuning(ks_fused=mode)
        out = empty_words(ct.size)
        ext.rotate(g, 1, to_dev(ct), dk, out, work)
        assert np.array_equal(to_host(out).reshape(want.shape), want), mode
    ext.set_tuning(ks_fused=1)
