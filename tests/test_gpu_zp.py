"""GPU parity of the Z_P variant (Sec. 6.1): slot encoding and decoding over
a prime t, the diagonal layout, the scaled weight plaintexts, and the
multiply-accumulate-rotate linear kernel, word for word against the oracle
(slots, diagonals, plaintexts, and the encrypted kernel composed of the
oracle's rotation and ciphertext-plaintext product), plus decryption of the
kernel's output to W x mod t, up to a 1000 x 2048 matrix at N=8192."""
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

# (N, L, bits of the q's, bits of t): a 37-bit t needs the 180-bit Q of
# N=8192, L=3 for the ciphertext-plaintext products to decode
PARAMS = [(4096, 2, 50, 20), (8192, 3, 60, 37)]


def setup(N, L, bits, tbits):
    """(base context with plaintext modulus t, extended context (P last),
    t-context, base Params, P, t)."""
    key = (N, L, bits, tbits)
    if key not in _cache:
        require_gpu()
        ensure_built()
        from paper_2506_11586_amd import heconv
        primes = oracle.find_primes(N, bits, L + 1)
        t = oracle.find_primes(N, tbits, 1)[0]
        prm = oracle.Params(N, L, bits, t, q=primes[:L])
        _cache[key] = (heconv.Context(N, primes[:L], t), heconv.Context(N, primes, t), heconv.Context(N, [t]), prm,
                       primes[L], t)
    return _cache[key]


def galois_key_dev(ext, prm, P, sk, g, seed):
    eprm = oracle.ext_params(prm, P)
    a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (prm.L, prm.L + 1, prm.N), eprm.q)
    e = Stream(seed, synth.ERROR).cbd(prm.L * prm.N, wl.ETA).reshape(prm.L, prm.N)
    dk = empty_words(prm.L * 2 * (prm.L + 1) * prm.N)
    ext.galois_key(g, to_dev(np.asarray(sk, dtype=np.int64)), to_dev(a), to_dev(e.astype(np.int64)), dk,
                   empty_words(ext.galois_key_work_words()))
    return dk, (a, e)


@pytest.mark.parametrize("N,L,bits,tbits", PARAMS)
def test_simd_encode_decode_match_oracle(N, L, bits, tbits):
    _, _, tctx, prm, P, t = setup(N, L, bits, tbits)
    n = 3
    v = Stream(100, synth.UNIFORM).below(n * N, t).reshape(n, N)
    v[0, :3] = [0, 1, t - 1]
    coeffs = empty_words(n * N)
    tctx.simd_encode(n, to_dev(v), coeffs)
    want = oracle.centred_lift(oracle.simd_encode(v, t), t)
    got = coeffs.cpu().numpy().reshape(n, N)
    assert np.array_equal(got, want)
    slots = empty_words(n * N)
    tctx.simd_decode(n, coeffs, slots, empty_words(n * N))
    assert np.array_equal(to_host(slots).reshape(n, N), v)
    # decoding takes any integers: shift every coefficient by a multiple of t
    shifted = got + (Stream(101, synth.MIX).below(n * N, 5).reshape(n, N).astype(np.int64) - 2) * t
    tctx.simd_decode(n, to_dev(shifted), slots, empty_words(n * N))
    assert np.array_equal(to_host(slots).reshape(n, N), v)


@pytest.mark.parametrize("rows,cols,n", [(5, 7, 8), (16, 16, 16), (3, 32, 32), (64, 1, 64)])
def test_diagonals_match_oracle(rows, cols, n):
    _, _, tctx, prm, P, t = setup(4096, 2, 50, 20)
    N = prm.N
    W = Stream(102 + n, synth.WEIGHT).ints(rows * cols, -t, t).reshape(rows, cols)  # signed, reduced mod t
    slots = empty_words(n * N)
    tctx.zp_diagonals(to_dev(W.astype(np.int64)), rows, cols, n, slots)
    assert np.array_equal(to_host(slots).reshape(n, N).astype(object), oracle.zp_diagonals(W, n, N, t))


@pytest.mark.parametrize("N,L,bits,tbits", PARAMS)
def test_encode_plain_matches_oracle(N, L, bits, tbits):
    _, ext, _, prm, P, t = setup(N, L, bits, tbits)
    n = 2
    c = oracle.centred_lift(Stream(103, synth.UNIFORM).below(n * N, t).reshape(n, N), t)
    w = empty_words(n * L * N)
    ext.zp_encode_plain(n, to_dev(c), w)
    lifted = np.array([[[int(v) % q * ((-P) % q) % q for v in c[i].tolist()] for q in prm.q] for i in range(n)],
                      dtype=np.uint64)
    assert np.array_equal(to_host(w).reshape(n, L, N), oracle.ntt(lifted, prm))


def encrypted_inputs(base, tctx, prm, t, xs, sk, seed):
    """Encrypt the slot vectors xs [B][N] on the GPU; returns (ct, ct_ntt)."""
    B, N, L = xs.shape[0], prm.N, prm.L
    coeffs = empty_words(B * N)
    tctx.simd_encode(B, to_dev(xs), coeffs)
    skn = empty_words(L * N)
    base.key_encode(to_dev(np.asarray(sk, dtype=np.int64)), skn)
    a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (B, L, N), prm.q)
    e = Stream(seed, synth.ERROR).cbd(B * N, wl.ETA).reshape(B, N)
    ct = empty_words(B * 2 * L * N)
    base.encrypt(B, coeffs, to_dev(a), to_dev(e.astype(np.int64)), skn, ct, empty_words(B * L * N))
    ct_ntt = ct.clone()
    base.ntt_fwd(ct_ntt, 2 * B)
    return ct, ct_ntt, skn


def weights_dev(tctx, ext, prm, W, n):
    """Diagonals of W as scaled NTT plaintexts [n][L][N], and their centred
    coefficients (host) for the oracle."""
    N, L = prm.N, prm.L
    rows, cols = W.shape
    slots = empty_words(n * N)
    tctx.zp_diagonals(to_dev(W.astype(np.int64)), rows, cols, n, slots)
    coeffs = empty_words(n * N)
    tctx.simd_encode(n, slots, coeffs)
    w = empty_words(n * L * N)
    ext.zp_encode_plain(n, coeffs, w)
    return w, coeffs.cpu().numpy().reshape(n, N)


def decrypt_slots(base, tctx, prm, out, skn, B):
    N, L = prm.N, prm.L
    dec = empty_words(B * N)
    base.decrypt(B, out, skn, dec, empty_words(B * L * N))
    slots = empty_words(B * N)
    tctx.simd_decode(B, dec, slots, empty_words(B * N))
    return to_host(slots).reshape(B, N)


@pytest.mark.parametrize("N,L,bits,tbits,rows,cols,n,B", [(4096, 2, 50, 20, 3, 4, 4, 2),
                                                          (4096, 2, 50, 20, 5, 8, 8, 3),
                                                          (8192, 3, 60, 37, 2, 2, 2, 1)])
def test_matvec_matches_oracle_word_for_word(N, L, bits, tbits, rows, cols, n, B):
    base, ext, tctx, prm, P, t = setup(N, L, bits, tbits)
    sk = wl.secret_key(104, N)
    dk, _ = galois_key_dev(ext, prm, P, sk, 5, 105)
    # the oracle's key from the same random values, in coefficient form
    eprm = oracle.ext_params(prm, P)
    a = synth.uniform_mod(Stream(105, synth.UNIFORM), (L, L + 1, N), eprm.q)
    e = Stream(105, synth.ERROR).cbd(L * N, wl.ETA).reshape(L, N)
    ksk = oracle.galois_key(sk, 5, a, e, prm, P)
    W = Stream(106, synth.WEIGHT).below(rows * cols, t).reshape(rows, cols)
    xv = Stream(107, synth.INPUT).below(B * cols, t).reshape(B, cols)
    xs = np.stack([oracle.zp_input_slots(x, n, N, t) for x in xv]).astype(np.uint64)
    ct, ct_ntt, skn = encrypted_inputs(base, tctx, prm, t, xs, sk, 108)
    w, diag_coeffs = weights_dev(tctx, ext, prm, W, n)
    out = empty_words(B * 2 * L * N)
    ext.zp_matvec(5, B, ct_ntt, w, n, dk, out, empty_words(ext.zp_work_words(B)))
    want = oracle.zp_matvec_ct(to_host(ct).reshape(B, 2, L, N), list(diag_coeffs), 5, ksk, prm, P)
    assert np.array_equal(to_host(out).reshape(want.shape), want)
    y = decrypt_slots(base, tctx, prm, out, skn, B)
    for b in range(B):
        assert np.array_equal(y[b, :rows].astype(object), (W.astype(object) @ xv[b].astype(object)) % t)


def test_matvec_fc_2048_to_1000_decrypts():
    """N=8192, L=3, 37-bit t: a 1000 x 2048 matrix (2048 diagonals, 2047
    rotations) on 4 ciphertexts in one call, the shape the bench times;
    every output decrypts to W x mod t in both slot rows, and a ciphertext
    alone gives the same words as in the batch."""
    base, ext, tctx, prm, P, t = setup(8192, 3, 60, 37)
    N, L, rows, cols, n, B = prm.N, prm.L, 1000, 2048, 2048, 4
    sk = wl.secret_key(109, N)
    dk, _ = galois_key_dev(ext, prm, P, sk, 5, 110)
    W = Stream(111, synth.WEIGHT).below(rows * cols, t).reshape(rows, cols)
    xv = Stream(112, synth.INPUT).below(B * cols, t).reshape(B, cols)
    xs = np.stack([np.tile(x, N // cols) for x in xv]).astype(np.uint64)
    ct, ct_ntt, skn = encrypted_inputs(base, tctx, prm, t, xs, sk, 113)
    w, _ = weights_dev(tctx, ext, prm, W, n)
    out = empty_words(B * 2 * L * N)
    work = empty_words(ext.zp_work_words(B))
    ext.zp_matvec(5, B, ct_ntt, w, n, dk, out, work)
    y = decrypt_slots(base, tctx, prm, out, skn, B)
    Wo = W.astype(object)
    h = N // 2
    for b in range(B):
        want = (Wo @ xv[b].astype(object)) % t
        assert np.array_equal(y[b, :rows].astype(object), want), b
        assert np.array_equal(y[b, h:h + rows].astype(object), want), b
    one = empty_words(2 * L * N)
    ext.zp_matvec(5, 1, ct_ntt[2 * 2 * L * N:3 * 2 * L * N].clone(), w, n, dk, one, work)
    assert np.array_equal(to_host(one), to_host(out)[2 * 2 * L * N:3 * 2 * L * N])


def test_zp_argument_errors():
    from paper_2506_11586_amd import heconv
    base, ext, tctx, prm, P, t = setup(4096, 2, 50, 20)
    N = prm.N
    x = empty_words(4 * N)
    with pytest.raises(heconv.HeError) as e:
        base.simd_encode(1, x, empty_words(N))  # two primes: not a t-context
    assert e.value.status == heconv.HE_EPARAM
    for n in (3, 4096, 0):
        with pytest.raises(heconv.HeError) as e:
            tctx.zp_diagonals(x, 1, 1, n, empty_words(max(n, 1) * N))
        assert e.value.status == heconv.HE_ESHAPE
    with pytest.raises(heconv.HeError) as e:
        tctx.zp_diagonals(x, 9, 1, 8, empty_words(8 * N))  # more rows than n
    assert e.value.status == heconv.HE_ESHAPE
    ct = empty_words(2 * prm.L * N)
    w = empty_words(prm.L * N)
    ksk = empty_words(prm.L * 2 * (prm.L + 1) * N)
    work = empty_words(ext.zp_work_words(1))
    with pytest.raises(heconv.HeError) as e:
        ext.zp_matvec(5, 1, ct, w, 0, ksk, ct, work)
    assert e.value.status == heconv.HE_EINVAL
    with pytest.raises(heconv.HeError) as e:
        ext.zp_matvec(4, 1, ct, w, 1, ksk, ct, work)
    assert e.value.status == heconv.HE_EINVAL


def test_zp_matvec_needs_n_at_most_8192():
    from paper_2506_11586_amd import heconv
    require_gpu()
    ensure_built()
    N = 16384
    primes = oracle.find_primes(N, 60, 3)
    ext = heconv.Context(N, primes)
    L = 2
    ct = empty_words(2 * L * N)
    with pytest.raises(heconv.HeError) as e:
        ext.zp_matvec(5, 1, ct, empty_words(L * N), 1, empty_words(L * 2 * 3 * N), empty_words(2 * L * N),
                      empty_words(ext.zp_work_words(1)))
    assert e.value.status == heconv.HE_EPARAM
    ext.close()


@pytest.mark.parametrize("G", [2, 4])
def test_grouped_matvec_matches_oracle_word_for_word(G):
    """The chains schedule (N=4096, 20-bit t, 5 x 8 matrix at n = 8, two
    ciphertexts) against the oracle's grouped kernel word for word, and
    decrypting to W x."""
    base, ext, tctx, prm, P, t = setup(4096, 2, 50, 20)
    N, L, n, B = prm.N, prm.L, 8, 2
    sk = wl.secret_key(155, N)
    eprm = oracle.ext_params(prm, P)
    keys = []
    for gg, seed in ((5, 156), (pow(5, n // G, 2 * N), 157)):
        dk, _ = galois_key_dev(ext, prm, P, sk, gg, seed)
        a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (L, L + 1, N), eprm.q)
        e = Stream(seed, synth.ERROR).cbd(L * N, wl.ETA).reshape(L, N)
        keys.append((gg, dk, oracle.galois_key(sk, gg, a, e, prm, P)))
    W = Stream(158, synth.WEIGHT).below(40, t).reshape(5, 8)
    xv = Stream(159, synth.INPUT).below(B * 8, t).reshape(B, 8)
    xs = np.stack([oracle.zp_input_slots(x, n, N, t) for x in xv]).astype(np.uint64)
    ct, ct_ntt, skn = encrypted_inputs(base, tctx, prm, t, xs, sk, 160)
    w, diag_coeffs = weights_dev(tctx, ext, prm, W, n)
    out = empty_words(B * 2 * L * N)
    ext.zp_matvec_grouped(5, B, ct_ntt, w, n, G, keys[0][1], keys[1][0], keys[1][1], out,
                          empty_words(ext.zp_grouped_work_words(B, G)))
    want = oracle.zp_matvec_grouped_ct(to_host(ct).reshape(B, 2, L, N), list(diag_coeffs), G, 5, keys[0][2],
                                       keys[1][0], keys[1][2], prm, P)
    assert np.array_equal(to_host(out).reshape(want.shape), want)
    y = decrypt_slots(base, tctx, prm, out, skn, B)
    for b in range(B):
        assert np.array_equal(y[b, :5].astype(object), (W.astype(object) @ xv[b].astype(object)) % t)


def test_grouped_fc_2048_to_1000_decrypts():
    """N=8192, L=3, 37-bit t, the 1000 x 2048 matrix as 8 chains of 256
    iterations combined by 7 rotations of 256 slots: every output decrypts
    to W x mod t; groups = 1 gives he_zp_matvec's words."""
    base, ext, tctx, prm, P, t = setup(8192, 3, 60, 37)
    N, L, rows, cols, n, B, G = prm.N, prm.L, 1000, 2048, 2048, 3, 8
    sk = wl.secret_key(161, N)
    dk, _ = galois_key_dev(ext, prm, P, sk, 5, 162)
    dk2, _ = galois_key_dev(ext, prm, P, sk, pow(5, n // G, 2 * N), 163)
    W = Stream(164, synth.WEIGHT).below(rows * cols, t).reshape(rows, cols)
    xv = Stream(165, synth.INPUT).below(B * cols, t).reshape(B, cols)
    xs = np.stack([np.tile(x, N // cols) for x in xv]).astype(np.uint64)
    ct, ct_ntt, skn = encrypted_inputs(base, tctx, prm, t, xs, sk, 166)
    w, _ = weights_dev(tctx, ext, prm, W, n)
    out = empty_words(B * 2 * L * N)
    ext.zp_matvec_grouped(5, B, ct_ntt, w, n, G, dk, pow(5, n // G, 2 * N), dk2, out,
                          empty_words(ext.zp_grouped_work_words(B, G)))
    y = decrypt_slots(base, tctx, prm, out, skn, B)
    Wo = W.astype(object)
    for b in range(B):
        assert np.array_equal(y[b, :rows].astype(object), (Wo @ xv[b].astype(object)) % t), b
    one = empty_words(B * 2 * L * N)
    two = empty_words(B * 2 * L * N)
    ext.zp_matvec_grouped(5, B, ct_ntt, w, 64, 1, dk, 1, None, one, empty_words(ext.zp_grouped_work_words(B, 1)))
    ext.zp_matvec(5, B, ct_ntt, w, 64, dk, two, empty_words(ext.zp_work_words(B)))
    assert np.array_equal(to_host(one), to_host(two))


@pytest.mark.parametrize("rows,cols,n_out,n_in", [(5, 16, 8, 16), (3, 32, 4, 32), (1000, 2048, 1024, 2048)])
def test_rectangular_diagonals_match_oracle(rows, cols, n_out, n_in):
    _, _, tctx, prm, P, t = setup(8192, 3, 60, 37)
    N = prm.N
    W = Stream(180 + n_in, synth.WEIGHT).ints(rows * cols, -t, t).reshape(rows, cols)
    slots = empty_words(n_out * N)
    tctx.zp_diagonals_rect(to_dev(W.astype(np.int64)), rows, cols, n_out, n_in, slots)
    got = to_host(slots).reshape(n_out, N)
    if n_out <= 8:
        assert np.array_equal(got.astype(object), oracle.zp_diagonals_rect(W, n_out, n_in, N, t))
    else:  # sampled rows of the large layout against the oracle's definition
        want = oracle.zp_diagonals_rect(W[:, :], n_out, n_in, N, t)
        for i in (0, 1, 511, 1023):
            assert np.array_equal(got[i].astype(object), want[i]), i


def test_fold_matches_oracle_word_for_word():
    """out = ct + rotate(ct, g2) on arbitrary words (N=4096), against the
    oracle's rotation and addition."""
    base, ext, tctx, prm, P, t = setup(4096, 2, 50, 20)
    N, L, n = prm.N, prm.L, 2
    g2 = pow(5, 4, 2 * N)
    sk = wl.secret_key(185, N)
    dk, (a, e) = galois_key_dev(ext, prm, P, sk, g2, 186)
    ksk = oracle.galois_key(sk, g2, a, e, prm, P)
    ct = synth.uniform_mod(Stream(187, synth.UNIFORM), (n, 2, L, N), prm.q)
    out = empty_words(ct.size)
    ext.zp_fold(g2, n, to_dev(ct), dk, out, empty_words(ext.keyswitch_work_words(n)))
    want = oracle.zp_fold_ct(ct, g2, ksk, prm, P)
    assert np.array_equal(to_host(out).reshape(want.shape), want)
    from paper_2506_11586_amd import heconv
    d = to_dev(ct)
    with pytest.raises(heconv.HeError) as exc:
        ext.zp_fold(g2, n, d, dk, d, empty_words(ext.keyswitch_work_words(n)))
    assert exc.value.status == heconv.HE_EINVAL


@pytest.mark.parametrize("G", [1, 8])
def test_rectangular_fc_2048_to_1000_decrypts(G):
    """N=8192, L=3, 37-bit t: the 1000 x 2048 matrix as 1024 generalized
    diagonals (as one chain, or as 8 chains) and one fold by 1024 slots:
    every output decrypts to W x mod t."""
    base, ext, tctx, prm, P, t = setup(8192, 3, 60, 37)
    N, L, rows, cols, n_out, B = prm.N, prm.L, 1000, 2048, 1024, 3
    sk = wl.secret_key(188, N)
    dk, _ = galois_key_dev(ext, prm, P, sk, 5, 189)
    gf = pow(5, n_out, 2 * N)
    dkf, _ = galois_key_dev(ext, prm, P, sk, gf, 190)
    W = Stream(191, synth.WEIGHT).below(rows * cols, t).reshape(rows, cols)
    xv = Stream(192, synth.INPUT).below(B * cols, t).reshape(B, cols)
    xs = np.stack([np.tile(x, N // cols) for x in xv]).astype(np.uint64)
    ct, ct_ntt, skn = encrypted_inputs(base, tctx, prm, t, xs, sk, 193)
    slots = empty_words(n_out * N)
    tctx.zp_diagonals_rect(to_dev(W.astype(np.int64)), rows, cols, n_out, cols, slots)
    coeffs = empty_words(n_out * N)
    tctx.simd_encode(n_out, slots, coeffs)
    w = empty_words(n_out * L * N)
    ext.zp_encode_plain(n_out, coeffs, w)
    z = empty_words(B * 2 * L * N)
    if G == 1:
        ext.zp_matvec(5, B, ct_ntt, w, n_out, dk, z, empty_words(ext.zp_work_words(B)))
    else:
        g2 = pow(5, n_out // G, 2 * N)
        dk2, _ = galois_key_dev(ext, prm, P, sk, g2, 194)
        ext.zp_matvec_grouped(5, B, ct_ntt, w, n_out, G, dk, g2, dk2, z, empty_words(ext.zp_grouped_work_words(B, G)))
    out = empty_words(B * 2 * L * N)
    ext.zp_fold(gf, B, z, dkf, out, empty_words(ext.keyswitch_work_words(B)))
    y = decrypt_slots(base, tctx, prm, out, skn, B)
    Wo = W.astype(object)
    for b in range(B):
        assert np.array_equal(y[b, :rows].astype(object), (Wo @ xv[b].astype(object)) % t), b
