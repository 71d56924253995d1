"""Pins for the oracle's Z_P variant (Sec. 6.1): batched plaintext slots
over a prime t = 1 mod 2N and the iterative multiply-accumulate-rotate
linear kernel.

Slots are pinned by evaluation written out at a tiny ring (decode(m)[s] =
m(psi^e_s) by a plain double loop), by the slot-wise product law, and by the
rotation law that fixes their order (X -> X^5 moves every row left by one
slot, X -> X^-1 swaps the rows); the diagonal layout by the iteration on
plain slot vectors against the matrix product; the encrypted kernel by
decryption to W x mod t."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests import workload as wl


def test_simd_decode_is_evaluation_at_the_slot_exponents():
    N, t = 16, 97  # 97 = 1 mod 32
    psi = oracle.Params(N, 1, 7, t, q=[t]).psi[0]
    assert pow(psi, N, t) == t - 1
    m = Stream(90, synth.UNIFORM).below(N, t).astype(np.int64)
    e = oracle.simd_exponents(N)
    assert sorted(int(v) for v in e) == list(range(1, 2 * N, 2))
    want = []
    for s in range(N):
        acc = 0
        for k in range(N):
            acc += int(m[k]) * pow(psi, int(e[s]) * k, t)
        want.append(acc % t)
    assert [int(v) for v in oracle.simd_decode(m, t)] == want


@pytest.fixture(scope="module")
def tp():
    N = 4096
    return N, oracle.find_primes(N, 37, 1)[0]


def test_simd_roundtrip_and_product(tp):
    N, t = tp
    a = Stream(91, synth.UNIFORM).below(N, t)
    b = Stream(92, synth.UNIFORM).below(N, t)
    ea, eb = oracle.simd_encode(a, t), oracle.simd_encode(b, t)
    assert np.array_equal(oracle.simd_decode(ea, t).astype(np.uint64), a)
    prod = oracle.negacyclic_mul(ea, eb, t)
    assert np.array_equal(oracle.simd_decode(prod, t).astype(object), (a.astype(object) * b.astype(object)) % t)


def test_simd_rotation_law(tp):
    N, t = tp
    h = N // 2
    v = Stream(93, synth.UNIFORM).below(N, t)
    m = oracle.simd_encode(v, t)
    left = oracle.simd_decode(oracle.automorphism(m[None], 5, [t])[0], t)
    assert np.array_equal(left[:h], np.roll(v[:h], -1)) and np.array_equal(left[h:], np.roll(v[h:], -1))
    swap = oracle.simd_decode(oracle.automorphism(m[None], 2 * N - 1, [t])[0], t)
    assert np.array_equal(swap[:h], v[h:]) and np.array_equal(swap[h:], v[:h])


@pytest.mark.parametrize("rows,cols,n", [(5, 7, 8), (16, 16, 16), (3, 32, 32)])
def test_diagonal_iteration_is_the_matrix_product(tp, rows, cols, n):
    N, t = tp
    W = Stream(94 + n, synth.WEIGHT).below(rows * cols, t).reshape(rows, cols)
    x = Stream(95 + n, synth.INPUT).below(cols, t)
    d = oracle.zp_diagonals(W, n, N, t)
    xs = oracle.zp_input_slots(x, n, N, t)
    h = N // 2
    rot = lambda v: np.concatenate([np.roll(v[:h], -1), np.roll(v[h:], -1)])
    acc = (d[n - 1] * xs) % t
    for i in range(n - 2, -1, -1):
        acc = (rot(acc) + d[i] * xs) % t
    want = (W.astype(object) @ x.astype(object)) % t
    assert np.array_equal(acc[:rows], want)
    assert np.array_equal(acc[h:h + rows], want)


def test_encrypted_kernel_decrypts_to_the_matrix_product():
    """N=4096, L=2 (50-bit) plus a special prime, a 3 x 4 matrix at n = 4:
    three rotations with the Galois key for g = 5.  The plaintext prime is
    below 2^20 here: the ciphertext-plaintext product of BFV decodes only
    while (Q mod t) * N * t^2 / 4 stays well below Q, which a 37-bit t
    breaks at Q ~ 2^100 (it needs the 180-bit Q of N=8192, L=3)."""
    N, L, bits, n = 4096, 2, 50, 4
    t = oracle.find_primes(N, 20, 1)[0]
    primes = oracle.find_primes(N, bits, L + 1)
    prm = oracle.Params(N, L, bits, t, q=primes[:L])
    P = primes[L]
    sk = wl.secret_key(96, N)
    ext = oracle.ext_params(prm, P)
    a = synth.uniform_mod(Stream(96, synth.UNIFORM), (L, L + 1, N), ext.q)
    e = Stream(96, synth.ERROR).cbd(L * N, wl.ETA).reshape(L, N)
    ksk = oracle.galois_key(sk, 5, a, e, prm, P)
    W = Stream(97, synth.WEIGHT).below(12, t).reshape(3, 4)
    x = Stream(97, synth.INPUT).below(4, t)
    msg = oracle.simd_encode(oracle.zp_input_slots(x, n, N, t), t).astype(np.uint64)
    ct = wl.encrypt_polys(msg[None], prm, 98, sk)
    diags = [oracle.centred_lift(oracle.simd_encode(dv, t), t) for dv in oracle.zp_diagonals(W, n, N, t)]
    out = oracle.zp_matvec_ct(ct, diags, 5, ksk, prm, P)
    dec, bits_used = oracle.bfv_decrypt(out, sk, prm, with_noise=True)
    y = oracle.simd_decode(dec[0], t)
    assert np.array_equal(y[:3], (W.astype(object) @ x.astype(object)) % t)
    assert bits_used < prm.delta.bit_length() - 2


def test_grouped_iteration_decrypts_to_the_matrix_product():
    """The iteration as G = 2 chains of n/G diagonals combined by one
    rotation by n/G slots (N=4096, 20-bit t, a 5 x 8 matrix at n = 8) also
    decrypts to W x; on plain slot vectors the grouped schedule equals W x
    for G = 1, 2, 4, 8."""
    N, L, bits, n = 4096, 2, 50, 8
    t = oracle.find_primes(N, 20, 1)[0]
    W = Stream(150, synth.WEIGHT).below(40, t).reshape(5, 8)
    x = Stream(150, synth.INPUT).below(8, t)
    d = oracle.zp_diagonals(W, n, N, t)
    xs = oracle.zp_input_slots(x, n, N, t)
    h = N // 2
    rot = lambda v, k: np.concatenate([np.roll(v[:h], -k), np.roll(v[h:], -k)])
    want = (W.astype(object) @ x.astype(object)) % t
    for G in (1, 2, 4, 8):
        per = n // G
        chains = []
        for c in range(G):
            acc = (d[c * per + per - 1] * xs) % t
            for i in range(per - 2, -1, -1):
                acc = (rot(acc, 1) + d[c * per + i] * xs) % t
            chains.append(acc)
        acc = chains[-1]
        for c in range(G - 2, -1, -1):
            acc = (rot(acc, per) + chains[c]) % t
        assert np.array_equal(acc[:5], want), G
    primes = oracle.find_primes(N, bits, L + 1)
    prm = oracle.Params(N, L, bits, t, q=primes[:L])
    P = primes[L]
    ext = oracle.ext_params(prm, P)
    sk = wl.secret_key(151, N)
    keys = []
    for gg, seed in ((5, 152), (pow(5, n // 2, 2 * N), 153)):
        a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (L, L + 1, N), ext.q)
        e = Stream(seed, synth.ERROR).cbd(L * N, wl.ETA).reshape(L, N)
        keys.append((gg, oracle.galois_key(sk, gg, a, e, prm, P)))
    msg = oracle.simd_encode(xs, t).astype(np.uint64)
    ct = wl.encrypt_polys(msg[None], prm, 154, sk)
    diags = [oracle.centred_lift(oracle.simd_encode(dv, t), t) for dv in d]
    out = oracle.zp_matvec_grouped_ct(ct, diags, 2, keys[0][0], keys[0][1], keys[1][0], keys[1][1], prm, P)
    y = oracle.simd_decode(oracle.bfv_decrypt(out, sk, prm)[0], t)
    assert np.array_equal(y[:5], want)


@pytest.mark.parametrize("rows,cols,n_out,n_in", [(5, 16, 8, 16), (3, 32, 4, 32), (8, 8, 8, 8), (1, 64, 1, 64)])
def test_rectangular_diagonals_and_folds_give_the_matrix_product(tp, rows, cols, n_out, n_in):
    """n_out generalized diagonals through the iteration, then
    log2(n_in/n_out) rotate-and-add steps, on plain slot vectors: W x."""
    N, t = tp
    W = Stream(170 + n_in, synth.WEIGHT).below(rows * cols, t).reshape(rows, cols)
    x = Stream(171 + n_in, synth.INPUT).below(cols, t)
    d = oracle.zp_diagonals_rect(W, n_out, n_in, N, t)
    xs = oracle.zp_input_slots(x, n_in, N, t)
    h = N // 2
    rot = lambda v, k: np.concatenate([np.roll(v[:h], -k), np.roll(v[h:], -k)])
    acc = (d[n_out - 1] * xs) % t
    for i in range(n_out - 2, -1, -1):
        acc = (rot(acc, 1) + d[i] * xs) % t
    s = n_out
    while s < n_in:
        acc = (acc + rot(acc, s)) % t
        s *= 2
    want = (W.astype(object) @ x.astype(object)) % t
    assert np.array_equal(acc[:rows], want)
    if n_out == n_in:
        assert np.array_equal(d, oracle.zp_diagonals(W, n_in, N, t))


def test_rectangular_kernel_with_fold_decrypts_to_the_matrix_product():
    """N=4096, 20-bit t: a 3 x 8 matrix with 4 diagonals of period 8, three
    rotations by one slot and one fold by 4 slots (two Galois keys)."""
    N, L, bits = 4096, 2, 50
    t = oracle.find_primes(N, 20, 1)[0]
    primes = oracle.find_primes(N, bits, L + 1)
    prm = oracle.Params(N, L, bits, t, q=primes[:L])
    P = primes[L]
    ext = oracle.ext_params(prm, P)
    sk = wl.secret_key(172, N)
    keys = {}
    for gg, seed in ((5, 173), (pow(5, 4, 2 * N), 174)):
        a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (L, L + 1, N), ext.q)
        e = Stream(seed, synth.ERROR).cbd(L * N, wl.ETA).reshape(L, N)
        keys[gg] = oracle.galois_key(sk, gg, a, e, prm, P)
    W = Stream(175, synth.WEIGHT).below(24, t).reshape(3, 8)
    x = Stream(175, synth.INPUT).below(8, t)
    msg = oracle.simd_encode(oracle.zp_input_slots(x, 8, N, t), t).astype(np.uint64)
    ct = wl.encrypt_polys(msg[None], prm, 176, sk)
    diags = [oracle.centred_lift(oracle.simd_encode(dv, t), t) for dv in oracle.zp_diagonals_rect(W, 4, 8, N, t)]
    out = oracle.zp_matvec_ct(ct, diags, 5, keys[5], prm, P)
    out = oracle.zp_fold_ct(out, pow(5, 4, 2 * N), keys[pow(5, 4, 2 * N)], prm, P)
    y = oracle.simd_decode(oracle.bfv_decrypt(out, sk, prm)[0], t)
    assert np.array_equal(y[:3], (W.astype(object) @ x.astype(object)) % t)
