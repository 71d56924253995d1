"""Pins for the oracle's ciphertext rotation (the Z_P variant's building
block: App. C, rotation; Sec. 6.1): the Galois automorphism a(X) -> a(X^g)
and hybrid key switching with a special prime.

The automorphism is pinned by ring-homomorphism and composition laws and by
g = 1 and g = 2N-1 (the inverse map X -> X^-1) written out; key switching by
decryption: a rotated encryption of m decrypts under the original key to
m(X^g), and with g = 1 key switching alone decrypts to m."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests import workload as wl


def small_ring():
    N = 64
    q = oracle.find_primes(N, 50, 1)[0]
    return N, q


def test_automorphism_is_a_ring_homomorphism():
    N, q = small_ring()
    a = synth.uniform_mod(Stream(81, synth.UNIFORM), (1, N), [q])[0]
    b = synth.uniform_mod(Stream(82, synth.UNIFORM), (1, N), [q])[0]
    for g in (3, 5, 2 * N - 1, 77):
        lhs = oracle.automorphism(oracle.negacyclic_mul(a, b, q)[None], g, [q])[0]
        rhs = oracle.negacyclic_mul(oracle.automorphism(a[None], g, [q])[0], oracle.automorphism(b[None], g, [q])[0], q)
        assert np.array_equal(lhs, rhs), g


def test_automorphism_composition_and_special_cases():
    N, q = small_ring()
    a = synth.uniform_mod(Stream(83, synth.UNIFORM), (1, N), [q])
    assert np.array_equal(oracle.automorphism(a, 1, [q]), a)
    for g, h in ((3, 5), (5, 2 * N - 1), (7, 9)):
        assert np.array_equal(oracle.automorphism(oracle.automorphism(a, g, [q]), h, [q]),
                              oracle.automorphism(a, (g * h) % (2 * N), [q]))
    # X -> X^-1 = -X^(N-1): a_0 stays, a_i (i >= 1) goes to -a_i at N - i
    inv = oracle.automorphism(a, 2 * N - 1, [q])[0]
    want = np.zeros(N, dtype=object)
    want[0] = int(a[0, 0])
    for i in range(1, N):
        want[N - i] = (-int(a[0, i])) % q
    assert np.array_equal(inv.astype(object), want)


def _rotation_case(N, L, bits, g, seed):
    primes = oracle.find_primes(N, bits, L + 1)
    prm = oracle.Params(N, L, bits, 2 ** synth.T_BITS, q=primes[:L])
    P = primes[L]
    sk = wl.secret_key(seed, N)
    msgs = Stream(seed, synth.INPUT).below(2 * N, prm.t).reshape(2, N)
    ct = wl.encrypt_polys(msgs, prm, seed, sk)
    ext = oracle.ext_params(prm, P)
    a = synth.uniform_mod(Stream(seed + 1, synth.UNIFORM), (L, L + 1, N), ext.q)
    e = Stream(seed + 1, synth.ERROR).cbd(L * N, wl.ETA).reshape(L, N)
    ksk = oracle.galois_key(sk, g, a, e, prm, P)
    return prm, P, sk, msgs, ct, ksk


@pytest.mark.parametrize("g", [3, 2 * 4096 - 1, 25])
def test_rotation_decrypts_to_automorphism_of_message(g):
    prm, P, sk, msgs, ct, ksk = _rotation_case(4096, 2, 50, g, 84)
    rot = oracle.rotate(ct, g, ksk, prm, P)
    dec, bits = oracle.bfv_decrypt(rot, sk, prm, with_noise=True)
    want = oracle.automorphism(msgs.astype(np.uint64)[:, None, :], g, [prm.t])[:, 0, :]
    assert np.array_equal(dec, oracle.centre_mod(want.astype(object), prm.t))
    assert bits < prm.delta.bit_length() - 2


def test_key_switch_with_identity_key_keeps_the_message():
    prm, P, sk, msgs, ct, ksk = _rotation_case(4096, 2, 50, 1, 85)
    out = oracle.key_switch(ct, ksk, prm, P)
    assert not np.array_equal(out, ct)  # a fresh a component
    assert np.array_equal(oracle.bfv_decrypt(out, sk, prm), oracle.centre_mod(msgs.astype(object), prm.t))
