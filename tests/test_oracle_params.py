"""Pins for the oracle's parameter search (primes, roots of unity, BFV scale).

The paper states no HE parameters; the reading is: the L largest primes below
2^bits with q = 1 mod 2N, descending, and psi the smallest primitive 2N-th
root of unity mod q.  These tests prove the oracle's choices with arithmetic
that shares nothing with its C core: Lucas certificates, Fermat witnesses of
compositeness, and a primitive root from the certificate."""
import math

import pytest

import oracle
from tests import numtheory as nt

CASES = [(4096, 50, 2), (8192, 60, 3), (64, 50, 2), (16, 60, 2)]


@pytest.mark.parametrize("N,bits,L", CASES)
def test_primes_certified_and_congruent(N, bits, L):
    qs = oracle.find_primes(N, bits, L)
    assert qs == sorted(qs, reverse=True) and len(set(qs)) == L
    for q in qs:
        assert q < 2 ** bits and q % (2 * N) == 1
        ok, g = nt.certify_prime(q)
        assert ok, q


@pytest.mark.parametrize("N,bits,L", CASES[:2])
def test_primes_are_the_largest(N, bits, L):
    """Every candidate = 1 mod 2N between q_{L-1} and 2^bits that was skipped
    is proved composite."""
    qs = oracle.find_primes(N, bits, L)
    step = 2 * N
    c = (2 ** bits - 2) // step * step + 1
    skipped = 0
    while c > qs[-1]:
        if c not in qs:
            assert nt.is_composite_proved(c), c
            skipped += 1
        c -= step
    assert skipped > 0


@pytest.mark.parametrize("N,bits,L", CASES)
def test_psi_is_smallest_primitive_root(N, bits, L):
    """psi^N = -1, and psi is the minimum of the N primitive 2N-th roots,
    enumerated from a primitive root g of the Lucas certificate (a different
    generator than the oracle's search uses)."""
    for q in oracle.find_primes(N, bits, L):
        psi = oracle.find_psi(q, N)
        assert pow(psi, N, q) == q - 1
        ok, g = nt.certify_prime(q)
        w = pow(g, (q - 1) // (2 * N), q)
        roots = {pow(w, k, q) for k in range(1, 2 * N, 2)}
        assert len(roots) == N
        assert all(pow(r, N, q) == q - 1 for r in list(roots)[:16])
        assert psi == min(roots)


def test_is_prime_small_range():
    """The C Miller-Rabin agrees with trial division on [0, 5000) and on the
    Carmichael numbers below 10^6 (all composite)."""
    for n in range(5000):
        td = n >= 2 and all(n % d for d in range(2, math.isqrt(n) + 1))
        assert oracle.is_prime(n) == td, n
    for n in (561, 1105, 1729, 2465, 2821, 6601, 8911, 10585, 15841, 29341, 41041, 46657, 52633, 62745,
              63973, 75361, 101101, 115921, 126217, 162401, 172081, 188461, 252601, 278545, 294409, 314821,
              334153, 340561, 399001, 410041, 449065, 488881, 512461):
        assert not oracle.is_prime(n)


def test_bfv_scale(prm4096, prm8192):
    for p in (prm4096, prm8192):
        assert p.Q == math.prod(p.q)
        assert p.delta * p.t <= p.Q < (p.delta + 1) * p.t
        assert all(d == p.delta % q for d, q in zip(p.delta_l, p.q))
    assert prm4096.Q.bit_length() == 100 and prm8192.Q.bit_length() == 180
