"""Pins for the oracle's transforms and ring products (App. C, App. C.1).

Checks: the by-definition NTT against the independent big-integer mirror,
its closed forms, INTT o NTT = id, the fast mode against the definition, the
schoolbook product against numpy's integer polynomial product folded by
X^N = -1, and the convolution theorem INTT(NTT(a) . NTT(b)) = a * b."""
import numpy as np
import pytest

import oracle
from oracle import mirror
from synth import Stream

SMALL = [(8, 50), (16, 60), (32, 50), (64, 60), (256, 60)]


def rand_poly(seed, N, q):
    return Stream(seed, 2).below(N, q)


def brv(i, logn):
    return int(format(i, f"0{logn}b")[::-1], 2)


@pytest.mark.parametrize("N,bits", SMALL[:4])
def test_ntt_def_matches_bigint_mirror(N, bits):
    for q in oracle.find_primes(N, bits, 2):
        psi = oracle.find_psi(q, N)
        a = rand_poly(N + bits, N, q)
        got = oracle.ntt_def(a, q, psi)
        want = mirror.ntt_def([int(v) for v in a], q, psi)
        assert [int(v) for v in got] == want


@pytest.mark.parametrize("N,bits", SMALL)
def test_ntt_closed_forms(N, bits):
    """NTT(1) = (1, ..., 1) and NTT(X^k)[i] = psi^((2 brv(i) + 1) k)."""
    q = oracle.find_primes(N, bits, 1)[0]
    psi = oracle.find_psi(q, N)
    logn = N.bit_length() - 1
    one = np.zeros(N, dtype=np.uint64)
    one[0] = 1
    assert np.all(oracle.ntt_def(one, q, psi) == 1)
    for k in (1, 2, N // 2 + 1, N - 1):
        xk = np.zeros(N, dtype=np.uint64)
        xk[k] = 1
        got = oracle.ntt_def(xk, q, psi)
        want = [pow(psi, (2 * brv(i, logn) + 1) * k, q) for i in range(N)]
        assert [int(v) for v in got] == want


@pytest.mark.parametrize("N,bits", SMALL)
def test_inverse_and_fast_mode(N, bits):
    for q in oracle.find_primes(N, bits, 2):
        psi = oracle.find_psi(q, N)
        a = rand_poly(3 * N, N, q)
        A = oracle.ntt_def(a, q, psi)
        assert np.array_equal(oracle.intt_def(A, q, psi), a)
        assert np.array_equal(oracle.ntt_fast(a, q, psi), A)
        assert np.array_equal(oracle.intt_fast(A, q, psi), a)


@pytest.mark.parametrize("N,bits", [(4096, 50), (8192, 60)])
def test_fast_mode_equals_definition_at_full_size(N, bits):
    """For every (N, q) the configurations use: one random polynomial, every
    word, forward and inverse."""
    for q in oracle.find_primes(N, bits, 2 if N == 4096 else 3):
        psi = oracle.find_psi(q, N)
        a = rand_poly(q % 1000, N, q)
        A = oracle.ntt_fast(a, q, psi)
        assert np.array_equal(A, oracle.ntt_def(a, q, psi))
        assert np.array_equal(oracle.intt_def(A, q, psi), a)


def numpy_negacyclic(a, b, q):
    """Integer polynomial product by numpy (object dtype, exact), folded by
    X^N = -1, then reduced mod q."""
    N = len(a)
    full = np.convolve(np.array([int(v) for v in a], dtype=object), np.array([int(v) for v in b], dtype=object))
    full = np.concatenate([full, np.zeros(2 * N - full.size, dtype=object)])
    return [int(v) % q for v in (full[:N] - full[N:])]


@pytest.mark.parametrize("N,bits", SMALL)
def test_schoolbook_product(N, bits):
    q = oracle.find_primes(N, bits, 1)[0]
    a, b = rand_poly(5, N, q), rand_poly(6, N, q)
    c = oracle.negacyclic_mul(a, b, q)
    assert [int(v) for v in c] == numpy_negacyclic(a, b, q)
    if N <= 64:
        assert [int(v) for v in c] == mirror.negacyclic_mul([int(v) for v in a], [int(v) for v in b], q)
    for k in (0, 1, N // 2, N - 1):
        assert oracle.negacyclic_coeff(a, b, k, q) == int(c[k])
    # X * X^(N-1) = X^N = -1
    x1 = np.zeros(N, dtype=np.uint64)
    x1[1] = 1
    xn1 = np.zeros(N, dtype=np.uint64)
    xn1[N - 1] = 1
    m1 = oracle.negacyclic_mul(x1, xn1, q)
    assert int(m1[0]) == q - 1 and int(m1[1:].sum()) == 0


@pytest.mark.parametrize("N,bits", SMALL + [(4096, 50)])
def test_convolution_theorem(N, bits):
    """INTT(NTT(a) . NTT(b)) equals the schoolbook negacyclic product."""
    q = oracle.find_primes(N, bits, 1)[0]
    psi = oracle.find_psi(q, N)
    a, b = rand_poly(7, N, q), rand_poly(8, N, q)
    A, B = oracle.ntt_fast(a, q, psi), oracle.ntt_fast(b, q, psi)
    C = np.array([int(x) * int(y) % q for x, y in zip(A, B)], dtype=np.uint64)
    assert np.array_equal(oracle.intt_fast(C, q, psi), oracle.negacyclic_mul(a, b, q))


def test_batched_transform_layout(prm4096):
    """ntt() over [n][L][N] transforms limb l with (q_l, psi_l), in both modes."""
    p = prm4096
    x = np.stack([np.stack([rand_poly(10 * i + l, p.N, p.q[l]) for l in range(p.L)]) for i in range(2)])
    y = oracle.ntt(x, p, oracle.MODE_FAST)
    for i in range(2):
        for l in range(p.L):
            assert np.array_equal(y[i, l], oracle.ntt_fast(x[i, l], p.q[l], p.psi[l]))
    assert np.array_equal(oracle.intt(y, p, oracle.MODE_FAST), x)
    y0 = oracle.ntt(x[:1], p, oracle.MODE_DEF)
    assert np.array_equal(y0, y[:1])
