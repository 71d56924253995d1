"""Pure-Python big-integer mirror of the oracle for tiny N (N <= 64).

TEST INFRASTRUCTURE ONLY.  Independent of heoracle.c: Python integers, no
RNS (a single modulus Q = prod q_l is used directly), no fast transforms.
It exists to check the C core and the RNS/CRT flow against arithmetic that
shares nothing with them.

Passages: ring Z_Q[X]/(X^N+1) (Sec. 2.1); BFV b = a*sk + delta*m + e and
its decryption (App. C); NTT as evaluation at the odd powers of a primitive
2N-th root (App. C.1).
"""
from __future__ import annotations


def brv(i: int, logn: int) -> int:
    """Bit reversal of i over logn bits, via its binary string."""
    return int(format(i, f"0{logn}b")[::-1], 2) if logn else 0


def ntt_def(a: list[int], q: int, psi: int) -> list[int]:
    """out[i] = a(psi^(2*brv(i)+1)) mod q, by Horner's rule."""
    N = len(a)
    logn = N.bit_length() - 1
    out = []
    for i in range(N):
        x = pow(psi, 2 * brv(i, logn) + 1, q)
        acc = 0
        for c in reversed(a):
            acc = (acc * x + c) % q
        out.append(acc)
    return out


def negacyclic_mul(a: list[int], b: list[int], Q: int) -> list[int]:
    """Product in Z_Q[X]/(X^N+1): full integer product, then fold the upper
    half back with a minus sign (X^N = -1)."""
    N = len(a)
    full = [0] * (2 * N)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            full[i + j] += ai * bj
    return [(full[k] - full[k + N]) % Q for k in range(N)]


def bfv_encrypt(m: list[int], sk: list[int], a: list[int], e: list[int], Q: int, t: int) -> tuple[list[int], list[int]]:
    """(a, b) with b = a*sk + floor(Q/t)*m + e over Z_Q."""
    delta = Q // t
    as_ = negacyclic_mul(a, sk, Q)
    b = [(as_[k] + delta * m[k] + e[k]) % Q for k in range(len(m))]
    return list(a), b


def bfv_decrypt(ct: tuple[list[int], list[int]], sk: list[int], Q: int, t: int) -> list[int]:
    """m = round(t * (b - a*sk mod Q) / Q) mod t, centred in [-t/2, t/2)."""
    a, b = ct
    as_ = negacyclic_mul(a, sk, Q)
    out = []
    for k in range(len(a)):
        v = (b[k] - as_[k]) % Q
        m = ((t * v + Q // 2) // Q) % t
        out.append(m - t if 2 * m >= t else m)
    return out


def ct_mul_plain(ct, w: list[int], Q: int):
    """Ciphertext times a plaintext polynomial with signed integer coefficients."""
    a, b = ct
    return negacyclic_mul(a, w, Q), negacyclic_mul(b, w, Q)


def ct_add(x, y, Q: int):
    return [(u + v) % Q for u, v in zip(x[0], y[0])], [(u + v) % Q for u, v in zip(x[1], y[1])]
