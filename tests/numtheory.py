"""Number theory for the tests, independent of the oracle's C core: Python
integers, pow() and gcd only.  Used to pin the oracle's parameter search."""
from __future__ import annotations

import math
import random


def _probable_prime(n: int, rounds: int = 24) -> bool:
    """Miller-Rabin with random bases -- used only to steer factoring; every
    primality claim in the tests rests on a certificate below."""
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    rng = random.Random(n)
    for _ in range(rounds):
        a = rng.randrange(2, n - 1)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _rho(n: int) -> int:
    """A non-trivial factor of composite n (Pollard rho, Brent's cycle)."""
    if n % 2 == 0:
        return 2
    rng = random.Random(n ^ 0x5DEECE66D)
    while True:
        y, c, m = rng.randrange(1, n), rng.randrange(1, n), 128
        g, r, qq = 1, 1, 1
        while g == 1:
            x = y
            for _ in range(r):
                y = (y * y + c) % n
            k = 0
            while k < r and g == 1:
                ys = y
                for _ in range(min(m, r - k)):
                    y = (y * y + c) % n
                    qq = qq * abs(x - y) % n
                g = math.gcd(qq, n)
                k += m
            r *= 2
        if g == n:
            g = 1
            while g == 1:
                ys = (ys * ys + c) % n
                g = math.gcd(abs(x - ys), n)
        if g != n:
            return g


def factor(n: int) -> dict[int, int]:
    """Prime factorisation {p: e} of n >= 1."""
    out: dict[int, int] = {}
    for p in range(2, 1000):
        while n % p == 0:
            out[p] = out.get(p, 0) + 1
            n //= p
    stack = [n] if n > 1 else []
    while stack:
        m = stack.pop()
        if _probable_prime(m):
            out[m] = out.get(m, 0) + 1
            continue
        f = _rho(m)
        stack += [f, m // f]
    return out


def certify_prime(n: int) -> tuple[bool, int | None]:
    """Lucas primality proof: n is prime iff some g has g^(n-1) = 1 and
    g^((n-1)/p) != 1 for every prime p | n-1.  The factors of n-1 are
    certified recursively (trial division below 2^32).  Returns (is_prime,
    g) where g is the witness, a primitive root mod n."""
    if n < 2:
        return False, None
    if n < (1 << 32):
        r = math.isqrt(n)
        for d in range(2, r + 1):
            if n % d == 0:
                return False, None
        # small primes: still find a primitive root for the caller
    fac = factor(n - 1)
    for p in fac:
        if p >= (1 << 32) and not certify_prime(p)[0]:
            return False, None
        if p < (1 << 32) and any(p % d == 0 for d in range(2, math.isqrt(p) + 1)):
            return False, None
    for g in range(2, min(n, 10_000)):
        if pow(g, n - 1, n) != 1:
            return False, None
        if all(pow(g, (n - 1) // p, n) != 1 for p in fac):
            return True, g
    return False, None


def is_composite_proved(n: int) -> bool:
    """True when n is shown composite: a Fermat witness (2^(n-1) != 1 mod n)
    or an explicit factor."""
    if n % 2 == 0 or pow(2, n - 1, n) != 1:
        return True
    f = _rho(n) if not _probable_prime(n) else None
    return f is not None and 1 < f < n and n % f == 0
