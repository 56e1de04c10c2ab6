"""Number theory for the parameter sets (test infrastructure; see package doc).

Prime chain and root of unity conventions (the paper fixes none of them; it
only states that the ring dimension and modulus are chosen for 128-bit
security, Section 2.1 and Section 5 "Cryptosystem Settings"):
  * a modulus of b bits is the largest prime q < 2^b with q = 1 (mod 2N); the
    next modulus of the same size is the largest such prime below the previous;
  * the 2N-th root psi is x^((q-1)/(2N)) for x the smallest quadratic
    non-residue mod q, so that psi^N = -1.
"""
from __future__ import annotations

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (the first 12 prime bases)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
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


def primes_below(bits: int, count: int, two_n: int, below: int | None = None) -> list[int]:
    """`count` primes q = 1 mod two_n, scanning downward from 2^bits (or from `below`)."""
    start = (1 << bits) if below is None else below
    q = ((start - 1) // two_n) * two_n + 1
    if q >= start:
        q -= two_n
    out = []
    while len(out) < count:
        if q < 2:
            raise ValueError("ran out of candidates")
        if is_prime(q):
            out.append(q)
        q -= two_n
    return out


def smallest_nonresidue(q: int) -> int:
    x = 2
    while pow(x, (q - 1) // 2, q) != q - 1:
        x += 1
    return x


def root_2n(q: int, n: int) -> int:
    """psi with psi^n = -1 mod q (a primitive 2n-th root of unity)."""
    assert (q - 1) % (2 * n) == 0
    return pow(smallest_nonresidue(q), (q - 1) // (2 * n), q)


def inv(a: int, q: int) -> int:
    return pow(a % q, -1, q)


def bit_reverse(i: int, bits: int) -> int:
    r = 0
    for _ in range(bits):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r
