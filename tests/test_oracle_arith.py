"""Pins for the oracle's modular arithmetic and parameter generation.

Residue products are checked against Python's arbitrary-precision integers;
primes are certified by a Lucas (Pocklington-style) proof built from a full
factorisation of q - 1 by trial division, independent of the Miller-Rabin
routine that generated them; every skipped candidate of the downward scan is
shown composite by a small factor or a Fermat witness.
"""
import numpy as np
import pytest

from oracle import modq, nt, params as P

PRIMES = [
    nt.primes_below(30, 1, 8192)[0],
    nt.primes_below(36, 1, 8192)[0],
    nt.primes_below(40, 1, 32768)[0],
    nt.primes_below(60, 1, 32768)[0],
    nt.primes_below(62, 1, 64)[0],
]


@pytest.mark.parametrize("q", PRIMES)
def test_mul_add_sub_against_python_ints(q):
    rng = np.random.default_rng(q % 1000)
    a = rng.integers(0, q, 4000, dtype=np.uint64)
    b = rng.integers(0, q, 4000, dtype=np.uint64)
    edge = np.array([0, 1, q - 1, q - 2, q // 2, (q + 1) // 2], dtype=np.uint64)
    a = np.concatenate([a, np.repeat(edge, len(edge))])
    b = np.concatenate([b, np.tile(edge, len(edge))])
    ai, bi = [int(v) for v in a], [int(v) for v in b]
    assert [int(v) for v in modq.mul(a, b, q)] == [x * y % q for x, y in zip(ai, bi)]
    assert [int(v) for v in modq.add(a, b, q)] == [(x + y) % q for x, y in zip(ai, bi)]
    assert [int(v) for v in modq.sub(a, b, q)] == [(x - y) % q for x, y in zip(ai, bi)]
    assert [int(v) for v in modq.neg(a, q)] == [(-x) % q for x in ai]
    c = modq.centered(a, q)
    assert all(abs(int(v)) <= (q - 1) // 2 and (int(v) - x) % q == 0 for v, x in zip(c, ai))
    s = rng.integers(-(1 << 62), 1 << 62, 1000)
    assert [int(v) for v in modq.from_signed(s, q)] == [int(x) % q for x in s]


def _factor(n):
    """Full factorisation by trial division (cofactor below the bound squared is prime)."""
    f = {}
    for p in (2, 3, 5):
        while n % p == 0:
            f[p] = f.get(p, 0) + 1
            n //= p
    bound = int(n ** 0.5) + 1
    cand = np.arange(7, min(bound, 1 << 23) + 1, 2, dtype=np.int64)
    for lo in range(0, len(cand), 1 << 20):
        chunk = cand[lo: lo + (1 << 20)]
        if n < (1 << 62):
            hits = chunk[(np.int64(n) % chunk) == 0]
        else:
            hits = [int(c) for c in chunk if n % int(c) == 0]
        for p in hits:
            p = int(p)
            while n % p == 0:
                f[p] = f.get(p, 0) + 1
                n //= p
    assert n == 1 or n < (1 << 46), "cofactor must be provably prime"
    if n > 1:
        f[n] = f.get(n, 0) + 1
    return f


def _lucas_prime(q):
    fac = _factor(q - 1)
    for a in range(2, 200):
        if pow(a, q - 1, q) != 1:
            return False
        if all(pow(a, (q - 1) // p, q) != 1 for p in fac):
            return True
    return False


def _composite(n):
    for p in range(3, 2000, 2):
        if n % p == 0:
            return n != p
    return any(pow(a, n - 1, n) != 1 for a in (2, 3, 5, 7, 11))


@pytest.mark.parametrize("maker", [P.plain_n4096, P.ffconv_n8192, P.cifar_n16384])
def test_parameter_sets_prime_chain(maker):
    p = maker()
    two_n = 2 * p.n
    bits = list(p.q_bits)
    prev = {}
    for q, b in zip(p.q, bits):
        assert q % two_n == 1 and q < (1 << b)
        upper = prev.get(b, 1 << b)
        for cand in range(q + two_n, upper, two_n):
            assert _composite(cand), cand
        prev[b] = q
        assert _lucas_prime(q)
    assert p.p % two_n == 1 and p.p < (1 << p.p_bits) and _lucas_prime(p.p)
    for cand in range(p.p + two_n, 1 << p.p_bits, two_n):
        assert _composite(cand)
    for m in p.q + [p.p]:
        psi = p.psi[m]
        assert pow(psi, p.n, m) == m - 1  # psi^N = -1, hence order exactly 2N
    assert len(set(p.q + [p.p])) == len(p.q) + 1
