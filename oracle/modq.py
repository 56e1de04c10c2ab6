"""Exact elementwise arithmetic modulo one prime on numpy uint64 arrays.

Test infrastructure (see package doc).  Residues are integers in [0, q) held
as uint64.  For q < 2^32 the product of two residues fits in 64 bits and is
reduced with numpy's integer remainder.  For 2^32 <= q < 2^62 the quotient
floor(a*b/q) is estimated in 64-bit-mantissa extended precision (off by at
most a few units), the remainder a*b - quot*q is then formed exactly with
wrapping 64-bit integer arithmetic (the true remainder lies in a small window
around [0, q), so it is recovered exactly as a signed 64-bit value), and a few
conditional corrections bring it into [0, q).
"""
from __future__ import annotations

import numpy as np

U64 = np.uint64
_LD = np.longdouble
assert np.finfo(_LD).nmant >= 63, "extended precision (64-bit mantissa) is required"


def asu64(x) -> np.ndarray:
    return np.asarray(x, dtype=U64)


def add(a, b, q: int) -> np.ndarray:
    s = asu64(a) + asu64(b)
    return np.where(s >= U64(q), s - U64(q), s)


def sub(a, b, q: int) -> np.ndarray:
    a = asu64(a)
    b = asu64(b)
    return np.where(a >= b, a - b, a + (U64(q) - b))


def neg(a, q: int) -> np.ndarray:
    a = asu64(a)
    return np.where(a == 0, a, U64(q) - a)


def mul(a, b, q: int) -> np.ndarray:
    a = asu64(a)
    b = asu64(b)
    if q < (1 << 32):
        return (a * b) % U64(q)
    assert q < (1 << 62)
    quot = np.floor(a.astype(_LD) * b.astype(_LD) / _LD(q))
    quot = np.clip(quot, 0, None).astype(U64)
    with np.errstate(over="ignore"):
        r = (a * b - quot * U64(q)).view(np.int64)
    qi = np.int64(q)
    for _ in range(3):
        r = np.where(r < 0, r + qi, r)
        r = np.where(r >= qi, r - qi, r)
    return r.astype(U64)


def from_signed(x, q: int) -> np.ndarray:
    """Reduce signed integers (int64 array, |x| < 2^63) into [0, q)."""
    x = np.asarray(x, dtype=np.int64)
    r = np.mod(x, np.int64(q))  # numpy mod takes the sign of the divisor
    return r.astype(U64)


def centered(a, q: int) -> np.ndarray:
    """Map residues in [0, q) to the representative in [-(q-1)/2, (q-1)/2] (q odd)."""
    a = asu64(a)
    half = U64((q - 1) // 2)
    return np.where(a > half, a.astype(np.int64) - np.int64(q), a.astype(np.int64))


def pow_table(base: int, count: int, q: int) -> np.ndarray:
    """[base^0, base^1, ..., base^(count-1)] mod q."""
    out = np.empty(count, dtype=U64)
    x = 1
    for i in range(count):
        out[i] = x
        x = x * base % q
    return out
