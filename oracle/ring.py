"""Ring helpers over Z_q[X]/(X^N + 1) (test infrastructure; see package doc).

Galois automorphisms sigma_g : a(X) -> a(X^g) for odd g (they implement the
paper's slot rotation, Rot, used by the DensePack dot product of Section 3.2):
  * coefficient domain: X^i goes to (-1)^floor(i*g / N) * X^(i*g mod N);
  * NTT domain (evaluations at psi^(2*brv(i)+1), see `ntt`): a pure index
    permutation, out[i] = in[src(i)] with 2*brv(src(i)) + 1 = (2*brv(i)+1)*g mod 2N.
The tests check that the two agree through the transform.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import modq
from .nt import bit_reverse


def automorph_coeff(a, g: int, q: int) -> np.ndarray:
    """sigma_g on coefficient-domain residues (last axis), exact."""
    a = modq.asu64(a)
    n = a.shape[-1]
    out = np.zeros_like(a)
    for i in range(n):
        e = (i * g) % (2 * n)
        if e < n:
            out[..., e] = a[..., i]
        else:
            out[..., e - n] = modq.neg(a[..., i], q)
    return out


@lru_cache(maxsize=None)
def automorph_ntt_src(n: int, g: int) -> np.ndarray:
    """src(i) for the NTT-domain permutation of sigma_g."""
    bits = n.bit_length() - 1
    rev = {bit_reverse(i, bits): i for i in range(n)}
    src = np.empty(n, dtype=np.int64)
    for i in range(n):
        e = ((2 * bit_reverse(i, bits) + 1) * g) % (2 * n)
        src[i] = rev[(e - 1) // 2]
    return src


def automorph_ntt(ahat, g: int) -> np.ndarray:
    ahat = modq.asu64(ahat)
    return ahat[..., automorph_ntt_src(ahat.shape[-1], g)]


def galois_for_rotation(k: int, n: int) -> int:
    """Galois element 5^k mod 2N; rotates the slot vector left by k (k may be negative)."""
    two_n = 2 * n
    slots = n // 2
    return pow(5, k % slots, two_n)


def negacyclic_schoolbook(a, b, q: int) -> list[int]:
    """a*b mod (X^N + 1, q) by the O(N^2) product, Python ints (small N only)."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            t = ai * int(b[j])
            if k < n:
                out[k] += t
            else:
                out[k - n] -= t
    return [x % q for x in out]
