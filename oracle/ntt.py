"""Negacyclic number-theoretic transform (test infrastructure; see package doc).

Definition (the convention fixed here; the paper does not discuss the
transform, which sits inside every rotation and square it times): for a
polynomial a of degree < N over Z_q and psi a primitive 2N-th root of unity,

    ahat[i] = a(psi^(2*brv(i) + 1)) = sum_j a_j * psi^((2*brv(i)+1)*j)   (mod q),

with brv the log2(N)-bit reversal, i.e. evaluations at the odd powers of psi
listed in bit-reversed order.  `ntt_definition` writes this sum out with Python
ints (small N only).  The fast route used everywhere else is written as
"twist by psi^j, cyclic DFT with omega = psi^2 in natural order, then read the
outputs at bit-reversed positions"; the cyclic DFT is the textbook iterative
radix-2 decimation-in-time recursion on bit-reversed input.  `intt` undoes each
step in reverse order and scales by N^-1.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import modq
from .nt import bit_reverse, inv


@lru_cache(maxsize=None)
def brv_perm(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    return np.array([bit_reverse(i, bits) for i in range(n)], dtype=np.int64)


def ntt_definition(a, q: int, psi: int) -> list[int]:
    """O(N^2) evaluation of the definition with Python ints (small N only)."""
    n = len(a)
    bits = n.bit_length() - 1
    out = []
    for i in range(n):
        e = 2 * bit_reverse(i, bits) + 1
        x = pow(psi, e, q)
        acc = 0
        xp = 1
        for j in range(n):
            acc = (acc + int(a[j]) * xp) % q
            xp = xp * x % q
        out.append(acc)
    return out


@lru_cache(maxsize=None)
def _tables(n: int, q: int, psi: int):
    omega = psi * psi % q
    omega_inv = inv(omega, q)
    psi_pow = modq.pow_table(psi, n, q)
    psi_inv_pow = modq.pow_table(inv(psi, q), n, q)
    stage_fwd, stage_inv = [], []
    size = 2
    while size <= n:
        half = size // 2
        stage_fwd.append(modq.pow_table(pow(omega, n // size, q), half, q))
        stage_inv.append(modq.pow_table(pow(omega_inv, n // size, q), half, q))
        size *= 2
    return psi_pow, psi_inv_pow, stage_fwd, stage_inv, inv(n, q)


def _cyclic_dft(x: np.ndarray, q: int, stage_tw) -> np.ndarray:
    """Natural-order cyclic DFT over Z_q along the last axis (radix-2 DIT)."""
    n = x.shape[-1]
    lead = x.shape[:-1]
    x = x[..., brv_perm(n)]
    size = 2
    s = 0
    while size <= n:
        half = size // 2
        y = x.reshape(lead + (n // size, 2, half))
        even = y[..., 0, :]
        odd = modq.mul(y[..., 1, :], stage_tw[s], q)
        x = np.stack([modq.add(even, odd, q), modq.sub(even, odd, q)], axis=-2).reshape(lead + (n,))
        size *= 2
        s += 1
    return x


def ntt(a, q: int, psi: int) -> np.ndarray:
    """Forward negacyclic NTT along the last axis (any leading batch shape)."""
    a = modq.asu64(a)
    n = a.shape[-1]
    psi_pow, _, stage_fwd, _, _ = _tables(n, q, psi)
    twisted = modq.mul(a, psi_pow, q)
    return _cyclic_dft(twisted, q, stage_fwd)[..., brv_perm(n)]


def intt(ahat, q: int, psi: int) -> np.ndarray:
    """Inverse of `ntt` along the last axis."""
    ahat = modq.asu64(ahat)
    n = ahat.shape[-1]
    _, psi_inv_pow, _, stage_inv, n_inv = _tables(n, q, psi)
    natural = np.empty_like(ahat)
    natural[..., brv_perm(n)] = ahat
    x = _cyclic_dft(natural, q, stage_inv)
    x = modq.mul(x, np.uint64(n_inv), q)
    return modq.mul(x, psi_inv_pow, q)
