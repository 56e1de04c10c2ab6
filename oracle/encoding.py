"""CKKS slot encoding and decoding (test infrastructure; see package doc).

The paper packs one message per slot (Section 1, packed SIMD encryption;
Section 3.2, DensePack and ConvPack) but uses BFV's integer slots.  Here we
use the CKKS canonical embedding over n = N/2 complex slots:
  * slot j corresponds to the root zeta^(5^j mod 2N), zeta = exp(i*pi/N);
  * a real vector z (length <= n, zero padded) maps to the real polynomial
    m_k = (2/N) * Re sum_j z_j zeta^(-k*5^j), k < N, i.e. the unique real
    polynomial with m(zeta^(5^j)) = z_j;
  * the plaintext is round-half-away(scale * m_k) reduced into each limb and
    moved to the NTT domain.
Decoding reverses this: centered CRT of the limbs, divide by the scale, and
evaluate at zeta^(5^j).  Both sums are evaluated with a length-2N FFT.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import modq
from .ntt import intt, ntt


@lru_cache(maxsize=None)
def slot_exponents(n_ring: int) -> np.ndarray:
    """5^j mod 2N for j < N/2."""
    two_n = 2 * n_ring
    out = np.empty(n_ring // 2, dtype=np.int64)
    x = 1
    for j in range(n_ring // 2):
        out[j] = x
        x = x * 5 % two_n
    return out


def round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def embed_inverse(z, n_ring: int) -> np.ndarray:
    """Real coefficients m_k (float64, length N) of the polynomial carrying slots z."""
    z = np.asarray(z, dtype=np.complex128)
    slots = n_ring // 2
    zz = np.zeros(slots, dtype=np.complex128)
    zz[: len(z)] = z
    e = slot_exponents(n_ring)
    v = np.zeros(2 * n_ring, dtype=np.complex128)
    v[e] = zz
    v[(2 * n_ring - e) % (2 * n_ring)] = np.conj(zz)
    return (np.fft.fft(v)[:n_ring] / n_ring).real


def embed(m, n_ring: int) -> np.ndarray:
    """Slot values m(zeta^(5^j)), j < N/2, of real coefficients m (complex128)."""
    m = np.asarray(m, dtype=np.float64)
    padded = np.zeros(2 * n_ring, dtype=np.complex128)
    padded[:n_ring] = m
    w = np.fft.ifft(padded) * (2 * n_ring)
    return w[slot_exponents(n_ring)]


def encode_int(z, n_ring: int, scale: float) -> np.ndarray:
    """Integer coefficients round(scale * m) as int64 (|value| < 2^62 asserted)."""
    c = round_half_away(scale * embed_inverse(z, n_ring))
    assert np.all(np.abs(c) < 2.0**62)
    return c.astype(np.int64)


def to_rns_ntt(coeffs_int64, moduli, psis) -> np.ndarray:
    """Signed integer coefficients -> NTT-domain residues, shape (len(moduli), N)."""
    return np.stack([ntt(modq.from_signed(coeffs_int64, q), q, psis[q]) for q in moduli])


def encode(z, params, level: int, scale: float) -> np.ndarray:
    moduli = params.moduli(level)
    return to_rns_ntt(encode_int(z, params.n, scale), moduli, params.psi)


def encode_constant_int(value: int, params, level: int) -> np.ndarray:
    """The constant polynomial `value` in NTT form (every evaluation equals value)."""
    moduli = params.moduli(level)
    return np.stack([np.full(params.n, value % q, dtype=np.uint64) for q in moduli])


def crt_centered(limbs_coeff, moduli) -> list[int]:
    """Centered representatives mod prod(moduli) of coefficient-domain residues."""
    big_q = 1
    for q in moduli:
        big_q *= q
    terms = []
    for q in moduli:
        qhat = big_q // q
        terms.append((qhat, pow(qhat % q, -1, q)))
    n = limbs_coeff.shape[-1]
    out = []
    for k in range(n):
        x = 0
        for t, q in enumerate(moduli):
            qhat, qhat_inv = terms[t]
            x += (int(limbs_coeff[t, k]) * qhat_inv % q) * qhat
        x %= big_q
        if x > big_q // 2:
            x -= big_q
        out.append(x)
    return out


def decode_poly(limbs_ntt, params, scale: float, n_values: int | None = None) -> np.ndarray:
    """Real slot values of an NTT-domain plaintext (e.g. a decrypted message)."""
    level = limbs_ntt.shape[0]
    moduli = params.moduli(level)
    coeff = np.stack([intt(limbs_ntt[t], q, params.psi[q]) for t, q in enumerate(moduli)])
    ints = crt_centered(coeff, moduli)
    m = np.array([float(x) for x in ints]) / scale
    z = embed(m, params.n).real
    return z if n_values is None else z[:n_values]
