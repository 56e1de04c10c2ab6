"""Pins for the negacyclic NTT, the automorphisms and the slot encoding.

* The fast NTT equals its O(N^2) definition on small rings, for 30-, 40- and
  60-bit primes; INTT(NTT(a)) = a; pointwise products in the NTT domain equal
  the schoolbook negacyclic product mod (X^N + 1).
* sigma_g is pinned as the ring homomorphism sending X to X^g: it is additive,
  multiplicative (checked with schoolbook products), fixes constants and sends
  X to X^g; composition follows g*h mod 2N; the NTT-domain permutation equals
  the transform of the coefficient-domain map.
* Encoding: a constant encodes to the constant polynomial (closed form); the
  one-hot slot-0 vector has coefficients (2/N) cos(pi k / N) (closed form);
  each slot is the value of the polynomial at zeta^(5^j), evaluated here by a
  direct sum; decode(encode(z)) is within the deterministic rounding bound
  N / (2 scale); sigma_{5^k} rotates the slots left by k.
"""
import numpy as np
import pytest

from oracle import encoding as E
from oracle import modq, nt
from oracle import ntt as T
from oracle import params as P
from oracle import ring

SMALL_PRIMES = {
    16: [nt.primes_below(b, 1, 32)[0] for b in (30, 40, 60)],
    32: [nt.primes_below(b, 1, 64)[0] for b in (30, 36, 60)],
}


@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("bits", [30, 40, 60])
def test_ntt_matches_definition(n, bits):
    q = nt.primes_below(bits, 1, 2 * n)[0]
    psi = nt.root_2n(q, n)
    rng = np.random.default_rng(n + bits)
    a = rng.integers(0, q, n, dtype=np.uint64)
    assert [int(v) for v in T.ntt(a, q, psi)] == T.ntt_definition(a, q, psi)
    assert (T.intt(T.ntt(a, q, psi), q, psi) == a).all()


@pytest.mark.parametrize("n", [16, 32])
def test_negacyclic_product(n):
    for q in SMALL_PRIMES[n]:
        psi = nt.root_2n(q, n)
        rng = np.random.default_rng(q % 97)
        a = rng.integers(0, q, n, dtype=np.uint64)
        b = rng.integers(0, q, n, dtype=np.uint64)
        prod = T.intt(modq.mul(T.ntt(a, q, psi), T.ntt(b, q, psi), q), q, psi)
        assert [int(v) for v in prod] == ring.negacyclic_schoolbook(a, b, q)


def test_large_ntt_roundtrip_batched():
    p = P.cifar_n16384()
    rng = np.random.default_rng(3)
    for m in (p.q[0], p.p):
        a = rng.integers(0, m, (2, p.n), dtype=np.uint64)
        f = T.ntt(a, m, p.psi[m])
        assert (T.intt(f, m, p.psi[m]) == a).all()
        assert (f[1] == T.ntt(a[1], m, p.psi[m])).all()


def _monomial(n, e, q):
    """X^e reduced mod X^N + 1 as residues."""
    v = np.zeros(n, dtype=np.uint64)
    e %= 2 * n
    if e < n:
        v[e] = 1
    else:
        v[e - n] = q - 1
    return v


@pytest.mark.parametrize("g", [3, 5, 25, 31, 63])
def test_automorphism_is_the_substitution_homomorphism(g):
    n = 32
    q = SMALL_PRIMES[32][0]
    rng = np.random.default_rng(g)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    sa, sb = ring.automorph_coeff(a, g, q), ring.automorph_coeff(b, g, q)
    # multiplicative
    ab = np.array(ring.negacyclic_schoolbook(a, b, q), dtype=np.uint64)
    assert [int(v) for v in ring.automorph_coeff(ab, g, q)] == ring.negacyclic_schoolbook(sa, sb, q)
    # additive, fixes constants, X -> X^g
    assert (ring.automorph_coeff(modq.add(a, b, q), g, q) == modq.add(sa, sb, q)).all()
    const = np.zeros(n, dtype=np.uint64)
    const[0] = 7
    assert (ring.automorph_coeff(const, g, q) == const).all()
    assert (ring.automorph_coeff(_monomial(n, 1, q), g, q) == _monomial(n, g, q)).all()
    # composition and NTT-domain agreement
    h = 5
    comp = ring.automorph_coeff(ring.automorph_coeff(a, h, q), g, q)
    assert (comp == ring.automorph_coeff(a, (g * h) % (2 * n), q)).all()
    psi = nt.root_2n(q, n)
    assert (ring.automorph_ntt(T.ntt(a, q, psi), g) == T.ntt(sa, q, psi)).all()


def test_encode_closed_forms():
    n = 64
    m = E.embed_inverse(np.full(n // 2, 0.75), n)
    assert abs(m[0] - 0.75) < 1e-12 and np.abs(m[1:]).max() < 1e-12
    z = np.zeros(n // 2)
    z[0] = 1.0
    k = np.arange(n)
    assert np.abs(E.embed_inverse(z, n) - (2.0 / n) * np.cos(np.pi * k / n)).max() < 1e-12
    assert (E.encode_int(np.full(n // 2, 0.5), n, 2.0**20) == np.concatenate([[2**19], np.zeros(n - 1)])).all()


def test_slots_are_evaluations_at_powers_of_five():
    n = 64
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, n // 2)
    m = E.embed_inverse(z, n)
    zeta = np.exp(1j * np.pi / n)
    for j in range(n // 2):
        root = zeta ** pow(5, j, 2 * n)
        val = sum(m[k] * root**k for k in range(n))
        assert abs(val - z[j]) < 1e-9
    assert np.abs(E.embed(m, n) - z).max() < 1e-9


def test_decode_encode_rounding_bound_and_rotation():
    p = P.Params(256, (30, 30), 36, float(2**20))
    rng = np.random.default_rng(11)
    z = rng.uniform(-1, 1, p.slots)
    pt = E.encode(z, p, 2, p.scale)
    back = E.decode_poly(pt, p, p.scale)
    assert np.abs(back - z).max() <= p.n / (2 * p.scale)
    for k in (1, 3, -2):
        g = ring.galois_for_rotation(k, p.n)
        rot = E.decode_poly(ring.automorph_ntt(pt, g), p, p.scale)
        assert np.abs(rot - np.roll(z, -k)).max() <= p.n / (2 * p.scale)
