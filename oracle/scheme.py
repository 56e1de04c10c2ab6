"""RNS CKKS-style scheme operations (test infrastructure; see package doc).

The paper's primitives are MulPC (plaintext x ciphertext), AddCC, Rot and
Square (Table I caption; Section 2.1; Square in Table VI).  They are realised
here as follows; every step is written out plainly, limb by limb.

Ciphertext: (c0, c1), each `level` limbs of N residues in the NTT domain, plus
a float scale.  Decryption is c0 + c1*s.

Keys (client side, from the draws of `synth`): a secret s with ternary
coefficients; for a target key s' (sigma_g(s) for a rotation, s^2 for
relinearisation) a hybrid switching key with one digit per ciphertext prime:
for digit j and every modulus t of {q_0..q_{L-1}, P},
    b_j = -a_j*s + e_j + [t == j] * (P mod q_t) * s'   (mod m_t),   a_j uniform.

Key switching of a polynomial d at level l (limbs q_0..q_{l-1}):
  1. d_j = d mod q_j in the coefficient domain, centred into (-q_j/2, q_j/2);
  2. each centred digit is reduced mod every q_t (t < l) and mod P, then NTT;
  3. (u0, u1) = sum_j D_j * (b_j, a_j) over those l+1 moduli;
  4. ModDown: r = centred(u mod P) (coefficient domain), u_t <- (u_t - r) * P^-1.
Then u0 + u1*s = d*s' + small.

Rotation left by k: g = 5^k mod 2N, Rot(c) = (sigma_g(c0) + u0, u1) with
(u0, u1) = KeySwitch(sigma_g(c1)) under the key for sigma_g(s).
Hoisted rotations decompose c1 once and apply sigma_g to the lifted digits; the
digits of sigma_g(c1) are exactly sigma_g of the digits of c1 (the centred
representative commutes with the signed coefficient permutation because every
q_j is odd), so the two routes give identical bits.

Rescale at level l: r = centred(c mod q_{l-1}) (coefficient domain),
c_t <- (c_t - r) * q_{l-1}^-1 mod q_t for t < l-1, and scale /= q_{l-1}.
Square: (c0^2, 2*c0*c1, c1^2), then key switch of the c1^2 part under the key
for s^2 (relinearisation).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import modq
from .encoding import decode_poly
from .ntt import intt, ntt
from .ring import automorph_ntt, galois_for_rotation


@dataclass
class Ciphertext:
    c: np.ndarray  # uint64, shape (..., 2, level, N), NTT domain (leading batch dims allowed)
    scale: float

    @property
    def level(self) -> int:
        return self.c.shape[-2]

    def copy(self) -> "Ciphertext":
        return Ciphertext(self.c.copy(), self.scale)


@dataclass
class SwitchKey:
    b: np.ndarray  # uint64 (dnum, L+1, N): moduli q_0..q_{L-1}, then P
    a: np.ndarray  # uint64 (dnum, L+1, N)


class Context:
    """Holds the parameter set and the client's keys (secret + switching keys)."""

    def __init__(self, params, secret_coeffs):
        self.params = params
        self.all_moduli = params.q + [params.p]
        self.s_coeff = np.asarray(secret_coeffs, dtype=np.int64)
        # s in the NTT domain for every modulus (ciphertext primes then P)
        self.s_ntt = np.stack(
            [ntt(modq.from_signed(self.s_coeff, m), m, params.psi[m]) for m in self.all_moduli]
        )
        self.rot_keys: dict[int, SwitchKey] = {}
        self.relin_key: SwitchKey | None = None

    # ---- keys -------------------------------------------------------------
    def make_switch_key(self, s_prime_ntt, a_draws, e_draws) -> SwitchKey:
        """a_draws: (dnum, L+1, N) uniform residues (NTT domain); e_draws: (dnum, N) ints."""
        p = self.params
        big_l = p.max_level
        b = np.empty((big_l, big_l + 1, p.n), dtype=np.uint64)
        for j in range(big_l):
            for t, m in enumerate(self.all_moduli):
                e_hat = ntt(modq.from_signed(e_draws[j], m), m, p.psi[m])
                val = modq.sub(e_hat, modq.mul(a_draws[j, t], self.s_ntt[t], m), m)
                if t == j:
                    val = modq.add(val, modq.mul(s_prime_ntt[t], np.uint64(p.p % m), m), m)
                b[j, t] = val
        return SwitchKey(b=b, a=np.asarray(a_draws, dtype=np.uint64).copy())

    def add_rotation_key(self, k: int, a_draws, e_draws) -> int:
        g = galois_for_rotation(k, self.params.n)
        s_rot = automorph_ntt(self.s_ntt, g)
        self.rot_keys[g] = self.make_switch_key(s_rot, a_draws, e_draws)
        return g

    def set_relin_key(self, a_draws, e_draws):
        s2 = np.stack([modq.mul(self.s_ntt[t], self.s_ntt[t], m) for t, m in enumerate(self.all_moduli)])
        self.relin_key = self.make_switch_key(s2, a_draws, e_draws)

    # ---- client: encrypt / decrypt ---------------------------------------
    def encrypt(self, pt_ntt, scale: float, a_draws, e_draw) -> Ciphertext:
        """Secret-key encryption of an NTT-domain plaintext at its level."""
        p = self.params
        level = pt_ntt.shape[0]
        c = np.empty((2, level, p.n), dtype=np.uint64)
        for t in range(level):
            m = p.q[t]
            e_hat = ntt(modq.from_signed(e_draw, m), m, p.psi[m])
            c0 = modq.sub(modq.add(pt_ntt[t], e_hat, m), modq.mul(a_draws[t], self.s_ntt[t], m), m)
            c[0, t] = c0
            c[1, t] = a_draws[t]
        return Ciphertext(c, scale)

    def decrypt_poly(self, ct: Ciphertext) -> np.ndarray:
        p = self.params
        out = np.empty((ct.level, p.n), dtype=np.uint64)
        for t in range(ct.level):
            m = p.q[t]
            out[t] = modq.add(ct.c[0, t], modq.mul(ct.c[1, t], self.s_ntt[t], m), m)
        return out

    def decrypt(self, ct: Ciphertext, n_values: int | None = None) -> np.ndarray:
        return decode_poly(self.decrypt_poly(ct), self.params, ct.scale, n_values)


# ---- server-side operations (no secret needed) ------------------------------
# All of them accept leading batch dimensions on the ciphertext arrays; limbs
# are always the second-to-last axis and components the third-to-last.

def add(params, x: Ciphertext, y: Ciphertext) -> Ciphertext:
    assert x.level == y.level
    out = np.empty(np.broadcast_shapes(x.c.shape, y.c.shape), dtype=np.uint64)
    for t in range(x.level):
        out[..., t, :] = modq.add(x.c[..., t, :], y.c[..., t, :], params.q[t])
    return Ciphertext(out, x.scale)


def mul_plain(params, x: Ciphertext, pt_ntt, pt_scale: float) -> Ciphertext:
    """MulPC: slot-wise product with an NTT-domain plaintext (limbs on axis -2)."""
    pt_ntt = np.asarray(pt_ntt, dtype=np.uint64)
    batch = np.broadcast_shapes(x.c.shape[:-3], pt_ntt.shape[:-2])
    out = np.empty(batch + x.c.shape[-3:], dtype=np.uint64)
    for t in range(x.level):
        # the plaintext limb broadcasts over both ciphertext components
        out[..., t, :] = modq.mul(x.c[..., t, :], np.expand_dims(pt_ntt[..., t, :], -2), params.q[t])
    return Ciphertext(out, x.scale * pt_scale)


def mul_int(params, x: Ciphertext, w: int) -> Ciphertext:
    """Product with an exact integer (a constant plaintext); the caller tracks its scale."""
    out = np.empty_like(x.c)
    for t in range(x.level):
        q = params.q[t]
        out[..., t, :] = modq.mul(x.c[..., t, :], np.uint64(int(w) % q), q)
    return Ciphertext(out, x.scale)


def _drop_last_limb(params, c, divisor_modulus: int, keep: int):
    """(c_t - centred(c mod m)) * m^-1 mod q_t for t < keep; c[..., keep, :] is mod m."""
    r = modq.centered(intt(c[..., keep, :], divisor_modulus, params.psi[divisor_modulus]), divisor_modulus)
    out = np.empty(c.shape[:-2] + (keep, params.n), dtype=np.uint64)
    for t in range(keep):
        q = params.q[t]
        r_hat = ntt(modq.from_signed(r, q), q, params.psi[q])
        out[..., t, :] = modq.mul(modq.sub(c[..., t, :], r_hat, q), np.uint64(pow(divisor_modulus, -1, q)), q)
    return out


def rescale(params, x: Ciphertext) -> Ciphertext:
    level = x.level
    assert level >= 2
    ql = params.q[level - 1]
    out = _drop_last_limb(params, x.c, ql, level - 1)
    return Ciphertext(out, x.scale / ql)


def decompose(params, d_ntt) -> list[np.ndarray]:
    """Centred digits (int64, coefficient domain) of an NTT-domain polynomial (limbs on axis -2)."""
    level = d_ntt.shape[-2]
    digits = []
    for j in range(level):
        qj = params.q[j]
        digits.append(modq.centered(intt(d_ntt[..., j, :], qj, params.psi[qj]), qj))
    return digits


def lift_digits(params, digits) -> list[list[np.ndarray]]:
    """lifted[j][t]: NTT of digit j modulo the t-th of (q_0..q_{l-1}, P)."""
    level = len(digits)
    moduli = params.q[:level] + [params.p]
    return [[ntt(modq.from_signed(dj, m), m, params.psi[m]) for m in moduli] for dj in digits]


def inner_product(params, lifted, key: SwitchKey) -> np.ndarray:
    """u = sum_j lifted_j * (b_j, a_j) over (q_0..q_{l-1}, P): (..., 2, level + 1, N)."""
    level = len(lifted)
    moduli = params.q[:level] + [params.p]
    key_index = list(range(level)) + [params.max_level]
    batch = lifted[0][0].shape[:-1]
    u = np.zeros(batch + (2, level + 1, params.n), dtype=np.uint64)
    for j in range(level):
        for t, m in enumerate(moduli):
            kt = key_index[t]
            u[..., 0, t, :] = modq.add(u[..., 0, t, :], modq.mul(lifted[j][t], key.b[j, kt], m), m)
            u[..., 1, t, :] = modq.add(u[..., 1, t, :], modq.mul(lifted[j][t], key.a[j, kt], m), m)
    return u


def mod_down(params, u: np.ndarray) -> np.ndarray:
    """ModDown: (..., level + 1, N) over (q_0..q_{l-1}, P) to
    round(u / P) over (q_0..q_{l-1})."""
    return _drop_last_limb(params, u, params.p, u.shape[-2] - 1)


def inner_product_moddown(params, lifted, key: SwitchKey):
    """(u0, u1) = ModDown(sum_j lifted_j * (b_j, a_j)), each (..., level, N)."""
    out = mod_down(params, inner_product(params, lifted, key))
    return out[..., 0, :, :], out[..., 1, :, :]


def key_switch(params, d_ntt, key: SwitchKey):
    return inner_product_moddown(params, lift_digits(params, decompose(params, d_ntt)), key)


def _finish_rotation(params, x: Ciphertext, g: int, u0, u1) -> Ciphertext:
    c0 = automorph_ntt(x.c[..., 0, :, :], g)
    out = np.empty_like(x.c)
    for t in range(x.level):
        out[..., 0, t, :] = modq.add(c0[..., t, :], u0[..., t, :], params.q[t])
    out[..., 1, :, :] = u1
    return Ciphertext(out, x.scale)


def rotate(params, keys: Context, x: Ciphertext, k: int) -> Ciphertext:
    """Rot: slot rotation left by k (one key switch)."""
    g = galois_for_rotation(k, params.n)
    key = keys.rot_keys[g]
    u0, u1 = key_switch(params, automorph_ntt(x.c[..., 1, :, :], g), key)
    return _finish_rotation(params, x, g, u0, u1)


def rotate_hoisted(params, keys: Context, x: Ciphertext, ks) -> list[Ciphertext]:
    """Several rotations of one ciphertext sharing one digit decomposition."""
    lifted = lift_digits(params, decompose(params, x.c[..., 1, :, :]))
    outs = []
    for k in ks:
        g = galois_for_rotation(k, params.n)
        moved = [[automorph_ntt(v, g) for v in row] for row in lifted]
        u0, u1 = inner_product_moddown(params, moved, keys.rot_keys[g])
        outs.append(_finish_rotation(params, x, g, u0, u1))
    return outs


def square(params, keys: Context, x: Ciphertext) -> Ciphertext:
    """ct x ct square with relinearisation (the scale squares; no rescale here)."""
    level = x.level
    shape = x.c.shape[:-3] + (level, params.n)
    d0 = np.empty(shape, dtype=np.uint64)
    d1 = np.empty(shape, dtype=np.uint64)
    d2 = np.empty(shape, dtype=np.uint64)
    for t in range(level):
        q = params.q[t]
        c0, c1 = x.c[..., 0, t, :], x.c[..., 1, t, :]
        d0[..., t, :] = modq.mul(c0, c0, q)
        d1[..., t, :] = modq.mul(modq.mul(c0, c1, q), np.uint64(2), q)
        d2[..., t, :] = modq.mul(c1, c1, q)
    u0, u1 = key_switch(params, d2, keys.relin_key)
    out = np.empty(x.c.shape, dtype=np.uint64)
    for t in range(level):
        q = params.q[t]
        out[..., 0, t, :] = modq.add(d0[..., t, :], u0[..., t, :], q)
        out[..., 1, t, :] = modq.add(d1[..., t, :], u1[..., t, :], q)
    return Ciphertext(out, x.scale * x.scale)
