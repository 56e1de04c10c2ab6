"""Pins for the oracle's scheme operations (encrypt, rotate, key switch, rescale, square).

Decrypted results are compared with the slot-wise operation on the cleartext
(rotation = np.roll, product = elementwise), within bounds set by the noise of
each step; hoisted rotations must equal one-at-a-time rotations bit for bit; a
key switch under the key for s itself must leave the decryption unchanged;
rescale obeys the deterministic per-coefficient bound (1 + ||s||_1) / 2.
"""
import numpy as np

import synth
from oracle import encoding as E
from oracle import params as P
from oracle import scheme as S
from oracle import workloads as Wk
from oracle.ntt import intt
from oracle.encoding import crt_centered

W = "unit"


def _setup(rotations=(1, 2, 7, -5), relin=True, n=512):
    p = P.Params(n, (30, 30, 30), 36, float(2**25))
    ctx = Wk.make_context(p, W, rotations=rotations, relin=relin)
    z = synth.message(W, p.slots)
    ct = Wk.encrypt_slots(ctx, z, 3, p.scale, W, 0)
    return p, ctx, z, ct


def test_encrypt_decrypt_and_rotations():
    p, ctx, z, ct = _setup()
    assert np.abs(ctx.decrypt(ct) - z).max() < 1e-5
    for k in (1, 2, 7, -5):
        r = S.rotate(p, ctx, ct, k)
        assert np.abs(ctx.decrypt(r) - np.roll(z, -k)).max() < 1e-4
    hs = S.rotate_hoisted(p, ctx, ct, [1, 2, 7, -5])
    for k, h in zip((1, 2, 7, -5), hs):
        assert np.array_equal(h.c, S.rotate(p, ctx, ct, k).c)


def test_batched_ops_equal_single():
    p, ctx, z, ct = _setup(rotations=(3,), relin=False, n=256)
    ct2 = Wk.encrypt_slots(ctx, -z, 3, p.scale, W, 1)
    both = S.Ciphertext(np.stack([ct.c, ct2.c]), ct.scale)
    rb = S.rotate(p, ctx, both, 3)
    assert np.array_equal(rb.c[0], S.rotate(p, ctx, ct, 3).c)
    assert np.array_equal(rb.c[1], S.rotate(p, ctx, ct2, 3).c)
    sb = S.rescale(p, both)
    assert np.array_equal(sb.c[1], S.rescale(p, ct2).c)


def test_key_switch_with_identity_key():
    p, ctx, z, ct = _setup(rotations=(), relin=False, n=256)
    a, e = synth.switch_key_draws(W, 12345, p.q + [p.p], p.n, p.max_level)
    key = ctx.make_switch_key(ctx.s_ntt, a, e)
    u0, u1 = S.key_switch(p, ct.c[1], key)
    out = ct.c.copy()
    for t in range(3):
        out[0, t] = (ct.c[0, t].astype(object) + u0[t].astype(object)) % p.q[t]
    out[1] = u1
    assert np.abs(ctx.decrypt(S.Ciphertext(out.astype(np.uint64), ct.scale)) - z).max() < 1e-4


def test_rescale_deterministic_bound():
    p, ctx, z, ct = _setup(rotations=(), relin=False, n=256)
    big = S.mul_plain(p, ct, E.encode(z, p, 3, p.q[2]), p.q[2])
    small = S.rescale(p, big)
    s_l1 = int(np.abs(ctx.s_coeff).sum())

    def coeffs(c):
        m = ctx.decrypt_poly(c)
        lim = np.stack([intt(m[t], p.q[t], p.psi[p.q[t]]) for t in range(c.level)])
        return crt_centered(lim, p.q[: c.level])

    before, after = coeffs(big), coeffs(small)
    ql = p.q[2]
    worst = max(abs(a * ql - b) for a, b in zip(after, before)) / ql
    assert worst <= (1 + s_l1) / 2
    assert small.scale == big.scale / ql
    assert np.abs(ctx.decrypt(small) - z * z).max() < 1e-4


def test_square_relinearise_rescale():
    p, ctx, z, ct = _setup(rotations=(), relin=True, n=512)
    # pre-square scale chosen so that the square and its rescale return to 2^25
    target = np.sqrt(p.q[1] * p.scale)
    x = S.rescale(p, S.mul_plain(p, ct, E.encode(np.ones(p.slots), p, 3, p.q[2] * target / p.scale),
                                 p.q[2] * target / p.scale))
    y = S.rescale(p, S.square(p, ctx, x))
    assert abs(y.scale / p.scale - 1) < 1e-9
    assert np.abs(ctx.decrypt(y) - z * z).max() < 1e-4
