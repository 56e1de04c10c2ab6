"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Ring-level results must match the oracle bit for bit (integer work); decrypted
layer outputs must be within 1e-3 absolute of the FP64 convolution (Eq. 1).
Inputs (ciphertexts, plaintexts) are produced by the oracle from the seeded
`synth` draws and uploaded; the GPU side generates its own switching keys from
the same draws, so any key-generation mistake shows up as a rotation mismatch.
Small rings (N = 1024) span many workgroups and ragged output counts; the
full-size layers are checked on sampled outputs and by decrypted accuracy.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import conv as C  # noqa: E402
from oracle import encoding as E  # noqa: E402
from oracle import params as P  # noqa: E402
from oracle import reference as R  # noqa: E402
from oracle import scheme as S  # noqa: E402
from oracle import workloads as Wk  # noqa: E402
from oracle.ntt import intt as o_intt  # noqa: E402
from oracle.ntt import ntt as o_ntt  # noqa: E402

W = "unit"


def _he():
    from paper_2102_03494_amd import he
    return he


def _ctx(p, ws=1 << 28):
    he = _he()
    c = he.HEContext(p.n, p.q_bits, p.p_bits, workspace_bytes=ws)
    assert c.moduli == p.q + [p.p]
    return c


def _client(ctx, rotations=(), relin=False):
    from paper_2102_03494_amd.client import Client
    cl = Client(ctx, W)
    cl.gen_rotation_keys(rotations)
    if relin:
        cl.gen_relin_key()
    return cl


def _dev(a):
    return _he().to_device(a)


def _host(t):
    torch.cuda.synchronize()
    return _he().to_host(t)


SMALL = dict(n=1024, q_bits=(30, 30, 30, 30), p_bits=40)


@pytest.mark.parametrize("n,q_bits,p_bits", [
    (1024, (30, 30, 30), 36), (4096, (30, 30), 36), (8192, (30, 30, 30, 30), 40), (16384, (40,) * 6, 60),
    (2048, (42, 41), 40),  # f64 class at its largest primes (2^42 limit)
    (4096, (42, 41), 40),  # the same through a first radix-16 inverse pass (canonical input, 16 q sums)
])
def test_ntt_intt_bit_exact(n, q_bits, p_bits):
    p = P.Params(n, q_bits, p_bits, 1.0)
    ctx = _ctx(p, ws=1 << 20)
    mods = p.q + [p.p]
    rng = np.random.default_rng(n)
    a = np.stack([np.stack([rng.integers(0, m, n, dtype=np.uint64) for m in mods]) for _ in range(3)])
    d = _dev(a)
    ctx.ntt(d)
    got = _host(d)
    for t, m in enumerate(mods):
        assert np.array_equal(got[:, t], o_ntt(a[:, t], m, p.psi[m])), (t, m)
    ctx.intt(d)
    assert np.array_equal(_host(d), a)


# a second small chain in the f64 width class (40-bit ciphertext primes) with a
# wide-class (60-bit) P, so the 64-bit branches of every kernel are compared
# bit for bit too
SMALL40 = dict(n=2048, q_bits=(40, 40, 40, 40), p_bits=60, scale=2.0**30)


def _small_setup(rotations=(), relin=False, n=1024, chain=None):
    if chain is not None:
        p = P.Params(chain["n"], chain["q_bits"], chain["p_bits"], chain["scale"])
        octx = Wk.make_context(p, W, rotations=rotations, relin=relin)
        gctx = _ctx(p)
        return p, octx, gctx, _client(gctx, rotations, relin)
    p = P.Params(n, SMALL["q_bits"], SMALL["p_bits"], 2.0**25)
    octx = Wk.make_context(p, W, rotations=rotations, relin=relin)
    gctx = _ctx(p)
    cl = _client(gctx, rotations, relin)
    return p, octx, gctx, cl


def test_encrypt_and_decrypt_bit_exact():
    p, octx, gctx, cl = _small_setup()
    z = synth.message(W, p.slots)
    pt = E.encode(z, p, 4, p.scale)
    a, e = synth.encryption_draws(W, 0, p.q, p.n)
    oct_ = octx.encrypt(pt, p.scale, a, e)
    gct = cl.encrypt_pt(_dev(pt), p.scale, 0)
    assert np.array_equal(_host(gct.data)[0], oct_.c)
    dec = _host(gctx.decrypt(gct.data[0], cl.s_ntt))
    assert np.array_equal(dec, octx.decrypt_poly(oct_))
    vals = cl.decrypt(gct.data[0], p.scale)
    assert np.abs(vals - z).max() < 1e-5


def _enc_batch(octx, p, count, level=4, index0=0):
    cts = []
    for i in range(count):
        z = synth.message(W, p.slots, index=index0 + i)
        cts.append(Wk.encrypt_slots(octx, z, level, p.scale, W, index0 + i).c)
    return np.stack(cts)


def test_rotate_batch_bit_exact():
    steps = (1, 3, -7, 100)
    p, octx, gctx, cl = _small_setup(rotations=steps)
    batch = _enc_batch(octx, p, 5)
    he = _he()
    for k in steps:
        got = _host(gctx.rotate(he.Ct(_dev(batch), p.scale), k).data)
        want = S.rotate(p, octx, S.Ciphertext(batch, p.scale), k).c
        assert np.array_equal(got, want), k
    # in place (out aliases in) and at a lower level
    low = np.ascontiguousarray(batch[:, :, :2])
    d = _dev(low)
    gctx.rotate(he.Ct(d, p.scale), 3, out=d)
    assert np.array_equal(_host(d), S.rotate(p, octx, S.Ciphertext(low, p.scale), 3).c)


@pytest.mark.parametrize("q_bits,p_bits", [
    ((40,) * 6, 60),        # f64 primes + wide P: the two-class half-ring ModUp
    ((40, 40, 40), 41),     # one class (f64)
    ((30, 30, 30), 40),     # narrow primes + f64 P
    ((30, 30), 60),         # narrow primes + wide P
])
def test_rotate_n16384_half_ring_modup(q_bits, p_bits):
    """At N = 16384 ModUp runs as two half-ring workgroups per target (first
    transform stage fused into the lift); every class pair and every P
    grouping gives the oracle's bits."""
    n = 16384
    p = P.Params(n, q_bits, p_bits, 2.0**30)
    steps = (1, -3)
    octx = Wk.make_context(p, W, rotations=steps)
    gctx = _ctx(p, ws=1 << 27)
    _client(gctx, steps)
    he = _he()
    level = len(q_bits)
    cts = np.stack([np.stack([np.stack([synth.rng(W, "test", 900 + i, c, t).integers(0, p.q[t], n, dtype=np.uint64)
                                        for t in range(level)]) for c in range(2)]) for i in range(2)])
    want = {k: S.rotate(p, octx, S.Ciphertext(cts, 1.0), k).c for k in steps}
    for pg in range(1, min(level, 4) + 1):
        gctx.set_tuning("p_groups", level, pg)
        for k in steps:
            got = _host(gctx.rotate(he.Ct(_dev(cts), 1.0), k).data)
            assert np.array_equal(got, want[k]), (pg, k)
    # a lower level of the same chain (ragged jobs share the launch geometry)
    low = np.ascontiguousarray(cts[:, :, :level - 1])
    got = _host(gctx.rotate(he.Ct(_dev(low), 1.0), 1).data)
    assert np.array_equal(got, S.rotate(p, octx, S.Ciphertext(low, 1.0), 1).c)


@pytest.mark.parametrize("n,q_bits,p_bits", [(2048, (30,) * 4, 40), (8192, (30,) * 4, 40), (4096, (40,) * 3, 60)])
def test_modup_halves_knob_bit_exact(n, q_bits, p_bits):
    """ModUp as one workgroup per target or as two half-ring workgroups gives
    the oracle's bits on smaller rings too (the knob the autotuner sets)."""
    p = P.Params(n, q_bits, p_bits, 2.0**25)
    octx = Wk.make_context(p, W, rotations=(3,))
    gctx = _ctx(p, ws=1 << 27)
    _client(gctx, (3,))
    he = _he()
    level = len(q_bits)
    cts = np.stack([np.stack([np.stack([synth.rng(W, "test", 950 + i, c, t).integers(0, p.q[t], n, dtype=np.uint64)
                                        for t in range(level)]) for c in range(2)]) for i in range(3)])
    want = S.rotate(p, octx, S.Ciphertext(cts, 1.0), 3).c
    for halves in (0, 1):
        gctx.set_tuning("modup_halves", 0, halves)
        assert gctx.get_tuning("modup_halves", 0) == halves
        for pg in (1, 2):
            gctx.set_tuning("p_groups", level, pg)
            assert np.array_equal(_host(gctx.rotate(he.Ct(_dev(cts), 1.0), 3).data), want), (halves, pg)


@pytest.mark.parametrize("n,q_bits,p_bits", [(2048, (30,) * 4, 40), (4096, (40,) * 3, 60)])
def test_moddown_halves_knob_bit_exact(n, q_bits, p_bits):
    """ModDown as one workgroup per limb or as two half-ring workgroups gives
    the oracle's bits: rotations, an in-place rotate-and-sum (packed chains
    keep the whole-limb kernel, so the narrow chain checks that path), hoisted
    rotations and x^2 with relinearisation."""
    p = P.Params(n, q_bits, p_bits, 2.0**25)
    steps = [1 << j for j in range(5)]
    octx = Wk.make_context(p, W, rotations=steps + [3], relin=True)
    gctx = _ctx(p, ws=1 << 27)
    _client(gctx, steps + [3], True)
    he = _he()
    level = len(q_bits)
    cts = np.stack([np.stack([np.stack([synth.rng(W, "test", 970 + i, c, t).integers(0, p.q[t], n, dtype=np.uint64)
                                        for t in range(level)]) for c in range(2)]) for i in range(3)])
    ct = S.Ciphertext(cts, p.scale)
    want_rot = S.rotate(p, octx, ct, 3).c
    want_sum = C.rotate_and_sum(p, octx, ct, 5, C.Counts()).c
    want_hoist = [S.rotate(p, octx, S.Ciphertext(cts[:1], p.scale), k).c for k in (1, 3)]
    want_sq = S.square(p, octx, ct).c
    for halves in (0, 1, -1):
        gctx.set_tuning("moddown_halves", 0, halves)
        assert gctx.get_tuning("moddown_halves", 0) == (halves if halves >= 0 else 0)
        assert np.array_equal(_host(gctx.rotate(he.Ct(_dev(cts), p.scale), 3).data), want_rot), halves
        d = _dev(cts)
        gctx.rotsum(he.Ct(d, p.scale), 5)
        assert np.array_equal(_host(d), want_sum), halves
        hoisted = _host(gctx.rotate_hoisted(he.Ct(_dev(cts[:1]), p.scale), [1, 3]).data)
        for k in range(2):
            assert np.array_equal(hoisted[k], want_hoist[k][0]), (halves, k)
        assert np.array_equal(_host(gctx.square(he.Ct(_dev(cts), p.scale)).data), want_sq), halves
    with pytest.raises(he.HEError):
        gctx.set_tuning("moddown_halves", 0, 2)


def test_uploaded_oracle_keys_rotate_bit_exact():
    """The server context gets only keys: the oracle makes them on the CPU (the
    client), they are uploaded from host memory in the exchange layout, and
    rotations and the square then match the oracle bit for bit.  The GPU
    client helper makes the same key bits, and bad uploads leave the store
    unchanged."""
    steps = (1, -3, 17)
    p, octx, _, _ = _small_setup(rotations=steps, relin=True)
    he = _he()
    srv = _ctx(p)  # no secret ever enters this context
    gal = [S.galois_for_rotation(k, p.n) for k in steps]
    keys = np.stack([np.stack([octx.rot_keys[g].b, octx.rot_keys[g].a], axis=1) for g in gal])
    srv.upload_keys(gal, keys)
    rk = octx.relin_key
    srv.upload_keys([0], np.stack([rk.b, rk.a], axis=1)[None])
    batch = _enc_batch(octx, p, 3)
    for k in steps:
        got = _host(srv.rotate(he.Ct(_dev(batch), p.scale), k).data)
        assert np.array_equal(got, S.rotate(p, octx, S.Ciphertext(batch, p.scale), k).c), k
    got = _host(srv.square(he.Ct(_dev(batch[:, :, :3].copy()), p.scale)).data)
    assert np.array_equal(got, S.square(p, octx, S.Ciphertext(batch[:, :, :3].copy(), p.scale)).c)
    # the GPU client helper writes the same bits in the exchange layout
    from paper_2102_03494_amd.client import Client
    cl = Client(srv, W)
    assert np.array_equal(_host(cl.switch_key(gal[1])), keys[1])
    # a residue not below its modulus is refused and the store keeps the old key
    bad = keys[:1].copy()
    bad[0, 0, 0, 0, 5] = p.q[0]
    with pytest.raises(he.HEError, match="code -1"):
        srv.upload_keys(gal[:1], bad)
    with pytest.raises(he.HEError, match="code -1"):
        srv.upload_keys([gal[0], gal[0]], np.concatenate([keys[:1], keys[:1]]))
    got = _host(srv.rotate(he.Ct(_dev(batch), p.scale), steps[0]).data)
    assert np.array_equal(got, S.rotate(p, octx, S.Ciphertext(batch, p.scale), steps[0]).c)
    # freeing: a missing key frees nothing; then the rotation reports the missing key
    with pytest.raises(he.HEError, match="code -4"):
        srv.drop_keys([gal[0], 12345 | 1])
    assert srv.has_key(gal[0])
    srv.drop_keys([gal[0]])
    assert not srv.has_key(gal[0]) and srv.has_key(gal[1])
    with pytest.raises(he.HEError, match="code -4"):
        srv.rotate(he.Ct(_dev(batch), p.scale), steps[0])


def test_caller_owned_workspace():
    """A context given the caller's device buffer as its workspace computes the
    same bits; too small a buffer gives HE_ENOMEM, not an allocation."""
    steps = (1, 2)
    p, octx, gctx, cl = _small_setup(rotations=steps)
    he = _he()
    srv = he.HEContext(p.n, p.q_bits, p.p_bits)
    cl.gen_rotation_keys(steps, server=srv)
    batch = _enc_batch(octx, p, 4)
    want = _host(gctx.rotate(he.Ct(_dev(batch), p.scale), 2).data)
    tiny = torch.empty(16, dtype=torch.int64, device="cuda")
    srv.set_workspace(tiny)
    with pytest.raises(he.HEError, match="code -5"):
        srv.rotate(he.Ct(_dev(batch), p.scale), 2)
    buf = torch.empty((8 << 20) // 8, dtype=torch.int64, device="cuda")
    srv.set_workspace(buf)
    assert np.array_equal(_host(srv.rotate(he.Ct(_dev(batch), p.scale), 2).data), want)
    srv.set_workspace(None)
    srv.reserve(8 << 20)
    assert np.array_equal(_host(srv.rotate(he.Ct(_dev(batch), p.scale), 2).data), want)


def test_p_groups_do_not_change_bits():
    """Every split of the P target's digits (1..4 groups) gives the oracle's bits."""
    p, octx, gctx, cl = _small_setup(rotations=(5,))
    batch = _enc_batch(octx, p, 3)
    want = S.rotate(p, octx, S.Ciphertext(batch, p.scale), 5).c
    he = _he()
    gctx.set_tuning("p_groups", 4, 0)  # the cost model's choice
    default = gctx.get_tuning("p_groups", 4)
    assert 1 <= default <= 4
    for pg in (1, 2, 3, 4):
        gctx.set_tuning("p_groups", 4, pg)
        assert gctx.get_tuning("p_groups", 4) == pg
        got = _host(gctx.rotate(he.Ct(_dev(batch), p.scale), 5).data)
        assert np.array_equal(got, want), pg
    gctx.set_tuning("p_groups", 4, 0)
    assert gctx.get_tuning("p_groups", 4) == default
    with pytest.raises(he.HEError):
        gctx.set_tuning("p_groups", 4, 5)


def test_split_streams_do_not_change_bits():
    """DensePack with its outputs split into 2, 3 or 4 chains on as many
    streams gives the one-stream bits."""
    p, octx, gctx, cl = _small_setup(rotations=[1 << j for j in range(9)])
    geom = C.ConvGeom(9, 9, 2, 3, 1, 1)
    x = synth.image(W, (9, 9, 2), index=3)
    w = synth.weights(W, 31, (3, 3, 2, 2), 0.3)
    ct = Wk.encrypt_slots(octx, C.densepack_slots(x, geom, p.slots)[0], 3, p.scale, W, 9)
    pts = C.densepack_pt_scale(p, 3, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w, geom, 3, pts)
    he = _he()
    desc = he.HEContext.conv_desc(9, 9, 2, 3, 1, 1, 2, 9)
    outs = {}
    for split, parts in ((0, 2), (1, 2), (1, 3), (1, 4)):
        gctx.set_tuning("split_streams", 0, split)
        gctx.set_tuning("split_parts", 0, parts)
        assert gctx.get_tuning("split_streams", 0) == split and gctx.get_tuning("split_parts", 0) == parts
        outs[split, parts] = _host(gctx.conv_densepack(he.Ct(_dev(ct.c[None]), p.scale), desc, _dev(bf), pts).data)
    gctx.set_tuning("split_parts", 0, 2)
    for bad in (1, 5):
        with pytest.raises(he.HEError):
            gctx.set_tuning("split_parts", 0, bad)
    assert outs[0, 2].shape[0] == 162  # 81 outputs x 2 channels: chains of 81, 54 or 40-41
    for key in ((1, 2), (1, 3), (1, 4)):
        assert np.array_equal(outs[0, 2], outs[key]), key
    sample = [0, 40, 41, 80, 81, 108, 161]
    want, _ = C.conv_densepack(p, octx, ct, geom, bf, pts, outputs=[C.output_list(geom, 2)[i] for i in sample])
    for k, i in enumerate(sample):
        assert np.array_equal(outs[1, 4][i], want.c[k]), i


@pytest.mark.parametrize("chain", [None, SMALL40], ids=["30bit", "40bit"])
@pytest.mark.parametrize("fused", [1, 0])
def test_rotate_hoisted_bit_exact(chain, fused):
    """Hoisted rotations with ModDown fused into the inner product (1) or
    after it (0) give the bits of one-at-a-time rotations (the oracle's)."""
    steps = [1, 2, 5, 17, 255, -3]
    p, octx, gctx, cl = _small_setup(rotations=steps, chain=chain)
    gctx.set_tuning("hoist_fused", 0, fused)
    assert gctx.get_tuning("hoist_fused", 0) == fused
    ct = _enc_batch(octx, p, 1)[0]
    got = _host(gctx.rotate_hoisted(_he().Ct(_dev(ct), p.scale), steps).data)
    for r, k in enumerate(steps):
        assert np.array_equal(got[r], S.rotate(p, octx, S.Ciphertext(ct, p.scale), k).c), k


def test_rotsum_rescale_add_bit_exact():
    p, octx, gctx, cl = _small_setup(rotations=[1 << j for j in range(9)])
    batch = _enc_batch(octx, p, 3)
    he = _he()
    d = _dev(batch)
    gctx.rotsum(he.Ct(d, p.scale), 9)
    want = C.rotate_and_sum(p, octx, S.Ciphertext(batch, p.scale), 9, C.Counts())
    assert np.array_equal(_host(d), want.c)
    r = gctx.rescale(he.Ct(d, p.scale))
    assert np.array_equal(_host(r.data), S.rescale(p, want).c)
    out = torch.empty_like(d)
    gctx.add(out, he.Ct(d, p.scale), he.Ct(_dev(batch), p.scale))
    assert np.array_equal(_host(out), S.add(p, want, S.Ciphertext(batch, p.scale)).c)
    # operands at different scales are refused before any launch, output untouched
    before = out.clone()
    with pytest.raises(he.HEError, match="code -3"):
        gctx.add(out, he.Ct(d, p.scale), he.Ct(_dev(batch), p.scale * 2))
    assert torch.equal(out, before)


def test_square_bit_exact():
    p, octx, gctx, cl = _small_setup(relin=True)
    batch = _enc_batch(octx, p, 3, level=3)
    got = _host(gctx.square(_he().Ct(_dev(batch), p.scale)).data)
    assert np.array_equal(got, S.square(p, octx, S.Ciphertext(batch, p.scale)).c)


@pytest.mark.parametrize("chain", [None, SMALL40], ids=["30bit", "40bit"])
def test_hma_plain_and_scalar_bit_exact(chain):
    p, octx, gctx, cl = _small_setup(chain=chain)
    batch = _enc_batch(octx, p, 4, level=3)
    pts = np.stack([E.encode(synth.message(W, p.slots, index=40 + i), p, 4, 2.0**20) for i in range(4)])
    gal = [1, 5, 25, 2 * p.n - 5]
    acc = torch.empty((2, 3, p.n), dtype=torch.int64, device="cuda")
    he = _he()
    cts = he.Ct(_dev(batch), p.scale)
    got = gctx.hma_plain(acc, cts, _dev(pts), 1, 2.0**20, galois=gal)
    assert got.scale == p.scale * 2.0**20
    want = None
    from oracle.ring import automorph_ntt
    for i in range(4):
        prod = S.mul_plain(p, S.Ciphertext(batch[i], p.scale), automorph_ntt(pts[i], gal[i]), 2.0**20)
        want = prod if want is None else S.add(p, want, prod)
    assert np.array_equal(_host(acc), want.c)
    # accumulating into it: a second MulPC of the same scale adds, another scale is refused
    got2 = gctx.hma_plain(acc, he.Ct(cts.data[:1].contiguous(), p.scale), _dev(pts[:1]), 0, 2.0**20,
                          acc_scale=got.scale)
    want = S.add(p, want, S.mul_plain(p, S.Ciphertext(batch[0], p.scale), pts[0], 2.0**20))
    assert np.array_equal(_host(acc), want.c) and got2.scale == want.scale
    with pytest.raises(he.HEError, match="code -3"):
        gctx.hma_plain(acc, cts, _dev(pts), 1, 2.0**21, acc_scale=got.scale)
    w = [3, -7, 1 << 40, -(1 << 35) + 11]
    got = gctx.hma_scalar(acc, cts, w, w_scale=1.0)
    want = None
    for i in range(4):
        prod = S.mul_int(p, S.Ciphertext(batch[i], p.scale), w[i])
        want = prod if want is None else S.add(p, want, prod)
    assert np.array_equal(_host(acc), want.c) and got.scale == p.scale
    with pytest.raises(he.HEError, match="code -3"):
        gctx.hma_scalar(acc, cts, w, w_scale=4.0, acc_scale=p.scale)


def _densepack_case(p, octx, gctx, geom, o_c, level, outputs=None, std=0.1, wid=7):
    x = synth.image(W, (geom.h, geom.w, geom.c_in))
    w = synth.weights(W, wid, (geom.d, geom.d, geom.c_in, o_c), std)
    cts = [Wk.encrypt_slots(octx, v, level, p.scale, W, m).c for m, v in enumerate(C.densepack_slots(x, geom, p.slots))]
    xin = np.stack(cts)
    pts = C.densepack_pt_scale(p, level, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w, geom, level, pts)
    he = _he()
    desc = he.HEContext.conv_desc(geom.h, geom.w, geom.c_in, geom.d, geom.stride, geom.pad, o_c,
                                  int(math.log2(p.slots)))
    gout = gctx.conv_densepack(he.Ct(_dev(xin), p.scale), desc, _dev(bf), pts)
    return x, w, xin, bf, pts, gout


@pytest.mark.parametrize("shape,d,stride,pad,o_c", [
    ((6, 6, 3), 3, 1, 1, 3),    # 9 border classes, 108 outputs (ragged vs the chunking)
    ((5, 5, 8), 3, 2, 1, 2),    # 200 values over 512 slots -> 1 ct; stride 2 with padding
    ((8, 8, 12), 3, 1, 0, 1),   # 768 values over 512 slots: two input ciphertexts
])
def test_densepack_bit_exact_small(shape, d, stride, pad, o_c):
    p, octx, gctx, cl = _small_setup(rotations=[1 << j for j in range(9)])
    geom = C.ConvGeom(shape[0], shape[1], shape[2], d, stride, pad)
    x, w, xin, bf, pts, gout = _densepack_case(p, octx, gctx, geom, o_c, 3)
    got = _host(gout.data)
    want, _ = C.conv_densepack(p, octx, S.Ciphertext(xin, p.scale), geom, bf, pts)
    assert got.shape == want.c.shape
    assert np.array_equal(got, want.c)
    cnt = gctx.last_counts()
    assert cnt["rot"] == geom.spatial * o_c * 9 and cnt["mulpc"] == geom.spatial * o_c * geom.n_cts(p.slots)
    ref = R.conv2d(x, w, stride, pad)
    for idx in (0, len(got) // 2, len(got) - 1):
        o, rem = divmod(idx, geom.spatial)
        i, j = divmod(rem, geom.out_w)
        v = cl.decrypt(gout.data[idx], gout.scale, 4)
        assert np.abs(v - ref[i, j, o]).max() < 1e-3


def test_convpack_bit_exact():
    p, octx, gctx, cl = _small_setup()
    batch = _enc_batch(octx, p, 3, level=3)
    wts = synth.weights(W, 11, (3, 4), 0.2)
    want, _ = C.convpack(p, S.Ciphertext(batch, p.scale), wts, p.scale)
    got = gctx.conv_convpack(_he().Ct(_dev(batch), p.scale), wts, p.scale)
    assert np.array_equal(_host(got.data), want.c)
    assert got.scale == want.scale
    cnt = gctx.last_counts()
    assert cnt["mulpc"] == 3 * 4 and cnt["addcc"] == 4 * 2  # Table II: O_c K MulPC, O_c (K-1) AddCC
    # an input scale that cannot reach the target at this level is refused
    with pytest.raises(_he().HEError, match="code -3"):
        gctx.conv_convpack(_he().Ct(_dev(batch), p.q[2] * p.scale * 4), wts, p.scale)


@pytest.mark.parametrize("chain", [None, SMALL40], ids=["30bit", "40bit"])
def test_ffconv_layer_bit_exact_small(chain):
    """Whole FFConv layer (W1 DensePack, gather, 1x1 ConvPack, x^2) on a small
    ring: 30-bit primes (narrow class) and 40-bit primes with a 60-bit P (f64
    and wide classes: the 64-bit branches of the gather, the scalar MAC, the
    tensor square, relinearisation and ModDown)."""
    r_steps = 9 if chain is None else int(math.log2(chain["n"] // 2))
    p, octx, gctx, cl = _small_setup(rotations=[1 << j for j in range(r_steps)], relin=True, chain=chain)
    geom = C.ConvGeom(7, 7, 2, 3, 2, 1)
    x = synth.image(W, (7, 7, 2))
    w1 = synth.weights(W, 21, (3, 3, 2, 2), 0.3)
    w2 = synth.weights(W, 22, (2, 3), 0.4)
    level = 4
    ct = Wk.encrypt_slots(octx, C.densepack_slots(x, geom, p.slots)[0], level, p.scale, W, 0)
    pts = C.densepack_pt_scale(p, level, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w1, geom, level, pts)
    y, _ = C.conv_densepack(p, octx, ct, geom, bf, pts)
    target = C.pre_square_target(p, level - 2, p.scale)
    ms = C.gather_mask_scale(p, y.level, y.scale, target, 12)
    mask = C.encode_onehot(p, y.level, ms)
    z, _ = C.gather_convpack(p, y, geom.spatial, w2, 12, mask, ms)
    want, _ = C.square_rescale(p, octx, z)
    he = _he()
    desc = he.HEContext.conv_desc(7, 7, 2, 3, 2, 1, 2, r_steps)
    got = gctx.ffconv_layer(he.Ct(_dev(ct.c[None]), p.scale), desc, _dev(bf), pts, _dev(mask), ms, w2, 12, True)
    assert np.array_equal(_host(got.data), want.c)
    assert abs(got.scale - want.scale) <= 1e-12 * want.scale
    ref = R.ffconv_reference(x, w1, w2, 2, 1, square=True)
    for o in range(3):
        v = cl.decrypt(got.data[o], got.scale, geom.spatial)
        assert np.abs(v - ref[:, :, o].reshape(-1)).max() < 1e-3


def test_factorized_layer_bit_exact():
    """Eq. 2 end to end: W factorised by the product's truncated SVD at rank
    2, then the FFConv layer on the GPU equals the oracle's layer on the same
    factors bit for bit, and decrypts to the FP64 rank-2 conv within 1e-3;
    at full rank the factors reproduce W's conv."""
    from paper_2102_03494_amd import factorize as F
    p, octx, gctx, cl = _small_setup(rotations=[1 << j for j in range(9)])
    geom = C.ConvGeom(6, 6, 2, 3, 1, 1)
    x = synth.image(W, (6, 6, 2))
    w = synth.weights(W, 23, (3, 3, 2, 4), 0.2)
    level = 3
    ct = Wk.encrypt_slots(octx, C.densepack_slots(x, geom, p.slots)[0], level, p.scale, W, 0)
    he = _he()
    for r in (2, 4):
        w1, w2 = F.factorize(w, r)
        pts = C.densepack_pt_scale(p, level, p.scale, p.scale)
        bf = C.densepack_base_filters(p, w1, geom, level, pts)
        y, _ = C.conv_densepack(p, octx, ct, geom, bf, pts)
        ms = C.gather_mask_scale(p, y.level, y.scale, p.scale, 12)
        mask = C.encode_onehot(p, y.level, ms)
        want, _ = C.gather_convpack(p, y, geom.spatial, w2, 12, mask, ms)
        desc = he.HEContext.conv_desc(6, 6, 2, 3, 1, 1, r, 9)
        got = gctx.ffconv_layer(he.Ct(_dev(ct.c[None]), p.scale), desc, _dev(bf), pts, _dev(mask), ms, w2, 12, False)
        assert np.array_equal(_host(got.data), want.c), r
        ref = R.ffconv_reference(x, w1, w2, 1, 1)
        ref_w = R.conv2d(x, w, 1, 1)
        for o in range(4):
            v = cl.decrypt(got.data[o], got.scale, geom.spatial)
            assert np.abs(v - ref[:, :, o].reshape(-1)).max() < 1e-3
            if r == 4:  # full rank: the factorisation is exact
                assert np.abs(v - ref_w[:, :, o].reshape(-1)).max() < 1e-3


@pytest.mark.parametrize("chain,square", [(None, True), (None, False), (SMALL40, True)],
                         ids=["30bit-sq", "30bit", "40bit-sq"])
def test_ffconv_convpack_convpack_bit_exact(chain, square):
    """FFConv with both factors under ConvPack (CP-HI2C-CP, d = 1): the GPU
    layer on the client's Im2Col ciphertexts equals the oracle's bit for bit,
    executes no rotation, and decrypts to the FP64 reference within 1e-3."""
    p, octx, gctx, cl = _small_setup(relin=square, chain=chain)
    geom = C.ConvGeom(7, 7, 2, 3, 2, 1)
    x = synth.image(W, (7, 7, 2))
    w1 = synth.weights(W, 71, (3, 3, 2, 3), 0.3)
    w2 = synth.weights(W, 72, (3, 4), 0.4)
    level = 4
    vecs = C.im2col_slots(x, geom, p.slots)
    from paper_2102_03494_amd import layers as Ly
    gvecs = Ly.im2col_layout(x, Ly.Geometry(7, 7, 2, 3, 2, 1), p.slots)
    assert all(np.array_equal(a, b) for a, b in zip(vecs, gvecs))  # the product's layout is the oracle's
    cts = np.stack([Wk.encrypt_slots(octx, v, level, p.scale, W, 400 + k).c for k, v in enumerate(vecs)])
    w1m = R.filters_as_matrix(w1)
    want, cnt = C.convpack_convpack(p, octx, S.Ciphertext(cts, p.scale), w1m, w2, p.scale, square=square)
    he = _he()
    got = gctx.ffconv_layer_convpack(he.Ct(_dev(cts), p.scale), w1m, w2, p.scale, square=square)
    assert np.array_equal(_host(got.data), want.c)
    assert got.scale == want.scale
    gc = gctx.last_counts()
    assert (gc["mulpc"], gc["addcc"], gc["rot"], gc["square"]) == (cnt.mulpc, cnt.addcc, 0, cnt.square)
    ref = R.ffconv_reference(x, w1, w2, 2, 1, square=square)
    for o in range(4):
        v = cl.decrypt(got.data[o], got.scale, geom.spatial)
        assert np.abs(v - ref[:, :, o].reshape(-1)).max() < 1e-3


def test_batch_rotate_ragged_levels():
    """One launch set over items at levels 4, 2, 3, 4, 1 with different steps (0 copies)."""
    steps = [1, 3, -7, 0, 100]
    levels = [4, 2, 3, 4, 1]
    p, octx, gctx, cl = _small_setup(rotations=[k for k in steps if k])
    cts = [_enc_batch(octx, p, 1, level=lv, index0=20 + i)[0] for i, lv in enumerate(levels)]
    ins = [_dev(c) for c in cts]
    outs = [torch.empty_like(t) for t in ins]
    gctx.batch_rotate(outs, ins, steps)

    def rot(c, k):
        return c if k == 0 else S.rotate(p, octx, S.Ciphertext(c, p.scale), k).c

    for c, o, k in zip(cts, outs, steps):
        assert np.array_equal(_host(o), rot(c, k)), k
    gctx.batch_rotate(ins, ins, steps, accumulate=True)  # in place: t + Rot(t, k)
    for c, t, k in zip(cts, ins, steps):
        want = S.add(p, S.Ciphertext(c, p.scale), S.Ciphertext(rot(c, k), p.scale)).c
        assert np.array_equal(_host(t), want), k


def test_batch_rescale_and_mul_plain_ragged():
    p, octx, gctx, cl = _small_setup()
    levels = [4, 2, 3, 2]
    cts = [_enc_batch(octx, p, 1, level=lv, index0=40 + i)[0] for i, lv in enumerate(levels)]
    pts = [E.encode(synth.message(W, p.slots, index=60 + i), p, lv, 2.0**20) for i, lv in enumerate(levels)]
    ins = [_dev(c) for c in cts]
    prods = [torch.empty_like(t) for t in ins]
    gctx.batch_mul_plain(prods, ins, [_dev(x) for x in pts])
    for c, pt, o in zip(cts, pts, prods):
        assert np.array_equal(_host(o), S.mul_plain(p, S.Ciphertext(c, 1.0), pt, 1.0).c)
    outs = [torch.empty((2, lv - 1, p.n), dtype=torch.int64, device="cuda") for lv in levels]
    gctx.batch_rescale(outs, ins)
    for c, o in zip(cts, outs):
        assert np.array_equal(_host(o), S.rescale(p, S.Ciphertext(c, p.scale)).c)


def test_combine_cp_dp_bit_exact():
    """CP -> DP combine of 5 channel ciphertexts (16 values each) into one dense ciphertext."""
    offsets = C.combine_offsets(5, 16, 8)
    p, octx, gctx, cl = _small_setup(rotations=offsets)
    vals = synth.message(W, 80, index=7)
    chans = np.stack([Wk.encrypt_slots(octx, np.concatenate([vals[16 * o:16 * o + 16], np.zeros(p.slots - 16)]),
                                       3, p.scale, W, 70 + o).c for o in range(5)])
    want, cnt = C.combine_cp_to_dp(p, octx, S.Ciphertext(chans, p.scale), 16, 8)
    got = gctx.combine_cp_dp(_he().Ct(_dev(chans), p.scale), 16, 8)
    assert np.array_equal(_host(got.data), want.c)
    assert gctx.last_counts()["rot"] == cnt.rot == 4
    dense = cl.decrypt(got.data[0], p.scale, 80)
    assert np.abs(dense - vals).max() < 1e-4


def test_empty_and_out_of_range_inputs_are_refused():
    """Empty batches and levels outside 1..L are refused with an error code
    before any launch (the output buffers keep their contents)."""
    import ctypes
    p, octx, gctx, cl = _small_setup(rotations=(1,))
    he = _he()
    lib = gctx.lib
    L = len(p.q_bits)
    buf = torch.full((2, L, p.n), 7, dtype=torch.int64, device="cuda")
    out = torch.full_like(buf, 9)
    ptr = he._ptr
    # count 0
    assert lib.he_rotate(gctx.h, ptr(out), ptr(buf), 0, L, 1, None) == -1
    assert lib.he_square(gctx.h, ptr(out), ptr(buf), 0, L, None) == -1
    assert lib.he_rotsum(gctx.h, ptr(buf), 0, L, 1, None) == -1
    steps = (ctypes.c_int32 * 1)(1)
    assert lib.he_rotate_hoisted(gctx.h, ptr(buf), L, steps, 0, ptr(out), None) == -1
    # levels outside 1..L
    assert lib.he_rotate(gctx.h, ptr(out), ptr(buf), 1, L + 1, 1, None) == -1
    assert lib.he_rotate(gctx.h, ptr(out), ptr(buf), 1, 0, 1, None) == -1
    assert lib.he_rescale(gctx.h, ptr(out), ptr(buf), 1, 1, None) in (-1, -2)
    torch.cuda.synchronize()
    assert bool((buf == 7).all()) and bool((out == 9).all())
    # the context still works afterwards
    ct = _enc_batch(octx, p, 1)
    got = _host(gctx.rotate(he.Ct(_dev(ct), p.scale), 1).data)
    assert np.array_equal(got, S.rotate(p, octx, S.Ciphertext(ct, p.scale), 1).c)


@pytest.mark.parametrize("parts", [2, 3])
def test_densepack_chunked_workspace_same_bits(parts):
    """A workspace that holds only part of a layer's outputs makes the layer
    run in chunks (the last one ragged, each split over `parts` chains where
    it is large enough); the bits equal the one-chunk run and the oracle's."""
    p, octx, gctx, cl = _small_setup(rotations=[1 << j for j in range(9)])
    geom = C.ConvGeom(9, 9, 2, 3, 1, 1)
    x = synth.image(W, (9, 9, 2), index=5)
    w = synth.weights(W, 33, (3, 3, 2, 2), 0.3)
    ct = Wk.encrypt_slots(octx, C.densepack_slots(x, geom, p.slots)[0], 3, p.scale, W, 11)
    pts = C.densepack_pt_scale(p, 3, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w, geom, 3, pts)
    he = _he()
    desc = he.HEContext.conv_desc(9, 9, 2, 3, 1, 1, 2, 9)
    gctx.set_tuning("split_parts", 0, parts)
    whole = _host(gctx.conv_densepack(he.Ct(_dev(ct.c[None]), p.scale), desc, _dev(bf), pts).data)
    # about 100 outputs' key-switch temporaries: chunks of ~100 and ~62 of the 162
    per_output = ((3 * 3 + 2 + 2) * p.n + 2 * 3 * p.n + 2 * p.n + 128) * 8
    small = torch.empty((100 * per_output + (1 << 20)) // 8, dtype=torch.int64, device="cuda")
    gctx.set_workspace(small)
    chunked = _host(gctx.conv_densepack(he.Ct(_dev(ct.c[None]), p.scale), desc, _dev(bf), pts).data)
    gctx.set_workspace(None)
    gctx.set_tuning("split_parts", 0, 2)
    assert chunked.shape[0] == 162
    assert np.array_equal(whole, chunked)
    sample = [0, 99, 100, 161]
    want, _ = C.conv_densepack(p, octx, ct, geom, bf, pts, outputs=[C.output_list(geom, 2)[i] for i in sample])
    for k, i in enumerate(sample):
        assert np.array_equal(chunked[i], want.c[k]), i
