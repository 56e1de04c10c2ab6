"""Pins for the FP64 reference, the packed HE conv layers of the oracle and the count model.

* conv2d (Eq. 1, im2col + one matrix product) equals a direct six-loop
  convolution; W1 followed by the 1x1 W2 equals the conv with W1 W2 (Eq. 2 is
  an exact identity at full rank); the truncated SVD residual equals the tail
  of the spectrum computed from eigenvalues of W^T W (Eckart-Young-Mirsky).
* The HE layers decrypt to the FP64 reference within 1e-3 absolute: an
  all-ones rotate-and-sum gives N/2 in every slot; a single-tap filter returns
  the shifted input; DensePack with padding (several border classes) and with
  the input split over several ciphertexts; gather + 1x1 ConvPack with an
  identity W2 returns the gathered channels; the full FFConv layer with x^2;
  the CP->DP combine lays channels out exactly as DensePack does; the
  one-hot arrangement puts replicated value j in slot j and zeros elsewhere.
* The standalone ConvPack layer (Table II) decrypts to the FP64 per-pixel
  matrix product, counts O_c K MulPC and O_c (K - 1) AddCC, lands on its
  target scale, returns its inputs for W = I and is linear in W.
* Tap-style DensePack (hoisted tap rotations, masked weight plaintexts, a
  block sum): the binary block schedule sums blocks without wrapping; the
  dataflow run on plain slot vectors equals Eq. 1 exactly; encrypted, the
  conv and the FFConv built on it decrypt to the FP64 reference with the
  stated rotation and MulPC counts.
"""
import math

import numpy as np
import pytest

import synth
from oracle import conv as C
from oracle import counts
from oracle import encoding as E
from oracle import params as P
from oracle import reference as R
from oracle import scheme as S
from oracle import workloads as Wk

W = "unit"


def direct_conv(x, w, stride, pad):
    h, wd, c = x.shape
    d, _, _, o = w.shape
    oh = (h + 2 * pad - d) // stride + 1
    ow = (wd + 2 * pad - d) // stride + 1
    out = np.zeros((oh, ow, o))
    for i in range(oh):
        for j in range(ow):
            for oc in range(o):
                s = 0.0
                for kh in range(d):
                    for kw in range(d):
                        for ch in range(c):
                            y, xx = stride * i - pad + kh, stride * j - pad + kw
                            if 0 <= y < h and 0 <= xx < wd:
                                s += x[y, xx, ch] * w[kh, kw, ch, oc]
                out[i, j, oc] = s
    return out


@pytest.mark.parametrize("shape,d,stride,pad", [((7, 6, 2), 3, 1, 1), ((9, 9, 1), 5, 2, 0), ((8, 8, 3), 3, 2, 1)])
def test_conv2d_matches_direct(shape, d, stride, pad):
    rng = np.random.default_rng(1)
    x = rng.random(shape)
    w = rng.normal(0, 0.1, (d, d, shape[2], 4))
    assert np.abs(R.conv2d(x, w, stride, pad) - direct_conv(x, w, stride, pad)).max() < 1e-12


def test_factorisation_identities():
    rng = np.random.default_rng(2)
    x = rng.random((8, 8, 3))
    w1 = rng.normal(0, 0.1, (3, 3, 3, 2))
    w2 = rng.normal(0, 0.1, (2, 5))
    lhs = R.ffconv_reference(x, w1, w2, 1, 1)
    rhs = R.conv2d(x, R.compose_factors(w1, w2), 1, 1)
    assert np.abs(lhs - rhs).max() < 1e-12
    wm = rng.normal(0, 1, (27, 6))
    ev = np.sort(np.linalg.eigvalsh(wm.T @ wm))[::-1]
    for r in (1, 3, 5):
        a, b = R.truncated_svd_factors(wm, r)
        assert abs(np.linalg.norm(wm - a @ b) ** 2 - ev[r:].sum()) < 1e-8
        for _ in range(5):  # no random rank-r factorisation does better
            u = rng.normal(size=(27, r))
            v = np.linalg.lstsq(u, wm, rcond=None)[0]
            assert np.linalg.norm(wm - u @ v) >= np.linalg.norm(wm - a @ b) - 1e-9


def _ctx(n, rotations, relin=False, levels=3, scale=2.0**25):
    p = P.Params(n, (30,) * levels, 36, scale)
    return p, Wk.make_context(p, W, rotations=rotations, relin=relin)


def test_rotate_and_sum_of_ones():
    p, ctx = _ctx(256, C.rotate_and_sum_steps(P.Params(256, (30,), 36, 1.0)))
    ct = Wk.encrypt_slots(ctx, np.ones(p.slots), 3, p.scale, W, 0)
    out = C.rotate_and_sum(p, ctx, ct, int(math.log2(p.slots)), C.Counts())
    assert np.abs(ctx.decrypt(out) - p.slots).max() < 1e-3


def _run_densepack(p, ctx, x, w, geom, level, outputs=None):
    cts = [Wk.encrypt_slots(ctx, v, level, p.scale, W, m) for m, v in enumerate(C.densepack_slots(x, geom, p.slots))]
    xin = S.Ciphertext(np.stack([c.c for c in cts]), p.scale)
    pts = C.densepack_pt_scale(p, level, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w, geom, level, pts)
    return C.conv_densepack(p, ctx, xin, geom, bf, pts, outputs=outputs)


def test_single_tap_filter_shifts_input():
    p, ctx = _ctx(256, C.rotate_and_sum_steps(P.Params(256, (30,), 36, 1.0)))
    geom = C.ConvGeom(6, 6, 2, 3, 1, 1)
    x = synth.image(W, (6, 6, 2))
    w = np.zeros((3, 3, 2, 1))
    w[2, 0, 1, 0] = 1.0  # picks x[i+1][j-1][1]
    y, cnt = _run_densepack(p, ctx, x, w, geom, 3)
    for idx, (o, i, j) in enumerate(C.output_list(geom, 1)):
        want = x[i + 1, j - 1, 1] if (i + 1 < 6 and j - 1 >= 0) else 0.0
        got = ctx.decrypt(S.Ciphertext(y.c[idx], y.scale))
        assert abs(got[0] - want) < 1e-3 and abs(got[77] - want) < 1e-3
    assert cnt.rot == 36 * 7 and cnt.mulpc == 36


@pytest.mark.parametrize("shape,d,stride,pad,o_c,n", [
    ((6, 6, 3), 3, 1, 1, 2, 256),   # one ciphertext, 9 border classes
    ((4, 4, 8), 3, 1, 1, 2, 128),   # 128 values over 64 slots: two input ciphertexts
    ((7, 7, 1), 3, 2, 0, 3, 128),   # stride 2, no padding, one class
])
def test_densepack_matches_fp64(shape, d, stride, pad, o_c, n):
    p, ctx = _ctx(n, C.rotate_and_sum_steps(P.Params(n, (30,), 36, 1.0)))
    geom = C.ConvGeom(shape[0], shape[1], shape[2], d, stride, pad)
    x = synth.image(W, shape)
    w = synth.weights(W, 7, (d, d, shape[2], o_c), 0.1)
    y, cnt = _run_densepack(p, ctx, x, w, geom, 3)
    ref = R.conv2d(x, w, stride, pad)
    for idx, (o, i, j) in enumerate(C.output_list(geom, o_c)):
        got = ctx.decrypt(S.Ciphertext(y.c[idx], y.scale))
        assert np.abs(got - ref[i, j, o]).max() < 1e-3
    m = geom.n_cts(p.slots)
    assert cnt.mulpc == geom.spatial * o_c * m
    assert cnt.rot == geom.spatial * o_c * int(math.log2(p.slots))


def _ffconv(p, ctx, geom, x, w1, w2, square, k_bits=12):
    level = p.max_level
    ct = Wk.encrypt_slots(ctx, C.densepack_slots(x, geom, p.slots)[0], level, p.scale, W, 0)
    pts = C.densepack_pt_scale(p, level, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w1, geom, level, pts)
    y, cnt = C.conv_densepack(p, ctx, ct, geom, bf, pts)
    target = C.pre_square_target(p, level - 2, p.scale) if square else p.scale
    ms = C.gather_mask_scale(p, y.level, y.scale, target, k_bits)
    mask = C.encode_onehot(p, y.level, ms)
    z, cnt = C.gather_convpack(p, y, geom.spatial, w2, k_bits, mask, ms, cnt)
    if square:
        z, cnt = C.square_rescale(p, ctx, z, cnt)
    return z, cnt


def test_gather_identity_w2_returns_channels():
    p, ctx = _ctx(256, C.rotate_and_sum_steps(P.Params(256, (30,), 36, 1.0)), levels=3)
    geom = C.ConvGeom(5, 5, 1, 3, 1, 0)
    x = synth.image(W, (5, 5, 1))
    w1 = synth.weights(W, 8, (3, 3, 1, 2), 0.3)
    z, _ = _ffconv(p, ctx, geom, x, w1, np.eye(2), square=False)
    y = R.conv2d(x, w1, 1, 0)
    for c in range(2):
        got = ctx.decrypt(S.Ciphertext(z.c[c], z.scale))
        assert np.abs(got[: geom.spatial] - y[:, :, c].reshape(-1)).max() < 1e-3
        assert np.abs(got[geom.spatial:]).max() < 1e-3  # zeros outside the S compact slots


def test_ffconv_with_square_matches_fp64():
    p, ctx = _ctx(512, C.rotate_and_sum_steps(P.Params(512, (30,), 36, 1.0)), relin=True, levels=4)
    geom = C.ConvGeom(8, 8, 2, 3, 1, 1)
    x = synth.image(W, (8, 8, 2))
    w1 = synth.weights(W, 9, (3, 3, 2, 2), 0.3)
    w2 = synth.weights(W, 10, (2, 3), 0.5)
    z, cnt = _ffconv(p, ctx, geom, x, w1, w2, square=True)
    ref = R.ffconv_reference(x, w1, w2, 1, 1, square=True)
    assert z.level == 1 and abs(z.scale / p.scale - 1) < 1e-9
    for o in range(3):
        got = ctx.decrypt(S.Ciphertext(z.c[o], z.scale))
        assert np.abs(got[: geom.spatial] - ref[:, :, o].reshape(-1)).max() < 1e-3
    assert cnt.rot == 64 * 2 * 8 and cnt.scalar_mul == 6 and cnt.square == 3


def test_combine_cp_to_dp_layout():
    n = 256
    geom_next = C.ConvGeom(4, 4, 3, 1)
    p = P.Params(n, (30, 30), 36, 2.0**25)
    offsets = C.combine_offsets(3, 16, 8)
    ctx = Wk.make_context(p, W, rotations=offsets)
    vals = synth.message(W, 48)
    chans = [Wk.encrypt_slots(ctx, np.concatenate([vals[16 * o: 16 * o + 16], np.zeros(p.slots - 16)]), 2, p.scale, W, o)
             for o in range(3)]
    z = S.Ciphertext(np.stack([c.c for c in chans]), p.scale)
    dense, cnt = C.combine_cp_to_dp(p, ctx, z, 16, 8)
    tensor = vals.reshape(3, 4, 4).transpose(1, 2, 0)  # [h][w][c]
    want = C.densepack_slots(tensor, geom_next, p.slots)[0]
    assert np.abs(ctx.decrypt(S.Ciphertext(dense.c[0], dense.scale)) - want).max() < 1e-4
    assert cnt.rot == 2


def test_gather_onehot_places_value_j_in_slot_j():
    n = 256
    p = P.Params(n, (30, 30), 36, 2.0**25)
    ctx = Wk.make_context(p, W)
    k = 10
    vals = synth.message(W, 2 * k, index=5)
    reps = np.stack([Wk.encrypt_slots(ctx, np.full(p.slots, v), 2, p.scale, W, 60 + i).c for i, v in enumerate(vals)])
    ms = p.q[1] * p.scale / p.scale  # the rescale lands back on the input scale
    mask = C.encode_onehot(p, 2, ms)
    g, cnt = C.gather_onehot(p, S.Ciphertext(reps, p.scale), k, mask, ms)
    g = S.rescale(p, g)
    assert g.c.shape[0] == 2 and cnt.mulpc == 2 * k and cnt.addcc == 2 * (k - 1)
    for z in range(2):
        got = ctx.decrypt(S.Ciphertext(g.c[z], g.scale))
        want = np.zeros(p.slots)
        want[:k] = vals[z * k:(z + 1) * k]
        assert np.abs(got - want).max() < 1e-4


def _convpack_inputs(p, ctx, k_in, hw):
    """K channel ciphertexts in ConvPack form: channel k's hw x hw plane at slots 0..S-1."""
    x = synth.image(W, (hw, hw, k_in), index=7)
    s = hw * hw
    cts = [Wk.encrypt_slots(ctx, np.concatenate([x[:, :, k].ravel(), np.zeros(p.slots - s)]), p.max_level,
                            p.scale, W, 200 + k) for k in range(k_in)]
    return x.reshape(s, k_in), S.Ciphertext(np.stack([c.c for c in cts]), p.scale)


@pytest.mark.parametrize("k_in,o_c", [(4, 3), (1, 2), (6, 1)])
def test_convpack_matches_per_pixel_matmul(k_in, o_c):
    """Standalone ConvPack (Table II): output channel o decrypts to the FP64
    per-pixel product sum_k W[k, o] x_k in slots 0..S-1 and zeros elsewhere;
    MulPC = O_c K and AddCC = O_c (K - 1) as Table II counts them; the
    rescale lands on the target scale (up to rounding of the scale algebra)."""
    p = P.Params(512, (30, 30, 30), 36, 2.0**25)
    ctx = Wk.make_context(p, W)
    pix, cts = _convpack_inputs(p, ctx, k_in, 7)
    w = synth.weights(W, 40 + k_in, (k_in, o_c), 0.4)
    target = 2.0**24
    z, cnt = C.convpack(p, cts, w, target)
    assert z.level == p.max_level - 1 and z.c.shape[0] == o_c
    assert abs(z.scale - target) <= 4 * np.spacing(target)
    want_counts = counts.convpack_lola(o_c, k_in)
    assert (cnt.mulpc, cnt.addcc, cnt.rot, cnt.rescale) == (want_counts["mulpc"], want_counts["addcc"], 0, o_c)
    assert want_counts["mulpc"] == o_c * k_in and want_counts["addcc"] == o_c * (k_in - 1)
    ref = pix @ w  # (S, O_c), plain FP64
    for o in range(o_c):
        got = ctx.decrypt(S.Ciphertext(z.c[o], z.scale))
        assert np.abs(got[: pix.shape[0]] - ref[:, o]).max() < 1e-4
        assert np.abs(got[pix.shape[0]:]).max() < 1e-4


def test_convpack_identity_and_linearity():
    """ConvPack with W = I returns its inputs (after the rescale), and
    ConvPack(W_a + W_b) decrypts to ConvPack(W_a) + ConvPack(W_b)."""
    p = P.Params(512, (30, 30, 30), 36, 2.0**25)
    ctx = Wk.make_context(p, W)
    pix, cts = _convpack_inputs(p, ctx, 3, 6)
    z, _ = C.convpack(p, cts, np.eye(3), p.scale)
    for k in range(3):
        got = ctx.decrypt(S.Ciphertext(z.c[k], z.scale))
        assert np.abs(got[: pix.shape[0]] - pix[:, k]).max() < 1e-4
    wa = synth.weights(W, 50, (3, 2), 0.3)
    wb = synth.weights(W, 51, (3, 2), 0.3)
    za, _ = C.convpack(p, cts, wa, p.scale)
    zb, _ = C.convpack(p, cts, wb, p.scale)
    zs, _ = C.convpack(p, cts, wa + wb, p.scale)
    for o in range(2):
        da = ctx.decrypt(S.Ciphertext(za.c[o], za.scale))
        db = ctx.decrypt(S.Ciphertext(zb.c[o], zb.scale))
        ds = ctx.decrypt(S.Ciphertext(zs.c[o], zs.scale))
        assert np.abs(ds - (da + db)).max() < 1e-4


def test_im2col_slots_are_patch_columns():
    """Client-side Im2Col: vector k holds, for every output p = i O_w + j, the
    input pixel under tap k = (kh d + kw) I_c + c (zero outside the image),
    written out here by direct indexing, in slots 0..S-1."""
    geom = C.ConvGeom(7, 6, 2, 3, 2, 1)
    x = synth.image(W, (7, 6, 2))
    vecs = C.im2col_slots(x, geom, 64)
    assert len(vecs) == 3 * 3 * 2
    for kh in range(3):
        for kw in range(3):
            for c in range(2):
                v = vecs[(kh * 3 + kw) * 2 + c]
                for i in range(geom.out_h):
                    for j in range(geom.out_w):
                        y, xx = 2 * i - 1 + kh, 2 * j - 1 + kw
                        want = x[y, xx, c] if 0 <= y < 7 and 0 <= xx < 6 else 0.0
                        assert v[i * geom.out_w + j] == want
                assert not v[geom.spatial:].any()


@pytest.mark.parametrize("square", [False, True])
def test_convpack_convpack_ffconv_matches_fp64_and_counts(square):
    """FFConv with both factors under ConvPack (CP-HI2C-CP, d = 1): decrypts to
    the FP64 W1-then-W2 reference (with x^2) within 1e-3; executes Table II's
    FFConv counts (derived AddCC form) and Table III's zero HGrouping cost
    (no rotation at all); lands on the target scale."""
    p = P.Params(512, (30, 30, 30, 30), 36, 2.0**25)
    ctx = Wk.make_context(p, W, relin=square)
    geom = C.ConvGeom(8, 8, 2, 3, 1, 1)
    x = synth.image(W, (8, 8, 2))
    w1 = synth.weights(W, 61, (3, 3, 2, 3), 0.3)
    w2 = synth.weights(W, 62, (3, 4), 0.5)
    cts = [Wk.encrypt_slots(ctx, v, 4, p.scale, W, 300 + k).c for k, v in enumerate(C.im2col_slots(x, geom, p.slots))]
    z, cnt = C.convpack_convpack(p, ctx, S.Ciphertext(np.stack(cts), p.scale), R.filters_as_matrix(w1), w2, p.scale,
                                 square=square)
    k = 3 * 3 * 2
    want = counts.convpack_ffconv_derived(4, 3, k)
    hg = counts.him2col("CP-CP", 1)
    assert (cnt.mulpc, cnt.addcc, cnt.rot) == (want["mulpc"] + hg["mulpc"], want["addcc"] + hg["addcc"], 0)
    assert cnt.square == (4 if square else 0)
    assert z.level == (1 if square else 2) and abs(z.scale / p.scale - 1) < 1e-9
    ref = R.ffconv_reference(x, w1, w2, 1, 1, square=square)
    for o in range(4):
        got = ctx.decrypt(S.Ciphertext(z.c[o], z.scale))
        assert np.abs(got[: geom.spatial] - ref[:, :, o].reshape(-1)).max() < 1e-3
        assert np.abs(got[geom.spatial:]).max() < 1e-3


@pytest.mark.parametrize("blocks", list(range(1, 21)))
def test_tap_block_schedule_sums_blocks_without_wrap(blocks):
    """The binary block-sum schedule, run on a plain slot vector (rotation =
    np.roll), leaves sum_{b < blocks} block b in block 0, reads no slot at or
    beyond blocks * H W, and uses floor(log2 B) doublings plus popcount(B) - 1
    increments."""
    hw = 7
    slots = blocks * hw + 5
    rng = np.random.default_rng(blocks)
    t = np.zeros(slots)
    t[: blocks * hw] = rng.normal(size=blocks * hw)
    # poison the tail: any read of it shows up in block 0
    t[blocks * hw:] = 1e6
    s = t.copy()
    sched = C.tap_block_schedule(blocks, hw)
    for kind, amount in sched:
        s = (s if kind == "double" else t) + np.roll(s, -amount)
    want = t[: blocks * hw].reshape(blocks, hw).sum(axis=0)
    assert np.allclose(s[:hw], want, rtol=0, atol=1e-9)
    assert sum(k == "double" for k, _ in sched) == blocks.bit_length() - 1
    assert sum(k == "inc" for k, _ in sched) == bin(blocks).count("1") - 1


TAP_GEOMS = [((6, 6, 3), 3, 1, 1), ((9, 9, 1), 5, 2, 0), ((5, 5, 12), 3, 1, 1), ((8, 8, 1), 5, 2, 1),
             ((7, 5, 2), 3, 2, 1)]


@pytest.mark.parametrize("shape,d,stride,pad", TAP_GEOMS)
def test_tap_layout_in_the_clear(shape, d, stride, pad):
    """The tap-style dataflow on plain slot vectors (np.roll for Rot, float
    products for MulPC): sum over ciphertexts and taps of
    filter * roll(x_m, -shift), then the block schedule, equals Eq. 1's
    convolution at every output slot.  Pins the shifts, the masked filter
    layout and the output slots without any encryption."""
    slots = 256
    geom = C.ConvGeom(shape[0], shape[1], shape[2], d, stride, pad)
    x = synth.image(W, shape)
    w = synth.weights(W, 91, (d, d, shape[2], 3), 0.3)
    xs = C.densepack_slots(x, geom, slots)
    shifts = C.tap_shifts(geom)
    ref = R.conv2d(x, w, stride, pad)
    where = C.tap_output_slots(geom)
    for o in range(3):
        t = np.zeros(slots)
        for m, xm in enumerate(xs):
            for k, sh in enumerate(shifts):
                t += C.tap_filter_slots(w, geom, slots, o, m, k) * np.roll(xm, -sh)
        s = t.copy()
        for kind, amount in C.tap_block_schedule(geom.channels_per_ct(slots), geom.h * geom.w):
            s = (s if kind == "double" else t) + np.roll(s, -amount)
        assert np.allclose(s[where], ref[:, :, o].reshape(-1), rtol=0, atol=1e-12)


def _tap_setup(shape, d, stride, pad, relin=False, q=(30, 30, 30), level=3):
    p = P.Params(512, q, 36, 2.0**25)
    geom = C.ConvGeom(shape[0], shape[1], shape[2], d, stride, pad)
    ctx = Wk.make_context(p, W, rotations=C.tap_rotation_steps(geom, p.slots), relin=relin)
    x = synth.image(W, shape)
    xs = S.Ciphertext(np.stack([Wk.encrypt_slots(ctx, v, level, p.scale, W, 600 + m).c
                                for m, v in enumerate(C.densepack_slots(x, geom, p.slots))]), p.scale)
    return p, geom, ctx, x, xs


@pytest.mark.parametrize("shape,d,stride,pad", TAP_GEOMS)
def test_tap_conv_matches_fp64_and_counts(shape, d, stride, pad):
    """Tap-style DensePack decrypts to Eq. 1's conv within 1e-3 at the output
    slots, lands on its target scale, and executes M (d^2 - 1) hoisted
    rotations (d odd, pad = (d - 1) / 2: the centre tap needs none; else d^2
    when no tap has shift 0), O len(schedule) block-sum rotations, O M d^2
    MulPC and O rescales."""
    o_c = 3
    p, geom, ctx, x, xs = _tap_setup(shape, d, stride, pad)
    w = synth.weights(W, 81, (d, d, shape[2], o_c), 0.2)
    target = p.scale
    pt_scale = p.q[2] * target / xs.scale
    filt = C.tap_filters(p, w, geom, 3, pt_scale)
    z, cnt = C.tap_conv(p, ctx, xs, geom, filt, pt_scale)
    assert z.level == 2 and abs(z.scale / target - 1) < 1e-12
    ref = R.conv2d(x, w, stride, pad)
    where = C.tap_output_slots(geom)
    for o in range(o_c):
        got = ctx.decrypt(S.Ciphertext(z.c[o], z.scale))
        assert np.abs(got[where] - ref[:, :, o].reshape(-1)).max() < 1e-3
    m_cts = geom.n_cts(p.slots)
    zero_tap = 1 if 0 in C.tap_shifts(geom) else 0
    sched = C.tap_block_schedule(geom.channels_per_ct(p.slots), geom.h * geom.w)
    assert cnt.rot == m_cts * (d * d - zero_tap) + o_c * len(sched)
    assert cnt.mulpc == o_c * m_cts * d * d and cnt.rescale == o_c


@pytest.mark.parametrize("square", [False, True])
def test_tap_ffconv_matches_fp64(square):
    """Tap-style FFConv (W1 tap-style DensePack, masked gather, 1x1 ConvPack
    with 2^12-scaled integers, optional x^2) decrypts to the FP64 W1-then-W2
    reference within 1e-3 at the output slots and to 0 elsewhere, on the
    target scale."""
    p, geom, ctx, x, xs = _tap_setup((6, 6, 3), 3, 1, 1, relin=square, q=(30,) * 5, level=5)
    w1 = synth.weights(W, 71, (3, 3, 3, 2), 0.3)
    w2 = synth.weights(W, 72, (2, 4), 0.5)
    target = p.scale
    w1_scale = p.q[4] * target / xs.scale
    filt = C.tap_filters(p, w1, geom, 5, w1_scale)
    t2 = C.pre_square_target(p, 3, target) if square else target
    mask_scale = C.gather_mask_scale(p, 4, target, t2, 12)
    mask = E.encode(C.tap_output_mask_slots(geom, p.slots), p, 4, mask_scale)
    z, cnt = C.tap_ffconv(p, ctx, xs, geom, filt, w1_scale, w2, 12, mask, mask_scale, square=square)
    assert z.level == (2 if square else 3) and abs(z.scale / target - 1) < 1e-9
    ref = R.ffconv_reference(x, w1, w2, 1, 1, square=square)
    where = C.tap_output_slots(geom)
    rest = np.ones(p.slots, bool)
    rest[where] = False
    for o in range(4):
        got = ctx.decrypt(S.Ciphertext(z.c[o], z.scale))
        assert np.abs(got[where] - ref[:, :, o].reshape(-1)).max() < 1e-3
        assert np.abs(got[rest]).max() < 1e-3
    assert cnt.square == (4 if square else 0)


@pytest.mark.parametrize("shape,d,stride,pad", [((6, 6, 3), 3, 1, 1), ((9, 9, 2), 4, 2, 0), ((5, 5, 12), 3, 1, 1),
                                                ((7, 5, 2), 3, 2, 1)])
def test_him2col_columns_and_counts(shape, d, stride, pad):
    """Homomorphic Im2Col from a DensePack input: ciphertext k decrypts to
    column k of Eq. 1's matrix I (conv2d's im2col, an independent numpy
    routine) at the output slots and to 0 elsewhere; ConvPack of the
    columns decrypts to the FP64 conv; executed counts are K MulPC and
    sum_m (B_m - 1 + B_m #nonzero shifts) rotations (K - #zero-shift columns
    when every ciphertext is full and pad = 0 keeps one zero shift)."""
    p = P.Params(512, (30, 30, 30, 30), 36, 2.0**25)
    geom = C.ConvGeom(shape[0], shape[1], shape[2], d, stride, pad)
    ctx = Wk.make_context(p, W, rotations=C.him2col_rotation_steps(geom, p.slots))
    x = synth.image(W, shape)
    xs = S.Ciphertext(np.stack([Wk.encrypt_slots(ctx, v, 4, p.scale, W, 800 + m).c
                                for m, v in enumerate(C.densepack_slots(x, geom, p.slots))]), p.scale)
    ms = float(p.q[3])
    masks = [E.encode(C.him2col_mask_slots(geom, p.slots, t), p, 4, ms) for t in range(d * d)]
    y, cnt = C.him2col(p, ctx, xs, geom, masks, ms)
    assert y.level == 3 and abs(y.scale / p.scale - 1) < 1e-12
    cols = R.im2col(x, d, stride, pad)
    where = C.tap_output_slots(geom)
    rest = np.ones(p.slots, bool)
    rest[where] = False
    assert y.c.shape[0] == cols.shape[1] == d * d * shape[2]
    for k in range(cols.shape[1]):
        got = ctx.decrypt(S.Ciphertext(y.c[k], y.scale))
        assert np.abs(got[where] - cols[:, k]).max() < 1e-3, k
        assert np.abs(got[rest]).max() < 1e-3, k
    per = geom.channels_per_ct(p.slots)
    nz = sum(1 for s in C.tap_shifts(geom) if s % p.slots)
    want = sum((min(per, shape[2] - m * per) - 1) + min(per, shape[2] - m * per) * nz for m in range(xs.c.shape[0]))
    assert cnt.rot == want and cnt.mulpc == d * d * shape[2] and cnt.rescale == d * d * shape[2]
    w = synth.weights(W, 85, (d, d, shape[2], 2), 0.2)
    z, _ = C.convpack(p, y, R.filters_as_matrix(w), p.scale)
    ref = R.conv2d(x, w, stride, pad)
    for o in range(2):
        got = ctx.decrypt(S.Ciphertext(z.c[o], z.scale))
        assert np.abs(got[where] - ref[:, :, o].reshape(-1)).max() < 1e-3


def test_moddown_absorbs_multiples_of_p():
    """ModDown(P a + b) = a + ModDown(b) exactly (the identity that lets the
    lazy tap conv fold the rotations' c0 terms into one ModDown)."""
    from oracle import modq
    p = P.Params(512, (30, 30, 30), 36, 2.0**25)
    rng = np.random.default_rng(5)
    level = 3
    moduli = p.q[:level] + [p.p]
    a = np.stack([rng.integers(0, q, p.n, dtype=np.uint64) for q in p.q[:level]])
    b = np.stack([rng.integers(0, q, p.n, dtype=np.uint64) for q in moduli])
    pa_b = b.copy()
    for i, q in enumerate(p.q[:level]):
        pa_b[i] = modq.add(modq.mul(a[i], np.uint64(p.p % q), q), b[i], q)
    lhs = S.mod_down(p, pa_b)
    rhs = S.mod_down(p, b)
    for i, q in enumerate(p.q[:level]):
        rhs[i] = modq.add(rhs[i], a[i], q)
    assert np.array_equal(lhs, rhs)


def test_tap_conv_lazy_single_unit_tap_is_a_rotation():
    """With the constant plaintext 1 on one tap and 0 on the others, the
    lazy tap conv's output is rescale(Rot(x, shift)) bit for bit: the one
    ModDown after the products equals the rotation's own."""
    p = P.Params(512, (30, 30, 30), 36, 2.0**25)
    geom = C.ConvGeom(6, 6, 1, 3, 1, 1)
    ctx = Wk.make_context(p, W, rotations=C.tap_rotation_steps(geom, p.slots))
    x = Wk.encrypt_slots(ctx, synth.message(W, p.slots), 3, p.scale, W, 5)
    shifts = C.tap_shifts(geom)
    for t in (0, 5, 8):
        filt = np.zeros((1, 1, 9, 3, p.n), dtype=np.uint64)
        filt_p = np.zeros((1, 1, 9, p.n), dtype=np.uint64)
        filt[0, 0, t] = 1
        filt_p[0, 0, t] = 1
        z, cnt = C.tap_conv_lazy(p, ctx, S.Ciphertext(x.c[None], x.scale), geom, filt, filt_p, 1.0)
        want = S.rescale(p, S.rotate(p, ctx, x, shifts[t] % p.slots))
        assert np.array_equal(z.c[0], want.c), t
        assert cnt.rot == 8 and cnt.extra["moddown"] == 1


@pytest.mark.parametrize("shape,d,stride,pad", TAP_GEOMS[:4])
def test_tap_conv_lazy_matches_fp64(shape, d, stride, pad):
    """The lazy tap conv decrypts to Eq. 1's conv within 1e-3 and to the
    per-rotation tap conv within 1e-4, with the same rotation and MulPC
    counts and one ModDown per output."""
    o_c = 3
    p, geom, ctx, x, xs = _tap_setup(shape, d, stride, pad)
    w = synth.weights(W, 81, (d, d, shape[2], o_c), 0.2)
    pt_scale = p.q[2] * p.scale / xs.scale
    filt = C.tap_filters(p, w, geom, 3, pt_scale)
    filt_p = C.tap_filters_p(p, w, geom, pt_scale)
    z, cnt = C.tap_conv_lazy(p, ctx, xs, geom, filt, filt_p, pt_scale)
    z1, cnt1 = C.tap_conv(p, ctx, xs, geom, filt, pt_scale)
    assert z.level == 2 and z.scale == z1.scale
    assert (cnt.rot, cnt.mulpc, cnt.rescale) == (cnt1.rot, cnt1.mulpc, cnt1.rescale)
    assert cnt.extra["moddown"] == o_c
    ref = R.conv2d(x, w, stride, pad)
    where = C.tap_output_slots(geom)
    for o in range(o_c):
        got = ctx.decrypt(S.Ciphertext(z.c[o], z.scale))
        per_rot = ctx.decrypt(S.Ciphertext(z1.c[o], z1.scale))
        assert np.abs(got[where] - ref[:, :, o].reshape(-1)).max() < 1e-3
        assert np.abs(got[where] - per_rot[where]).max() < 1e-4
