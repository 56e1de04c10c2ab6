"""Packed homomorphic convolution layers (test infrastructure; see package doc).

DensePack (Section 3.2, Fig. 1, Table I): the input tensor X[h][w][c] is laid
out in the slots of one ciphertext at slot c*H*W + h*W + w (channel slowest,
then rows; zeros elsewhere).  A tensor with more than N/2 values is split by
channel blocks over M ciphertexts.  Each output value (o, i, j) is one
homomorphic dot product: the filter, zero-padded to the input size, is placed
at the patch anchor a = (s*i - pad)*W + (s*j - pad), multiplied slot-wise with
the input (MulPC), and all slots are summed by R = log2(N/2) rotate-and-add
steps (Rot, AddCC).  The shifted filter is an exact slot rotation (Galois
permutation, rotation right by a) of one base filter plaintext per output
channel and border class; a border class is the set of filter taps that fall
inside the image, so the client never pads.  The result of each dot product
is left replicated in every slot, one ciphertext per output value.

Scale rule: a plaintext multiply that is followed by a rescale dropping q_l is
encoded at scale q_l * target / current, so the rescale lands exactly on the
target.  The rescale happens after the rotate-and-sum.

FFConv (Section 4, Eq. 2; DP-HI2C-CP of Section 4.2 and Table IX): W1 (d x d,
O'_c filters) runs under DensePack; the O'_c*S replicated results are gathered
into one ConvPack ciphertext per channel by multiplying each with a one-hot
mask moved to slot p = i*O_w + j (the DP->CP transition of Table III with
d = 1, written with masks instead of rotations because the DensePack outputs
are replicated); W2 (1 x 1) is then a ConvPack layer (Table II): output
channel o is sum_c round(W2[c,o] * 2^k) * G_c with exact integer scalars.
One rescale follows, so the factorized layer has depth 2.

CP->DP combine (Table III, CP-HI2C-DP): channel ciphertexts holding S values
at slots 0..S-1 are rotated right by (o mod B)*S and summed into dense
ciphertexts of B channels each.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import modq, scheme
from .encoding import encode, encode_int, round_half_away, to_rns_ntt
from .ring import automorph_ntt, galois_for_rotation


@dataclass(frozen=True)
class ConvGeom:
    h: int
    w: int
    c_in: int
    d: int
    stride: int = 1
    pad: int = 0

    @property
    def out_h(self) -> int:
        return (self.h + 2 * self.pad - self.d) // self.stride + 1

    @property
    def out_w(self) -> int:
        return (self.w + 2 * self.pad - self.d) // self.stride + 1

    @property
    def spatial(self) -> int:
        return self.out_h * self.out_w

    def channels_per_ct(self, slots: int) -> int:
        per = slots // (self.h * self.w)
        assert per >= 1, "one channel plane must fit in the slots"
        return min(per, self.c_in)

    def n_cts(self, slots: int) -> int:
        return math.ceil(self.c_in / self.channels_per_ct(slots))

    def tap_range(self, pos: int, size: int):
        """Valid filter taps [lo, hi) along one axis for output coordinate pos."""
        start = self.stride * pos - self.pad
        return max(0, -start), min(self.d, size - start)

    def border_classes(self):
        """(row_ranges, col_ranges, class_of_output[i][j]).

        Row (column) ranges are numbered in order of first appearance as the
        output row (column) index increases; class = row_class * n_cols + col_class.
        """
        rows, row_id = [], []
        for i in range(self.out_h):
            r = self.tap_range(i, self.h)
            if r not in rows:
                rows.append(r)
            row_id.append(rows.index(r))
        cols, col_id = [], []
        for j in range(self.out_w):
            c = self.tap_range(j, self.w)
            if c not in cols:
                cols.append(c)
            col_id.append(cols.index(c))
        cls = [[row_id[i] * len(cols) + col_id[j] for j in range(self.out_w)] for i in range(self.out_h)]
        return rows, cols, cls

    def anchor(self, i: int, j: int) -> int:
        return (self.stride * i - self.pad) * self.w + (self.stride * j - self.pad)


@dataclass
class Counts:
    mulpc: int = 0
    addcc: int = 0
    rot: int = 0
    rescale: int = 0
    square: int = 0
    scalar_mul: int = 0
    extra: dict = field(default_factory=dict)

    def merge(self, other: "Counts") -> "Counts":
        return Counts(
            self.mulpc + other.mulpc, self.addcc + other.addcc, self.rot + other.rot,
            self.rescale + other.rescale, self.square + other.square,
            self.scalar_mul + other.scalar_mul,
        )


# ---- DensePack ---------------------------------------------------------------

def densepack_slots(x: np.ndarray, geom: ConvGeom, slots: int) -> list[np.ndarray]:
    """Slot vectors (one per input ciphertext) of X[h][w][c]: slot c*H*W + h*W + w."""
    per = geom.channels_per_ct(slots)
    out = []
    for m in range(geom.n_cts(slots)):
        v = np.zeros(slots)
        for cl in range(per):
            c = m * per + cl
            if c >= geom.c_in:
                break
            v[cl * geom.h * geom.w: (cl + 1) * geom.h * geom.w] = x[:, :, c].reshape(-1)
        out.append(v)
    return out


def base_filter_slots(weights: np.ndarray, geom: ConvGeom, slots: int, o: int, cls: int, m: int) -> np.ndarray:
    """Slot vector of the base filter for output channel o, border class cls, input ct m."""
    rows, cols, _ = geom.border_classes()
    (kh_lo, kh_hi) = rows[cls // len(cols)]
    (kw_lo, kw_hi) = cols[cls % len(cols)]
    per = geom.channels_per_ct(slots)
    v = np.zeros(slots)
    for cl in range(per):
        c = m * per + cl
        if c >= geom.c_in:
            break
        for kh in range(kh_lo, kh_hi):
            for kw in range(kw_lo, kw_hi):
                v[cl * geom.h * geom.w + kh * geom.w + kw] = weights[kh, kw, c, o]
    return v


def densepack_pt_scale(params, level: int, in_scale: float, target_scale: float) -> float:
    return params.q[level - 1] * target_scale / in_scale


def densepack_base_filters(params, weights, geom: ConvGeom, level: int, pt_scale: float) -> np.ndarray:
    """Encoded base filters, uint64 array [O_c][classes][M][level][N] (NTT domain)."""
    rows, cols, _ = geom.border_classes()
    n_cls = len(rows) * len(cols)
    m_cts = geom.n_cts(params.slots)
    o_c = weights.shape[3]
    out = np.empty((o_c, n_cls, m_cts, level, params.n), dtype=np.uint64)
    for o in range(o_c):
        for b in range(n_cls):
            for m in range(m_cts):
                out[o, b, m] = encode(base_filter_slots(weights, geom, params.slots, o, b, m), params, level, pt_scale)
    return out


def rotate_and_sum(params, keys, t: scheme.Ciphertext, r_steps: int, counts: Counts) -> scheme.Ciphertext:
    """t <- t + Rot(t, 2^j) for j < r_steps (all slots end up holding the total)."""
    for j in range(r_steps):
        t = scheme.add(params, t, scheme.rotate(params, keys, t, 1 << j))
        counts.rot += int(np.prod(t.c.shape[:-3], dtype=np.int64))
        counts.addcc += int(np.prod(t.c.shape[:-3], dtype=np.int64))
    return t


def output_list(geom: ConvGeom, o_c: int):
    """All (o, i, j) in output order index = o*S + i*O_w + j."""
    return [(o, i, j) for o in range(o_c) for i in range(geom.out_h) for j in range(geom.out_w)]


def conv_densepack(params, keys, x: scheme.Ciphertext, geom: ConvGeom, base_filters: np.ndarray,
                   pt_scale: float, outputs=None, r_steps: int | None = None, counts: Counts | None = None):
    """DensePack conv (Table I): returns (ciphertexts of the requested outputs, rescaled)."""
    counts = counts if counts is not None else Counts()
    o_c = base_filters.shape[0]
    outputs = output_list(geom, o_c) if outputs is None else outputs
    r_steps = int(math.log2(params.slots)) if r_steps is None else r_steps
    _, _, cls = geom.border_classes()
    xc = x.c if x.c.ndim == 4 else x.c[None]  # (M, 2, level, N)
    m_cts = xc.shape[0]
    level = xc.shape[-2]
    acc = np.empty((len(outputs), 2, level, params.n), dtype=np.uint64)
    for idx, (o, i, j) in enumerate(outputs):
        g = galois_for_rotation(-geom.anchor(i, j), params.n)
        term = None
        for m in range(m_cts):
            f = automorph_ntt(base_filters[o, cls[i][j], m, :level], g)
            prod = scheme.mul_plain(params, scheme.Ciphertext(xc[m], x.scale), f, pt_scale)
            counts.mulpc += 1
            if term is None:
                term = prod
            else:
                term = scheme.add(params, term, prod)
                counts.addcc += 1
        acc[idx] = term.c
    t = scheme.Ciphertext(acc, x.scale * pt_scale)
    t = rotate_and_sum(params, keys, t, r_steps, counts)
    t = scheme.rescale(params, t)
    counts.rescale += len(outputs)
    return t, counts


# ---- DP -> CP gather and the 1x1 ConvPack -------------------------------------

def gather_mask_scale(params, level: int, y_scale: float, target_scale: float, k_bits: int) -> float:
    return params.q[level - 1] * target_scale / (y_scale * 2.0**k_bits)


def encode_onehot(params, level: int, scale: float) -> np.ndarray:
    z = np.zeros(params.slots)
    z[0] = 1.0
    return encode(z, params, level, scale)


def w2_integers(w2: np.ndarray, k_bits: int) -> np.ndarray:
    """round-half-away(W2 * 2^k) as int64 (the exact integer scalars of the 1x1 conv)."""
    return round_half_away(np.asarray(w2, dtype=np.float64) * 2.0**k_bits).astype(np.int64)


def gather_convpack(params, y: scheme.Ciphertext, spatial: int, w2: np.ndarray, k_bits: int,
                    mask_pt: np.ndarray, mask_scale: float, counts: Counts | None = None):
    """y: (r*S) replicated DensePack outputs, index c*S + p.  Returns O_c ConvPack cts (rescaled)."""
    counts = counts if counts is not None else Counts()
    r, o_c = w2.shape
    level = y.level
    gathered = []
    for c in range(r):
        acc = None
        for p in range(spatial):
            e = automorph_ntt(mask_pt[:level], galois_for_rotation(-p, params.n))
            prod = scheme.mul_plain(params, scheme.Ciphertext(y.c[c * spatial + p], y.scale), e, mask_scale)
            counts.mulpc += 1
            if acc is None:
                acc = prod
            else:
                acc = scheme.add(params, acc, prod)
                counts.addcc += 1
        gathered.append(acc)
    wint = w2_integers(w2, k_bits)
    outs = []
    for o in range(o_c):
        z = None
        for c in range(r):
            term = scheme.mul_int(params, gathered[c], int(wint[c, o]))
            counts.scalar_mul += 1
            if z is None:
                z = term
            else:
                z = scheme.add(params, z, term)
                counts.addcc += 1
        outs.append(z.c)
    z = scheme.Ciphertext(np.stack(outs), gathered[0].scale * 2.0**k_bits)
    z = scheme.rescale(params, z)
    counts.rescale += o_c
    return z, counts


def gather_onehot(params, y: scheme.Ciphertext, k: int, mask_pt: np.ndarray, mask_scale: float,
                  counts: Counts | None = None):
    """Output arrangement of replicated DensePack outputs (the step Table I
    leaves uncounted, Sec. 3.2): for each group of k ciphertexts, the sum over
    j of y_j times the one-hot plaintext E shifted right by j, i.e.
    sigma_{5^-j}(E); the value of ciphertext j lands in slot j.  y.c holds
    (groups * k, 2, level, N); returns (groups, 2, level, N), not rescaled."""
    counts = counts if counts is not None else Counts()
    level = y.level
    groups = y.c.shape[0] // k
    out = []
    for z in range(groups):
        acc = None
        for j in range(k):
            e = automorph_ntt(mask_pt[:level], galois_for_rotation(-j, params.n))
            prod = scheme.mul_plain(params, scheme.Ciphertext(y.c[z * k + j], y.scale), e, mask_scale)
            counts.mulpc += 1
            if acc is None:
                acc = prod
            else:
                acc = scheme.add(params, acc, prod)
                counts.addcc += 1
        out.append(acc.c)
    return scheme.Ciphertext(np.stack(out), y.scale * mask_scale), counts


def convpack(params, cts: scheme.Ciphertext, w: np.ndarray, target_scale: float,
             counts: Counts | None = None):
    """Standalone ConvPack layer (Table II): K input cts, weights (K, O_c) as integers.

    Each weight is round-half-away(w * D_w) with D_w = q_l * target / input scale,
    so the rescale that follows lands on `target_scale`.
    """
    counts = counts if counts is not None else Counts()
    k_in, o_c = w.shape
    level = cts.level
    dw = params.q[level - 1] * target_scale / cts.scale
    wint = round_half_away(np.asarray(w, np.float64) * dw)
    outs = []
    for o in range(o_c):
        z = None
        for k in range(k_in):
            term = scheme.mul_int(params, scheme.Ciphertext(cts.c[k], cts.scale), int(wint[k, o]))
            counts.mulpc += 1
            if z is None:
                z = term
            else:
                z = scheme.add(params, z, term)
                counts.addcc += 1
        outs.append(z.c)
    z = scheme.Ciphertext(np.stack(outs), cts.scale * dw)
    z = scheme.rescale(params, z)
    counts.rescale += o_c
    return z, counts


def square_rescale(params, keys, x: scheme.Ciphertext, counts: Counts | None = None):
    counts = counts if counts is not None else Counts()
    y = scheme.rescale(params, scheme.square(params, keys, x))
    n = int(np.prod(x.c.shape[:-3], dtype=np.int64))
    counts.square += n
    counts.rescale += n
    return y, counts


def pre_square_target(params, level_after_rescale: int, scale: float) -> float:
    """Scale to aim for before a square so that square + rescale returns to `scale`."""
    return math.sqrt(params.q[level_after_rescale - 1] * scale)


def im2col_slots(x: np.ndarray, geom: ConvGeom, slots: int) -> list[np.ndarray]:
    """Client-side plaintext Im2Col for a ConvPack input (Sec. 3.3, Eq. 1):
    K = d^2 I_c slot vectors, vector k holding column k of the S x K matrix I
    (the S = O_w O_h patch values at tap k = (kh d + kw) I_c + c, zero for
    taps outside the image) in slots 0..S-1 and zeros elsewhere."""
    from .reference import im2col
    cols = im2col(x, geom.d, geom.stride, geom.pad)
    s_out, k = cols.shape
    if s_out > slots:
        raise ValueError("S exceeds the slot count")
    out = []
    for j in range(k):
        v = np.zeros(slots)
        v[:s_out] = cols[:, j]
        out.append(v)
    return out


def convpack_convpack(params, keys, cts: scheme.Ciphertext, w1: np.ndarray, w2: np.ndarray, target_scale: float,
                      square: bool = False, counts: Counts | None = None):
    """FFConv with both factors under ConvPack (Sec. 4.2.2 "ConvPack for W1",
    Fig. 5; CP-HI2C-CP with d = 1 in Table III).

    cts: the K Im2Col ciphertexts of the input (im2col_slots).  W1 (K x O'_c,
    the d x d low-rank filters flattened as Eq. 1) under ConvPack gives O'_c
    channel ciphertexts, each holding its S outputs in slots 0..S-1; for the
    1 x 1 W2 these already are the per-channel ConvPack inputs (HGrouping with
    d = 1 moves no slot: no MulPC, no rotation), so W2 (O'_c x O_c) under
    ConvPack follows directly.  Each ConvPack rescales once; with `square`,
    W2 lands on the pre-square scale and x^2 (relinearised, rescaled) returns
    to target_scale.
    """
    counts = counts if counts is not None else Counts()
    level = cts.level
    t2 = pre_square_target(params, level - 2, target_scale) if square else target_scale
    y, _ = convpack(params, cts, w1, target_scale, counts)
    z, _ = convpack(params, y, w2, t2, counts)
    if square:
        z, _ = square_rescale(params, keys, z, counts)
    return z, counts


# ---- Tap-style DensePack (hoisted rotations) ----------------------------------
# A variant of the DensePack conv beyond the paper's own designs (Table I
# counts R rotations per output; Sec. 3.2): instead of one rotate-and-sum
# chain per output, each input ciphertext is rotated once per filter tap,
# all those rotations share one digit decomposition, and plaintexts that
# hold the tap's weights at the output slots do the rest.  Layout: input as
# C10 (channel c of ciphertext m in block b = c - m B at slots b H W + h W +
# w); output o's value for (i, j) at slot (s i) W + s j.

def tap_shifts(geom: ConvGeom) -> list[int]:
    """Left rotation of tap t = kh d + kw: it moves the input pixel
    (s i - pad + kh, s j - pad + kw) of every block onto the output slot
    (s i) W + s j of that block."""
    return [(kh - geom.pad) * geom.w + (kw - geom.pad) for kh in range(geom.d) for kw in range(geom.d)]


def tap_output_slots(geom: ConvGeom) -> np.ndarray:
    """Slot of output (i, j), in output order (row-major)."""
    return np.array([geom.stride * i * geom.w + geom.stride * j
                     for i in range(geom.out_h) for j in range(geom.out_w)], dtype=np.int64)


def tap_filter_slots(weights: np.ndarray, geom: ConvGeom, slots: int, o: int, m: int, t: int) -> np.ndarray:
    """Masked weight plaintext of (output channel o, input ciphertext m, tap
    t): in block b (channel c = m B + b) the weight W[kh][kw][c][o] at the
    slot of every output whose tap t falls inside the image (zero padding
    elsewhere), zero in all other slots."""
    per = geom.channels_per_ct(slots)
    kh, kw = divmod(t, geom.d)
    hw = geom.h * geom.w
    v = np.zeros(slots)
    for c in range(m * per, min((m + 1) * per, geom.c_in)):
        b = c - m * per
        for i in range(geom.out_h):
            y = geom.stride * i - geom.pad + kh
            if not 0 <= y < geom.h:
                continue
            for j in range(geom.out_w):
                x = geom.stride * j - geom.pad + kw
                if 0 <= x < geom.w:
                    v[b * hw + geom.stride * i * geom.w + geom.stride * j] = weights[kh, kw, c, o]
    return v


def tap_filters(params, weights: np.ndarray, geom: ConvGeom, level: int, pt_scale: float) -> np.ndarray:
    """All tap plaintexts, NTT domain: (O, M, d^2, level, N)."""
    slots = params.slots
    o_c = weights.shape[3]
    m_cts = geom.n_cts(slots)
    out = np.empty((o_c, m_cts, geom.d * geom.d, level, params.n), dtype=np.uint64)
    for o in range(o_c):
        for m in range(m_cts):
            for t in range(geom.d * geom.d):
                out[o, m, t] = encode(tap_filter_slots(weights, geom, slots, o, m, t), params, level, pt_scale)
    return out


def tap_block_schedule(blocks: int, hw: int) -> list[tuple[str, int]]:
    """Steps that sum the first `blocks` blocks of H W slots into block 0,
    sum_{b < blocks} Rot(t, b H W), by the binary method over the bits of
    `blocks` below the leading one: ("double", k H W) takes a k-block sum S
    to S + Rot(S, k H W) (2k blocks), ("inc", H W) takes it to
    t + Rot(S, H W) (k + 1 blocks).  No slot wraps past the last block."""
    steps = []
    k = 1
    for bit in bin(blocks)[3:]:
        steps.append(("double", k * hw))
        k *= 2
        if bit == "1":
            steps.append(("inc", hw))
            k += 1
    return steps


def tap_rotation_steps(geom: ConvGeom, slots: int) -> list[int]:
    """Every rotation amount (mod slots, nonzero) a tap-style layer uses."""
    amounts = {s % slots for s in tap_shifts(geom)}
    amounts |= {a for _, a in tap_block_schedule(geom.channels_per_ct(slots), geom.h * geom.w)}
    return sorted(amounts - {0})


def tap_conv(params, keys, xs: scheme.Ciphertext, geom: ConvGeom, filters: np.ndarray, pt_scale: float,
             counts: Counts | None = None) -> tuple[scheme.Ciphertext, Counts]:
    """Tap-style DensePack conv of one input (xs.c: M ciphertexts).

    1. Each input ciphertext x_m is rotated by every nonzero tap shift, the
       rotations of one x_m hoisted over one digit decomposition
       (scheme.rotate_hoisted); the zero shift is x_m itself.
    2. t_o = sum_m sum_t F[o][m][t] * Rot(x_m, shift_t) (MulPC, AddCC):
       block b of t_o holds, at each output slot, channel m B + b's part of
       the dot product.
    3. The blocks are summed into block 0 (tap_block_schedule), then one
       rescale.  The rescale comes after all rotations, as for the
       rotate-and-sum of C10.
    Output (O cts at level - 1): output (i, j) of channel o at slot
    (s i) W + s j; other slots hold partial sums and noise."""
    counts = counts if counts is not None else Counts()
    slots = params.slots
    shifts = [s % slots for s in tap_shifts(geom)]
    moved = []
    for m in range(xs.c.shape[0]):
        x = scheme.Ciphertext(xs.c[m], xs.scale)
        nonzero = [s for s in shifts if s != 0]
        rot = dict(zip(nonzero, scheme.rotate_hoisted(params, keys, x, nonzero)))
        counts.rot += len(nonzero)
        moved.append([x if s == 0 else rot[s] for s in shifts])
    o_c = filters.shape[0]
    blocks = geom.channels_per_ct(slots)
    outs = []
    for o in range(o_c):
        t_o = None
        for m, row in enumerate(moved):
            for t, y in enumerate(row):
                term = scheme.mul_plain(params, y, filters[o, m, t], pt_scale)
                counts.mulpc += 1
                if t_o is None:
                    t_o = term
                else:
                    t_o = scheme.add(params, t_o, term)
                    counts.addcc += 1
        first = t_o
        for kind, amount in tap_block_schedule(blocks, geom.h * geom.w):
            r = scheme.rotate(params, keys, t_o, amount)
            t_o = scheme.add(params, t_o if kind == "double" else first, r)
            counts.rot += 1
            counts.addcc += 1
        outs.append(t_o.c)
    z = scheme.rescale(params, scheme.Ciphertext(np.stack(outs), xs.scale * pt_scale))
    counts.rescale += o_c
    return z, counts


def tap_filters_p(params, weights: np.ndarray, geom: ConvGeom, pt_scale: float) -> np.ndarray:
    """The tap plaintexts' residues modulo the special prime P, NTT domain:
    (O, M, d^2, N), for tap_conv_lazy."""
    slots = params.slots
    o_c = weights.shape[3]
    m_cts = geom.n_cts(slots)
    out = np.empty((o_c, m_cts, geom.d * geom.d, params.n), dtype=np.uint64)
    for o in range(o_c):
        for m in range(m_cts):
            for t in range(geom.d * geom.d):
                z = tap_filter_slots(weights, geom, slots, o, m, t)
                out[o, m, t] = to_rns_ntt(encode_int(z, params.n, pt_scale), [params.p], params.psi)[0]
    return out


def tap_conv_lazy(params, keys, xs: scheme.Ciphertext, geom: ConvGeom, filters: np.ndarray, filters_p: np.ndarray,
                  pt_scale: float, counts: Counts | None = None) -> tuple[scheme.Ciphertext, Counts]:
    """tap_conv with the ModDown of the hoisted rotations deferred past the
    plaintext products: one ModDown per output instead of one per rotation.
    A rotation by g is (sigma_g(c0) + ModDown(u_0), ModDown(u_1)) with
    u = the key inner product over (Q, P); since ModDown(P a + b) =
    a + ModDown(b) exactly, the products and sums run over (Q, P) on
    U_o = sum_m [ sum_{t: shift != 0} F[o][m][t] * (u_{m,t} + (P sigma_t(c0_m), 0))
                  + F[o][m][t0] * P x_m ]
    (F's residues mod P from filters_p, the P terms on the Q limbs only),
    and t_o = ModDown(U_o).  The block sum and the rescale follow as in
    tap_conv.  Different rounding from tap_conv (one ModDown instead of one
    per rotation), same value within noise."""
    counts = counts if counts is not None else Counts()
    slots = params.slots
    level = xs.level
    n = params.n
    shifts = [s % slots for s in tap_shifts(geom)]
    o_c = filters.shape[0]
    u_acc = np.zeros((o_c, 2, level + 1, n), dtype=np.uint64)
    moduli = params.q[:level] + [params.p]
    p_mod = [np.uint64(params.p % q) for q in params.q[:level]]
    for m in range(xs.c.shape[0]):
        c = xs.c[m]
        lifted = scheme.lift_digits(params, scheme.decompose(params, c[1]))
        for t, s in enumerate(shifts):
            if s == 0:
                term = np.zeros((2, level + 1, n), dtype=np.uint64)
                for i in range(level):
                    term[:, i] = modq.mul(c[:, i], p_mod[i], params.q[i])
            else:
                g = galois_for_rotation(s, n)
                moved = [[automorph_ntt(v, g) for v in row] for row in lifted]
                term = scheme.inner_product(params, moved, keys.rot_keys[g])
                c0 = automorph_ntt(c[0], g)
                for i in range(level):
                    term[0, i] = modq.add(term[0, i], modq.mul(c0[i], p_mod[i], params.q[i]), params.q[i])
                counts.rot += 1
            for o in range(o_c):
                for i, q in enumerate(moduli):
                    f = filters[o, m, t, i] if i < level else filters_p[o, m, t]
                    u_acc[o, :, i] = modq.add(u_acc[o, :, i], modq.mul(term[:, i], f, q), q)
                counts.mulpc += 1
    t_all = scheme.mod_down(params, u_acc)
    counts.extra["moddown"] = counts.extra.get("moddown", 0) + o_c
    blocks = geom.channels_per_ct(slots)
    outs = []
    for o in range(o_c):
        t_o = scheme.Ciphertext(t_all[o], xs.scale * pt_scale)
        first = t_o
        for kind, amount in tap_block_schedule(blocks, geom.h * geom.w):
            r = scheme.rotate(params, keys, t_o, amount)
            t_o = scheme.add(params, t_o if kind == "double" else first, r)
            counts.rot += 1
            counts.addcc += 1
        counts.addcc += xs.c.shape[0] * geom.d * geom.d - 1
        outs.append(t_o.c)
    z = scheme.rescale(params, scheme.Ciphertext(np.stack(outs), xs.scale * pt_scale))
    counts.rescale += o_c
    return z, counts


def tap_output_mask_slots(geom: ConvGeom, slots: int) -> np.ndarray:
    """E of the tap-style FFConv: 1 at every output slot (s i) W + s j."""
    v = np.zeros(slots)
    v[tap_output_slots(geom)] = 1.0
    return v


def tap_ffconv(params, keys, xs: scheme.Ciphertext, geom: ConvGeom, w1_filters: np.ndarray, w1_scale: float,
               w2: np.ndarray, k_bits: int, mask_pt: np.ndarray, mask_scale: float, square: bool = False,
               counts: Counts | None = None, w1_filters_p: np.ndarray | None = None
               ) -> tuple[scheme.Ciphertext, Counts]:
    """FFConv with W1 as a tap-style DensePack conv (tap_conv, r outputs),
    then C12's second half with one ciphertext per channel: G_c = y_c * E
    (E = tap_output_mask_slots at mask_scale; it clears the partial sums
    and leaves the outputs at their slots), Z_o = sum_c round(W2[c][o] 2^k)
    G_c, rescale, and with `square` x^2 relinearised and rescaled.
    Output: O_c ciphertexts, output (i, j) at slot (s i) W + s j, zero
    elsewhere.  With w1_filters_p (W1's residues mod P) W1 runs as
    tap_conv_lazy."""
    counts = counts if counts is not None else Counts()
    if w1_filters_p is None:
        y, _ = tap_conv(params, keys, xs, geom, w1_filters, w1_scale, counts)
    else:
        y, _ = tap_conv_lazy(params, keys, xs, geom, w1_filters, w1_filters_p, w1_scale, counts)
    z, _ = gather_convpack(params, y, 1, w2, k_bits, mask_pt, mask_scale, counts)
    if square:
        z, _ = square_rescale(params, keys, z, counts)
    return z, counts


# ---- Homomorphic Im2Col for d > 1 (Table III, CP-HI2C-*) ------------------------
# From a DensePack input to the K = d^2 I_c ConvPack input ciphertexts of
# Eq. 1.  The paper gives only the counts; this is one concrete algorithm
# with hoisted rotations, and its executed counts are reported beside
# Table III's.  Layout of Im2Col ciphertext k = (kh d + kw) I_c + c: the
# pixel under tap (kh, kw) of channel c for output (i, j) at slot
# (s i) W + s j, zero elsewhere.

def him2col_block_shifts(geom: ConvGeom, slots: int) -> list[int]:
    """Left rotations b H W, 0 < b < B, that bring block b to block 0."""
    per = geom.channels_per_ct(slots)
    return [b * geom.h * geom.w for b in range(1, per)]


def him2col_rotation_steps(geom: ConvGeom, slots: int) -> list[int]:
    amounts = {s % slots for s in tap_shifts(geom)} | set(him2col_block_shifts(geom, slots))
    return sorted(amounts - {0})


def him2col_mask_slots(geom: ConvGeom, slots: int, t: int) -> np.ndarray:
    """Mask of tap t: 1 at the slot of every output whose tap t lies inside
    the image."""
    kh, kw = divmod(t, geom.d)
    v = np.zeros(slots)
    for i in range(geom.out_h):
        y = geom.stride * i - geom.pad + kh
        if not 0 <= y < geom.h:
            continue
        for j in range(geom.out_w):
            x = geom.stride * j - geom.pad + kw
            if 0 <= x < geom.w:
                v[geom.stride * i * geom.w + geom.stride * j] = 1.0
    return v


def him2col(params, keys, xs: scheme.Ciphertext, geom: ConvGeom, masks: np.ndarray, mask_scale: float,
            counts: Counts | None = None) -> tuple[scheme.Ciphertext, Counts]:
    """Im2Col ciphertexts of a DensePack input xs (M ciphertexts).

    1. Per input ciphertext x_m, z_b = Rot(x_m, b H W) for 0 < b < B_m
       (B_m channels in x_m), hoisted over x_m's decomposition; z_0 = x_m.
    2. Per z_b, Rot(z_b, shift_t) for every nonzero tap shift, hoisted over
       z_b's decomposition (the zero shift is z_b).
    3. Ciphertext k = (kh d + kw) I_c + c (c = m B + b, t = kh d + kw) is
       mask_t * Rot(z_b, shift_t) (masks[t]: him2col_mask_slots at
       mask_scale, NTT domain), then all K are rescaled.
    Counts: Rot sum_m (B_m - 1 + B_m #nonzero shifts), MulPC K, K rescales."""
    counts = counts if counts is not None else Counts()
    slots = params.slots
    per = geom.channels_per_ct(slots)
    hw = geom.h * geom.w
    shifts = [s % slots for s in tap_shifts(geom)]
    nonzero = [s for s in shifts if s != 0]
    d2 = geom.d * geom.d
    out = [None] * (d2 * geom.c_in)
    for m in range(xs.c.shape[0]):
        x = scheme.Ciphertext(xs.c[m], xs.scale)
        b_m = min(per, geom.c_in - m * per)
        blocks = [x] + (scheme.rotate_hoisted(params, keys, x, [b * hw for b in range(1, b_m)]) if b_m > 1 else [])
        counts.rot += b_m - 1
        for b, z in enumerate(blocks):
            rot = dict(zip(nonzero, scheme.rotate_hoisted(params, keys, z, nonzero))) if nonzero else {}
            counts.rot += len(nonzero)
            c = m * per + b
            for t, s in enumerate(shifts):
                y = z if s == 0 else rot[s]
                out[t * geom.c_in + c] = scheme.mul_plain(params, y, masks[t], mask_scale).c
                counts.mulpc += 1
    y = scheme.rescale(params, scheme.Ciphertext(np.stack(out), xs.scale * mask_scale))
    counts.rescale += len(out)
    return y, counts


def combine_cp_to_dp(params, keys, z: scheme.Ciphertext, spatial: int, per_dense: int,
                     counts: Counts | None = None):
    """CP->DP: dense_m = sum_{o in block m} Rot(Z_o, -(o mod B)*S)."""
    counts = counts if counts is not None else Counts()
    o_c = z.c.shape[0]
    dense = []
    for m in range(math.ceil(o_c / per_dense)):
        acc = None
        for o in range(m * per_dense, min(o_c, (m + 1) * per_dense)):
            zo = scheme.Ciphertext(z.c[o], z.scale)
            shift = (o % per_dense) * spatial
            if shift:
                zo = scheme.rotate(params, keys, zo, -shift)
                counts.rot += 1
            if acc is None:
                acc = zo
            else:
                acc = scheme.add(params, acc, zo)
                counts.addcc += 1
        dense.append(acc.c)
    return scheme.Ciphertext(np.stack(dense), z.scale), counts


def combine_offsets(o_c: int, spatial: int, per_dense: int) -> list[int]:
    """Rotation amounts the combine step needs keys for (left rotations)."""
    return sorted({-(o % per_dense) * spatial for o in range(o_c) if o % per_dense})


def rotate_and_sum_steps(params) -> list[int]:
    return [1 << j for j in range(int(math.log2(params.slots)))]
