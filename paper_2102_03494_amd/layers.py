"""Server-side layer set-up: packing layouts, plaintext weights and scales.

The weights stay in plaintext on the server (Section 3, MLaaS scenario).
This module lays them out in slots as the C ABI expects (DensePack, Section
3.2 and Fig. 1; the DP->CP mask of FFConv, Section 4.2), encodes them with the
client-library encoder into NTT-domain plaintexts on the device, and computes
the plaintext scales.  The evaluation itself is one library call.

Scale rule: a plaintext multiply followed by a rescale that drops q_l is
encoded at q_l * target / current so the rescale lands on `target`; before a
square the target is sqrt(q_next * scale) so that square + rescale returns to
`scale`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .he import HEContext


@dataclass(frozen=True)
class Geometry:
    h: int
    w: int
    c_in: int
    d: int
    stride: int = 1
    pad: int = 0

    @property
    def out_h(self):
        return (self.h + 2 * self.pad - self.d) // self.stride + 1

    @property
    def out_w(self):
        return (self.w + 2 * self.pad - self.d) // self.stride + 1

    @property
    def spatial(self):
        return self.out_h * self.out_w

    def per_ct(self, slots):
        return min(self.c_in, slots // (self.h * self.w))

    def n_cts(self, slots):
        return -(-self.c_in // self.per_ct(slots))

    def _axis_classes(self, out, size):
        seen, ids = [], []
        for i in range(out):
            start = self.stride * i - self.pad
            r = (max(0, -start), min(self.d, size - start))
            if r not in seen:
                seen.append(r)
            ids.append(seen.index(r))
        return seen, ids

    def classes(self):
        """(row tap ranges, column tap ranges); class = row_class * n_cols + col_class."""
        rows, _ = self._axis_classes(self.out_h, self.h)
        cols, _ = self._axis_classes(self.out_w, self.w)
        return rows, cols


def densepack_layout(x: np.ndarray, g: Geometry, slots: int) -> list[np.ndarray]:
    """Slot vectors of X[h][w][c]: value (h, w, c) at slot (c mod B)*H*W + h*W + w of ct c // B."""
    per = g.per_ct(slots)
    vecs = []
    for m in range(g.n_cts(slots)):
        v = np.zeros(slots)
        for cl in range(per):
            c = m * per + cl
            if c < g.c_in:
                v[cl * g.h * g.w:(cl + 1) * g.h * g.w] = x[:, :, c].ravel()
        vecs.append(v)
    return vecs


def im2col_layout(x: np.ndarray, g: Geometry, slots: int) -> list[np.ndarray]:
    """Client-side plaintext Im2Col for a ConvPack input (Eq. 1): K = d^2 I_c
    slot vectors; vector (kh d + kw) I_c + c holds, at slot i O_w + j, the
    pixel X[s i - pad + kh][s j - pad + kw][c] (zero outside the image)."""
    h, w, c_in = x.shape
    s_out = g.out_h * g.out_w
    if s_out > slots:
        raise ValueError("more outputs than slots")
    xp = np.zeros((h + 2 * g.pad, w + 2 * g.pad, c_in))
    xp[g.pad:g.pad + h, g.pad:g.pad + w] = x
    out = []
    for kh in range(g.d):
        for kw in range(g.d):
            win = xp[kh:kh + g.stride * (g.out_h - 1) + 1:g.stride, kw:kw + g.stride * (g.out_w - 1) + 1:g.stride]
            for c in range(c_in):
                v = np.zeros(slots)
                v[:s_out] = win[:, :, c].reshape(-1)
                out.append(v)
    return out


def filter_layout(weights: np.ndarray, g: Geometry, slots: int, o: int, cls: int, m: int) -> np.ndarray:
    rows, cols = g.classes()
    kh0, kh1 = rows[cls // len(cols)]
    kw0, kw1 = cols[cls % len(cols)]
    per = g.per_ct(slots)
    v = np.zeros(slots)
    for cl in range(per):
        c = m * per + cl
        if c >= g.c_in:
            break
        for kh in range(kh0, kh1):
            for kw in range(kw0, kw1):
                v[cl * g.h * g.w + kh * g.w + kw] = weights[kh, kw, c, o]
    return v


# ---- tap-style DensePack (hoisted tap rotations; not one of the paper's designs) ----

def tap_shifts(g: Geometry) -> list[int]:
    """Left rotation of tap t = kh d + kw: (kh - pad) W + (kw - pad)."""
    return [(kh - g.pad) * g.w + (kw - g.pad) for kh in range(g.d) for kw in range(g.d)]


def tap_block_steps(blocks: int, hw: int) -> list[tuple[int, int]]:
    """The library's block-sum schedule: (0, k H W) doubles a k-block sum,
    (1, H W) adds one block, over the bits of `blocks` below the leading one."""
    steps, k = [], 1
    for bit in bin(blocks)[3:]:
        steps.append((0, k * hw))
        k *= 2
        if bit == "1":
            steps.append((1, hw))
            k += 1
    return steps


def tap_rotation_steps(g: Geometry, slots: int) -> list[int]:
    """Rotation keys a tap-style layer of this geometry needs."""
    amounts = {s % slots for s in tap_shifts(g)} | {a for _, a in tap_block_steps(g.per_ct(slots), g.h * g.w)}
    return sorted(amounts - {0})


def tap_output_slots(g: Geometry) -> np.ndarray:
    """Slot (s i) W + s j of output (i, j), row-major over outputs."""
    i = np.arange(g.out_h)[:, None]
    j = np.arange(g.out_w)[None, :]
    return (g.stride * i * g.w + g.stride * j).reshape(-1)


def tap_filter_layout(weights: np.ndarray, g: Geometry, slots: int, o: int, m: int, t: int) -> np.ndarray:
    """Plaintext (o, m, t): W[kh][kw][m B + b][o] in block b at the slot of
    every output whose tap (kh, kw) is inside the image; zero elsewhere."""
    kh, kw = divmod(t, g.d)
    per = g.per_ct(slots)
    hw = g.h * g.w
    ys = g.stride * np.arange(g.out_h) - g.pad + kh
    xs = g.stride * np.arange(g.out_w) - g.pad + kw
    valid = ((ys >= 0) & (ys < g.h))[:, None] & ((xs >= 0) & (xs < g.w))[None, :]
    where = tap_output_slots(g)[valid.reshape(-1)]
    v = np.zeros(slots)
    for b in range(per):
        c = m * per + b
        if c >= g.c_in:
            break
        v[b * hw + where] = weights[kh, kw, c, o]
    return v


def him2col_rotation_steps(g: Geometry, slots: int) -> list[int]:
    """Rotation keys of he_him2col: the nonzero tap shifts and the block
    shifts b H W, 0 < b < B."""
    amounts = {s % slots for s in tap_shifts(g)} | {b * g.h * g.w for b in range(1, g.per_ct(slots))}
    return sorted(amounts - {0})


def him2col_mask_layout(g: Geometry, slots: int, t: int) -> np.ndarray:
    """Mask of tap t: one at the slot of every output whose tap t is inside
    the image."""
    ones = np.ones((g.d, g.d, 1, 1))
    return tap_filter_layout(ones, Geometry(g.h, g.w, 1, g.d, g.stride, g.pad), slots, 0, 0, t)


def encode_him2col_masks(enc, g: Geometry, level: int, scale: float) -> torch.Tensor:
    slots = enc.ctx.n // 2
    return torch.stack([enc.encode(him2col_mask_layout(g, slots, t), level, scale) for t in range(g.d * g.d)])


def tap_output_mask_layout(g: Geometry, slots: int) -> np.ndarray:
    v = np.zeros(slots)
    v[tap_output_slots(g)] = 1.0
    return v


class PlainEncoder:
    """Keyless encoder for the server's plaintext weights: slot values to an
    NTT-domain plaintext [level][N] on the device (the client's encoding:
    host FFT of the canonical embedding, then the library's NTT)."""

    def __init__(self, ctx: HEContext):
        self.ctx = ctx

    def encode(self, z, level: int, scale: float) -> torch.Tensor:
        coeffs = torch.from_numpy(self.ctx.encode_coeffs(z, scale)).cuda()
        pt = self.ctx.from_signed(coeffs, level, 0)
        self.ctx.ntt(pt.view(1, level, self.ctx.n))
        return pt


def encode_filters(client, weights: np.ndarray, g: Geometry, level: int, pt_scale: float) -> torch.Tensor:
    """Base filter plaintexts [O_c][classes][M][level][N] on the device."""
    ctx = client.ctx
    rows, cols = g.classes()
    n_cls = len(rows) * len(cols)
    m_cts = g.n_cts(ctx.n // 2)
    o_c = weights.shape[3]
    out = torch.empty((o_c, n_cls, m_cts, level, ctx.n), dtype=torch.int64, device="cuda")
    for o in range(o_c):
        for b in range(n_cls):
            for m in range(m_cts):
                out[o, b, m] = client.encode(filter_layout(weights, g, ctx.n // 2, o, b, m), level, pt_scale)
    return out


def encode_tap_filters(client, weights: np.ndarray, g: Geometry, level: int, pt_scale: float,
                       threads: int = 16, with_p: bool = False):
    """Tap plaintexts [O][M][d^2][level][N] on the device (with_p: also their
    residues mod the special prime P, [O][M][d^2][N], returned as a pair).
    The host encodes run in a thread pool (the library's encoder releases
    the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    ctx = client.ctx
    slots = ctx.n // 2
    o_c = weights.shape[3]
    m_cts = g.n_cts(slots)
    d2 = g.d * g.d
    out = torch.empty((o_c, m_cts, d2, level, ctx.n), dtype=torch.int64, device="cuda")
    outp = torch.empty((o_c, m_cts, d2, ctx.n), dtype=torch.int64, device="cuda") if with_p else None
    big_l = len(ctx.q)
    idx = [(o, m, t) for o in range(o_c) for m in range(m_cts) for t in range(d2)]

    def coeffs(key):
        o, m, t = key
        return ctx.encode_coeffs(tap_filter_layout(weights, g, slots, o, m, t), pt_scale)

    with ThreadPoolExecutor(max_workers=threads) as pool:
        for (o, m, t), co in zip(idx, pool.map(coeffs, idx)):
            dco = torch.from_numpy(co).cuda()
            pt = ctx.from_signed(dco, level, 0)
            ctx.ntt(pt.view(1, level, ctx.n))
            out[o, m, t] = pt
            if with_p:
                pp = ctx.from_signed(dco, 1, big_l)
                ctx.ntt(pp.view(1, 1, ctx.n), big_l)
                outp[o, m, t] = pp[0]
    return (out, outp) if with_p else out


def pt_scale_for(ctx: HEContext, level: int, in_scale: float, target: float) -> float:
    return ctx.q[level - 1] * target / in_scale


def pre_square_target(ctx: HEContext, level_after_rescale: int, scale: float) -> float:
    return math.sqrt(ctx.q[level_after_rescale - 1] * scale)


def mask_scale_for(ctx: HEContext, level: int, y_scale: float, target: float, k_bits: int) -> float:
    return ctx.q[level - 1] * target / (y_scale * 2.0**k_bits)


def onehot_mask(client, level: int, scale: float) -> torch.Tensor:
    z = np.zeros(client.ctx.n // 2)
    z[0] = 1.0
    return client.encode(z, level, scale)


def rot_steps(ctx: HEContext) -> list[int]:
    return [1 << j for j in range(int(math.log2(ctx.n // 2)))]


def reference_conv2d(x: np.ndarray, weights: np.ndarray, stride: int = 1, pad: int = 0) -> np.ndarray:
    """FP64 plaintext convolution (for accuracy reports): Z[i][j][o]."""
    h, w, c = x.shape
    d = weights.shape[0]
    oh = (h + 2 * pad - d) // stride + 1
    ow = (w + 2 * pad - d) // stride + 1
    xp = np.zeros((h + 2 * pad, w + 2 * pad, c))
    xp[pad:pad + h, pad:pad + w] = x
    out = np.zeros((oh, ow, weights.shape[3]))
    for kh in range(d):
        for kw in range(d):
            patch = xp[kh:kh + stride * oh:stride, kw:kw + stride * ow:stride, :]  # (oh, ow, c)
            out += np.tensordot(patch, weights[kh, kw], axes=([2], [0]))
    return out


def compose_factors(w1: np.ndarray, w2: np.ndarray) -> np.ndarray:
    """d x d x I_c x O_c filters of W1 followed by the 1x1 W2 (O'_c x O_c)."""
    d1, d2, c, r = w1.shape
    return (w1.reshape(d1 * d2 * c, r) @ w2).reshape(d1, d2, c, w2.shape[1])
