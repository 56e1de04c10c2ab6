"""Encrypted networks of the serving workload, batched over requests.

Two nets with the shapes of Sec. 5's MNIST and CIFAR-10 experiments and
synthetic (seeded Gaussian) weights.  All requests of a batch run one model,
so every layer is one batched library call over all of them: the key
switches of a rotate-and-add step of every request share one Galois key.

MNIST-shaped net (N = 8192, 5 x 30-bit primes + 40-bit P, scale 2^25,
depth 4): FFConv 5x5 stride 2 pad 1, 1 -> 2 -> 5 channels (W1 under
DensePack, DP->CP gather, 1x1 W2 under ConvPack), x^2, CP->DP combine of the
five 13x13 channels into one DensePack ciphertext, then the 845 -> 10 fully
connected layer as a DensePack layer whose kernel covers the whole input.

CIFAR-shaped net (N = 16384, 6 x 40-bit primes + 60-bit P, scale 2^30,
depth 5): FFConv 3x3 pad 1, 3 -> 8 -> 64 channels with x^2, CP->DP combine
of the 64 32x32 channels into 8 DensePack ciphertexts, FFConv 3x3 pad 1,
64 -> 8 -> 64 over those 8 input ciphertexts.

The "plain" variant of each net replaces every FFConv by the conv with the
composed weights W1 W2 under DensePack (the comparator of Sec. 5), whose
replicated outputs are arranged into DensePack ciphertexts with shifted
one-hot masks before the next layer.

Each net takes its ring, weight shapes and geometry from a NetSpec, so the
same code runs the evaluated sizes and the small rings of the parity tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

import synth

from .he import Ct, HEContext
from .layers import (Geometry, PlainEncoder, compose_factors, densepack_layout, encode_filters, encode_tap_filters,
                     onehot_mask, pre_square_target, pt_scale_for, reference_conv2d, rot_steps, tap_output_mask_layout,
                     tap_rotation_steps)

K_BITS = 12


@dataclass(frozen=True)
class FFConvSpec:
    """One FFConv stage: W1 d x d (c_in -> r) under DensePack, 1x1 W2 (r -> o_c)."""
    geom: Geometry
    r: int
    o_c: int
    square: bool
    w1_id: int
    w2_id: int
    std: float


@dataclass(frozen=True)
class NetSpec:
    name: str
    n: int
    q_bits: tuple
    p_bits: int
    scale: float
    workload: str
    stages: tuple                  # FFConvSpec, ...: a CP->DP combine sits between consecutive stages
    fc: tuple | None = None        # (o, w_id, std): final dense layer on the combined last stage
    extra: dict = field(default_factory=dict)

    @property
    def level(self) -> int:
        return len(self.q_bits)


def mnist_spec(n=8192, q_bits=(30,) * 5, p_bits=40, image=28, d=5, stride=2, pad=1, r=2, o_c=5, fc_out=10):
    g = Geometry(image, image, 1, d, stride, pad)
    return NetSpec("mnist", n, tuple(q_bits), p_bits, 2.0**25, "serving",
                   (FFConvSpec(g, r, o_c, True, 1, 2, 0.1),), (fc_out, 3, 0.05))


def cifar_spec(n=16384, q_bits=(40,) * 6, p_bits=60, image=32, c_in=3, r1=8, o1=64, r2=8, o2=64):
    g1 = Geometry(image, image, c_in, 3, 1, 1)
    g2 = Geometry(image, image, o1, 3, 1, 1)
    return NetSpec("cifar", n, tuple(q_bits), p_bits, 2.0**30, "serving",
                   (FFConvSpec(g1, r1, o1, True, 11, 12, 0.05), FFConvSpec(g2, r2, o2, False, 13, 14, 0.05)))


def net_weights(spec: NetSpec) -> dict:
    """Seeded synthetic weights of the net (N(0, std^2))."""
    w = {}
    for k, st in enumerate(spec.stages):
        g = st.geom
        w[f"w1_{k}"] = synth.weights(spec.workload, 100 * st.w1_id + spec.n % 97, (g.d, g.d, g.c_in, st.r), st.std)
        w[f"w2_{k}"] = synth.weights(spec.workload, 100 * st.w2_id + spec.n % 97, (st.r, st.o_c), st.std)
    if spec.fc is not None:
        o, wid, std = spec.fc
        last = spec.stages[-1]
        g = last.geom
        w["fc"] = synth.weights(spec.workload, 100 * wid + spec.n % 97, (g.out_h, g.out_w, last.o_c, o), std)
    return w


def reference_forward(spec: NetSpec, weights: dict, x: np.ndarray, plain: bool = False) -> np.ndarray:
    """FP64 forward pass (Eq. 1 convolutions; W1 W2 composed for the plain
    variant, which is the same function)."""
    h = x
    for k, st in enumerate(spec.stages):
        g = st.geom
        w = compose_factors(weights[f"w1_{k}"], weights[f"w2_{k}"])
        h = reference_conv2d(h, w, g.stride, g.pad)
        if st.square:
            h = h * h
    if spec.fc is not None:
        h = reference_conv2d(h, weights["fc"], 1, 0).reshape(-1)
    return h


class EncryptedNet:
    """A net on one context, set up once (plaintext weights encoded on the
    device), run on batches of encrypted requests by forward()."""

    def __init__(self, ctx: HEContext, spec: NetSpec, weights: dict, plain: bool = False, encoder=None):
        """encoder: object with encode(z, level, scale) -> device plaintext
        (default: the library's keyless encoder)."""
        self.ctx, self.spec, self.plain = ctx, spec, plain
        enc = encoder if encoder is not None else PlainEncoder(ctx)
        n, slots = ctx.n, ctx.n // 2
        self.r_steps = int(math.log2(slots))
        scale = spec.scale
        level = spec.level
        self.stages = []
        self.combine_offsets = []
        cur_scale = scale
        for k, st in enumerate(spec.stages):
            g = st.geom
            rec = {"spec": st, "level": level, "in_scale": cur_scale}
            if not plain:
                desc = ctx.conv_desc(g.h, g.w, g.c_in, g.d, g.stride, g.pad, st.r, self.r_steps)
                pts = pt_scale_for(ctx, level, cur_scale, scale)
                y_scale = cur_scale * pts / ctx.q[level - 1]
                tgt = pre_square_target(ctx, level - 2, scale) if st.square else scale
                ms = ctx.q[level - 2] * tgt / (y_scale * 2.0**K_BITS)
                rec.update(desc=desc, pts=pts, ms=ms, mask=onehot_mask(enc, level - 1, ms),
                           filt=encode_filters(enc, weights[f"w1_{k}"], g, level, pts),
                           tab=ctx.int_weight_table(weights[f"w2_{k}"], K_BITS, level - 1))
                out_level = level - 2 - (1 if st.square else 0)
                z_scale = y_scale * ms * 2.0**K_BITS / ctx.q[level - 2]
                if st.square:
                    z_scale = z_scale * z_scale / ctx.q[level - 3]
            else:
                wp = compose_factors(weights[f"w1_{k}"], weights[f"w2_{k}"])
                desc = ctx.conv_desc(g.h, g.w, g.c_in, g.d, g.stride, g.pad, st.o_c, self.r_steps)
                pts = pt_scale_for(ctx, level, cur_scale, scale)
                y_scale = cur_scale * pts / ctx.q[level - 1]
                tgt = pre_square_target(ctx, level - 2, scale) if st.square else scale
                ms = ctx.q[level - 2] * tgt / y_scale
                per = min(st.o_c, slots // g.spatial)
                rec.update(desc=desc, pts=pts, ms=ms, mask=onehot_mask(enc, level - 1, ms),
                           filt=encode_filters(enc, wp, g, level, pts), per_dense=per)
                out_level = level - 2 - (1 if st.square else 0)
                z_scale = y_scale * ms / ctx.q[level - 2]
                if st.square:
                    z_scale = z_scale * z_scale / ctx.q[level - 3]
            rec.update(out_level=out_level, out_scale=z_scale)
            self.stages.append(rec)
            level, cur_scale = out_level, z_scale
            if not plain and (k + 1 < len(spec.stages) or spec.fc is not None):
                per = min(st.o_c, slots // g.spatial)
                rec["per_dense"] = per
                self.combine_offsets += [-(o % per) * g.spatial for o in range(st.o_c) if o % per]
        self.fc = None
        if spec.fc is not None:
            o, _, _ = spec.fc
            last = spec.stages[-1]
            gl = last.geom
            gf = Geometry(gl.out_h, gl.out_w, last.o_c, gl.out_h, 1, 0)
            desc = ctx.conv_desc(gf.h, gf.w, gf.c_in, gf.d, 1, 0, o, self.r_steps)
            pts = pt_scale_for(ctx, level, cur_scale, scale)
            self.fc = dict(desc=desc, pts=pts, level=level, filt=encode_filters(enc, weights["fc"], gf, level, pts),
                           out_scale=cur_scale * pts / ctx.q[level - 1])
        self.combine_offsets = sorted(set(self.combine_offsets))
        self._tabs = {}

    # ---- keys and sizes -------------------------------------------------------------
    def rotation_steps(self) -> list[int]:
        return rot_steps(self.ctx) + self.combine_offsets

    def needs_relin(self) -> bool:
        return any(st.square for st in self.spec.stages)

    def input_layout(self, x: np.ndarray) -> list[np.ndarray]:
        return densepack_layout(x, self.spec.stages[0].geom, self.ctx.n // 2)

    def workspace_need(self, batch: int) -> int:
        """Context workspace bytes of forward() on `batch` requests."""
        ctx = self.ctx
        need = 0
        for rec in self.stages:
            st = rec["spec"]
            if not self.plain:
                need = max(need, ctx.ffconv_workspace_need(batch, rec["level"], rec["desc"], st.o_c, st.square))
            else:
                g = st.geom
                need = max(need, ctx.workspace_need(min(batch * g.spatial * st.o_c, 16000), rec["level"]))
            need = max(need, ctx.workspace_need(batch * st.o_c, rec["out_level"]))
        if self.fc is not None:
            need = max(need, ctx.workspace_need(batch * self.fc["desc"].o_c, self.fc["level"]))
        return need

    def activation_bytes(self, batch: int) -> int:
        """Device bytes of the tensors forward() allocates besides the
        workspace (largest stage output; the plain variant's replicated
        DensePack outputs dominate)."""
        n = self.ctx.n
        most = 0
        for rec in self.stages:
            st = rec["spec"]
            g = st.geom
            count = g.spatial * st.o_c if self.plain else st.o_c
            most = max(most, batch * count * 2 * (rec["level"] - 1) * n * 8)
        return 2 * most

    def _w2_tabs(self, k: int, batch: int) -> torch.Tensor:
        key = (k, batch)
        if key not in self._tabs:
            self._tabs[key] = self.stages[k]["tab"].unsqueeze(0).repeat(batch, 1).contiguous()
        return self._tabs[key]

    # ---- evaluation ------------------------------------------------------------------
    def forward(self, xs: torch.Tensor) -> Ct:
        """xs: [B][M][2][level][N] (or [B][2][level][N]) requests at the spec's
        scale.  Returns [B][10][2][1][N] replicated FC outputs (MNIST) or the
        last stage's [B][o_c][2][level][N] ConvPack channels (CIFAR)."""
        ctx = self.ctx
        batch = xs.shape[0]
        cur = Ct(xs.contiguous(), self.spec.scale)
        for k, rec in enumerate(self.stages):
            st = rec["spec"]
            g = st.geom
            if not self.plain:
                z = ctx.ffconv_layer_batch(cur.data, cur.scale, rec["desc"], rec["filt"], rec["pts"], rec["mask"],
                                           rec["ms"], self._w2_tabs(k, batch), st.o_c, K_BITS, st.square,
                                           shared_w1=True)
                if "per_dense" in rec:
                    cur = ctx.combine_cp_dp_batch(z, g.spatial, rec["per_dense"])
                else:
                    cur = z
            else:
                y = ctx.conv_densepack_batch(cur.data, cur.scale, rec["desc"], rec["filt"], rec["pts"])
                lv = rec["level"] - 1
                per = rec["per_dense"]
                total = g.spatial * st.o_c
                n_dense = -(-st.o_c // per)
                # arrange the replicated outputs: channel o to slots (o mod per) * S + p of dense o // per
                yd = y.data.view(batch, total, 2, lv, ctx.n)
                k = per * g.spatial
                if n_dense * k > total:  # zero ciphertexts fill the last group
                    pad = torch.zeros((batch, n_dense * k - total, 2, lv, ctx.n), dtype=torch.int64, device="cuda")
                    yd = torch.cat([yd, pad], 1)
                grp = Ct(yd.reshape(batch * n_dense * k, 2, lv, ctx.n), y.scale)
                dense = ctx.gather_onehot(grp, k, rec["mask"], rec["ms"])
                dense = ctx.rescale(dense)
                if st.square:
                    dense = ctx.rescale(ctx.square(dense))
                cur = Ct(dense.data.view(batch, n_dense, 2, dense.level, ctx.n), dense.scale)
        if self.fc is not None:
            fc = self.fc
            data = cur.data if cur.data.dim() == 5 else cur.data.unsqueeze(1)
            out = ctx.conv_densepack_batch(data.contiguous(), cur.scale, fc["desc"], fc["filt"], fc["pts"])
            return Ct(out.data.view(batch, fc["desc"].o_c, 2, 1, ctx.n), out.scale)
        return cur

    def decode(self, client, out: Ct, b: int) -> np.ndarray:
        """Decrypted prediction of request b (FC values, or the last stage's channels)."""
        if self.fc is not None:
            return np.array([client.decrypt(out.data[b, o], out.scale, 1, limbs=1)[0]
                             for o in range(out.data.shape[1])])
        last = self.spec.stages[-1]
        s = last.geom.spatial
        if not self.plain:
            return np.stack([client.decrypt(out.data[b, o], out.scale, s, limbs=1) for o in range(last.o_c)], 1)
        per = self.stages[-1]["per_dense"]
        vals = [client.decrypt(out.data[b, m], out.scale, per * s, limbs=1) for m in range(out.data.shape[1])]
        flat = np.concatenate(vals)[: last.o_c * s]
        return flat.reshape(last.o_c, s).T


class TapNet:
    """The same nets with every FFConv stage as a tap-style FFConv
    (ffconv_layer_tap: hoisted tap rotations and masked W1 plaintexts
    instead of one rotate-and-sum chain per DensePack output, the rotations'
    ModDown deferred to one per W1 output; not one of the paper's designs).  A stage's output channel o holds output (i, j) at slot
    (s i) W + s j of its input plane (W: input width), zero elsewhere; the
    CP->DP combine packs B = floor(N / (2 H W)) channels per ciphertext with
    blocks of H W slots, so for stride 1 the next stage reads the usual
    DensePack layout.  The MNIST-shaped net's FC layer is a DensePack layer
    over that plane whose weights sit at the strided output positions (zero
    elsewhere): the same 845 -> 10 map.  Same interface as EncryptedNet
    (forward, decode, keys, sizes)."""

    plain = False

    def __init__(self, ctx: HEContext, spec: NetSpec, weights: dict, encoder=None):
        self.ctx, self.spec = ctx, spec
        enc = encoder if encoder is not None else PlainEncoder(ctx)
        slots = ctx.n // 2
        self.r_steps = int(math.log2(slots))
        scale = spec.scale
        level = spec.level
        cur_scale = scale
        self.stages = []
        steps = set()
        for k, st in enumerate(spec.stages):
            g = st.geom
            steps |= set(tap_rotation_steps(g, slots))
            desc = ctx.conv_desc(g.h, g.w, g.c_in, g.d, g.stride, g.pad, st.r, 0)
            w1s = pt_scale_for(ctx, level, cur_scale, scale)
            y_scale = cur_scale * w1s / ctx.q[level - 1]
            tgt = pre_square_target(ctx, level - 2, scale) if st.square else scale
            ms = ctx.q[level - 2] * tgt / (y_scale * 2.0**K_BITS)
            filt, filt_p = encode_tap_filters(enc, weights[f"w1_{k}"], g, level, w1s, with_p=True)
            rec = dict(spec=st, level=level, in_scale=cur_scale, desc=desc, w1s=w1s, ms=ms, filt=filt, filt_p=filt_p,
                       mask=enc.encode(tap_output_mask_layout(g, slots), level - 1, ms), w2=weights[f"w2_{k}"],
                       w2_tab=ctx.int_weight_table(weights[f"w2_{k}"], K_BITS, level - 1))
            out_level = level - 2 - (1 if st.square else 0)
            z_scale = y_scale * ms * 2.0**K_BITS / ctx.q[level - 2]
            if st.square:
                z_scale = z_scale * z_scale / ctx.q[level - 3]
            rec.update(out_level=out_level, out_scale=z_scale)
            if k + 1 < len(spec.stages) or spec.fc is not None:
                block = g.h * g.w
                per = min(st.o_c, slots // block)
                rec.update(block=block, per_dense=per)
                steps |= {(-(o % per) * block) % slots for o in range(st.o_c) if o % per}
            self.stages.append(rec)
            level, cur_scale = out_level, z_scale
        self.fc = None
        if spec.fc is not None:
            o, _, _ = spec.fc
            last = spec.stages[-1]
            gl = last.geom
            if gl.h != gl.w:
                raise ValueError("the FC layer over a stage's plane needs a square plane")
            wd = np.zeros((gl.h, gl.w, last.o_c, o))
            s_ = gl.stride
            wd[0:s_ * gl.out_h:s_, 0:s_ * gl.out_w:s_] = weights["fc"]
            gf = Geometry(gl.h, gl.w, last.o_c, gl.h, 1, 0)
            desc = ctx.conv_desc(gf.h, gf.w, gf.c_in, gf.d, 1, 0, o, self.r_steps)
            pts = pt_scale_for(ctx, level, cur_scale, scale)
            self.fc = dict(desc=desc, pts=pts, level=level, filt=encode_filters(enc, wd, gf, level, pts),
                           out_scale=cur_scale * pts / ctx.q[level - 1])
            steps |= set(rot_steps(ctx))
        self.steps = sorted(steps - {0})

    def rotation_steps(self) -> list[int]:
        return list(self.steps)

    def needs_relin(self) -> bool:
        return any(st.square for st in self.spec.stages)

    def input_layout(self, x: np.ndarray) -> list[np.ndarray]:
        return densepack_layout(x, self.spec.stages[0].geom, self.ctx.n // 2)

    def workspace_need(self, batch: int) -> int:
        ctx = self.ctx
        need = 0
        for rec in self.stages:
            st = rec["spec"]
            need = max(need, ctx.tap_workspace_need(batch, rec["level"], rec["desc"], st.o_c, st.square))
            need = max(need, ctx.workspace_need(batch * st.o_c, rec["out_level"]))
        if self.fc is not None:
            need = max(need, ctx.workspace_need(batch * self.fc["desc"].o_c, self.fc["level"]))
        return need

    def activation_bytes(self, batch: int) -> int:
        n = self.ctx.n
        most = max(batch * rec["spec"].o_c * 2 * (rec["level"] - 1) * n * 8 for rec in self.stages)
        return 2 * most

    def forward(self, xs: torch.Tensor) -> Ct:
        """xs: [B][M][2][level][N] (or [B][2][level][N]) requests; returns
        [B][10][2][1][N] replicated FC outputs (MNIST-shaped) or the last
        stage's [B][o_c][2][level][N] channels (CIFAR-shaped)."""
        ctx = self.ctx
        batch = xs.shape[0]
        data = xs.contiguous() if xs.dim() == 5 else xs.contiguous().unsqueeze(1)
        cur = Ct(data, self.spec.scale)
        for rec in self.stages:
            st = rec["spec"]
            z = ctx.ffconv_layer_tap(cur.data, cur.scale, rec["desc"], rec["filt"], rec["w1s"], rec["mask"],
                                     rec["ms"], rec["w2"], K_BITS, square=st.square, w1_p=rec["filt_p"],
                                     w2_tab=rec["w2_tab"])
            cur = ctx.combine_cp_dp_batch(z, rec["block"], rec["per_dense"]) if "per_dense" in rec else z
        if self.fc is not None:
            fc = self.fc
            out = ctx.conv_densepack_batch(cur.data.contiguous(), cur.scale, fc["desc"], fc["filt"], fc["pts"])
            return Ct(out.data.view(batch, fc["desc"].o_c, 2, 1, ctx.n), out.scale)
        return cur

    def decode(self, client, out: Ct, b: int) -> np.ndarray:
        """Decrypted prediction of request b (FC values, or the last stage's
        channels as [S][o_c])."""
        if self.fc is not None:
            return np.array([client.decrypt(out.data[b, o], out.scale, 1, limbs=1)[0]
                             for o in range(out.data.shape[1])])
        last = self.spec.stages[-1]
        g = last.geom
        i = np.arange(g.out_h)[:, None]
        j = np.arange(g.out_w)[None, :]
        where = (g.stride * i * g.w + g.stride * j).reshape(-1)
        return np.stack([client.decrypt(out.data[b, o], out.scale, limbs=1)[where] for o in range(last.o_c)], 1)
