#!/usr/bin/env python3
"""Encrypted conv-layer latency and rotations/s on one MI355X: FFConv vs plain.

Workload (the 28x28 MNIST-shaped layer, synthetic): a 28x28x1 image with
pixels uniform in [0, 1), client-encrypted under DensePack in one ciphertext
at N = 8192 (4 x 30-bit primes + a 40-bit special prime, scale 2^25).
  * FFConv layer (the step that is timed): 5x5 stride-2 low-rank conv 1 -> 2
    channels under DensePack (288 dot products, 12 rotate-and-add steps each),
    the DP->CP gather and a 1x1 conv 2 -> 5 under ConvPack, then x^2 and
    rescale -- one ffconv_layer call;
  * plain comparator: the 5x5 stride-2 conv 1 -> 5 with the composed weights
    W1 W2 under DensePack (720 dot products), then x^2 and rescale.
Weights are N(0, 0.1^2).  Inputs, keys and plaintext weights are resident in
HBM before the timed region.  One step = one FFConv layer on one encrypted
image; `value` is executed rotations per second of the timed steps.

Extra fields: the plain layer's latency and rotations/s, HMA/s, decrypted
max error of both against the FP64 convolution, executed operation counts,
the roofline of the dominant kernel (timed with HIP events around each of its
launches inside the timed region), and the CPU oracle timed on a bounded
sample of the same DensePack dot products.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "ffconv_n8192"
N, Q_BITS, P_BITS, SCALE = 8192, (30, 30, 30, 30), 40, 2.0**25
K_BITS = 12


def w2_bits(ctx) -> int:
    """Bits of W2's exact integers round(W2 2^k) for a chain: 12 with 30-bit
    primes (scale 2^25), 16 with 40-bit primes (scale 2^30).  Measured on the
    CIFAR-shaped layer (N = 16384), decrypted max error 1.5e-4 / 4.0e-5 /
    2.2e-5 / 5.1e-5 for k = 12 / 14 / 16 / 18 (W2 rounding against the one-hot
    mask's encoding at scale 2^(40 - k)); on the 30-bit chain k = 9..13 all
    gave 1.6e-4 .. 2.3e-4 (rescale noise dominates)."""
    return 16 if min(ctx.q) > (1 << 36) else K_BITS
HBM_PEAK_GBS = 8000.0
# 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
DOMINANT = "ks_modup_stage"

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (each
# scaled by what the counter reads for a 1 GiB device copy: x2.0 / x1.0),
# valid only for the kernel sources they were measured on: bench.py reports
# them when these sources hash to KERNEL_SHA256, else null.
KERNEL_SOURCES = ("modarith.h", "ntt_lds.h", "kernels.h", "capi.hip")
KERNEL_SHA256 = "a2e1876622bb806d24b6a4957695cf75a58db498a2ea55cb2bd448bc97dd381f"
# ks_modup_stage: mean over one layer's 25 launches (24 of 144 jobs at
# 123.0 MB, one relinearisation launch of 5 jobs at 6.3 MB); ip_perm: one
# launch over all 256 rotations; dp_hma: the one MulPC launch of a layer
TRAFFIC_BYTES = {"ks_modup_stage": 118295983, "ip_perm": 4454320155, "dp_hma": 78350999}


def kernel_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2102_03494_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    return TRAFFIC_BYTES.get(kernel) if KERNEL_SHA256 is not None and kernel_sha256() == KERNEL_SHA256 else None

# Algorithmic operation counts (VALU lane ops; an FP64 multiply, FMA or add
# counts as one, as it issues at the 32-bit rate) of the key-switch work per
# width class: narrow = 30-bit primes in 32-bit words (Harvey butterflies,
# 64-bit lazy inner-product sums), f64 = primes below 2^42 as exact integers
# in doubles, wide = 64-bit words.
COST = {
    "bfly": {"n32": 9, "f64": 9, "u64": 34},   # one butterfly with its twiddle product
    "mac": {"n32": 1, "f64": 8, "u64": 40},    # one key product accumulated
    "lift": {"n32": 3, "f64": 3, "u64": 12},   # centred lift of one digit coefficient
    "fin": {"n32": 10, "f64": 6, "u64": 0},    # final reduction of one output coefficient
}


def width_class(q: int) -> str:
    return "n32" if q < (1 << 30) else ("f64" if q < (1 << 42) else "u64")


def modup_ip_ops(count: int, level: int, n: int, moduli, pg: int, halves: bool = False) -> float:
    """Algorithmic VALU ops of the ModUp + inner-product stage (every target
    prime of every width class, P split over pg digit groups) over `count`
    ciphertexts at `level`: per target, a lift and an NTT of each digit but
    its own, one key product per digit and output polynomial, one final
    reduction per output coefficient; with one P group and whole-limb
    workgroups, the INTT of the P limb (which then runs in the same launch).
    With half-ring workgroups the work is the same (the duplicated
    first-stage products are not counted) and the P INTT runs in its own
    kernel."""
    bfly = (n // 2) * int(math.log2(n))
    ops = 0.0
    for t in range(level):
        c = width_class(moduli[t])
        ops += (level - 1) * (bfly * COST["bfly"][c] + n * COST["lift"][c])
        ops += 2 * n * (level * COST["mac"][c] + COST["fin"][c])
    c = width_class(moduli[-1])
    groups = -(-level // -(-level // pg))
    ops += level * (bfly * COST["bfly"][c] + n * COST["lift"][c] + 2 * n * COST["mac"][c])
    ops += groups * 2 * n * COST["fin"][c]
    if groups == 1 and not halves:  # the P workgroup also takes its limb back to the coefficient domain
        ops += 2 * (bfly * COST["bfly"][c] + n * COST["fin"][c])
    return ops * count


def modup_ip_bytes(count: int, level: int, n: int, moduli, pg: int, packed_in: bool = False) -> float:
    """Algorithmic HBM bytes of the ModUp + inner-product stage over `count`
    ciphertexts at `level`: per ciphertext its coefficient-domain digits and
    its own NTT-domain limbs read once, both output polynomials written once
    (the level ciphertext-prime rows, and the P limb as its coefficient-domain
    copy with one P group, else as one partial row per group), and the key
    (2 level (level + 1) limbs) read once.  Residues of narrow primes are
    packed 32-bit words in the scratch rows and keys, and in the input
    ciphertext when packed_in (a rotate-and-sum chain after its first step);
    all others are 64-bit words."""
    def width(q):
        return 4 if q < (1 << 30) else 8
    qs, p = moduli[:level], moduli[-1]
    groups = -(-level // -(-level // pg))
    q_row = sum(width(q) for q in qs) * n
    own = q_row if packed_in else 8 * n * level
    per = q_row + own + 2 * (q_row + groups * width(p) * n)
    key = 2 * level * (q_row + width(p) * n)
    return count * per + key


def dp_hma_bytes(n_out: int, m_cts: int, n_filters: int, level: int, n: int, moduli,
                 packed_out: bool = True) -> float:
    """Algorithmic HBM bytes of one DensePack MulPC launch (k_dp_hma) over
    n_out outputs: the m_cts input ciphertexts and the n_filters base filter
    plaintexts (one per output channel, border class and input ciphertext)
    read once, as 64-bit words, and the n_out products (two polynomials of
    `level` limbs) written once, narrow residues as packed 32-bit words when
    packed_out (the products then go straight into packed rotate-and-sum
    chains)."""
    qs = moduli[:level]
    out_row = sum(4 if (packed_out and q < (1 << 30)) else 8 for q in qs) * n
    return (2 * m_cts + n_filters) * level * 8 * n + n_out * 2 * out_row


def setup(ctx, client, x, w1, w2):
    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.he import Ct

    geom = Ly.Geometry(28, 28, 1, 5, 2, 0)
    level = len(Q_BITS)
    slots = N // 2
    ct = client.encrypt(Ly.densepack_layout(x, geom, slots)[0], level, SCALE, index=0)
    steps = Ly.rot_steps(ctx)
    desc_ff = ctx.conv_desc(28, 28, 1, 5, 2, 0, w1.shape[3], len(steps))
    pts1 = Ly.pt_scale_for(ctx, level, SCALE, SCALE)
    f1 = Ly.encode_filters(client, w1, geom, level, pts1)
    y_scale = SCALE * pts1 / ctx.q[level - 1]
    target = Ly.pre_square_target(ctx, level - 2, SCALE)
    ms = Ly.mask_scale_for(ctx, level - 1, y_scale, target, K_BITS)
    mask = Ly.onehot_mask(client, level - 1, ms)
    w_plain = Ly.compose_factors(w1, w2)
    desc_pl = ctx.conv_desc(28, 28, 1, 5, 2, 0, w_plain.shape[3], len(steps))
    target_pl = Ly.pre_square_target(ctx, level - 1, SCALE)
    pts_pl = Ly.pt_scale_for(ctx, level, SCALE, target_pl)
    f_pl = Ly.encode_filters(client, w_plain, geom, level, pts_pl)

    def ffconv_step():
        return ctx.ffconv_layer(ct, desc_ff, f1, pts1, mask, ms, w2, K_BITS, True)

    def plain_step():
        y = ctx.conv_densepack(ct, desc_pl, f_pl, pts_pl)
        return ctx.rescale(ctx.square(y))

    return geom, ct, ffconv_step, plain_step, w_plain


def paper_counts_dp_hi2c_cp(spatial: int, r: int, o_c: int, r_steps: int) -> dict:
    """The paper's formula counts of an FFConv layer packed DP-HI2C-CP with
    d = 1 (Table I for W1 with O' = S r, Table III DP-HI2C-CP d = 1: O^1_c
    MulPC and O^1_c Rot, Table II for W2 with K = r)."""
    o1 = spatial * r
    w1 = {"mulpc": o1, "addcc": o1 * r_steps, "rot": o1 * r_steps}
    hi2c = {"mulpc": r, "addcc": 0, "rot": r}
    w2 = {"mulpc": o_c * r, "addcc": o_c * (r - 1), "rot": 0}
    tot = {k: w1[k] + hi2c[k] + w2[k] for k in w1}
    return {"W1_densepack_table_I": w1, "HI2C_table_III_dp_cp_d1": hi2c, "W2_convpack_table_II": w2, "total": tot,
            "note": "executed: the DP->CP step is S r one-hot mask products and no rotation (CKKS replicated "
                    "DensePack outputs), plus x^2 with its relinearisation where configured"}


def paper_counts_dp(spatial: int, o_c: int, r_steps: int) -> dict:
    """Table I counts of a plain DensePack layer (O = S O_c dot products)."""
    o = spatial * o_c
    return {"mulpc": o, "addcc": o * r_steps, "rot": o * r_steps}


def chain_parts(n_out: int, split_streams: int, split_parts: int) -> int:
    """Chains (one stream each) the library splits a DensePack rotate-and-sum
    of n_out outputs into: split_parts when splitting is on and there are at
    least 64 outputs, at most one chain per 32 outputs; else one."""
    if not split_streams or n_out < 64:
        return 1
    return max(1, min(split_parts, n_out // 32))


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def hoisted_section(torch, steps: int):
    """256 seeded rotations of one level-6 ciphertext at N = 16384 (6 x 40-bit +
    60-bit P) sharing one ModUp, against 256 one-at-a-time rotations.  The
    per-rotation inner product (k_ip_perm) streams each rotation's key once:
    it is the HBM-bound kernel of the path."""
    import synth
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import HEContext

    wl = "batched_n16384"
    n, level = 16384, 6
    ctx = HEContext(n, (40,) * level, 60)
    ctx.reserve(3 << 30)
    cl = Client(ctx, wl)
    amounts = [int(k) for k in synth.rotation_amounts(wl, 256, n // 2)]
    cl.gen_rotation_keys(amounts)
    ct = cl.encrypt(synth.message(wl, n // 2), level, 2.0**30, index=0)
    ctx.rotate_hoisted(ct, amounts)
    torch.cuda.synchronize()
    ctx.prof_select("ip_perm")
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.rotate_hoisted(ct, amounts)
    torch.cuda.synchronize()
    t_h = (time.perf_counter() - t0) / steps
    ip_ms, ip_launches = ctx.prof_read()
    ctx.prof_select(None)
    # the variant with the inner product fused into ModDown (no u round trip)
    ctx.set_tuning("hoist_fused", 0, 1)
    t_fused, _ = timed(lambda: ctx.rotate_hoisted(ct, amounts), steps, 1, torch)
    ctx.set_tuning("hoist_fused", 0, 0)
    # two streams: a chunk's inner products beside the previous chunk's ModDown
    ctx.set_tuning("hoist_pipeline", 0, 1)
    t_twostreams, _ = timed(lambda: ctx.rotate_hoisted(ct, amounts), steps, 1, torch)
    ctx.set_tuning("hoist_pipeline", 0, 0)
    out = torch.empty_like(ct.data)
    t0 = time.perf_counter()
    for k in amounts:
        ctx.rotate(ct, k, out=out)
    torch.cuda.synchronize()
    t_u = time.perf_counter() - t0
    limb = 8 * n
    m = len(amounts)
    # the whole call: the input ciphertext once, then per rotation its key
    # (2 L (L + 1) limbs) and its output (2 L limbs)
    call_bytes = 2 * level * limb + m * (2 * level * limb + 2 * level * (level + 1) * limb)
    # the inner-product kernel: per rotation its key and its 2 (L + 1) output
    # rows, and the shared lifted digits once
    # (the shared lifted digits counted once per launch)
    per_call = max(1, ip_launches // max(1, steps))
    ip_bytes = (m * (2 * level * (level + 1) * limb + 2 * (level + 1) * limb)
                + per_call * level * (level + 1) * limb) // per_call
    avg = ip_ms / max(1, ip_launches)
    ach = ip_bytes / (avg * 1e-3) / 1e9
    ach_call = call_bytes / t_h / 1e9
    return {
        "workload": "one ciphertext, N=16384, level 6 (6x40-bit + 60-bit P), 256 seeded rotation amounts",
        "hoisted_ms": t_h * 1e3, "unhoisted_ms": t_u * 1e3, "speedup": t_u / t_h,
        "hoisted_fused_moddown_ms": t_fused * 1e3,
        "hoisted_two_streams_ms": t_twostreams * 1e3,
        "rotations_per_s": m / t_h,
        "roofline": {"kernel": "he_rotate_hoisted end to end (one ModUp; the inner products of all 256 rotations "
                               "in one launch; P INTT; ModDown)",
                     "bound": "hbm", "achieved": ach_call, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach_call / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes_per_call": call_bytes},
        "roofline_ip_kernel": {"kernel": "k_ip_perm (key inner product of all 256 rotations, one launch)",
                               "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic("ip_perm"),
                               "avg_launch_ms": avg, "algorithmic_bytes_per_launch": ip_bytes},
    }


def batched_layers_section(torch, ctx, client, n_layers: int, reps: int):
    """n_layers independent FFConv layers of the timed workload's shape (each
    with its own seeded image, W1 and W2), three ways: n_layers sequential
    ffconv_layer calls, one ffconv_layer_batch call, and that call captured
    once in a HIP graph and replayed."""
    import numpy as np

    import synth
    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.he import Ct

    geom = Ly.Geometry(28, 28, 1, 5, 2, 0)
    level = len(Q_BITS)
    steps = Ly.rot_steps(ctx)
    desc = ctx.conv_desc(28, 28, 1, 5, 2, 0, 2, len(steps))
    pts = Ly.pt_scale_for(ctx, level, SCALE, SCALE)
    y_scale = SCALE * pts / ctx.q[level - 1]
    ms = Ly.mask_scale_for(ctx, level - 1, y_scale, Ly.pre_square_target(ctx, level - 2, SCALE), K_BITS)
    mask = Ly.onehot_mask(client, level - 1, ms)
    xs, filts, tabs, w1s, w2s, imgs = [], [], [], [], [], []
    for li in range(n_layers):
        x = synth.image(WORKLOAD, (28, 28, 1), index=1000 + li)
        w1 = synth.weights(WORKLOAD, 1000 + 2 * li, (5, 5, 1, 2), 0.1)
        w2 = synth.weights(WORKLOAD, 1001 + 2 * li, (2, 5), 0.1)
        xs.append(client.encrypt(Ly.densepack_layout(x, geom, N // 2)[0], level, SCALE, index=1000 + li).data[0])
        filts.append(Ly.encode_filters(client, w1, geom, level, pts))
        tabs.append(ctx.int_weight_table(w2, K_BITS, level - 1))
        imgs.append(x)
        w1s.append(w1)
        w2s.append(w2)
    xs = torch.stack(xs).contiguous()
    filts = torch.stack(filts).contiguous()
    tabs = torch.stack(tabs).contiguous()
    ctx.reserve(ctx.ffconv_workspace_need(n_layers, level, desc, 5, True))
    out = torch.empty((n_layers, 5, 2, level - 3, N), dtype=torch.int64, device="cuda")
    print(f"# batched layers: {n_layers} layers set up", file=sys.stderr, flush=True)

    def sequential():
        for li in range(n_layers):
            ctx.ffconv_layer(Ct(xs[li:li + 1], SCALE), desc, filts[li], pts, mask, ms, w2s[li], K_BITS, True,
                             out=out[li])

    def batched():
        return ctx.ffconv_layer_batch(xs, SCALE, desc, filts, pts, mask, ms, tabs, 5, K_BITS, True, out=out)

    t_seq, _ = timed(sequential, 1, 1, torch)
    seq_bits = out.cpu().clone()
    t_bat, z = timed(batched, reps, 1, torch)
    bat_bits = out.cpu().clone()
    graph, _ = ctx.capture(batched)
    out.zero_()
    t_gr, _ = timed(graph.launch, reps, 1, torch)
    gr_bits = out.cpu().clone()
    graph.close()
    same = bool(torch.equal(seq_bits, bat_bits) and torch.equal(bat_bits, gr_bits))
    err = 0.0
    for li in (0, n_layers // 2, n_layers - 1):
        ref = (Ly.reference_conv2d(imgs[li], w1s[li], 2, 0) @ w2s[li]) ** 2
        for o in range(5):
            v = client.decrypt(out[li, o], z.scale, geom.spatial, limbs=1)
            err = max(err, float(np.abs(v - ref[:, :, o].ravel()).max()))
    rot = n_layers * 288 * 12
    return {
        "workload": f"{n_layers} independent FFConv layers 28x28x1, 5x5 s2 1->2 + 1x1 2->5 + x^2, N=8192, "
                    "each with its own seeded image, W1 and W2",
        "sequential_ms_per_layer": t_seq * 1e3 / n_layers,
        "batched_ms_per_layer": t_bat * 1e3 / n_layers,
        "graph_ms_per_layer": t_gr * 1e3 / n_layers,
        "graph_rotations_per_s": rot / t_gr,
        "speedup_graph_vs_sequential": t_seq / t_gr,
        "outputs_identical_sequential_batched_graph": same,
        "decrypted_max_abs_err_sampled_layers": err,
        "p_groups": ctx.get_tuning("p_groups", level),
    }


def ragged_section(torch, reps: int):
    """64 ciphertexts at N = 16384 (6 x 40-bit + 60-bit P), ciphertext i at
    level 2 + (i mod 5): one batched MulPC, one batched rescale and the 13
    rotate-and-add steps (each one batched key switch over all 64, every item
    at its own level), against the same work issued per ciphertext."""
    import numpy as np

    import synth
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import Ct, HEContext

    wl = "batched_n16384"
    n = 16384
    ctx = HEContext(n, (40,) * 6, 60)
    ctx.reserve(4 << 30)
    cl = Client(ctx, wl)
    r_steps = 13
    cl.gen_rotation_keys([1 << j for j in range(r_steps)])
    levels = [2 + (i % 5) for i in range(64)]
    msgs = [synth.message(wl, n // 2, index=100 + i) for i in range(64)]
    cts = [cl.encrypt(msgs[i], levels[i], 2.0**30, index=100 + i).data[0] for i in range(64)]
    pts = [cl.encode(synth.message(wl, n // 2, index=300 + i), levels[i], 2.0**30) for i in range(64)]
    prod = [torch.empty_like(c) for c in cts]
    resc = [torch.empty((2, lv - 1, n), dtype=torch.int64, device="cuda") for lv in levels]
    acc = [c.clone() for c in cts]

    def b_mul():
        ctx.batch_mul_plain(prod, cts, pts)

    def u_mul():
        for i in range(64):
            ctx.batch_mul_plain(prod[i:i + 1], cts[i:i + 1], pts[i:i + 1])

    def b_resc():
        ctx.batch_rescale(resc, prod)

    def u_resc():
        for i in range(64):
            ctx.batch_rescale(resc[i:i + 1], prod[i:i + 1])

    def b_rot():
        for j in range(r_steps):
            ctx.batch_rotate(acc, acc, [1 << j] * 64, accumulate=True)

    def u_rot():
        for j in range(r_steps):
            for i in range(64):
                ctx.batch_rotate(acc[i:i + 1], acc[i:i + 1], [1 << j], accumulate=True)

    res = {}
    for name, fb, fu in (("mulpc", b_mul, u_mul), ("rescale", b_resc, u_resc), ("rotate_and_sum", b_rot, u_rot)):
        tb, _ = timed(fb, reps, 1, torch)
        tu, _ = timed(fu, reps, 1, torch)
        res[name] = {"batched_ms": tb * 1e3, "per_ciphertext_ms": tu * 1e3, "speedup": tu / tb}
    res["rotate_and_sum"]["rotations_per_s"] = 64 * r_steps / (res["rotate_and_sum"]["batched_ms"] * 1e-3)
    # check: rotate-and-sum of a fresh copy sums all slots
    for i in (0, 1, 4):
        acc[i].copy_(cts[i])
    for j in range(r_steps):
        ctx.batch_rotate(acc[:5], acc[:5], [1 << j] * 5, accumulate=True)
    err = 0.0
    for i in (0, 1, 4):
        v = cl.decrypt(acc[i], 2.0**30, 4)
        err = max(err, float(np.abs(v - msgs[i].sum()).max()))
    res["workload"] = ("64 ciphertexts, N=16384 (6x40-bit + 60-bit P), levels 2 + (i mod 5); MulPC, rescale and "
                       "13 rotate-and-add steps, each one batched launch chain over all 64 vs per-ciphertext calls")
    res["rotate_and_sum_decrypted_max_abs_err"] = err
    return res


def convpack_ffconv(torch, ctx, cl, x, w1, w2, stride, pad, level, scale, square, reps: int, index0: int):
    """FFConv with both factors under ConvPack (CP-HI2C-CP, d = 1; Sec. 4.2.2,
    Fig. 5): the client encrypts the K = d^2 I_c columns of the plaintext
    Im2Col, W1 and W2 run as two ConvPack layers with no rotation.  Reports
    latency, executed and paper-formula counts and the decrypted error."""
    import numpy as np

    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.he import Ct

    h, w_, c_in = x.shape
    d, r, o_c = w1.shape[0], w1.shape[3], w2.shape[1]
    geom = Ly.Geometry(h, w_, c_in, d, stride, pad)
    vecs = Ly.im2col_layout(x, geom, ctx.n // 2)
    cts = torch.stack([cl.encrypt(v, level, scale, index=index0 + k).data[0] for k, v in enumerate(vecs)])
    xin = Ct(cts.contiguous(), scale)
    w1m = w1.reshape(-1, r)
    ctx.reserve(ctx.workspace_need(max(r, o_c) * 3, level) + (64 << 20))
    t, z = timed(lambda: ctx.ffconv_layer_convpack(xin, w1m, w2, scale, square=square), reps, 1, torch)
    cnt = ctx.last_counts()
    ref = Ly.reference_conv2d(x, w1, stride, pad) @ w2
    if square:
        ref = ref * ref
    err = 0.0
    for o in range(o_c):
        v = cl.decrypt(z.data[o], z.scale, geom.spatial, limbs=1)
        err = max(err, float(np.abs(v - ref[:, :, o].ravel()).max()))
    k = len(vecs)
    return {"layer_ms": t * 1e3, "input_ciphertexts": k, "counts": cnt,
            "paper_counts": {"mulpc": r * (k + o_c), "addcc": r * (k - 1) + o_c * (r - 1), "rot": 0,
                             "source": "Table II (FFConv, both factors ConvPack; AddCC derived form) + Table III "
                                       "CP-HI2C-CP d = 1 (0, 0, 0)"},
            "decrypted_max_abs_err": err}


def rank_sweep(torch, ctx, cl, shape, stride, pad, level, scale, ranks, wl, reps: int):
    """Eq. 2 / Table X: a synthetic W (d x d x I_c x O_c) whose K x O_c matrix
    has singular values 0.3 * 0.7^i is factorised at each rank r (truncated
    SVD, factorize.py) and evaluated as an FFConv layer (W1 under DensePack,
    gather, W2 under ConvPack, rescale; no x^2).  Per rank: layer latency,
    executed rotations, the relative Frobenius error of W1 W2, the max
    decrypted error against the FP64 rank-r conv (HE error) and against the
    FP64 conv with W (factorisation + HE error)."""
    import numpy as np

    import synth
    from paper_2102_03494_amd import factorize as F
    from paper_2102_03494_amd import layers as Ly

    h, w_, c_in, d, o_c = shape[0], shape[1], shape[2], shape[3], shape[4]
    geom = Ly.Geometry(h, w_, c_in, d, stride, pad)
    k = d * d * c_in
    m = min(k, o_c)
    sigma = 0.3 * 0.7 ** np.arange(m)
    rng = synth.rng(wl, "weight", 900)
    w = F.with_spectrum(rng.normal(size=(k, m)), rng.normal(size=(o_c, m)), sigma, (d, d, c_in, o_c))
    x = synth.image(wl, (h, w_, c_in))
    ct = cl.encrypt(Ly.densepack_layout(x, geom, ctx.n // 2)[0], level, scale, index=0)
    ref_full = Ly.reference_conv2d(x, w, stride, pad)
    r_steps = int(math.log2(ctx.n // 2))
    rows = []
    for r in ranks:
        w1, w2 = F.factorize(w, r)
        desc = ctx.conv_desc(h, w_, c_in, d, stride, pad, r, r_steps)
        pts = Ly.pt_scale_for(ctx, level, scale, scale)
        f1 = Ly.encode_filters(cl, w1, geom, level, pts)
        ms = Ly.mask_scale_for(ctx, level - 1, scale * pts / ctx.q[level - 1], scale, w2_bits(ctx))
        mask = Ly.onehot_mask(cl, level - 1, ms)
        ctx.reserve(ctx.ffconv_workspace_need(1, level, desc, o_c, False))
        t, z = timed(lambda: ctx.ffconv_layer(ct, desc, f1, pts, mask, ms, w2, w2_bits(ctx), False), reps, 1, torch)
        rot = ctx.last_counts()["rot"]
        ref_r = Ly.reference_conv2d(x, w1, stride, pad) @ w2
        e_he = e_full = 0.0
        for o in range(o_c):
            v = cl.decrypt(z.data[o], z.scale, geom.spatial, limbs=1)
            e_he = max(e_he, float(np.abs(v - ref_r[:, :, o].ravel()).max()))
            e_full = max(e_full, float(np.abs(v - ref_full[:, :, o].ravel()).max()))
        rows.append({"rank": r, "layer_ms": t * 1e3, "rotations": rot, "w_rel_frobenius_error": F.relative_error(w, w1, w2),
                     "decrypted_max_abs_err_vs_rank_r_fp64": e_he, "decrypted_max_abs_err_vs_full_w_fp64": e_full})
        del z, f1
    return {"workload": f"{h}x{w_}x{c_in} input, {d}x{d} stride {stride} pad {pad} conv {c_in}->{o_c}, synthetic W "
                        f"with singular values 0.3*0.7^i, N={ctx.n}; FFConv at each rank (no x^2)",
            "ranks": rows}


def cifar_section(torch, steps: int, plain: bool, digests_path: str):
    """The CIFAR-shaped layer: a 32x32x3 image (U[0,1)) under DensePack in one
    ciphertext at N = 16384 (6 x 40-bit primes + 60-bit P, scale 2^30).
      * FFConv: 3x3 pad 1 conv 3 -> r = 8 under DensePack (8192 dot products,
        13 rotate-and-add steps each: 106,496 rotations), the DP->CP gather and
        a 1x1 conv 8 -> 64 under ConvPack (16-bit integer weights, w2_bits), rescale;
      * plain comparator: the 3x3 pad 1 conv 3 -> 64 with W = W1 W2 under
        DensePack (65,536 dot products: 851,968 rotations), rescale.
    Weights N(0, 0.05^2).  Reports latency, rotations/s, HMA/s, decrypted max
    error against FP64, the ModUp stage's ALU roofline, and a bit-for-bit
    check of 72 W1 outputs (every channel x border class) against digests the
    oracle wrote offline for the same seeded inputs."""
    import hashlib

    import numpy as np

    import synth
    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import HEContext

    wl = "cifar_n16384"
    n, level, scale = 16384, 6, 2.0**30
    ctx = HEContext(n, (40,) * level, 60)
    cl = Client(ctx, wl)
    r_steps = int(math.log2(n // 2))
    cl.gen_rotation_keys([1 << j for j in range(r_steps)])
    geom = Ly.Geometry(32, 32, 3, 3, 1, 1)
    x = synth.image(wl, (32, 32, 3))
    w1 = synth.weights(wl, 1, (3, 3, 3, 8), 0.05)
    w2 = synth.weights(wl, 2, (8, 64), 0.05)
    ct = cl.encrypt(Ly.densepack_layout(x, geom, n // 2)[0], level, scale, index=0)
    desc = ctx.conv_desc(32, 32, 3, 3, 1, 1, 8, r_steps)
    pts = Ly.pt_scale_for(ctx, level, scale, scale)
    f1 = Ly.encode_filters(cl, w1, geom, level, pts)
    y_scale = scale * pts / ctx.q[level - 1]
    kb = w2_bits(ctx)
    ms = Ly.mask_scale_for(ctx, level - 1, y_scale, scale, kb)
    mask = Ly.onehot_mask(cl, level - 1, ms)
    ctx.reserve(ctx.ffconv_workspace_need(1, level, desc, 64, False))
    out = torch.empty((64, 2, level - 2, n), dtype=torch.int64, device="cuda")

    def ffconv():
        return ctx.ffconv_layer(ct, desc, f1, pts, mask, ms, w2, kb, False, out=out)

    ffconv()
    torch.cuda.synchronize()
    ctx.prof_select(DOMINANT)
    t0 = time.perf_counter()
    for _ in range(steps):
        z = ffconv()
    torch.cuda.synchronize()
    t_ff = (time.perf_counter() - t0) / steps
    dom_ms, dom_busy_ms, dom_launches = ctx.prof_read_busy()
    ctx.prof_select(None)
    counts_ff = ctx.last_counts()
    print(f"# cifar ffconv: {t_ff * 1e3:.1f} ms/layer", file=sys.stderr, flush=True)
    ref = Ly.reference_conv2d(x, w1, 1, 1) @ w2
    err_ff = 0.0
    for o in range(64):
        v = cl.decrypt(z.data[o], z.scale, geom.spatial, limbs=1)
        err_ff = max(err_ff, float(np.abs(v - ref[:, :, o].ravel()).max()))
    pg = ctx.get_tuning("p_groups", level)
    n_dp = 8 * geom.spatial
    ops = r_steps * modup_ip_ops(n_dp, level, n, ctx.moduli, pg, ctx.get_tuning("modup_halves", level) == 1)
    roof = {"kernel": "k_ks_modup_half<14, f64, wide>: ModUp NTTs + key inner product into the six 40-bit primes "
                      "(f64 class) and P (wide), two half-ring workgroups per target, one launch per rotate-and-add "
                      "step of the 8192 W1 outputs (split into concurrent chains when split_streams)",
            "bound": "alu", "achieved": ops * steps / (dom_busy_ms * 1e-3) / 1e12 if dom_busy_ms else None,
            "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s (VALU lane ops)",
            "avg_launch_ms": dom_ms / max(1, dom_launches), "launches": dom_launches, "busy_ms": dom_busy_ms,
            "algorithmic_ops_per_layer": ops, "p_groups": pg}
    if roof["achieved"] is not None:
        roof["frac"] = roof["achieved"] / roof["peak"]
    # 72 W1 dot products bit for bit against the oracle's digests
    bit = None
    if os.path.exists(digests_path):
        with open(digests_path) as f:
            gold = json.load(f).get(wl)
        if gold:
            y = ctx.conv_densepack(ct, desc, f1, pts)
            torch.cuda.synchronize()
            got = [hashlib.sha256(np.ascontiguousarray(y.data[i].cpu().numpy().view(np.uint64), dtype="<u8")
                                  .tobytes()).hexdigest() for i in gold["w1_sample"]]
            bit = {"sampled_w1_outputs": len(got),
                   "identical": sum(g == w for g, w in zip(got, gold["w1_sample_sha256"]))}
            del y
    print("# cifar ConvPack-ConvPack FFConv", file=sys.stderr, flush=True)
    cpcp = convpack_ffconv(torch, ctx, cl, x, w1, w2, 1, 1, level, scale, False, max(1, steps), 500)
    cpcp["speedup_vs_dp_hi2c_cp"] = t_ff * 1e3 / cpcp["layer_ms"]
    print("# cifar rank sweep", file=sys.stderr, flush=True)
    del out, z
    torch.cuda.empty_cache()
    sweep = rank_sweep(torch, ctx, cl, (32, 32, 3, 3, 64), 1, 1, level, scale, (1, 2, 4, 8, 16), wl, 1)
    res = {
        "rank_sweep": sweep,
        "ffconv_convpack_convpack": cpcp,
        "workload": "CIFAR-shaped layer 32x32x3, N=16384 (6x40-bit + 60-bit P, scale 2^30): FFConv 3x3 pad 1 "
                    "3->8 DensePack + 1x1 8->64 ConvPack vs plain 3x3 pad 1 3->64 DensePack (W = W1 W2)",
        "ffconv_layer_ms": t_ff * 1e3, "ffconv_rotations_per_s": counts_ff["rot"] / t_ff,
        "ffconv_hma_per_s": (counts_ff["mulpc"] + counts_ff["scalar_mul"]) / t_ff,
        "counts_ffconv": counts_ff, "paper_counts_ffconv": paper_counts_dp_hi2c_cp(geom.spatial, 8, 64, r_steps),
        "ffconv_decrypted_max_abs_err": err_ff, "roofline": roof,
        "w1_bit_exact_vs_oracle": bit,
    }
    if plain:
        wp = Ly.compose_factors(w1, w2)
        pts_pl = Ly.pt_scale_for(ctx, level, scale, scale)
        fp = Ly.encode_filters(cl, wp, geom, level, pts_pl)
        descp = ctx.conv_desc(32, 32, 3, 3, 1, 1, 64, r_steps)
        # outputs (65,536 replicated ciphertexts at level 5: 80 GiB) plus a
        # workspace that runs the layer in chunks of about 8000 dot products
        yp = torch.empty((64 * geom.spatial, 2, level - 1, n), dtype=torch.int64, device="cuda")
        ctx.reserve(ctx.workspace_need(8000, level))
        print("# cifar plain comparator: 65,536 dot products", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        zp = ctx.conv_densepack(ct, descp, fp, pts_pl, out=yp)
        torch.cuda.synchronize()
        t_pl = time.perf_counter() - t0
        counts_pl = ctx.last_counts()
        refp = Ly.reference_conv2d(x, wp, 1, 1)
        err_pl = err_pl0 = 0.0
        rng = np.random.default_rng(7)
        for idx in rng.choice(yp.shape[0], 256, replace=False):
            o, rem = divmod(int(idx), geom.spatial)
            i, j = divmod(rem, geom.out_w)
            v = cl.decrypt(yp[idx], zp.scale, rem + 1, limbs=1)  # slot p, as in the N=8192 section
            err_pl = max(err_pl, abs(float(v[rem]) - refp[i, j, o]))
            err_pl0 = max(err_pl0, abs(float(v[0]) - refp[i, j, o]))
        res.update(plain_layer_ms=t_pl * 1e3, plain_rotations_per_s=counts_pl["rot"] / t_pl,
                   plain_hma_per_s=counts_pl["mulpc"] / t_pl, counts_plain=counts_pl,
                   paper_counts_plain=paper_counts_dp(geom.spatial, 64, r_steps),
                   plain_decrypted_max_abs_err_256_sampled=err_pl,
                   plain_decrypted_max_abs_err_256_sampled_slot0=err_pl0, speedup_vs_plain=t_pl / t_ff)
        print(f"# cifar plain: {t_pl * 1e3:.1f} ms/layer", file=sys.stderr, flush=True)
        del yp, zp
    del ctx, cl
    torch.cuda.empty_cache()
    return res


def packing_ablation_section(torch, reps: int) -> dict:
    """The four packings of FFConv's two factors (Table IX) at the shapes of
    WideNet's second conv (Sec. 5: 14x14x83 input, W1 6x6 stride 2 to 20
    channels, W2 1x1 20 -> 163), synthetic input and weights, one input
    ciphertext set at N = 16384 (6 x 40-bit + 60-bit P, scale 2^30):
      DP-HI2C-CP  W1 DensePack, gather (HI2C, d = 1), W2 ConvPack (ffconv_layer)
      DP-DP       W1 DensePack, one-hot arrangement into a DensePack input, W2 DensePack
      CP-HI2C-CP  homomorphic Im2Col (d = 6), W1 ConvPack, W2 ConvPack (HGrouping: nothing)
      CP-HI2C-DP  homomorphic Im2Col, W1 ConvPack, combine (I_c - 1 rotations), W2 DensePack
    Per variant: time of each part, executed counts, and the paper's
    formula counts (Tables I-III, log2 N rotations per DensePack dot
    product).  Timing and counts only; the DensePack W2 after the
    Im2Col-based W1 runs on a 9 x 14 plane (the W1 outputs keep their
    stride-2 slots), so it computes 5 x 7 positions per channel, 10 of them
    outside the 5 x 5 output."""
    import numpy as np

    import synth
    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import Ct, HEContext

    wl = "widenet_n16384"
    n, level, scale = 16384, 6, 2.0**30
    slots = n // 2
    ctx = HEContext(n, (40,) * level, 60)
    cl = Client(ctx, wl)
    g1 = Ly.Geometry(14, 14, 83, 6, 2, 0)
    r, o_c = 20, 163
    r_steps = int(math.log2(slots))
    g2p = Ly.Geometry(9, 14, r, 1, 2, 0)  # W2 DensePack over the W1 outputs' stride-2 slots
    steps = set(Ly.rot_steps(ctx)) | set(Ly.him2col_rotation_steps(g1, slots))
    steps |= {(-(c * g2p.h * g2p.w)) % slots for c in range(1, r)}
    cl.gen_rotation_keys(sorted(steps))
    x = synth.image(wl, (14, 14, 83))
    cts = torch.stack([cl.encrypt(v, level, scale, index=m).data[0] for m, v in enumerate(Ly.densepack_layout(x, g1, slots))])
    xct = Ct(cts, scale)
    w1 = synth.weights(wl, 1, (6, 6, 83, r), 0.02)
    w2 = synth.weights(wl, 2, (r, o_c), 0.05)
    w1m = w1.reshape(-1, r)
    enc = Ly.PlainEncoder(ctx)
    s_out = g1.spatial  # 25
    k_cols = 6 * 6 * 83
    lg = math.log2(n)
    out = {"workload": "WideNet conv2 shapes (14x14x83, W1 6x6 s2 -> 20, W2 1x1 -> 163), synthetic U[0,1) input "
                       "and N(0, 0.02^2) / N(0, 0.05^2) weights, N=16384 (6x40-bit + 60-bit P), scale 2^30",
           "paper_table_ix_s": {"CP-HI2C-DP": 3269.65, "CP-HI2C-CP": 2560.49, "DP-DP": 784.45, "DP-HI2C-CP": 75.27}}

    def run(parts):
        """parts: [(name, fn)]; time each part (median of reps) and collect counts."""
        res, counts = {}, {}
        for name, fn in parts:
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res[name + "_s"] = sorted(ts)[len(ts) // 2]
            counts[name] = ctx.last_counts()
        res["total_s"] = sum(v for k, v in res.items() if k.endswith("_s"))
        return res, counts

    state = {}
    # ---- DP-HI2C-CP (ours)
    desc1 = ctx.conv_desc(14, 14, 83, 6, 2, 0, r, r_steps)
    pts1 = Ly.pt_scale_for(ctx, level, scale, scale)
    f1 = Ly.encode_filters(enc, w1, g1, level, pts1)
    ms = Ly.mask_scale_for(ctx, level - 1, scale, scale, w2_bits(ctx))
    onehot = Ly.onehot_mask(enc, level - 1, ms)
    ctx.reserve(ctx.ffconv_workspace_need(1, level, desc1, o_c, False))
    res, cnt = run([("W1+HI2C+W2", lambda: ctx.ffconv_layer(xct, desc1, f1, pts1, onehot, ms, w2, w2_bits(ctx),
                                                            False))])
    out["DP-HI2C-CP"] = {"time": res, "executed": cnt,
                         "paper": {"W1 DP": {"mulpc": r * s_out, "rot": r * s_out * lg, "addcc": r * s_out * lg},
                                   "HI2C d=1": {"mulpc": r, "rot": r, "addcc": 0},
                                   "W2 CP": {"mulpc": o_c * r, "rot": 0, "addcc": o_c * (r - 1)}}}
    print(f"# ablation DP-HI2C-CP {res['total_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # ---- DP-DP
    ms_arr = float(ctx.q[level - 2])
    arr_mask = Ly.onehot_mask(enc, level - 1, ms_arr)
    g2 = Ly.Geometry(5, 5, r, 1, 1, 0)
    desc2 = ctx.conv_desc(5, 5, r, 1, 1, 0, o_c, r_steps)
    f2 = Ly.encode_filters(enc, w2.reshape(1, 1, r, o_c), g2, level - 2, float(ctx.q[level - 3]))
    ctx.reserve(ctx.workspace_need(min(o_c * s_out, 16000), level - 2) + ctx.workspace_need(r * s_out, level))

    def dp_w1():
        state["y"] = ctx.conv_densepack(xct, desc1, f1, pts1)

    def dp_arrange():
        dense = ctx.gather_onehot(Ct(state["y"].data, state["y"].scale), r * s_out, arr_mask, ms_arr)
        state["dense"] = ctx.rescale(dense)

    def dp_w2():
        state["z"] = ctx.conv_densepack(Ct(state["dense"].data, state["dense"].scale), desc2, f2,
                                        float(ctx.q[level - 3]))

    res, cnt = run([("W1", dp_w1), ("arrange", dp_arrange), ("W2", dp_w2)])
    out["DP-DP"] = {"time": res, "executed": cnt,
                    "paper": {"W1 DP": {"mulpc": r * s_out, "rot": r * s_out * lg, "addcc": r * s_out * lg},
                              "W2 DP": {"mulpc": o_c * s_out, "rot": o_c * s_out * lg, "addcc": o_c * s_out * lg}}}
    print(f"# ablation DP-DP {res['total_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    state.clear()
    del f1, f2
    torch.cuda.empty_cache()
    # ---- CP-HI2C-CP and CP-HI2C-DP share the homomorphic Im2Col and the W1 ConvPack
    descm = ctx.conv_desc(14, 14, 83, 6, 2, 0, 1, 0)
    ms_i = float(ctx.q[level - 1])
    masks = Ly.encode_him2col_masks(enc, g1, level, ms_i)
    ctx.reserve(ctx.him2col_workspace_need(1, level, descm))

    def hi2c():
        state["cols"] = ctx.him2col(cts[None], scale, descm, masks, ms_i)

    def cp_w1():
        c_ = state["cols"]
        state["y"] = ctx.conv_convpack(Ct(c_.data[0], c_.scale), w1m, scale)

    def cp_w2():
        state["z"] = ctx.conv_convpack(state["y"], w2, scale)

    res, cnt = run([("HI2C", hi2c), ("W1", cp_w1), ("W2", cp_w2)])
    paper_hi2c = {"mulpc": 14 * 14 * 83, "rot": s_out * k_cols, "addcc": s_out * k_cols}
    # per-rotation time of a batched (not hoisted) rotation of the K Im2Col
    # ciphertexts at level 6, to price Table III's HI2C count
    ctx.reserve(max(ctx.him2col_workspace_need(1, level, descm), ctx.workspace_need(k_cols, level)))
    big = Ct(state["cols"].data[0].new_zeros((k_cols, 2, level, n)), scale)
    big.data[:, :, :, :] = cts[0][None]
    ctx.rotate(big, 1, out=big.data)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.rotate(big, 1, out=big.data)
    torch.cuda.synchronize()
    t_rot = (time.perf_counter() - t0) / k_cols
    del big
    out["batched_rotation_ms_level6"] = t_rot * 1e3
    out["table_iii_hi2c_projected_s"] = paper_hi2c["rot"] * t_rot
    out["CP-HI2C-CP"] = {"time": res, "executed": cnt,
                         "paper": {"HI2C d=6": paper_hi2c,
                                   "W1 CP": {"mulpc": r * k_cols, "rot": 0, "addcc": r * (k_cols - 1)},
                                   "HGrouping d=1": {"mulpc": 0, "rot": 0, "addcc": 0},
                                   "W2 CP": {"mulpc": o_c * r, "rot": 0, "addcc": o_c * (r - 1)}}}
    print(f"# ablation CP-HI2C-CP {res['total_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    block = g2p.h * g2p.w
    desc2p = ctx.conv_desc(9, 14, r, 1, 2, 0, o_c, r_steps)
    f2p = Ly.encode_filters(enc, w2.reshape(1, 1, r, o_c), g2p, level - 2, float(ctx.q[level - 3]))
    ctx.reserve(ctx.workspace_need(min(o_c * g2p.spatial, 16000), level - 2))

    def combine():
        y = state["y"]
        state["dense"] = ctx.combine_cp_dp(Ct(y.data, y.scale), block, r)

    def dp_w2p():
        d_ = state["dense"]
        state["z"] = ctx.conv_densepack(Ct(d_.data, d_.scale), desc2p, f2p, float(ctx.q[level - 3]))

    res, cnt = run([("HI2C", hi2c), ("W1", cp_w1), ("combine", combine), ("W2", dp_w2p)])
    out["CP-HI2C-DP"] = {"time": res, "executed": cnt,
                         "paper": {"HI2C d=6": paper_hi2c,
                                   "W1 CP": {"mulpc": r * k_cols, "rot": 0, "addcc": r * (k_cols - 1)},
                                   "combine": {"mulpc": 0, "rot": r - 1, "addcc": r - 1},
                                   "W2 DP": {"mulpc": o_c * s_out, "rot": o_c * s_out * lg,
                                             "addcc": o_c * s_out * lg}}}
    print(f"# ablation CP-HI2C-DP {res['total_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    state.clear()
    ctx.close()
    order = sorted(["DP-HI2C-CP", "DP-DP", "CP-HI2C-CP", "CP-HI2C-DP"], key=lambda k: out[k]["time"]["total_s"])
    out["fastest_first"] = order
    # the same ranking with the HI2C priced at Table III's rotation count
    proj = {k: out[k]["time"]["total_s"] for k in ("DP-HI2C-CP", "DP-DP")}
    for k in ("CP-HI2C-CP", "CP-HI2C-DP"):
        proj[k] = out[k]["time"]["total_s"] - out[k]["time"]["HI2C_s"] + out["table_iii_hi2c_projected_s"]
    out["total_s_with_table_iii_hi2c"] = proj
    out["fastest_first_with_table_iii_hi2c"] = sorted(proj, key=proj.get)
    return out


TAP_KERNELS = ("ip_perm", "modup_store", "ks_digits", "intt_last", "drop_last", "tap_hma", "ks_modup_stage",
               "hma_perm", "scalar_mac", "tensor_sq")


def tap_case(torch, name, ring, shape, d, stride, pad, level, r, o_c, square, batch, reps, plain=True):
    """One tap-style layer shape: FFConv (W1 d x d -> r under tap-style
    DensePack, masked gather, 1x1 r -> o_c ConvPack, optional x^2) and the
    plain conv (W1 W2 under tap-style DensePack, optional x^2), on `batch`
    seeded inputs in one call.  Latency, executed counts, rotations/s,
    per-kernel busy time, decrypted error against FP64."""
    import numpy as np

    import synth
    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import Ct, HEContext

    n, q_bits, p_bits, scale = ring
    wl = f"tap_{name}"
    ctx = HEContext(n, q_bits, p_bits)
    cl = Client(ctx, wl)
    g = Ly.Geometry(*shape, d, stride, pad)
    slots = n // 2
    cl.gen_rotation_keys(Ly.tap_rotation_steps(g, slots))
    if square:
        cl.gen_relin_key()
    xs = [synth.image(wl, shape, index=b) for b in range(batch)]
    cts = torch.stack([torch.stack([cl.encrypt(v, level, scale, index=100 * b + m).data[0]
                                    for m, v in enumerate(Ly.densepack_layout(x, g, slots))]) for b, x in enumerate(xs)])
    w1 = synth.weights(wl, 1, (d, d, shape[2], r), 0.05)
    w2 = synth.weights(wl, 2, (r, o_c), 0.05)
    enc = Ly.PlainEncoder(ctx)
    w1_scale = Ly.pt_scale_for(ctx, level, scale, scale)
    t0 = time.perf_counter()
    f1, f1p = Ly.encode_tap_filters(enc, w1, g, level, w1_scale, with_p=True)
    t_enc = time.perf_counter() - t0
    t2 = Ly.pre_square_target(ctx, level - 2, scale) if square else scale
    ms = Ly.mask_scale_for(ctx, level - 1, scale, t2, w2_bits(ctx))
    mask = enc.encode(Ly.tap_output_mask_layout(g, slots), level - 1, ms)
    desc = ctx.conv_desc(*shape, d, stride, pad, r, 0)
    ctx.reserve(ctx.tap_workspace_need(batch, level, desc, o_c, square))
    where = Ly.tap_output_slots(g)

    def ff(lazy=False):
        return ctx.ffconv_layer_tap(cts, scale, desc, f1, w1_scale, mask, ms, w2, w2_bits(ctx), square=square,
                                    w1_p=f1p if lazy else None)

    def kernel_ms(fn):
        busy = {}
        for k in TAP_KERNELS:
            ctx.prof_select(k)
            fn()
            b_ms, _, launches = ctx.prof_read_busy()
            if launches:
                busy[k] = round(b_ms, 4)
        ctx.prof_select(None)
        return busy

    t_ff, z = timed(ff, reps, 1, torch)
    counts_ff = ctx.last_counts()
    busy = kernel_ms(ff)
    # one ModDown per W1 output instead of one per hoisted rotation
    t_lazy, zl = timed(lambda: ff(True), reps, 1, torch)
    busy_lazy = kernel_ms(lambda: ff(True))
    err = err_l = 0.0
    for b in range(batch if batch <= 2 else 2):
        ref = Ly.reference_conv2d(xs[b], w1, stride, pad) @ w2
        ref = ref * ref if square else ref
        for o in range(o_c):
            v = cl.decrypt(z.data[b, o], z.scale)
            err = max(err, float(np.abs(v[where] - ref[:, :, o].ravel()).max()))
            v = cl.decrypt(zl.data[b, o], zl.scale)
            err_l = max(err_l, float(np.abs(v[where] - ref[:, :, o].ravel()).max()))
    out = {"batch": batch, "ffconv_ms": t_ff * 1e3, "ffconv_ms_per_input": t_ff * 1e3 / batch,
           "ffconv_counts_per_input": {k: v // batch for k, v in counts_ff.items()},
           "ffconv_rotations_per_s": counts_ff["rot"] / t_ff, "ffconv_decrypted_max_abs_err": err,
           "ffconv_kernel_ms": busy, "w1_plaintexts": int(f1.shape[0] * f1.shape[1] * f1.shape[2]),
           "w1_encode_s": t_enc,
           "ffconv_moddown_per_output_ms": t_lazy * 1e3, "ffconv_moddown_per_output_ms_per_input": t_lazy * 1e3 / batch,
           "ffconv_moddown_per_output_kernel_ms": busy_lazy,
           "ffconv_moddown_per_output_decrypted_max_abs_err": err_l}
    del f1, f1p
    if plain:
        wp = Ly.compose_factors(w1, w2)
        tp = Ly.pre_square_target(ctx, level - 1, scale) if square else scale
        ps = Ly.pt_scale_for(ctx, level, scale, tp)
        t0 = time.perf_counter()
        fp = Ly.encode_tap_filters(enc, wp, g, level, ps)
        t_enc = time.perf_counter() - t0
        desc_p = ctx.conv_desc(*shape, d, stride, pad, o_c, 0)
        ctx.reserve(ctx.tap_workspace_need(batch, level, desc_p) + (batch * o_c * 4 * level * n * 8 if square else 0))

        def pl():
            y = ctx.conv_tap(cts, scale, desc_p, fp, ps)
            if not square:
                return y
            sq = ctx.square(Ct(y.data.view(-1, 2, level - 1, n), y.scale))
            return ctx.rescale(sq)

        t_pl, zp = timed(pl, reps, 1, torch)
        err_p = 0.0
        zd = zp.data.view(batch, o_c, 2, -1, n)
        for b in range(batch if batch <= 2 else 2):
            ref = Ly.reference_conv2d(xs[b], wp, stride, pad)
            ref = ref * ref if square else ref
            for o in range(o_c):
                v = cl.decrypt(zd[b, o], zp.scale)
                err_p = max(err_p, float(np.abs(v[where] - ref[:, :, o].ravel()).max()))
        out.update(plain_ms=t_pl * 1e3, plain_ms_per_input=t_pl * 1e3 / batch, plain_decrypted_max_abs_err=err_p,
                   plain_plaintexts=int(fp.shape[0] * fp.shape[1] * fp.shape[2]), plain_encode_s=t_enc)
        del fp
    print(f"# tap {name} b{batch}: ffconv {t_ff * 1e3:.2f} ms (one ModDown per output: {t_lazy * 1e3:.2f} ms)" +
          (f", plain {out['plain_ms']:.2f} ms" if plain else ""), file=sys.stderr, flush=True)
    ctx.close()
    return out


def tap_graph_section(torch, n_inputs: int = 128) -> dict:
    """Launch-bound layers: the MNIST-shaped tap-style FFConv (one ModDown per
    output, W2 from a device table, so the call copies nothing from the
    host) on n_inputs encrypted images three ways: one call per image, one
    captured call replayed per image (the next image copied into its input
    buffer first), and one batched call over all images."""
    import synth
    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import HEContext

    wl = "tap_mnist"
    ctx = HEContext(N, Q_BITS, P_BITS)
    cl = Client(ctx, wl)
    g = Ly.Geometry(28, 28, 1, 5, 2, 0)
    slots = N // 2
    level = len(Q_BITS)
    cl.gen_rotation_keys(Ly.tap_rotation_steps(g, slots))
    cl.gen_relin_key()
    imgs = [synth.image(wl, (28, 28, 1), index=b) for b in range(n_inputs)]
    cts = torch.stack([cl.encrypt(Ly.densepack_layout(x, g, slots)[0], level, SCALE, index=b).data
                       for b, x in enumerate(imgs)])  # [B][1][2][level][N]
    w1 = synth.weights(wl, 1, (5, 5, 1, 2), 0.05)
    w2 = synth.weights(wl, 2, (2, 5), 0.05)
    enc = Ly.PlainEncoder(ctx)
    w1s = Ly.pt_scale_for(ctx, level, SCALE, SCALE)
    f1, f1p = Ly.encode_tap_filters(enc, w1, g, level, w1s, with_p=True)
    t2 = Ly.pre_square_target(ctx, level - 2, SCALE)
    ms = Ly.mask_scale_for(ctx, level - 1, SCALE, t2, K_BITS)
    mask = enc.encode(Ly.tap_output_mask_layout(g, slots), level - 1, ms)
    tab = ctx.int_weight_table(w2, K_BITS, level - 1)
    desc = ctx.conv_desc(28, 28, 1, 5, 2, 0, 2, 0)
    ctx.reserve(ctx.tap_workspace_need(n_inputs, level, desc, 5, True))
    x1 = cts[0:1].clone()
    out1 = torch.empty((1, 5, 2, level - 3, N), dtype=torch.int64, device="cuda")

    def one(xs, out=None):
        return ctx.ffconv_layer_tap(xs, SCALE, desc, f1, w1s, mask, ms, w2, K_BITS, square=True, w1_p=f1p,
                                    w2_tab=tab, out=out)

    def eager_all():
        for b in range(n_inputs):
            one(cts[b:b + 1])

    graph, _ = ctx.capture(lambda: one(x1, out1))

    def graph_all():
        for b in range(n_inputs):
            x1.copy_(cts[b:b + 1])
            graph.launch()

    t_eager, _ = timed(eager_all, 2, 1, torch)
    t_graph, _ = timed(graph_all, 2, 1, torch)
    t_batch, zb = timed(lambda: one(cts), 3, 1, torch)
    x1.copy_(cts[n_inputs - 1:n_inputs])
    graph.launch()
    torch.cuda.synchronize()
    same = bool(torch.equal(out1[0], zb.data[n_inputs - 1]))
    graph.close()
    ctx.close()
    print(f"# tap graph: eager {t_eager * 1e3 / n_inputs:.3f}, graph {t_graph * 1e3 / n_inputs:.3f}, "
          f"batched {t_batch * 1e3 / n_inputs:.3f} ms per image", file=sys.stderr, flush=True)
    return {"workload": f"{n_inputs} MNIST-shaped images (28x28x1), tap-style FFConv 5x5 s2 1->2->5 + x^2 at N=8192",
            "eager_ms_per_image": t_eager * 1e3 / n_inputs, "graph_ms_per_image": t_graph * 1e3 / n_inputs,
            "batched_ms_per_image": t_batch * 1e3 / n_inputs, "graph_speedup": t_eager / t_graph,
            "batched_speedup": t_eager / t_batch, "graph_bits_equal_batched": same}


def tap_section(torch, reps: int) -> dict:
    """Tap-style DensePack (hoisted tap rotations; a variant that is not one
    of the paper's designs) on the MNIST-shaped layer of the timed workload
    and on the two conv stages of the CIFAR-shaped serving net."""
    ring8 = (N, Q_BITS, P_BITS, SCALE)
    ring16 = (16384, (40,) * 6, 60, 2.0**30)
    out = {"note": "tap-style DensePack: per input ciphertext one hoisted rotation per nonzero tap shift, masked "
                   "weight plaintexts per (output, ciphertext, tap), a block sum of ceil-log rotations per output; "
                   "outputs at slot (s i) W + s j"}
    out["mnist_28x28x1_d5s2_b1"] = tap_case(torch, "mnist", ring8, (28, 28, 1), 5, 2, 0, len(Q_BITS), 2, 5, True, 1,
                                            reps)
    out["mnist_28x28x1_d5s2_b32"] = tap_case(torch, "mnist", ring8, (28, 28, 1), 5, 2, 0, len(Q_BITS), 2, 5, True,
                                             32, reps)
    out["cifar_stage1_32x32x3_r8_o64"] = tap_case(torch, "cifar1", ring16, (32, 32, 3), 3, 1, 1, 6, 8, 64, False, 1,
                                                  reps)
    out["cifar_stage2_32x32x64_r8_o64_level3"] = tap_case(torch, "cifar2", ring16, (32, 32, 64), 3, 1, 1, 3, 8, 64,
                                                          False, 1, reps)
    torch.cuda.empty_cache()
    out["launch_bound_graph_vs_batch"] = tap_graph_section(torch)
    return out


def serving_section(window: float, cap: float, mix_cap: float):
    """Serving (Poisson arrivals at 200 requests/s, 70% MNIST-shaped):
    * the 70/30 mix of MNIST- and CIFAR-shaped requests served by FFConv nets
      with continuous (iteration-level) batching: per class p50/p99 latency,
      completed requests per second and backlog (the CIFAR-shaped load is far
      beyond one GPU, so the run is capped and the backlog reported);
    * the same mix served by tap-style FFConv nets (hoisted tap rotations)
      in whole-request batches;
    * the MNIST-shaped share alone, served by FFConv nets and by the plain
      comparator nets in whole-request batches (sequential plain-conv
      evaluation), for reference."""
    from paper_2102_03494_amd import serve
    out = {}
    args = serve.parse_args(["--window", str(window), "--cap", str(mix_cap), "--classes", "mnist,cifar",
                             "--variant", "ffconv", "--mode", "continuous"])
    rep = serve.run(args)
    out["continuous_mix"] = {
        "classes": rep["classes"], "makespan_s": rep["makespan_s"], "completed_per_s": rep["completed_per_s"],
        "peak_backlog": rep["peak_backlog"], "backlog_at_end": rep["backlog_at_end"],
        "decrypted_max_abs_err": rep["decrypted_max_abs_err"],
        "workload": f"{window:g} s Poisson window at 200 requests/s, 70% MNIST-shaped (FFConv 5x5 s2 pad 1 1->2->5 "
                    "+ x^2, combine, FC 845->10 at N=8192) and 30% CIFAR-shaped (FFConv 3x3 3->8->64 + x^2, "
                    "combine, FFConv 64->8->64 at N=16384); continuous batching, drain capped at "
                    f"{mix_cap:g} s"}
    # the same mix with tap-style FFConv nets (whole-request batches, shortest class first)
    args = serve.parse_args(["--window", str(window), "--cap", str(mix_cap), "--classes", "mnist,cifar",
                             "--variant", "tap", "--mode", "queue", "--max-batch-cifar", "8"])
    rep = serve.run(args)
    out["tap_mix"] = {
        "classes": rep["classes"], "makespan_s": rep["makespan_s"], "completed_per_s": rep["completed_per_s"],
        "peak_backlog": rep["peak_backlog"], "backlog_at_end": rep["backlog_at_end"],
        "decrypted_max_abs_err": rep["decrypted_max_abs_err"], "max_batch": rep["max_batch"],
        "ms_per_request": {c: 1e3 * v for c, v in rep["cost_per_request_s"].items()},
        "workload": "the same arrivals; every FFConv stage tap-style (hoisted tap rotations, masked W1 "
                    "plaintexts), whole-request batches of up to 32 (MNIST-shaped) / 8 (CIFAR-shaped), "
                    "shortest class first"}
    for variant in ("ffconv", "plain"):
        args = serve.parse_args(["--window", str(window), "--cap", str(cap), "--classes", "mnist",
                                 "--variant", variant, "--mode", "queue"])
        rep = serve.run(args)
        c = rep["classes"]["mnist"]
        out[f"{variant}_queue_mnist"] = {k: c[k] for k in ("offered", "completed", "batches", "deferrals",
                                                           "p50_latency_s", "p99_latency_s")}
        out[f"{variant}_queue_mnist"].update(
            makespan_s=rep["makespan_s"], peak_backlog=rep["peak_backlog"], backlog_at_end=rep["backlog_at_end"],
            ms_per_request=1e3 * rep["cost_per_request_s"]["mnist"],
            decrypted_max_abs_err=rep["decrypted_max_abs_err"]["mnist"])
    out["queue_workload"] = (f"MNIST-shaped requests of the same {window:g} s window in whole-request batches of up "
                             "to 32, FFConv nets and plain-conv comparator nets (sequential evaluation)")
    return out


def cpu_baseline(x, w1, n_outputs: int):
    """The oracle's DensePack dot products (HMA + 12 rotate-and-add + rescale)
    on a sample of W1 outputs of the same workload, single process."""
    from threadpoolctl import threadpool_limits

    import synth  # noqa: F401
    from oracle import conv as C
    from oracle import params as P
    from oracle import workloads as Wk

    p = P.ffconv_n8192()
    ctx = Wk.make_context(p, WORKLOAD, rotations=C.rotate_and_sum_steps(p))
    geom = C.ConvGeom(28, 28, 1, 5, 2, 0)
    ct = Wk.encrypt_slots(ctx, C.densepack_slots(x, geom, p.slots)[0], p.max_level, p.scale, WORKLOAD, 0)
    pts = C.densepack_pt_scale(p, p.max_level, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w1, geom, p.max_level, pts)
    outs = C.output_list(geom, w1.shape[3])
    sample = [outs[i] for i in range(0, len(outs), max(1, len(outs) // n_outputs))][:n_outputs]
    with threadpool_limits(limits=1):  # BLAS/OpenMP pools held to one thread
        t0 = time.perf_counter()
        _, cnt = C.conv_densepack(p, ctx, ct, geom, bf, pts, outputs=sample)
        dt = time.perf_counter() - t0
    return {"value": cnt.rot / dt, "unit": "rotations/s", "cores": 1, "kind": "oracle",
            "cores_available": len(os.sched_getaffinity(0)),
            "sample": f"{len(sample)} of the {len(outs)} W1 DensePack dot products (HMA, 12 rotate-and-add, "
                      f"rescale) at N=8192, {dt:.1f} s single-threaded numpy"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=4)
    ap.add_argument("--spread-layers", type=int, default=20,
                    help="layers timed one by one with HIP events after the timed steps (0: none)")
    ap.add_argument("--cpu-sample", type=int, default=12, help="oracle dot products timed (0 = skip)")
    ap.add_argument("--no-hoisted", action="store_true", help="skip the N=16384 hoisted-rotation section")
    ap.add_argument("--batched-layers", type=int, default=128,
                    help="independent layers in the batched/graph section (0 = skip)")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged 64-ciphertext batch section")
    ap.add_argument("--no-tap", action="store_true", help="skip the tap-style DensePack section")
    ap.add_argument("--no-ablation", action="store_true", help="skip the packing-variant ablation (WideNet shapes)")
    ap.add_argument("--no-cifar", action="store_true", help="skip the N=16384 CIFAR-shaped layer section")
    ap.add_argument("--no-rank-sweep", action="store_true", help="skip the low-rank factorisation sweep (N=8192)")
    ap.add_argument("--no-cifar-plain", action="store_true",
                    help="skip the CIFAR-shaped plain comparator (65,536 dot products, about 80 GiB of outputs)")
    ap.add_argument("--serve-window", type=float, default=1.0,
                    help="arrival window (s) of the serving section (0 = skip)")
    ap.add_argument("--mix-cap", type=float, default=20.0,
                    help="drain cap (s) of the continuous-batching 70/30 serving mix")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU sharding is a design note, not a built path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe > 0:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "copies": 3}))
        return

    import synth
    from paper_2102_03494_amd import layers as Ly
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import HEContext

    torch.cuda.set_device(0)
    x = synth.image(WORKLOAD, (28, 28, 1))
    w1 = synth.weights(WORKLOAD, 1, (5, 5, 1, 2), 0.1)
    w2 = synth.weights(WORKLOAD, 2, (2, 5), 0.1)

    ctx = HEContext(N, Q_BITS, P_BITS)
    ctx.reserve(ctx.workspace_need(720, len(Q_BITS)) + (1 << 28))
    client = Client(ctx, WORKLOAD)
    client.gen_rotation_keys(Ly.rot_steps(ctx))
    client.gen_relin_key()
    geom, ct, ffconv_step, plain_step, w_plain = setup(ctx, client, x, w1, w2)
    print(f"# setup done: N={N}, moduli={ctx.moduli}", file=sys.stderr, flush=True)

    # ---- timed FFConv steps (dominant kernel bracketed by HIP events) ----------
    for _ in range(args.warmup):
        ffconv_step()
    torch.cuda.synchronize()
    ctx.prof_select(DOMINANT)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        z = ffconv_step()
    torch.cuda.synchronize()
    t_ff = (time.perf_counter() - t0) / args.steps
    dom_ms, dom_busy_ms, dom_launches = ctx.prof_read_busy()
    ctx.prof_select(None)
    counts_ff = ctx.last_counts()
    print(f"# ffconv: {t_ff * 1e3:.3f} ms/layer", file=sys.stderr, flush=True)
    # the DensePack MulPC kernel, bracketed by HIP events in a few more layers
    hma_steps = max(2, min(args.steps, 10))
    ctx.prof_select("dp_hma")
    for _ in range(hma_steps):
        ffconv_step()
    torch.cuda.synchronize()
    hma_ms, _hma_busy, hma_launches = ctx.prof_read_busy()
    ctx.prof_select(None)
    # spread of single layers: a HIP event pair on the library's stream (the
    # side streams join it before a call returns) around each of 20 layers
    layer_spread = None
    if args.spread_layers > 0:
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.spread_layers)]
        for a, b in ev:
            a.record()
            ffconv_step()
            b.record()
        torch.cuda.synchronize()
        lay_ms = np.array([a.elapsed_time(b) for a, b in ev])
        layer_spread = {"layers": len(lay_ms), "median_ms": float(np.median(lay_ms)),
                        "p10_ms": float(np.percentile(lay_ms, 10)), "p90_ms": float(np.percentile(lay_ms, 90)),
                        "note": "HIP events around each layer, after the timed steps"}

    # ---- plain comparator -------------------------------------------------------
    t_pl, zp, counts_pl = float("nan"), None, None
    if args.plain_steps > 0:
        t_pl, zp = timed(plain_step, args.plain_steps, 1, torch)
        counts_pl = ctx.last_counts()
        print(f"# plain: {t_pl * 1e3:.3f} ms/layer", file=sys.stderr, flush=True)

    # ---- decrypted accuracy vs FP64 ------------------------------------------------
    ref_y = Ly.reference_conv2d(x, w1, 2, 0)
    ref_ff = (ref_y @ w2) ** 2
    err_ff = 0.0
    for o in range(w2.shape[1]):
        v = client.decrypt(z.data[o], z.scale, geom.spatial, limbs=1)
        err_ff = max(err_ff, float(np.abs(v - ref_ff[:, :, o].ravel()).max()))
    # A DensePack output is replicated over the slots, but not equally
    # noisy: slot 0 decrypts with several times less noise than the others.
    # Each plain output (o, p) is read in slot p, the slot a DP->CP gather
    # takes it from (as FFConv's gather does with its own W1 outputs); the
    # slot-0 reading is reported beside it.
    ref_pl = Ly.reference_conv2d(x, w_plain, 2, 0) ** 2
    err_pl = err_pl0 = None if zp is None else 0.0
    for idx in range(0 if zp is None else zp.data.shape[0]):
        o, rem = divmod(idx, geom.spatial)
        i, j = divmod(rem, geom.out_w)
        v = client.decrypt(zp.data[idx], zp.scale, rem + 1, limbs=1)
        err_pl = max(err_pl, abs(float(v[rem]) - ref_pl[i, j, o]))
        err_pl0 = max(err_pl0, abs(float(v[0]) - ref_pl[i, j, o]))

    rot_ff = 288 * 12
    rot_pl = 720 * 12
    hma_ff = counts_ff["mulpc"] + counts_ff["scalar_mul"]
    level = len(Q_BITS)
    pg = ctx.get_tuning("p_groups", level)
    split = ctx.get_tuning("split_streams", 0)
    parts = chain_parts(288, split, ctx.get_tuning("split_parts", 0))
    # the timed region holds, per layer, 12 rotate-and-add steps of the 288 W1
    # outputs (one launch per chain and step) and the 5 relinearisations of
    # x^2 (level 2)
    hv = ctx.get_tuning("modup_halves", level) == 1
    ops_layer = 12 * modup_ip_ops(288, level, N, ctx.moduli, pg, hv) + \
        modup_ip_ops(5, 2, N, ctx.moduli[:2] + ctx.moduli[-1:], ctx.get_tuning("p_groups", 2),
                     ctx.get_tuning("modup_halves", 2) == 1)
    # the chain's accumulator is packed from its first step on (all primes
    # narrow: the MulPC kernel leaves its products packed)
    packed = all(q < (1 << 30) for q in ctx.moduli[:level])
    bytes_layer = 12 * modup_ip_bytes(288, level, N, ctx.moduli, pg, packed_in=packed) + \
        modup_ip_bytes(5, 2, N, ctx.moduli[:2] + ctx.moduli[-1:], ctx.get_tuning("p_groups", 2))
    launches_layer = 12 * parts + 1
    avg_ms = dom_ms / max(1, dom_launches)
    layers = dom_launches / launches_layer
    ops_per_launch = ops_layer / launches_layer
    # throughput while the stage runs: all its algorithmic work over the time
    # at least one of its launches was running (two overlap when split)
    achieved_ops = ops_layer * layers / (dom_busy_ms * 1e-3)
    per_launch_ops = ops_per_launch / (avg_ms * 1e-3)
    roofline = {
        "kernel": ("k_ks_modup_half<13, narrow, f64>: ModUp NTTs + key inner product into the four 30-bit primes "
                   "and P (f64), two half-ring workgroups per target" if hv else
                   "k_ks_modup_ip2<13, narrow, f64>: ModUp NTTs + key inner product into the four 30-bit primes and "
                   "P (f64), one workgroup per target") +
                  ", one launch per rotate-and-add step of each chain of W1 outputs at level 4 (the 288 outputs "
                  "split into concurrent chains on their own streams), plus one relinearisation launch per layer",
        "bound": "alu", "achieved": achieved_ops / 1e12, "peak": VALU_PEAK_OPS / 1e12,
        "unit": "Tops/s (VALU lane ops)", "frac": achieved_ops / VALU_PEAK_OPS,
        "traffic": measured_traffic("ks_modup_stage"),
        "avg_launch_ms": avg_ms, "launches": dom_launches, "busy_ms": dom_busy_ms,
        "concurrency": dom_ms / dom_busy_ms if dom_busy_ms > 0 else None,
        "algorithmic_ops_per_launch": ops_per_launch,
        "per_launch_achieved": per_launch_ops / 1e12,
        "p_groups": pg, "split_streams": split, "split_parts": parts,
        "hbm_gbs_algorithmic": bytes_layer * layers / (dom_busy_ms * 1e-3) / 1e9,
    }
    rows, cols = geom.classes()
    n_out_ff = geom.spatial * w1.shape[3]
    hma_bytes = dp_hma_bytes(n_out_ff, 1, w1.shape[3] * len(rows) * len(cols), level, N, ctx.moduli, packed)
    hma_avg_ms = hma_ms / max(1, hma_launches)
    hma_roofline = {
        "kernel": "k_dp_hma<13>: DensePack MulPC of the 288 W1 outputs (input times Galois-permuted base filter, "
                  "four 30-bit limbs), one launch per layer",
        "bound": "hbm", "achieved": hma_bytes / (hma_avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": hma_bytes / (hma_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic("dp_hma"),
        "avg_launch_ms": hma_avg_ms, "launches": hma_launches, "algorithmic_bytes_per_launch": hma_bytes,
        "hma_per_s_in_kernel": n_out_ff / (hma_avg_ms * 1e-3),
    }
    from paper_2102_03494_amd import tune as _tune
    tuning = {"source": ctx.tuning_source, **_tune.chosen(ctx)}

    batched = None
    if args.batched_layers > 0:
        print("# batched layers and graph", file=sys.stderr, flush=True)
        batched = batched_layers_section(torch, ctx, client, args.batched_layers, max(1, min(args.steps, 3)))

    print("# ConvPack-ConvPack FFConv at N=8192", file=sys.stderr, flush=True)
    cpcp = convpack_ffconv(torch, ctx, client, x, w1, w2, 2, 0, len(Q_BITS), SCALE, True, max(1, min(args.steps, 10)),
                           500)
    cpcp["speedup_vs_dp_hi2c_cp"] = t_ff * 1e3 / cpcp["layer_ms"]
    cpcp["workload"] = ("the same 28x28x1 layer with both factors under ConvPack: 25 Im2Col ciphertexts, W1 25->2, "
                        "W2 2->5, x^2 (CP-HI2C-CP, d = 1)")

    sweep = None
    if not args.no_rank_sweep:
        print("# rank sweep at N=8192", file=sys.stderr, flush=True)
        sweep = rank_sweep(torch, ctx, client, (28, 28, 1, 5, 5), 2, 0, len(Q_BITS), SCALE, (1, 2, 3, 4, 5), WORKLOAD,
                           max(1, min(args.steps, 5)))

    hoisted = None
    if not args.no_hoisted:
        del ctx, client
        torch.cuda.empty_cache()
        print("# hoisted rotations at N=16384", file=sys.stderr, flush=True)
        hoisted = hoisted_section(torch, max(1, min(args.steps, 5)))

    cifar = None
    if not args.no_cifar:
        torch.cuda.empty_cache()
        print("# CIFAR-shaped layer at N=16384", file=sys.stderr, flush=True)
        cifar = cifar_section(torch, max(1, min(args.steps, 3)), not args.no_cifar_plain,
                              os.path.join(ROOT, "tests", "golden", "fullsize_digests.json"))

    ragged = None
    if not args.no_ragged:
        torch.cuda.empty_cache()
        print("# ragged batch at N=16384", file=sys.stderr, flush=True)
        ragged = ragged_section(torch, max(1, min(args.steps, 3)))

    tap = None
    if not args.no_tap:
        torch.cuda.empty_cache()
        print("# tap-style DensePack section", file=sys.stderr, flush=True)
        tap = tap_section(torch, max(1, min(args.steps, 5)))

    ablation = None
    if not args.no_ablation:
        torch.cuda.empty_cache()
        print("# packing-variant ablation", file=sys.stderr, flush=True)
        ablation = packing_ablation_section(torch, max(1, min(args.steps, 2)))

    serving = None
    if args.serve_window > 0:
        torch.cuda.empty_cache()
        print("# serving section", file=sys.stderr, flush=True)
        serving = serving_section(args.serve_window, 30.0, args.mix_cap)

    cpu = None
    if args.cpu_sample > 0:
        print("# timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(x, w1, args.cpu_sample)

    line = {
        "metric": "encrypted conv-layer latency (ms) + rotations/s; FFConv batched vs plain",
        "value": rot_ff / t_ff,
        "unit": "rotations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_ff * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 (exact RNS residues, 30/40-bit primes)",
        "data": "synthetic (seeded U[0,1) 28x28x1 image, N(0,0.1^2) weights; no dataset)",
        "config": {"workload": "FFConv layer 28x28x1, 5x5 s2 1->2 DensePack + 1x1 2->5 ConvPack + x^2, "
                               "N=8192, 4x30-bit + 40-bit P, scale 2^25",
                   "global_batch": 1, "parallelism": "none (1 GPU)"},
        "ffconv_layer_ms": t_ff * 1e3,
        "ffconv_layer_spread": layer_spread,
        "plain_layer_ms": None if zp is None else t_pl * 1e3,
        "speedup_vs_plain": None if zp is None else t_pl / t_ff,
        "plain_rotations_per_s": None if zp is None else rot_pl / t_pl,
        "hma_per_s": hma_ff / t_ff,
        "counts_ffconv": counts_ff,
        "counts_plain_conv": counts_pl,
        "paper_counts_ffconv": paper_counts_dp_hi2c_cp(geom.spatial, w1.shape[3], w2.shape[1], 12),
        "paper_counts_plain_conv": paper_counts_dp(geom.spatial, w2.shape[1], 12),
        "decrypted_max_abs_err": {"ffconv": err_ff, "plain": err_pl, "plain_slot0": err_pl0,
                                  "note": "ffconv: all 144 output slots of each channel; plain: output (o, p) "
                                          "read in slot p of its replicated DensePack ciphertext (the slot a "
                                          "gather reads); plain_slot0: read in slot 0, which decrypts with less "
                                          "noise than the other slots"},
        "roofline": roofline,
        "hma_roofline": hma_roofline,
        "tuning": tuning,
        "batched_layers_graph": batched,
        "rank_sweep": sweep,
        "ffconv_convpack_convpack": cpcp,
        "ragged_batch": ragged,
        "serving": serving,
        "hoisted_rotations": hoisted,
        "cifar_layer": cifar,
        "tap_style_densepack": tap,
        "packing_ablation": ablation,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
