"""Writes fullsize_digests.json: SHA-256 digests of the oracle's ciphertexts at
the evaluated sizes, for the GPU tests to compare against bit for bit.

Run offline on the CPU (it calls only ``oracle`` and ``synth``; about 10
minutes with 8 worker processes):

    python tests/golden/make_fullsize_digests.py [-j 8]

Workloads (inputs and keys from the seeded ``synth`` draws, exactly as the GPU
tests make them):

* ``ffconv_n8192``: the 28x28x1 FFConv layer (5x5 stride 2, W1 1->2 under
  DensePack, DP->CP gather, W2 2->5 under ConvPack with 12-bit integer
  weights, x^2 and rescale) at N = 8192, 4 x 30-bit + 40-bit P: digest of the
  288 W1 DensePack outputs and of the layer's 5 output ciphertexts; and the
  plain comparator (W1 W2 composed, 1->5 DensePack, x^2 with
  relinearisation, rescale): digest of its 720 outputs.
* ``cifar_n16384``: the CIFAR-shaped FFConv W1 (3x3 pad 1, 3->8 under
  DensePack) at N = 16384, 6 x 40-bit + 60-bit P: per-output digests of 72
  sampled dot products, one per (output channel, border class) pair.
* ``tap``: the tap-style FFConv layers of bench.py's section (MNIST-shaped
  at N = 8192 with x^2; the CIFAR-shaped net's two stages at N = 16384):
  digests of the W1 output and of the layer output, with the hoisted
  rotations' ModDown per rotation and deferred to one per output.

A digest is the SHA-256 of the little-endian uint64 residues of the
ciphertext array [count][2][level][N] in C order.  Each DensePack output is
independent of the others (Table I: its own MulPC and rotate-and-sum), so the
outputs are split over worker processes and concatenated in output order.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import conv as C  # noqa: E402
from oracle import params as P  # noqa: E402
from oracle import reference as R  # noqa: E402
from oracle import scheme as S  # noqa: E402
from oracle import workloads as Wk  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_digests.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


# ---- config 2 (N = 8192) ------------------------------------------------------
W8 = "ffconv_n8192"
_G = {}  # state shared with forked workers


def _setup8():
    p = P.ffconv_n8192()
    steps = C.rotate_and_sum_steps(p)
    octx = Wk.make_context(p, W8, rotations=steps, relin=True)
    geom = C.ConvGeom(28, 28, 1, 5, 2, 0)
    x = synth.image(W8, (28, 28, 1))
    w1 = synth.weights(W8, 1, (5, 5, 1, 2), 0.1)
    w2 = synth.weights(W8, 2, (2, 5), 0.1)
    level = 4
    ct = Wk.encrypt_slots(octx, C.densepack_slots(x, geom, p.slots)[0], level, p.scale, W8, 0)
    pts = C.densepack_pt_scale(p, level, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w1, geom, level, pts)
    wp = R.compose_factors(w1, w2)
    target_pl = C.pre_square_target(p, level - 1, p.scale)
    pts_pl = C.densepack_pt_scale(p, level, p.scale, target_pl)
    bfp = C.densepack_base_filters(p, wp, geom, level, pts_pl)
    _G.update(p=p, octx=octx, geom=geom, ct=ct, pts=pts, bf=bf, pts_pl=pts_pl, bfp=bfp, w2=w2, level=level)


def _w1_chunk(idx):
    g = _G
    outs = C.output_list(g["geom"], 2)
    y, _ = C.conv_densepack(g["p"], g["octx"], g["ct"], g["geom"], g["bf"], g["pts"], outputs=[outs[i] for i in idx])
    return y.c, y.scale


def _plain_chunk(idx):
    g = _G
    outs = C.output_list(g["geom"], 5)
    y, _ = C.conv_densepack(g["p"], g["octx"], g["ct"], g["geom"], g["bfp"], g["pts_pl"],
                            outputs=[outs[i] for i in idx])
    z, _ = C.square_rescale(g["p"], g["octx"], y)
    return z.c, z.scale


def _chunks(total, parts):
    bounds = np.linspace(0, total, parts + 1).astype(int)
    return [list(range(bounds[k], bounds[k + 1])) for k in range(parts) if bounds[k + 1] > bounds[k]]


def config2(pool_size: int) -> dict:
    _setup8()
    g = _G
    p = g["p"]
    with mp.get_context("fork").Pool(pool_size) as pool:
        parts = pool.map(_w1_chunk, _chunks(288, 4 * pool_size))
        y = S.Ciphertext(np.concatenate([c for c, _ in parts]), parts[0][1])
        plain = pool.map(_plain_chunk, _chunks(720, 4 * pool_size))
    zp = np.concatenate([c for c, _ in plain])
    target = C.pre_square_target(p, g["level"] - 2, p.scale)
    ms = C.gather_mask_scale(p, y.level, y.scale, target, 12)
    mask = C.encode_onehot(p, y.level, ms)
    z, _ = C.gather_convpack(p, y, g["geom"].spatial, g["w2"], 12, mask, ms)
    out, _ = C.square_rescale(p, g["octx"], z)
    return {
        "w1_densepack": {"shape": list(y.c.shape), "sha256": digest(y.c)},
        "ffconv_layer_sq": {"shape": list(out.c.shape), "scale": out.scale, "sha256": digest(out.c)},
        "plain_comparator_sq": {"shape": list(zp.shape), "scale": plain[0][1], "sha256": digest(zp)},
    }


# ---- config 3 (N = 16384) -----------------------------------------------------
W16 = "cifar_n16384"


def cifar_w1_sample() -> list[int]:
    """One W1 output per (channel, border class) of the 32x32 pad-1 3x3 layer:
    rows/columns 0 and 31 are the edge classes, an interior row/column is
    drawn from the seeded stream."""
    rng = synth.rng(W16, "test", 3)
    picks = []
    for o in range(8):
        for rc in range(3):
            for cc in range(3):
                i = 0 if rc == 0 else (31 if rc == 2 else int(rng.integers(1, 31)))
                j = 0 if cc == 0 else (31 if cc == 2 else int(rng.integers(1, 31)))
                picks.append(o * 1024 + i * 32 + j)
    return picks


def _setup16():
    p = P.cifar_n16384()
    steps = C.rotate_and_sum_steps(p)
    octx = Wk.make_context(p, W16, rotations=steps)
    geom = C.ConvGeom(32, 32, 3, 3, 1, 1)
    x = synth.image(W16, (32, 32, 3))
    w1 = synth.weights(W16, 1, (3, 3, 3, 8), 0.05)
    level = 6
    ct = Wk.encrypt_slots(octx, C.densepack_slots(x, geom, p.slots)[0], level, p.scale, W16, 0)
    pts = C.densepack_pt_scale(p, level, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w1, geom, level, pts)
    _G.update(p16=p, octx16=octx, geom16=geom, ct16=ct, pts16=pts, bf16=bf)


def _cifar_one(i):
    g = _G
    outs = C.output_list(g["geom16"], 8)
    y, _ = C.conv_densepack(g["p16"], g["octx16"], g["ct16"], g["geom16"], g["bf16"], g["pts16"], outputs=[outs[i]])
    return digest(y.c[0])


def config3(pool_size: int) -> dict:
    _setup16()
    sample = cifar_w1_sample()
    with mp.get_context("fork").Pool(pool_size) as pool:
        digests = pool.map(_cifar_one, sample, chunksize=1)
    return {"w1_sample": sample, "w1_sample_sha256": digests}


# ---- tap-style DensePack FFConv at the bench's shapes ------------------------------
# (workload, ring, image shape, d, stride, pad, level, r, o_c, square)
TAP_CASES = {
    "tap_mnist": ("ffconv_n8192", (28, 28, 1), 5, 2, 0, 4, 2, 5, True),
    "tap_cifar1": ("cifar_n16384", (32, 32, 3), 3, 1, 1, 6, 8, 64, False),
    "tap_cifar2": ("cifar_n16384", (32, 32, 64), 3, 1, 1, 3, 8, 64, False),
}


def tap_case(name: str) -> dict:
    """The tap-style FFConv of bench.py's section for one workload: input
    image synth.image(name, shape), DensePack input ciphertext m encrypted
    with draw index m, W1 = synth.weights(name, 1, (d, d, c, r), 0.05),
    W2 = synth.weights(name, 2, (r, o_c), 0.05), W1 plaintexts at
    q_{level-1} (target = input scale), mask E at the gather scale for the
    (pre-square) target, 12-bit W2 integers.  Digests of the W1 output
    (r ciphertexts after the rescale) and of the layer output."""
    ring, shape, d, stride, pad, level, r, o_c, square = TAP_CASES[name]
    p = P.ffconv_n8192() if ring == "ffconv_n8192" else P.cifar_n16384()
    geom = C.ConvGeom(*shape, d, stride, pad)
    octx = Wk.make_context(p, name, rotations=C.tap_rotation_steps(geom, p.slots), relin=square)
    x = synth.image(name, shape)
    xs = S.Ciphertext(np.stack([Wk.encrypt_slots(octx, v, level, p.scale, name, m).c
                                for m, v in enumerate(C.densepack_slots(x, geom, p.slots))]), p.scale)
    w1 = synth.weights(name, 1, (d, d, shape[2], r), 0.05)
    w2 = synth.weights(name, 2, (r, o_c), 0.05)
    w1_scale = p.q[level - 1] * p.scale / p.scale
    filt = C.tap_filters(p, w1, geom, level, w1_scale)
    y, _ = C.tap_conv(p, octx, xs, geom, filt, w1_scale)
    t2 = C.pre_square_target(p, level - 2, p.scale) if square else p.scale
    ms = C.gather_mask_scale(p, level - 1, y.scale, t2, 12)
    mask = C.encode(C.tap_output_mask_slots(geom, p.slots), p, level - 1, ms)
    z, _ = C.gather_convpack(p, y, 1, w2, 12, mask, ms)
    if square:
        z, _ = C.square_rescale(p, octx, z)
    # the same with one ModDown per W1 output (tap_conv_lazy)
    filt_p = C.tap_filters_p(p, w1, geom, w1_scale)
    yl, _ = C.tap_conv_lazy(p, octx, xs, geom, filt, filt_p, w1_scale)
    zl, _ = C.tap_ffconv(p, octx, xs, geom, filt, w1_scale, w2, 12, mask, ms, square=square, w1_filters_p=filt_p)
    return {"w1_tap": {"shape": list(y.c.shape), "scale": y.scale, "sha256": digest(y.c)},
            "ffconv_tap": {"shape": list(z.c.shape), "scale": z.scale, "sha256": digest(z.c)},
            "w1_tap_lazy": {"shape": list(yl.c.shape), "scale": yl.scale, "sha256": digest(yl.c)},
            "ffconv_tap_lazy": {"shape": list(zl.c.shape), "scale": zl.scale, "sha256": digest(zl.c)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--only", choices=["ffconv_n8192", "cifar_n16384", "tap"], default=None)
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    res["format"] = "sha256 of little-endian uint64 [count][2][level][N], C order"
    if a.only in (None, "ffconv_n8192"):
        res["ffconv_n8192"] = config2(a.j)
        print("ffconv_n8192 done", flush=True)
    if a.only in (None, "cifar_n16384"):
        res["cifar_n16384"] = config3(a.j)
        print("cifar_n16384 done", flush=True)
    if a.only in (None, "tap"):
        with mp.get_context("fork").Pool(min(a.j, len(TAP_CASES))) as pool:
            got = pool.map(tap_case, list(TAP_CASES))
        res["tap"] = dict(zip(TAP_CASES, got))
        print("tap done", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
