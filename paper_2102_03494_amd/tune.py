"""Autotuner of the key-switch schedule and the layer schedule, with an
in-tree cache.

Knobs (none changes a result bit; all are GPU-tested for that):
* per key-switch level, the ModUp workgroup shape ("modup_halves": one
  workgroup of N/8 or N/16 threads per target prime, or two half-ring
  workgroups of N/16 threads with the transform's first stage fused into the
  lift) and the number of workgroups sharing the P target ("p_groups", the
  limb grouping: with P in a costlier width class, one P workgroup per
  ciphertext would finish long after the others);
* per ring, whether a DensePack layer runs its rotate-and-sum as several
  chains on as many streams ("split_streams"), and into how many (2 to 4,
  "split_parts").

`tune()` times one batched rotate-and-add step over `batch` ciphertexts at
every level for every (modup_halves, p_groups) pair, then a DensePack layer
of `layer_outputs` dot products unsplit and split into 2, 3 and 4 chains,
and keeps the fastest.  `apply()` loads the cached choice for a context's ring into the
library (he_ctx_set_tuning); HEContext does that at creation.  The cache is
`tuning_cache.json` beside this file, keyed by ring dimension and prime
sizes; every entry records the hash of the kernel sources it was measured
on, and an entry whose hash differs from the current sources is ignored
(the context keeps the library's defaults and reports "stale cache").

Usage (on the GPU): python -m paper_2102_03494_amd.tune --n 8192 --q 30,30,30,30 --p 40 --out FILE
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")


def ring_key(n: int, q_bits, p_bits: int) -> str:
    return f"n{n}_q{'-'.join(str(b) for b in q_bits)}_p{p_bits}"


def kernel_sha256() -> str:
    """Hash of the library's sources (csrc/ and the C header): a cache entry
    is valid only for the kernels it was measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    with open(os.path.join(os.path.dirname(HERE), "include", "ffconv_he.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def _device_name() -> str:
    import torch
    if not torch.cuda.is_available():
        return "none"
    props = torch.cuda.get_device_properties(0)
    return f"{torch.cuda.get_device_name(0)} ({getattr(props, 'gcnArchName', '?')})"


def load_cache(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(n: int, q_bits, p_bits: int, path: str = CACHE, sha: str | None = None):
    """(entry, status) for this ring: status "cache" with the entry, or
    "stale cache" / "no entry" with None."""
    entry = load_cache(path).get(ring_key(n, q_bits, p_bits))
    if not entry:
        return None, "no entry"
    if entry.get("kernel_sha256") != (sha or kernel_sha256()):
        return None, "stale cache"
    return entry, "cache"


def apply(ctx, path: str = CACHE) -> str:
    """Sets the cached choices on ctx; returns "cache", "stale cache" or
    "cost model" (no entry)."""
    entry, status = lookup(ctx.n, ctx.q_bits, ctx.p_bits, path)
    if entry is None:
        return "cost model" if status == "no entry" else status
    for level, pg in entry["p_groups"].items():
        if 1 <= int(level) <= ctx.L:
            ctx.set_tuning("p_groups", int(level), int(pg))
    for level, hv in entry.get("modup_halves", {}).items():
        if 1 <= int(level) <= ctx.L:
            ctx.set_tuning("modup_halves", int(level), int(hv))
    if "split_streams" in entry:
        ctx.set_tuning("split_streams", 0, int(entry["split_streams"]))
    if "split_parts" in entry:
        ctx.set_tuning("split_parts", 0, int(entry["split_parts"]))
    return "cache"


def chosen(ctx) -> dict:
    """The knob values in effect on ctx, per level."""
    return {"p_groups": {lv: ctx.get_tuning("p_groups", lv) for lv in range(1, ctx.L + 1)},
            "modup_halves": {lv: ctx.get_tuning("modup_halves", lv) for lv in range(1, ctx.L + 1)},
            "split_streams": ctx.get_tuning("split_streams", 0),
            "split_parts": ctx.get_tuning("split_parts", 0)}


def _time(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def tune(ctx, batch: int = 288, reps: int = 8, levels=None, layer_outputs: int = 288) -> dict:
    """Fastest (modup_halves, p_groups) per level for one rotate-and-add step
    over `batch` ciphertexts, then (split_streams, split_parts) for a
    DensePack layer of `layer_outputs` dot products (uniform random residues:
    timing does not depend on them)."""
    import math

    import numpy as np
    import torch

    from .client import Client
    from .he import Ct
    r_steps = int(math.log2(ctx.n // 2))
    client = Client(ctx, "unit")
    client.gen_rotation_keys([1 << j for j in range(r_steps)])
    levels = levels or list(range(2, ctx.L + 1))
    rng = np.random.default_rng(7)
    halves_opts = (0, 1) if ctx.n >= 2048 else (0,)
    out = {"levels": {}}
    for level in levels:
        mods = np.array(ctx.q[:level], dtype=np.uint64)
        data = rng.integers(0, mods[None, None, :, None], size=(batch, 2, level, ctx.n), dtype=np.uint64)
        ct = Ct(torch.from_numpy(data.view(np.int64)).cuda(), 1.0)
        ctx.reserve(ctx.workspace_need(batch, level))
        times = {}
        for hv in halves_opts:
            ctx.set_tuning("modup_halves", level, hv)
            for pg in range(1, min(level, 4) + 1):
                ctx.set_tuning("p_groups", level, pg)
                times[(hv, pg)] = _time(lambda: ctx.rotate(ct, 1, out=ct.data), reps, torch)
        best = min(times, key=times.get)
        ctx.set_tuning("modup_halves", level, best[0])
        ctx.set_tuning("p_groups", level, best[1])
        out["levels"][level] = {"modup_halves": best[0], "p_groups": best[1],
                                "ms": {f"h{k[0]}_pg{k[1]}": v for k, v in times.items()}}
        print(f"# level {level}: " + ", ".join(f"h{k[0]} pg{k[1]}: {v:.3f} ms" for k, v in times.items())
              + f" -> {best}", file=sys.stderr, flush=True)
        del ct
    # split_streams on a DensePack layer at the top level: a 1-channel image
    # with one output per slot-sized window (layer_outputs dot products)
    level = ctx.L
    side = int(math.isqrt(min(layer_outputs, ctx.n // 2)))
    desc = ctx.conv_desc(side, side, 1, 1, 1, 0, max(1, layer_outputs // (side * side)), r_steps)
    x = Ct(torch.from_numpy(rng.integers(0, np.array(ctx.q[:level], dtype=np.uint64)[None, :, None],
                                         size=(2, level, ctx.n), dtype=np.uint64).view(np.int64)).cuda()[None], 1.0)
    filt = torch.zeros((desc.o_c, 1, 1, level, ctx.n), dtype=torch.int64, device="cuda")
    total = side * side * desc.o_c
    ctx.reserve(ctx.workspace_need(total, level))
    split_t = {}
    for sp, parts in ((0, 2), (1, 2), (1, 3), (1, 4)):
        ctx.set_tuning("split_streams", 0, sp)
        ctx.set_tuning("split_parts", 0, parts)
        split_t[(sp, parts)] = _time(lambda: ctx.conv_densepack(x, desc, filt, 1.0), max(2, reps // 2), torch)
    best = min(split_t, key=split_t.get)
    ctx.set_tuning("split_streams", 0, best[0])
    ctx.set_tuning("split_parts", 0, best[1])
    out["split_streams"] = {"best": best[0], "parts": best[1], "outputs": total,
                            "ms": {("1" if sp == 0 else str(parts)): t for (sp, parts), t in split_t.items()}}
    print(f"# split (chains: ms): {out['split_streams']['ms']} -> {best}", file=sys.stderr, flush=True)
    return out


def entry_of(res: dict, batch: int) -> dict:
    lv = res["levels"]
    return {"p_groups": {str(k): v["p_groups"] for k, v in lv.items()},
            "modup_halves": {str(k): v["modup_halves"] for k, v in lv.items()},
            "split_streams": res["split_streams"]["best"],
            "split_parts": res["split_streams"]["parts"],
            "ms_per_step": {str(k): {kk: round(t, 4) for kk, t in v["ms"].items()} for k, v in lv.items()},
            "split_ms_per_layer": {k: round(t, 4) for k, t in res["split_streams"]["ms"].items()},
            "batch": batch, "device": _device_name(), "kernel_sha256": kernel_sha256()}


def main(argv=None):
    ap = argparse.ArgumentParser(description="tune the key-switch and layer schedule and cache the result")
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--q", required=True, help="comma-separated prime sizes, e.g. 30,30,30,30")
    ap.add_argument("--p", type=int, required=True)
    ap.add_argument("--batch", type=int, default=288)
    ap.add_argument("--reps", type=int, default=8)
    ap.add_argument("--layer-outputs", type=int, default=288)
    ap.add_argument("--write", action="store_true", help="store the result in the cache")
    ap.add_argument("--out", default=None, help="also write the entry (JSON) to this file")
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args(argv)
    from .he import HEContext
    q_bits = tuple(int(b) for b in args.q.split(","))
    ctx = HEContext(args.n, q_bits, args.p, tuned=False)
    res = tune(ctx, args.batch, args.reps, layer_outputs=args.layer_outputs)
    entry = entry_of(res, args.batch)
    line = json.dumps({ring_key(args.n, q_bits, args.p): entry})
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    if args.write:
        cache = load_cache(args.cache)
        cache[ring_key(args.n, q_bits, args.p)] = entry
        with open(args.cache, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
            f.write("\n")
    return entry


if __name__ == "__main__":
    main()
