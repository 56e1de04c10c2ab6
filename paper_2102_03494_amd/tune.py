"""Autotuner of the key-switch schedule, with an in-tree cache.

The one schedule knob of the key switch is the number of workgroups that
share the ModUp + inner product into the special prime P ("p_groups", the
limb grouping of the ModUp kernel): with P in a more expensive width class
than the ciphertext primes, one P workgroup per ciphertext would finish
long after the others.  It changes no result bit (GPU-tested), only speed.

`tune()` times one batched rotate-and-add step (the layer's hot loop) over
`batch` ciphertexts at every level for every legal value and keeps the
fastest; `apply()` loads the cached choice for a context's ring into the
library (he_ctx_set_tuning), and HEContext does that at creation.  The cache
is `tuning_cache.json` beside this file, keyed by ring dimension, prime sizes
and device name; a ring without an entry keeps the library's cost model.

Usage (on the GPU): python -m paper_2102_03494_amd.tune --n 8192 --q 30,30,30,30 --p 40 --write
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def ring_key(n: int, q_bits, p_bits: int) -> str:
    return f"n{n}_q{'-'.join(str(b) for b in q_bits)}_p{p_bits}"


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


def lookup(n: int, q_bits, p_bits: int, path: str = CACHE) -> dict | None:
    """Cached p_groups per level ({level: value}) for this ring, or None."""
    entry = load_cache(path).get(ring_key(n, q_bits, p_bits))
    if not entry:
        return None
    return {int(k): int(v) for k, v in entry["p_groups"].items()}


def apply(ctx, path: str = CACHE) -> str:
    """Sets the cached choices on ctx; returns "cache" or "cost model"."""
    choice = lookup(ctx.n, ctx.q_bits, ctx.p_bits, path)
    if not choice:
        return "cost model"
    for level, pg in choice.items():
        if 1 <= level <= ctx.L:
            ctx.set_tuning("p_groups", level, pg)
    return "cache"


def tune(ctx, batch: int = 288, reps: int = 8, levels=None) -> dict:
    """Fastest p_groups per level for one rotate-and-add step over `batch`
    ciphertexts (uniform random residues: timing does not depend on them)."""
    import numpy as np
    import torch

    from .he import Ct
    from .client import Client
    client = Client(ctx, "unit")
    client.gen_rotation_keys([1])
    levels = levels or list(range(2, ctx.L + 1))
    rng = np.random.default_rng(7)
    out = {}
    for level in levels:
        mods = np.array(ctx.q[:level], dtype=np.uint64)
        data = rng.integers(0, mods[None, None, :, None], size=(batch, 2, level, ctx.n), dtype=np.uint64)
        ct = Ct(torch.from_numpy(data.view(np.int64)).cuda(), 1.0)
        ctx.reserve(ctx.workspace_need(batch, level))
        times = {}
        for pg in range(1, min(level, 4) + 1):
            ctx.set_tuning("p_groups", level, pg)
            ctx.rotate(ct, 1, out=ct.data)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.rotate(ct, 1, out=ct.data)
            torch.cuda.synchronize()
            times[pg] = (time.perf_counter() - t0) / reps * 1e3
        best = min(times, key=times.get)
        ctx.set_tuning("p_groups", level, best)
        out[level] = {"best": best, "ms": times}
        print(f"# level {level}: " + ", ".join(f"pg={k}: {v:.3f} ms" for k, v in times.items()) + f" -> {best}",
              file=sys.stderr, flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="tune the key-switch P grouping and cache the result")
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--q", required=True, help="comma-separated prime sizes, e.g. 30,30,30,30")
    ap.add_argument("--p", type=int, required=True)
    ap.add_argument("--batch", type=int, default=288)
    ap.add_argument("--reps", type=int, default=8)
    ap.add_argument("--write", action="store_true", help="store the result in the cache")
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args(argv)
    from .he import HEContext
    q_bits = tuple(int(b) for b in args.q.split(","))
    ctx = HEContext(args.n, q_bits, args.p)
    res = tune(ctx, args.batch, args.reps)
    entry = {"p_groups": {str(k): v["best"] for k, v in res.items()},
             "ms_per_step": {str(k): {str(pg): round(t, 4) for pg, t in v["ms"].items()} for k, v in res.items()},
             "batch": args.batch, "device": _device_name()}
    print(json.dumps({ring_key(args.n, q_bits, args.p): entry}))
    if args.write:
        cache = load_cache(args.cache)
        cache[ring_key(args.n, q_bits, args.p)] = entry
        with open(args.cache, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
            f.write("\n")
    return entry


if __name__ == "__main__":
    main()
