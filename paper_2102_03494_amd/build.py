"""Builds libffconv_he.so for gfx950 in-tree with hipcc.

The library is split into translation units that compile in parallel: the
C-ABI unit (capi.hip), the host tables (host_params.cpp) and one launch unit
per ring size (launch_n10.hip .. launch_n14.hip, each instantiating the
kernels of one log2 N).  Objects go to _build/ beside this file; with
`incremental`, a unit whose sources (and every header of csrc/) are unchanged
since its object was made is not recompiled.

Usage: python -m paper_2102_03494_amd.build [--incremental] [-j JOBS]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libffconv_he.so")
OBJ_DIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wno-unused-value",
    # packed FP32 instructions stay off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
UNITS = ["capi.hip", "host_params.cpp"] + [f"launch_n{lg}.hip" for lg in range(10, 15)]


def _headers_digest() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".h"):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + f.read())
    with open(os.path.join(os.path.dirname(HERE), "include", "ffconv_he.h"), "rb") as f:
        h.update(f.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()


def _compile(hipcc: str, unit: str, hdr: str, incremental: bool, verbose: bool) -> str:
    src = os.path.join(CSRC, unit)
    obj = os.path.join(OBJ_DIR, unit + ".o")
    stamp = obj + ".sha"
    with open(src, "rb") as f:
        key = hashlib.sha256(f.read() + hdr.encode()).hexdigest()
    if incremental and os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == key:
        return obj
    cmd = [hipcc, *HIPCC_FLAGS, "-c", src, "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stderr)
        raise RuntimeError(f"hipcc failed on {unit}")
    os.replace(obj + ".tmp", obj)
    with open(stamp, "w") as f:
        f.write(key)
    return obj


def build(verbose: bool = True, incremental: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    hdr = _headers_digest()
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(hipcc, u, hdr, incremental, verbose), UNITS))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--incremental", action="store_true", help="reuse objects whose sources are unchanged")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    build(incremental=a.incremental, jobs=a.j)
