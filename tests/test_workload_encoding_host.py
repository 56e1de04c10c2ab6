"""The library's host FP64 encoder gives exactly the oracle's integer
plaintexts for every plaintext of the full-size workloads (no GPU needed).

Two independent FP64 encoders may differ by one unit at rounding near-ties
(test_capi_host counts those on random vectors).  For the seeded workloads
that bench.py and the full-size GPU tests run, the DensePack input, every
base filter plaintext (channel x border class) and the one-hot gather mask
must encode to the same integers on both sides: then a ciphertext the GPU
client encrypts from these draws is bit-identical to the oracle's, and the
oracle's stored digests (tests/golden/fullsize_digests.json) apply to it.
"""
import numpy as np
import pytest

import synth
from oracle import conv as C
from oracle import encoding as E
from oracle import params as P
from paper_2102_03494_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _same(lib, z, n, scale):
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty(n, dtype=np.int64)
    assert lib.he_encode_coeffs(n, z.ctypes.data_as(_lib.DP), len(z), scale, out.ctypes.data_as(_lib.I64P)) == 0
    return int((out != E.encode_int(z, n, scale)).sum())


def _workload_vectors(wl, p, geom, w, level, pt_scale):
    x = synth.image(wl, (geom.h, geom.w, geom.c_in))
    yield "input", C.densepack_slots(x, geom, p.slots)[0], p.scale
    o_c = w.shape[3]
    rows, cols, _ = geom.border_classes()
    for o in range(o_c):
        for b in range(len(rows) * len(cols)):
            yield f"filter {o},{b}", C.base_filter_slots(w, geom, p.slots, o, b, 0), pt_scale


@pytest.mark.parametrize("wl", ["ffconv_n8192", "cifar_n16384"])
def test_workload_plaintexts_encode_identically(lib, wl):
    if wl == "ffconv_n8192":
        p = P.ffconv_n8192()
        geom = C.ConvGeom(28, 28, 1, 5, 2, 0)
        w1 = synth.weights(wl, 1, (5, 5, 1, 2), 0.1)
        w2 = synth.weights(wl, 2, (2, 5), 0.1)
        from oracle import reference as R
        level = 4
        sets = [(w1, C.densepack_pt_scale(p, level, p.scale, p.scale)),
                (R.compose_factors(w1, w2),
                 C.densepack_pt_scale(p, level, p.scale, C.pre_square_target(p, level - 1, p.scale)))]
        y_scale = p.scale * sets[0][1] / p.q[level - 1]
        mask_scale = C.gather_mask_scale(p, level - 1, y_scale, C.pre_square_target(p, level - 2, p.scale), 12)
    else:
        p = P.cifar_n16384()
        geom = C.ConvGeom(32, 32, 3, 3, 1, 1)
        w1 = synth.weights(wl, 1, (3, 3, 3, 8), 0.05)
        level = 6
        sets = [(w1, C.densepack_pt_scale(p, level, p.scale, p.scale))]
        y_scale = p.scale * sets[0][1] / p.q[level - 1]
        mask_scale = C.gather_mask_scale(p, level - 1, y_scale, p.scale, 12)
    bad = []
    for w, pts in sets:
        for name, z, scale in _workload_vectors(wl, p, geom, w, level, pts):
            if _same(lib, z, p.n, scale):
                bad.append(name)
    onehot = np.zeros(p.slots)
    onehot[0] = 1.0
    if _same(lib, onehot, p.n, mask_scale):
        bad.append("mask")
    assert not bad, bad
