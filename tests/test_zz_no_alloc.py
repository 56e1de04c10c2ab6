"""The allocation-free rotation (he_rotate_static) against he_rotate.

he_rotate_static takes its key-switch temporaries from the library's fixed
per-GPU scratch array instead of the context workspace.  Called through the C
ABI, it must give the same bits as he_rotate on the same inputs, on two calls
in a row (the second smaller, at a lower level, so stale contents of the
array from the first call would show), and the first batch is larger than one
chunk of the array, so the chunk loop runs too.  The ring spans the f64 width
class (40-bit primes) and the wide class (60-bit P).  A batch that is too
large for the context workspace still works here (no workspace is reserved).
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402

W = "unit"


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _random_cts(moduli, count, level, n, index):
    rng = synth.rng(W, "test", 7000 + index)
    a = np.empty((count, 2, level, n), dtype=np.uint64)
    for t in range(level):
        a[:, :, t, :] = rng.integers(0, moduli[t], (count, 2, n), dtype=np.uint64)
    return a


def test_rotate_static_matches_rotate_twice():
    from paper_2102_03494_amd import he
    from paper_2102_03494_amd.client import Client

    n, q_bits, p_bits = 4096, (40, 40, 40), 60
    lib = he._lib.lib()
    # context without any workspace: he_rotate_static must not need one
    bare = he.HEContext(n, q_bits, p_bits)
    ref = he.HEContext(n, q_bits, p_bits, workspace_bytes=1 << 30)
    steps = (3, -5)
    for ctx in (bare, ref):
        Client(ctx, W).gen_rotation_keys(steps)
    cap0 = lib.he_rotate_static_max_batch(bare.h, 3)
    assert cap0 >= 1
    cases = [(cap0 + 7, 3, steps[0], 0), (5, 2, steps[1], 1)]  # second call smaller, lower level
    for count, level, k, idx in cases:
        x = he.to_device(_random_cts(bare.moduli, count, level, n, idx))
        out_static = torch.empty_like(x)
        out_ref = torch.empty_like(x)
        rc = lib.he_rotate_static(bare.h, _ptr(out_static), _ptr(x), count, level, k, _stream())
        assert rc == 0, lib.he_last_error(bare.h)
        ref.rotate(he.Ct(x, 1.0), k, out=out_ref)
        torch.cuda.synchronize()
        assert torch.equal(out_static, out_ref), (count, level, k)
        # the rotation is not the identity on these inputs
        assert not torch.equal(out_static, x)
    # a missing key is reported before any launch
    rc = lib.he_rotate_static(bare.h, _ptr(out_static), _ptr(x), 1, 2, 7, _stream())
    assert rc == -4
    bare.close()
    ref.close()
