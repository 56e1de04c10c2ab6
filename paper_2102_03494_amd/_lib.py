"""ctypes loader for libffconv_he.so (the gfx950 HIP library).

The library is built in-tree by ``python -m paper_2102_03494_amd.build``.  Importing this module never falls
back to anything else: if the shared object is missing or does not load, an
ImportError says so.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffconv_he.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ffconv_he.h")

HE_MAX_PRIMES = 16


class HeParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("n_q", ctypes.c_int32),
        ("q_bits", ctypes.c_int32 * HE_MAX_PRIMES),
        ("p_bits", ctypes.c_int32),
    ]


class HeConvDesc(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("h", "w", "c_in", "d", "stride", "pad", "o_c", "r_steps")]


class HeRotsumGroup(ctypes.Structure):
    _fields_ = [("acc", ctypes.c_void_p), ("count", ctypes.c_int32), ("level", ctypes.c_int32),
                ("step", ctypes.c_int32)]


class HeCounts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("mulpc", "addcc", "rot", "rescale", "square", "scalar_mul")]


P = ctypes.c_void_p
I = ctypes.c_int
U64P = ctypes.POINTER(ctypes.c_uint64)
I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)
DP = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "he_params_moduli": (I, [ctypes.POINTER(HeParams), U64P]),
    "he_ctx_create": (I, [ctypes.POINTER(HeParams), ctypes.POINTER(P)]),
    "he_ctx_destroy": (I, [P]),
    "he_ctx_reserve": (I, [P, ctypes.c_size_t]),
    "he_ctx_set_workspace": (I, [P, P, ctypes.c_size_t]),
    "he_ctx_workspace_need": (ctypes.c_size_t, [P, I, I]),
    "he_ctx_moduli": (I, [P, U64P]),
    "he_last_error": (ctypes.c_char_p, [P]),
    "he_ctx_set_tuning": (I, [P, ctypes.c_char_p, I, I]),
    "he_ctx_get_tuning": (I, [P, ctypes.c_char_p, I]),
    "he_ntt": (I, [P, P, I, I, I, P]),
    "he_intt": (I, [P, P, I, I, I, P]),
    "he_add": (I, [P, P, P, P, I, I, ctypes.c_double, ctypes.c_double, P]),
    "he_hma_plain": (I, [P, P, P, I, P, I, I, I32P, I, I, ctypes.c_double, ctypes.c_double, DP, P]),
    "he_hma_scalar": (I, [P, P, P, I, I64P, I, I, ctypes.c_double, ctypes.c_double, DP, P]),
    "he_rescale": (I, [P, P, P, I, I, P]),
    "he_keygen_switch": (I, [P, ctypes.c_int32, P, P, P, P, P]),
    "he_keys_upload": (I, [P, I32P, I, P, I, P]),
    "he_keys_free": (I, [P, I32P, I]),
    "he_has_key": (I, [P, ctypes.c_int32]),
    "he_from_signed": (I, [P, P, P, I, I, P]),
    "he_encrypt_sk": (I, [P, P, P, P, P, P, I, P]),
    "he_decrypt": (I, [P, P, P, P, I, P]),
    "he_encode_coeffs": (I, [I, DP, I, ctypes.c_double, I64P]),
    "he_decode_coeffs": (I, [I, DP, I, DP]),
    "he_rotate": (I, [P, P, P, I, I, I, P]),
    "he_rotate_hoisted": (I, [P, P, I, I32P, I, P, P]),
    "he_rotate_hoisted_batch": (I, [P, P, I, I, I32P, I, P, P]),
    "he_rotsum": (I, [P, P, I, I, I, P]),
    "he_rotate_static": (I, [P, P, P, I, I, I, P]),
    "he_rotate_static_max_batch": (I, [P, I]),
    "he_square": (I, [P, P, P, I, I, P]),
    "he_batch_rotate": (I, [P, ctypes.POINTER(P), ctypes.POINTER(P), I32P, I32P, I, I, P]),
    "he_batch_rescale": (I, [P, ctypes.POINTER(P), ctypes.POINTER(P), I32P, I, P]),
    "he_batch_mul_plain": (I, [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), I32P, I, P]),
    "he_combine_cp_dp": (I, [P, P, I, I, I, I, P, P]),
    "he_conv_densepack": (I, [P, P, I, ctypes.POINTER(HeConvDesc), P, P, P]),
    "he_conv_convpack": (I, [P, P, I, I, DP, I, ctypes.c_double, ctypes.c_double, P, DP, P]),
    "ffconv_layer": (I, [P, P, I, ctypes.POINTER(HeConvDesc), P, P, DP, I, I, I, P, P]),
    "ffconv_layer_convpack": (I, [P, P, I, I, DP, I, DP, I, ctypes.c_double, ctypes.c_double, I, P, DP, P]),
    "he_int_weight_table": (I, [P, DP, I, I, I, P, P]),
    "he_him2col_workspace_need": (ctypes.c_size_t, [P, I, I, ctypes.POINTER(HeConvDesc)]),
    "he_him2col": (I, [P, I, P, I, ctypes.POINTER(HeConvDesc), P, I, ctypes.c_double, ctypes.c_double, P, DP, P]),
    "he_tap_workspace_need": (ctypes.c_size_t, [P, I, I, ctypes.POINTER(HeConvDesc), I, I]),
    "he_conv_tap": (I, [P, I, P, I, ctypes.POINTER(HeConvDesc), P, I, P, ctypes.c_double, ctypes.c_double, P, DP,
                        P]),
    "ffconv_layer_tap": (I, [P, I, P, I, ctypes.POINTER(HeConvDesc), P, I, P, ctypes.c_double, ctypes.c_double, P,
                             ctypes.c_double, DP, P, I, I, I, P, DP, P]),
    "ffconv_layer_batch": (I, [P, I, P, ctypes.c_size_t, I, ctypes.POINTER(HeConvDesc), P, ctypes.c_size_t, P, P,
                               I, I, P, P]),
    "he_ffconv_workspace_need": (ctypes.c_size_t, [P, I, I, ctypes.POINTER(HeConvDesc), I, I]),
    "he_densepack_hma": (I, [P, I, P, ctypes.c_size_t, I, ctypes.POINTER(HeConvDesc), P, ctypes.c_size_t, P, P]),
    "he_rotsum_groups": (I, [P, ctypes.POINTER(HeRotsumGroup), I, P]),
    "ffconv_tail_batch": (I, [P, I, P, I, ctypes.POINTER(HeConvDesc), P, P, I, I, P, P]),
    "he_combine_cp_dp_batch": (I, [P, I, P, I, I, I, I, P, P]),
    "he_gather_onehot": (I, [P, I, P, I, P, I, P, P]),
    "he_conv_densepack_batch": (I, [P, I, P, ctypes.c_size_t, I, ctypes.POINTER(HeConvDesc), P, ctypes.c_size_t, P,
                                    P]),
    "he_graph_begin": (I, [P, P]),
    "he_graph_end": (I, [P, P, ctypes.POINTER(P)]),
    "he_graph_launch": (I, [P, P]),
    "he_graph_destroy": (I, [P]),
    "he_last_counts": (I, [P, ctypes.POINTER(HeCounts)]),
    "he_prof_select": (I, [P, ctypes.c_char_p]),
    "he_prof_read_busy": (I, [P, DP, DP, ctypes.POINTER(ctypes.c_int64)]),
    "he_prof_read": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
}


def header_symbols() -> list[str]:
    """Function names declared in include/ffconv_he.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)))


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first (python -m paper_2102_03494_amd.build)"
        )
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB
