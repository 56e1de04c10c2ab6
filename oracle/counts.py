"""The paper's operation-count model (test infrastructure; see package doc).

Table I (DensePack): LoLa #MulPC = O, #AddCC = #Rot = O * R; FFConv's W1 the
same with O' = O_w O_h O'_c.  The table writes R = log2 N; the printed counts
of Section 5 use R = 13, 14 and 12 at N = 16384 (see the tests), so R is a
parameter here.

Table II (ConvPack): LoLa #MulPC = O_c K, #AddCC = O_c (K - 1); FFConv with
both factors under ConvPack: #MulPC = O'_c (K + O_c) and #AddCC as printed
O'_c (K + O_c) - K - O'_c.  Adding the two ConvPack layers' own AddCC counts,
O'_c (K - 1) + O_c (O'_c - 1), gives O'_c (K + O_c) - O'_c - O_c instead; both
forms are provided and the executed counters follow the derived one.

Table III (homomorphic Im2Col between two layers, per kernel size d of the
second layer): CP-HI2C-CP d > 1: (O^1, O^2_w O^2_h K, O^2_w O^2_h K), d = 1:
(0, 0, 0); DP-HI2C-CP d > 1: same as CP-HI2C-CP d > 1, d = 1: (O^1_c, 0,
O^1_c); CP-HI2C-DP any d: (0, I^2_c - 1, I^2_c - 1), where I^2_c is the input
channel count of the second layer.  Tuples are (#MulPC, #AddCC, #Rot).
"""
from __future__ import annotations


def densepack(o: int, r_steps: int) -> dict:
    return {"mulpc": o, "addcc": o * r_steps, "rot": o * r_steps}


def convpack_lola(o_c: int, k: int) -> dict:
    return {"mulpc": o_c * k, "addcc": o_c * (k - 1), "rot": 0}


def convpack_ffconv_printed(o_c: int, o_c_low: int, k: int) -> dict:
    return {"mulpc": o_c_low * (k + o_c), "addcc": o_c_low * (k + o_c) - k - o_c_low, "rot": 0}


def convpack_ffconv_derived(o_c: int, o_c_low: int, k: int) -> dict:
    return {"mulpc": o_c_low * (k + o_c), "addcc": o_c_low * (k - 1) + o_c * (o_c_low - 1), "rot": 0}


def him2col(kind: str, d2: int, o1: int = 0, o1_c: int = 0, o2_w: int = 0, o2_h: int = 0,
            k2: int = 0, i2_c: int = 0) -> dict:
    if kind == "CP-CP":
        t = (o1, o2_w * o2_h * k2, o2_w * o2_h * k2) if d2 > 1 else (0, 0, 0)
    elif kind == "DP-CP":
        t = (o1, o2_w * o2_h * k2, o2_w * o2_h * k2) if d2 > 1 else (o1_c, 0, o1_c)
    elif kind == "CP-DP":
        t = (0, i2_c - 1, i2_c - 1)
    else:
        raise ValueError(kind)
    return {"mulpc": t[0], "addcc": t[1], "rot": t[2]}


def conv_params(d: int, c_in: int, c_out: int) -> int:
    return d * d * c_in * c_out


def ffconv_params(d: int, c_in: int, c_out: int, rank: int) -> int:
    """O'_c (K + O_c), Section 4.1."""
    return rank * (d * d * c_in + c_out)


def him2col_ciphertexts(d: int, c_in: int) -> int:
    """K = d^2 I_c ciphertexts after homomorphic Im2Col (Fig. 2b)."""
    return d * d * c_in
