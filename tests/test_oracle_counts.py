"""The count model against the paper's printed numbers (tests/golden/paper_counts.json).

Rotations per dot product: the paper's Table I writes log2 N; the printed
WideNet numbers use R = 13 (LoLa conv2), 14 (FFConv W1) and 12 (FC) at the
same N = 16384, so each printed number is reproduced with its own R.
"""
import json
import os

from oracle import conv as C
from oracle import counts as K

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))


def test_widenet_densepack_rotations():
    g = GOLD["widenet_conv2"]
    geom = C.ConvGeom(g["input"][0], g["input"][1], g["input"][2], g["d"], g["stride"], 0)
    assert [geom.out_h, geom.out_w] == g["out_hw"]
    o = geom.spatial * g["o_c"]
    o_low = geom.spatial * g["rank"]
    assert o_low == g["ffconv_w1_dot_products"]
    assert K.densepack(o, 13)["rot"] == g["lola_rotations"]
    assert K.densepack(o_low, 14)["rot"] == g["ffconv_w1_rotations"]
    assert K.him2col("CP-DP", 1, i2_c=g["o_c"])["rot"] == g["combine_rotations"]
    assert K.densepack(g["fc_outputs"], 12)["rot"] == g["fc_rotations"]
    total = K.densepack(o_low, 14)["rot"] + K.him2col("CP-DP", 1, i2_c=g["o_c"])["rot"]
    assert total == g["ffconv_rotations_total"]
    assert round(100 * (1 - total / g["lola_rotations"]), 2) == g["rotation_reduction_percent"]
    params = K.conv_params(g["d"], g["input"][2], g["o_c"])
    assert params == 487044 and abs(params - g["parameters_nearly"]) < 0.03 * g["parameters_nearly"]
    assert K.ffconv_params(g["d"], g["input"][2], g["o_c"], g["rank"]) == 20 * (2988 + 163)


def test_fig2b_ciphertext_counts():
    g = GOLD["fig2b"]
    assert K.him2col_ciphertexts(2, g["c_in"]) == g["k_d2"]
    assert K.him2col_ciphertexts(1, g["c_in"]) == g["k_d1"]


def test_convpack_tables():
    # Table II with K = 2988, O_c = 163, O'_c = 20
    lola = K.convpack_lola(163, 2988)
    assert lola == {"mulpc": 163 * 2988, "addcc": 163 * 2987, "rot": 0}
    pr = K.convpack_ffconv_printed(163, 20, 2988)
    de = K.convpack_ffconv_derived(163, 20, 2988)
    assert pr["mulpc"] == de["mulpc"] == 20 * (2988 + 163)
    # the derived AddCC is the sum of the two ConvPack layers' own counts
    assert de["addcc"] == K.convpack_lola(20, 2988)["addcc"] + K.convpack_lola(163, 20)["addcc"]
    assert pr["addcc"] - de["addcc"] == 163 - 2988
    # Table III rows
    assert K.him2col("CP-CP", 1) == {"mulpc": 0, "addcc": 0, "rot": 0}
    assert K.him2col("DP-CP", 1, o1_c=20) == {"mulpc": 20, "addcc": 0, "rot": 20}
    assert K.him2col("DP-CP", 3, o1=500, o2_w=5, o2_h=5, k2=180) == {"mulpc": 500, "addcc": 4500, "rot": 4500}


def test_percentages_and_printed_tinynet():
    for before, after, pct in (GOLD["percentages"]["mnist_latency"], GOLD["percentages"]["tinynet_conv"]):
        assert abs(100 * (1 - after / before) - pct) < 0.01
    # Table VI prints 53 rotations; with 54 channels the CP->DP rule gives I_c - 1 = 53
    assert K.him2col("CP-DP", 1, i2_c=54)["rot"] == GOLD["tinynet"]["combine_rotations_printed"]
