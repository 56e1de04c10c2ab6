"""Host-side checks of bench.py (no GPU): the one-GPU rule and the byte and
operation models its roofline divides by."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N = 8192
# four 30-bit primes and a 40-bit P (values only need the right sizes here)
MODULI = [(1 << 30) - 35, (1 << 30) - 107, (1 << 30) - 173, (1 << 30) - 179, (1 << 40) - 87]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_modup_bytes_count_rows():
    level, n = 4, N
    row32, row64 = 4 * n, 8 * n
    # per job: 4 packed digit rows, 4 own limbs, outputs: 2 x (4 packed rows + the P limb)
    per_job = 4 * row32 + 4 * row64 + 2 * (4 * row32 + row64)
    key = 2 * level * (4 * row32 + row64)
    assert bench.modup_ip_bytes(144, level, n, MODULI, 1) == 144 * per_job + key
    # a packed input ciphertext saves half of each own limb
    saved = bench.modup_ip_bytes(144, level, n, MODULI, 1) - bench.modup_ip_bytes(144, level, n, MODULI, 1, True)
    assert saved == 144 * 4 * (row64 - row32)
    # two P groups write one more P row per polynomial
    extra = bench.modup_ip_bytes(1, level, n, MODULI, 2) - bench.modup_ip_bytes(1, level, n, MODULI, 1)
    assert extra == 2 * row64


@pytest.mark.parametrize("pg", [1, 2, 4])
def test_modup_ops_scale_with_jobs_and_grouping(pg):
    one = bench.modup_ip_ops(1, 4, N, MODULI, pg)
    assert bench.modup_ip_ops(144, 4, N, MODULI, pg) == pytest.approx(144 * one)
    if pg > 1:  # no INTT of the P limb inside the stage, one more final reduction per extra group
        groups = -(-4 // -(-4 // pg))
        base = bench.modup_ip_ops(1, 4, N, MODULI, 1)
        bfly = (N // 2) * 13
        c = bench.width_class(MODULI[-1])
        expect = base - 2 * (bfly * bench.COST["bfly"][c] + N * bench.COST["fin"][c]) \
            + (groups - 1) * 2 * N * bench.COST["fin"][c]
        assert one == pytest.approx(expect)


def test_dp_hma_bytes_count_rows():
    level, n = 4, N
    row32, row64 = 4 * n, 8 * n
    # one input ciphertext and two base filters read as 64-bit rows; 288
    # products of two polynomials written as packed narrow rows
    packed = bench.dp_hma_bytes(288, 1, 2, level, n, MODULI)
    assert packed == (2 + 2) * level * row64 + 288 * 2 * level * row32
    # unpacked products take 64-bit words
    assert bench.dp_hma_bytes(288, 1, 2, level, n, MODULI, packed_out=False) - packed == \
        288 * 2 * level * (row64 - row32)
    # a 40-bit limb is never packed
    wide = [(1 << 40) - 87] * 2 + MODULI[-1:]
    assert bench.dp_hma_bytes(1, 1, 1, 2, n, wide) == 3 * 2 * row64 + 2 * 2 * row64


def test_chain_parts_follow_the_library_split():
    # the library splits a rotate-and-sum of cn outputs into
    # min(split_parts, cn / 32) chains when split_streams is on and cn >= 64
    assert bench.chain_parts(288, 1, 2) == 2
    assert bench.chain_parts(288, 1, 4) == 4
    assert bench.chain_parts(288, 0, 4) == 1
    assert bench.chain_parts(96, 1, 4) == 3
    assert bench.chain_parts(63, 1, 4) == 1
