"""Exactness of the library's FP64 width class, checked on the host.

Primes from 2^30 to 2^42 run their transforms and key products as exact
integers held in doubles (paper_2102_03494_amd/csrc/modarith.h).  The
claims that make those results bit-exact -- products with the FMA split and
a rounded quotient are exact and centred within 0.54 q for inputs below
2^46, centring and canonical reduction are exact, 15 unreduced products sum
below 8.2 q, and 14 unreduced forward butterfly stages stay below 8.6 q --
are checked by tests/host/f64_exact_check.cpp against 128-bit integer
arithmetic on about 13 million cases at the extreme magnitudes.  The program
is compiled here for the host with hipcc (no GPU involved).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_f64_class_exact(tmp_path):
    exe = str(tmp_path / "f64_exact_check")
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-O2", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", os.path.join(HERE, "host", "f64_exact_check.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0 and run.stdout.startswith("OK"), run.stdout + run.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_narrow_lazy_reduction(tmp_path):
    """reduce64_lazy32 (ModUp's store of narrow inner-product rows) lands
    below 2q and congruent to its 64-bit input, against exact remainders."""
    exe = str(tmp_path / "narrow_reduce_check")
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-O2", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", os.path.join(HERE, "host", "narrow_reduce_check.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0 and run.stdout.startswith("OK"), run.stdout + run.stderr
