"""Register spills of the built library's gfx950 kernels, read from the code
object metadata (each kernel's private segment size) on the host.

Every kernel on a default path must run without scratch.  The exceptions are
kernels no default path launches: the whole-limb ModUp at N >= 8192 (the
half-ring kernels are the default there; the whole-limb ones run only when
the modup_halves knob is 0), the whole-limb P-mode ModDown at N = 16384 (the
half-ring ModDown is the default there), and instances for 60-bit ciphertext
primes (width class 2), which no ring of the workloads has."""

import os
import re
import shutil
import struct
import subprocess
import tempfile

import pytest
import yaml

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2102_03494_amd", "libffconv_he.so")
LLVM = "/opt/rocm/llvm/bin"
BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"

# kernels that may use scratch (demangled name prefixes, see the module docstring)
ALLOWED = [
    re.compile(r"he::k_ks_modup_ip2?<1[34],"),
    re.compile(r"he::k_drop_last<14, 0,"),
    re.compile(r"he::k_drop_last<\d+, \d, \d, 2,"),
]


def _gfx950_objects(fatbin: bytes):
    """Code objects for gfx950 in a section of concatenated offload bundles
    (magic, entry count, then offset / size / target triple per entry)."""
    pos = 0
    while (i := fatbin.find(BUNDLE_MAGIC, pos)) >= 0:
        n = struct.unpack_from("<Q", fatbin, i + len(BUNDLE_MAGIC))[0]
        p = i + len(BUNDLE_MAGIC) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", fatbin, p)
            p += 24
            triple = fatbin[p:p + tlen].decode()
            p += tlen
            if "gfx950" in triple and size:
                yield fatbin[i + off:i + off + size]
        pos = i + len(BUNDLE_MAGIC)


def _kernel_scratch() -> dict:
    """Demangled kernel name -> private segment bytes per lane."""
    out = {}
    with tempfile.TemporaryDirectory() as td:
        fb = os.path.join(td, "fatbin")
        subprocess.run([f"{LLVM}/llvm-objcopy", "--dump-section", f".hip_fatbin={fb}", LIB,
                        os.path.join(td, "copy.so")], check=True, capture_output=True)
        with open(fb, "rb") as f:
            data = f.read()
        names = {}
        for k, co in enumerate(_gfx950_objects(data)):
            path = os.path.join(td, f"co{k}.o")
            with open(path, "wb") as f:
                f.write(co)
            notes = subprocess.run([f"{LLVM}/llvm-readelf", "--notes", path], check=True, capture_output=True,
                                   text=True).stdout
            meta = yaml.safe_load(notes[notes.index("---"):notes.rindex("...") + 3])
            for kern in meta["amdhsa.kernels"]:
                names[kern[".name"]] = kern[".private_segment_fixed_size"]
        demangled = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True,
                                   check=True).stdout.splitlines()
        for (mangled, size), dm in zip(names.items(), demangled):
            out[dm.split("(")[0].replace("void ", "")] = size
    return out


needs_tools = pytest.mark.skipif(
    not (os.path.exists(LIB) and os.path.exists(f"{LLVM}/llvm-objcopy") and os.path.exists(f"{LLVM}/llvm-readelf")
         and shutil.which("c++filt")),
    reason="needs the built library and the ROCm LLVM tools")


@needs_tools
def test_default_path_kernels_do_not_spill():
    scratch = _kernel_scratch()
    assert len(scratch) > 100
    bad = {k: v for k, v in scratch.items() if v and not any(p.search(k) for p in ALLOWED)}
    assert not bad, f"kernels with scratch on default paths: {bad}"
    # the N = 16384 half-ring ModUp (f64 ciphertext primes, 60-bit P) and the
    # DensePack MulPC at N = 16384 held hoisted addresses in scratch before
    for k in ("he::k_ks_modup_half<14, 1, 2>", "he::k_dp_hma<14, 1>", "he::k_drop_half<14, 2, 1>",
              "he::k_ks_modup_half<13, 0, 1>", "he::k_dp_hma<13, 0>"):
        assert k in scratch and scratch[k] == 0, (k, scratch.get(k))
