"""CPU oracle for the homomorphic convolution hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, exact implementation of what the GPU library
computes: RNS CKKS-style ring arithmetic (negacyclic NTT, automorphisms,
hybrid key switching with one special prime, rescale), the DensePack and
ConvPack convolution layers of the paper (Section 3.2, Tables I-III) and the
FFConv factorized layer (Section 4, Eq. 2), plus an FP64 reference convolution
(Eq. 1) and the paper's operation-count model.

Only the test suite, the package's smoke check and the CPU-baseline leg of the
benchmark may import it.  The GPU library never imports, links or calls
anything here, and this package imports nothing from the GPU library; the two
only share the seeded draws of the ``synth`` module.

Modular arithmetic is exact: residues are numpy uint64, products of residues
below 2^32 are formed directly, wider moduli go through an extended-precision
quotient estimate with an exact integer correction, and CRT / big-integer steps
use Python ints.

Parity status: every function is pinned by the CPU tests against closed forms,
brute force on tiny rings, or the FP64 convolution, except the exact bit
patterns of ciphertexts, which the paper does not fix; those are pinned only by
the oracle's own two-route cross checks (coefficient- vs NTT-domain
automorphism, hoisted vs one-at-a-time rotation): "parity unpinned" for the
ciphertext bits themselves.
"""
