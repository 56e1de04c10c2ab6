"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws random numbers: images, weights, the ternary secret,
rounded-Gaussian errors, uniform residues and serving arrivals.  It holds none
of the scheme's arithmetic (no modular products, no transforms, no encoding),
so that the oracle and the GPU library can both consume the same draws while
sharing no code of the method.

Every draw comes from numpy's PCG64 seeded by a ``SeedSequence`` whose entropy
is the paper's arXiv number and whose spawn key is ``(workload, purpose, *index)``.
A key or ciphertext can therefore be regenerated on its own (for sampled
parity checks at full size) without replaying any other stream.

Conventions fixed here (the paper is silent on them):
  * the secret is uniform over {-1, 0, 1} per coefficient;
  * errors are a continuous N(0, sigma^2) rounded to the nearest integer, with
    any draw of magnitude above 6 sigma drawn again (sigma = 3.2);
  * the uniform ``a`` part of keys and ciphertexts is drawn per modulus as an
    integer in [0, q) and is taken to be in the NTT (evaluation) domain, which
    has the same distribution as drawing it in the coefficient domain.
"""
from __future__ import annotations

import numpy as np

ROOT_ENTROPY = 2102_03494

# Stable numeric ids for each purpose (the spawn key must be integers).
PURPOSES = {
    "image": 1,
    "weight": 2,
    "secret": 3,
    "enc_a": 4,
    "enc_e": 5,
    "ksk_a": 6,
    "ksk_e": 7,
    "rot_amounts": 8,
    "arrivals": 9,
    "message": 10,
    "levels": 11,
    "test": 12,
}

# Workload ids used in spawn keys (one per evaluated configuration).
WORKLOADS = {
    "plain_n4096": 1,      # 28x28x1 plain 5x5 s2 conv, N=4096
    "ffconv_n8192": 2,     # 28x28x1 FFConv 1->2->5 + x^2, N=8192
    "cifar_n16384": 3,     # 32x32x3 layer, N=16384
    "batched_n16384": 4,   # mixed-level batch, hoisted rotations, many layers
    "serving": 5,          # request loop
    "tap_mnist": 6,        # tap-style DensePack, 28x28x1 5x5 s2 layer, N=8192
    "tap_cifar1": 7,       # tap-style DensePack, 32x32x3 3x3 layer, N=16384
    "tap_cifar2": 8,       # tap-style DensePack, 32x32x64 3x3 layer, N=16384
    "widenet_n16384": 9,   # packing-variant ablation at WideNet conv2 shapes
    "unit": 99,            # small unit-test rings
}


def _wid(workload) -> int:
    return WORKLOADS[workload] if isinstance(workload, str) else int(workload)


def rng(workload, purpose: str, *index: int) -> np.random.Generator:
    """Independent generator for (workload, purpose, *index)."""
    key = (_wid(workload), PURPOSES[purpose]) + tuple(int(i) for i in index)
    ss = np.random.SeedSequence(entropy=ROOT_ENTROPY, spawn_key=key)
    return np.random.Generator(np.random.PCG64(ss))


def image(workload, shape, index: int = 0) -> np.ndarray:
    """Pixels uniform in [0, 1), float64, laid out as [h][w][c]."""
    return rng(workload, "image", index).random(shape)


def weights(workload, name_id: int, shape, std: float) -> np.ndarray:
    """Gaussian weights N(0, std^2) (std is a standard deviation), float64."""
    return rng(workload, "weight", name_id).normal(0.0, std, size=shape)


def ternary_secret(workload, n: int, index: int = 0) -> np.ndarray:
    """Secret coefficients uniform over {-1, 0, 1}, int64, length n."""
    return rng(workload, "secret", index).integers(-1, 2, size=n).astype(np.int64)


def rounded_gaussian(workload, purpose: str, index, n: int, sigma: float = 3.2) -> np.ndarray:
    """Rounded N(0, sigma^2) with draws beyond 6 sigma redrawn; int64, length n."""
    idx = index if isinstance(index, tuple) else (index,)
    g = rng(workload, purpose, *idx)
    x = np.rint(g.normal(0.0, sigma, size=n))
    bad = np.abs(x) > 6.0 * sigma
    while bad.any():
        x[bad] = np.rint(g.normal(0.0, sigma, size=int(bad.sum())))
        bad = np.abs(x) > 6.0 * sigma
    return x.astype(np.int64)


def uniform_residues(workload, purpose: str, index, moduli, n: int) -> np.ndarray:
    """Row t holds n integers uniform in [0, moduli[t]); uint64, shape (len(moduli), n)."""
    idx = index if isinstance(index, tuple) else (index,)
    g = rng(workload, purpose, *idx)
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for t, q in enumerate(moduli):
        out[t] = g.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def message(workload, n: int, lo: float = -1.0, hi: float = 1.0, index: int = 0) -> np.ndarray:
    """Real slot values uniform in [lo, hi), float64, length n."""
    return rng(workload, "message", index).uniform(lo, hi, size=n)


def rotation_amounts(workload, count: int, n_slots: int) -> np.ndarray:
    """`count` distinct rotation amounts in [1, n_slots), sorted, int64."""
    g = rng(workload, "rot_amounts")
    return np.sort(g.choice(np.arange(1, n_slots), size=count, replace=False)).astype(np.int64)


def poisson_arrivals(workload, rate_per_s: float, window_s: float, p_first: float):
    """Arrival times (s) of a Poisson process and a Bernoulli(p_first) class flag each."""
    g = rng(workload, "arrivals")
    times = []
    t = 0.0
    while True:
        t += g.exponential(1.0 / rate_per_s)
        if t >= window_s:
            break
        times.append(t)
    times = np.asarray(times)
    first = g.random(len(times)) < p_first
    return times, first


RELIN_INDEX = 0  # key-stream index of the relinearisation key (Galois elements are odd)


def switch_key_draws(workload, key_index: int, moduli, n: int, dnum: int):
    """Draws of one switching key: a (dnum, len(moduli), n) uniform residues, e (dnum, n).

    `key_index` is the Galois element of a rotation key, or RELIN_INDEX.
    """
    a = np.stack([uniform_residues(workload, "ksk_a", (key_index, j), moduli, n) for j in range(dnum)])
    e = np.stack([rounded_gaussian(workload, "ksk_e", (key_index, j), n) for j in range(dnum)])
    return a, e


def encryption_draws(workload, index: int, moduli, n: int):
    """Draws of one secret-key encryption: a (len(moduli), n) residues, e (n,)."""
    return (uniform_residues(workload, "enc_a", (index,), moduli, n),
            rounded_gaussian(workload, "enc_e", (index,), n))
