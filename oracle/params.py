"""Parameter sets (test infrastructure; see package doc).

A parameter set is (N, bit sizes of the ciphertext primes, bit size of the one
special prime, default scale).  The prime chain q_0 > q_1 > ... is listed in
generation order; a ciphertext at level l holds limbs q_0..q_{l-1} and a
rescale drops the last of them.  The special prime P is only used inside key
switching.

The three parameter sets of the evaluated workloads (the paper runs BFV with
N = 8192 for MNIST and N = 16384 for CIFAR-10, Section 5 "Cryptosystem
Settings"; here an RNS CKKS-style scheme is used instead):
  * plain 28x28 conv:        N = 4096,  2 x 30-bit + 36-bit P, scale 2^25
  * FFConv 28x28 layer:      N = 8192,  4 x 30-bit + 40-bit P, scale 2^25
    (three 30-bit primes cannot hold the FFConv depth of 2 plus the square
    and its rescale, so a fourth is added)
  * CIFAR-shaped layer:      N = 16384, 6 x 40-bit + 60-bit P, scale 2^30
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .nt import inv, primes_below, root_2n


@dataclass
class Params:
    n: int
    q_bits: tuple
    p_bits: int
    scale: float
    q: list = field(init=False)
    p: int = field(init=False)
    psi: dict = field(init=False)

    def __post_init__(self):
        two_n = 2 * self.n
        qs: list[int] = []
        by_size: dict[int, int] = {}
        for b in self.q_bits:
            below = by_size.get(b)
            qv = primes_below(b, 1, two_n, below=below)[0]
            by_size[b] = qv
            qs.append(qv)
        self.q = qs
        below_p = by_size.get(self.p_bits)
        self.p = primes_below(self.p_bits, 1, two_n, below=below_p)[0]
        self.psi = {m: root_2n(m, self.n) for m in self.q + [self.p]}

    @property
    def slots(self) -> int:
        return self.n // 2

    @property
    def max_level(self) -> int:
        return len(self.q)

    def moduli(self, level: int) -> list[int]:
        return self.q[:level]

    def p_inv(self, qi: int) -> int:
        return inv(self.p, qi)


def plain_n4096() -> Params:
    return Params(4096, (30, 30), 36, float(2**25))


def ffconv_n8192() -> Params:
    return Params(8192, (30, 30, 30, 30), 40, float(2**25))


def cifar_n16384() -> Params:
    return Params(16384, (40,) * 6, 60, float(2**30))


def tiny(n: int = 16, q_bits=(30, 30, 30), p_bits: int = 36, scale: float = float(2**20)) -> Params:
    return Params(n, tuple(q_bits), p_bits, scale)
