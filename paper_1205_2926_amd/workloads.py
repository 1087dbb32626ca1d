"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and states workload parameters; it
holds none of the transform's arithmetic, so the GPU library and the CPU
oracle can both be fed from it without sharing any code path.

Random numbers come from numpy's ``Generator(PCG64(seed))``.  Residues are
uniform in [0, p); polynomial coefficients are uniform in [0, 2^20); lengths
that are "log-uniform in 2^a..2^b" are n = floor(2^U), U ~ Uniform[a, b].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

#: 30-bit NTT primes p < 2^30 = beta/4 for beta = 2^32, with a primitive root each.
#: 998244353 = 119 * 2^23 + 1, 754974721 = 45 * 2^24 + 1, 167772161 = 5 * 2^25 + 1.
P30 = 998244353
G30 = 3
CRT_PRIMES = ((998244353, 3), (754974721, 11), (167772161, 3))

#: The largest prime p < 2^62 with p = 1 mod 2^24 (below beta/4 for beta = 2^64),
#: and its smallest primitive root.  Both the oracle and the library search for it
#: themselves; the constant is what the search must return.
P62 = 4611686018326724609
G62 = 3


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_residues(seed: int, shape, p: int, dtype=np.uint32) -> np.ndarray:
    """Residues uniform in [0, p) of the given integer dtype."""
    return rng(seed).integers(0, p, size=shape, dtype=dtype)


def log_uniform_lengths(gen: np.random.Generator, count: int, lo_bits: float, hi_bits: float) -> np.ndarray:
    u = gen.uniform(lo_bits, hi_bits, size=count)
    return np.floor(np.exp2(u)).astype(np.int64)


@dataclass(frozen=True)
class NttBatch:
    """A batch of equal-length transforms over one prime."""
    p: int
    g: int
    log2_len: int
    batch: int
    word_bits: int
    seed: int

    @property
    def length(self) -> int:
        return 1 << self.log2_len

    @property
    def dtype(self):
        return np.uint32 if self.word_bits == 32 else np.uint64

    def data(self) -> np.ndarray:
        return uniform_residues(self.seed, (self.batch, self.length), self.p, self.dtype)

    @property
    def butterflies(self) -> int:
        """Radix-2 butterflies per direction: batch * l * L / 2."""
        return self.batch * self.log2_len * (self.length // 2)


#: One forward NTT of 1024 residues mod 998244353 (the small parity case).
SINGLE_1K = NttBatch(p=P30, g=G30, log2_len=10, batch=1, word_bits=32, seed=1)
#: 64 forward+inverse NTTs of length 2^20 mod 998244353 on 32-bit words (the headline case).
BATCH64_1M = NttBatch(p=P30, g=G30, log2_len=20, batch=64, word_bits=32, seed=2)
#: 8 NTTs of length 2^22 over the 62-bit prime on 64-bit words.
BATCH8_4M_U64 = NttBatch(p=P62, g=G62, log2_len=22, batch=8, word_bits=64, seed=3)


def polymul_pairs(seed: int = 4, pairs: int = 4096, lo_bits: float = 8, hi_bits: float = 16,
                  coeff_bits: int = 20):
    """Pairs of polynomials with one log-uniform length n per pair (both operands
    get n coefficients), coefficients uniform in [0, 2^coeff_bits)."""
    gen = rng(seed)
    ns = log_uniform_lengths(gen, pairs, lo_bits, hi_bits)
    out = []
    for n in ns:
        a = gen.integers(0, 1 << coeff_bits, size=int(n), dtype=np.uint32)
        b = gen.integers(0, 1 << coeff_bits, size=int(n), dtype=np.uint32)
        out.append((a, b))
    return out


def poisson_requests(seed: int, count: int, rate_per_s: float, lo_bits: float = 10, hi_bits: float = 20,
                     coeff_bits: int = 20):
    """A Poisson stream of polynomial-multiply requests: (arrival_s, a, b) with
    exponential inter-arrival times of mean 1/rate and log-uniform lengths."""
    gen = rng(seed)
    gaps = gen.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = log_uniform_lengths(gen, count, lo_bits, hi_bits)
    reqs = []
    for t, n in zip(arrivals, ns):
        a = gen.integers(0, 1 << coeff_bits, size=int(n), dtype=np.uint32)
        b = gen.integers(0, 1 << coeff_bits, size=int(n), dtype=np.uint32)
        reqs.append((float(t), a, b))
    return reqs
