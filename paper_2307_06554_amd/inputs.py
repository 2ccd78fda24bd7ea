"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the multiplication itself: it draws
coefficients and moduli.  Both the GPU library and the CPU oracle receive the
arrays it returns; neither is imported here.

Workloads follow the paper's parameter ranges (Sec. 2.3, Table 1: PQC n = 2^8..2^10,
FHE n = 2^10..2^14 with 32..54-bit coefficients) and the RNS batching of Sec. 2.4.
The paper names no dataset; every coefficient is uniform in [0, q) from a PCG64
stream seeded per workload.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

GOLDILOCKS = (1 << 64) - (1 << 32) + 1
KYBER_Q = 3329

# Deterministic Miller-Rabin witness set valid for every n < 3.3e24 (covers 64-bit).
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_prime(rng: np.random.Generator, bits: int, two_n: int, exclude=()) -> int:
    """A prime q with exactly `bits` bits and q = 1 (mod two_n): draw k uniformly
    with 2^(bits-1) < k*two_n + 1 < 2^bits and return the first prime hit."""
    lo = ((1 << (bits - 1)) - 1) // two_n + 1
    hi = ((1 << bits) - 2) // two_n
    while True:
        k = int(rng.integers(lo, hi + 1))
        q = k * two_n + 1
        if q.bit_length() == bits and q not in exclude and is_prime(q):
            return q


def uniform(rng: np.random.Generator, shape, q: int, dtype=np.uint32) -> np.ndarray:
    """Coefficients uniform in [0, q)."""
    if q <= (1 << 63):
        return rng.integers(0, q, size=shape, dtype=np.int64 if q <= (1 << 62) else np.uint64).astype(dtype)
    return rng.integers(0, q, size=shape, dtype=np.uint64).astype(dtype)


@dataclass
class Group:
    """`count` independent products of degree bound n over Z_q (one modulus per group)."""
    n: int
    q: int
    a: np.ndarray
    b: np.ndarray

    @property
    def count(self):
        return self.a.shape[0]


@dataclass
class Workload:
    name: str
    kind: str                      # "single" | "rns" | "grouped" | "u64"
    n: int = 0
    q: int = 0
    qs: List[int] = field(default_factory=list)
    a: np.ndarray = None
    b: np.ndarray = None
    groups: List[Group] = field(default_factory=list)

    def products(self) -> int:
        if self.kind == "grouped":
            return sum(g.count for g in self.groups)
        if self.kind == "rns":
            return self.a.shape[0] * self.a.shape[1]
        return self.a.shape[0]


WORKLOAD_NAMES = {
    0: "n256_q3329_b1024",
    1: "n1024_q30bit_b4096",
    2: "n4096_rns8x30bit_b256",
    3: "uneven_n256-8192_q30bit_2768jobs",
    4: "n65536_goldilocks_b16",
}

UNEVEN_GROUPS = ((2048, 256), (512, 1024), (128, 2048), (64, 4096), (16, 8192))


def make_workload(index: int, seed: int = None, scale: float = 1.0) -> Workload:
    """The five synthetic workloads.  `scale` < 1 shrinks batch counts (never n)
    for quick tests; seeds default to 1000 + index."""
    seed = 1000 + index if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))

    def cnt(x):
        return max(1, int(round(x * scale)))

    if index == 0:
        n, q, B = 256, KYBER_Q, cnt(1024)
        return Workload(WORKLOAD_NAMES[0], "single", n=n, q=q,
                        a=uniform(rng, (B, n), q), b=uniform(rng, (B, n), q))
    if index == 1:
        n, B = 1024, cnt(4096)
        q = ntt_prime(rng, 30, 2 * n)
        return Workload(WORKLOAD_NAMES[1], "single", n=n, q=q,
                        a=uniform(rng, (B, n), q), b=uniform(rng, (B, n), q))
    if index == 2:
        n, L, B = 4096, 8, cnt(256)
        qs = []
        for _ in range(L):
            qs.append(ntt_prime(rng, 30, 2 * n, exclude=qs))
        a = np.stack([uniform(rng, (B, n), q) for q in qs], axis=1)
        b = np.stack([uniform(rng, (B, n), q) for q in qs], axis=1)
        return Workload(WORKLOAD_NAMES[2], "rns", n=n, qs=qs, a=a, b=b)
    if index == 3:
        used = []
        for _, n in UNEVEN_GROUPS:
            used.append(ntt_prime(rng, 30, 2 * n, exclude=used))
        groups = []
        for (count, n), q in zip(UNEVEN_GROUPS, used):
            B = cnt(count)
            groups.append(Group(n, q, uniform(rng, (B, n), q), uniform(rng, (B, n), q)))
        return Workload(WORKLOAD_NAMES[3], "grouped", groups=groups)
    if index == 4:
        n, q, B = 65536, GOLDILOCKS, cnt(16)
        return Workload(WORKLOAD_NAMES[4], "u64", n=n, q=q,
                        a=uniform(rng, (B, n), q, np.uint64), b=uniform(rng, (B, n), q, np.uint64))
    raise ValueError(f"no workload {index}")
