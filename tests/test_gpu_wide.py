"""GPU parity for 64-bit moduli (up to 8 int8 limbs) and for degrees beyond the
LDS-resident path (K-streaming kernel, int32 sums folded into residues)."""
import numpy as np
import pytest

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu

GOLD = inputs.GOLDILOCKS
Q64 = [GOLD, (1 << 64) - 59, (1 << 63) + 1, (1 << 62) - 57, (1 << 40) - 87, (1 << 32) + 15, 3329, 17,
       (1 << 64) - 2]


def _rand64(rng, shape, q):
    return rng.integers(0, q, size=shape, dtype=np.uint64)


def _check64(a, b, q):
    want = oracle.negacyclic(a, b, q)
    got = to_host(pm.polymul_negacyclic_u64(to_dev(a), to_dev(b), q), np.uint64)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_u64_goldilocks_degrees(n):
    rng = np.random.Generator(np.random.PCG64(n + 64))
    B = 3
    _check64(_rand64(rng, (B, n), GOLD), _rand64(rng, (B, n), GOLD), GOLD)


@pytest.mark.parametrize("q", Q64)
def test_u64_moduli(q):
    rng = np.random.Generator(np.random.PCG64(q % 65521))
    for n in (64, 1024):
        _check64(_rand64(rng, (2, n), q), _rand64(rng, (2, n), q), q)


def test_u64_noncanonical_and_edges():
    rng = np.random.Generator(np.random.PCG64(3))
    n = 1024
    a = rng.integers(0, np.iinfo(np.uint64).max, size=(2, n), dtype=np.uint64, endpoint=True)
    b = rng.integers(0, np.iinfo(np.uint64).max, size=(2, n), dtype=np.uint64, endpoint=True)
    _check64(a, b, GOLD)
    special = np.array([0, 1, GOLD - 1, GOLD // 2, 0x7F7F7F7F7F7F7F7F, 0x7F7F7F7F7F7F7F80,
                        0x8080808080808080 % GOLD, 0x80, 0xFFFFFFFF], dtype=np.uint64)
    a = rng.choice(special, size=(2, n))
    b = rng.choice(special, size=(2, n))
    _check64(a, b, GOLD)
    full = np.full((1, n), GOLD - 1, dtype=np.uint64)
    _check64(full, full, GOLD)


@pytest.mark.parametrize("n", [8192, 16384, 32768])
def test_u64_streaming_kchunks(n):
    """Several K-chunks of 1024; from n = 16384 on (16 chunks, a flush every 15)
    at least one int32 flush between them."""
    rng = np.random.Generator(np.random.PCG64(n))
    _check64(_rand64(rng, (2, n), GOLD), _rand64(rng, (2, n), GOLD), GOLD)


def test_u64_worst_case_digits_flush():
    """All words q - 1 and 2^63-ish patterns over many K-chunks: the largest
    int32 class sums the flush interval allows."""
    n = 16384
    a = np.full((1, n), 0x8080808080808080 % GOLD, dtype=np.uint64)
    _check64(a, a, GOLD)


@pytest.mark.parametrize("sign", ["pos", "neg"])
def test_streaming_flush_extreme_class_sums(sign):
    """Every digit +127 (words 0x7F..7F, the window's top) against every digit +127 or
    words whose digits are mostly -128: the shift-class sums reach their largest
    magnitude within each flush interval, for 8 limbs (64-bit q) and 4 limbs (32-bit
    q, streamed above n = 8192).  The flush adds the classes four at a time into
    64-bit sums offset by 2^56 and removes the offset with a precomputed constant."""
    top8 = np.uint64(0x7F7F7F7F7F7F7F7F)
    # one past the window's top is stored as x - q: digits 127 x4, -128 x4 for this q
    other8 = top8 if sign == "pos" else np.uint64(0x7F7F7F7F7F7F7F80)
    n = 16384
    a = np.full((1, n), top8, dtype=np.uint64)
    b = np.full((1, n), other8, dtype=np.uint64)
    _check64(a, b, GOLD)
    q32 = (1 << 32) - 5
    top4 = np.uint32(0x7F7F7F7F)
    other4 = top4 if sign == "pos" else np.uint32(0x7F7F7F80)  # digits -123, -128, -128, -128
    n = 32768
    a = np.full((1, n), top4, dtype=np.uint32)
    b = np.full((1, n), other4, dtype=np.uint32)
    want = oracle.negacyclic(a, b, q32)
    got = to_host(pm.polymul_negacyclic(to_dev(a), to_dev(b), q32), np.uint32)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.mark.parametrize("n", [16384, 32768, 65536])
@pytest.mark.parametrize("q", [1068236801, (1 << 32) - 5])
def test_u32_streaming_large_degree(n, q):
    rng = np.random.Generator(np.random.PCG64(n ^ q))
    a = rng.integers(0, q, size=(1, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, size=(1, n), dtype=np.uint64).astype(np.uint32)
    want = oracle.negacyclic(a, b, q)
    got = to_host(pm.polymul_negacyclic(to_dev(a), to_dev(b), q), np.uint32)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_u32_streaming_rns_channels():
    rng = np.random.Generator(np.random.PCG64(44))
    n, B = 16384, 1
    qs = []
    while len(qs) < 10:  # more channels than one streaming launch carries
        qs.append(inputs.ntt_prime(rng, 30, 2 * n, exclude=qs))
    a = np.stack([rng.integers(0, q, size=(B, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(B, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    got = to_host(pm.polymul_negacyclic_rns(to_dev(a), to_dev(b), qs), np.uint32)
    pidx = np.zeros(64, dtype=np.uint64)
    jidx = rng.integers(0, n, size=64).astype(np.uint64)
    for l, q in enumerate(qs):
        want = oracle.negacyclic_sample(a[:, l], b[:, l], q, pidx, jidx)
        assert np.array_equal(got[0, l, jidx.astype(np.int64)], want), f"channel {l}"
