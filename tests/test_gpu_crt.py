"""GPU parity for the small-modulus residue path (the paper's RNS + CRT
coefficient method): word for word equal to the oracle."""
import numpy as np
import pytest

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu

MODULI = [2, 17, 3329, 65537, 1 << 20, 1068236801, (1 << 31) - 1, (1 << 32) - 5]


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 256, 1024, 2048, 4096])
@pytest.mark.parametrize("q", MODULI)
def test_crt_matches_oracle(n, q):
    rng = np.random.Generator(np.random.PCG64(n * 31 + q % 997))
    batch = 3 if n >= 2048 else 7
    a = rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32)
    got = to_host(pm.polymul_negacyclic_crt(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.negacyclic(a, b, q)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.mark.parametrize("q", [3329, 1068236801, (1 << 32) - 5])
@pytest.mark.parametrize("n", [64, 4096])
def test_crt_extreme_sums(q, n):
    # all coefficients floor(q/2) (the largest centred sums) and all q - 1 / 1 mixes
    h = q // 2
    a = np.stack([np.full(n, h), np.full(n, q - 1), np.arange(n) % 2 * h]).astype(np.uint32)
    b = np.stack([np.full(n, h), np.full(n, 1), np.full(n, q - h)]).astype(np.uint32)
    got = to_host(pm.polymul_negacyclic_crt(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.negacyclic(a, b, q)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_crt_noncanonical_words():
    rng = np.random.Generator(np.random.PCG64(8))
    q, n = 12289, 512
    a = rng.integers(0, 1 << 32, size=(5, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << 32, size=(5, n), dtype=np.uint64).astype(np.uint32)
    got = to_host(pm.polymul_negacyclic_crt(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.negacyclic(a, b, q)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_crt_rns_headline_shape():
    rng = np.random.Generator(np.random.PCG64(12))
    n, L, batch = 4096, 8, 24
    qs = []
    for _ in range(L):
        qs.append(inputs.ntt_prime(rng, 30, 2 * n, exclude=qs))
    a = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    da, db = to_dev(a), to_dev(b)
    got = to_host(pm.polymul_negacyclic_rns_crt(da, db, qs), np.uint32)
    want = oracle.negacyclic_rns(a, b, qs)
    assert np.array_equal(got, want), mismatch_report(got, want)
    limb = to_host(pm.polymul_negacyclic_rns(da, db, qs), np.uint32)
    assert np.array_equal(limb, want), mismatch_report(limb, want)


def test_crt_rns_many_channels_and_ragged_batch():
    # 11 q-level channels (two launches of at most 8) and a batch that leaves a partial group
    rng = np.random.Generator(np.random.PCG64(13))
    n, batch = 256, 13
    qs = [3329, 7681, 12289, 17, 65537, 257, 40961, 786433, 5, 1 << 16, 1068236801]
    a = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    got = to_host(pm.polymul_negacyclic_rns_crt(to_dev(a), to_dev(b), qs), np.uint32)
    want = oracle.negacyclic_rns(a, b, qs)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_crt_rejects_large_degree():
    import torch
    a = torch.zeros((1, 8192), dtype=torch.int32, device="cuda:0")
    with pytest.raises(pm.PolymulError):
        pm.polymul_negacyclic_crt(a, a, 17)
