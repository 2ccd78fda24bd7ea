"""GPU parity for the shared-operand entry points (one b for a whole batch):
word for word equal to the oracle's product of each a[i] with b."""
import numpy as np
import pytest

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu


def rep(b, batch):
    return np.ascontiguousarray(np.broadcast_to(b, (batch,) + b.shape))


SHARED_CASES = [(n, batch) for n in (1, 2, 4, 8, 32, 64, 256, 1024, 2048, 4096, 8192, 16384)
                for batch in (1, 5, 37) if n < 8192 or batch <= 5]


@pytest.mark.parametrize("n,batch", SHARED_CASES)
def test_shared_u32(n, batch):
    q = 1068236801 if n % 3 else (1 << 32) - 5
    rng = np.random.Generator(np.random.PCG64(n * 100 + batch))
    a = rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, size=(n,), dtype=np.uint64).astype(np.uint32)
    got = to_host(pm.polymul_negacyclic_shared(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.negacyclic(a, rep(b, batch), q)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.mark.parametrize("q", [2, 3329, 65537, 12289 * 4, (1 << 31) - 1])
def test_shared_moduli(q):
    rng = np.random.Generator(np.random.PCG64(q % 9973))
    batch, n = 9, 512
    a = rng.integers(0, 1 << 32, size=(batch, n), dtype=np.uint64).astype(np.uint32)  # non-canonical
    b = rng.integers(0, 1 << 32, size=(n,), dtype=np.uint64).astype(np.uint32)
    got = to_host(pm.polymul_negacyclic_shared(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.negacyclic(a, rep(b, batch), q)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_shared_rns_matches_oracle_and_direct():
    rng = np.random.Generator(np.random.PCG64(77))
    n, L, batch = 4096, 8, 12
    qs = []
    for _ in range(L):
        qs.append(inputs.ntt_prime(rng, 30, 2 * n, exclude=qs))
    a = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(n,), dtype=np.uint64).astype(np.uint32) for q in qs], axis=0)
    da, db = to_dev(a), to_dev(b)
    got = to_host(pm.polymul_negacyclic_rns_shared(da, db, qs), np.uint32)
    want = oracle.negacyclic_rns(a, rep(b, batch), qs)
    assert np.array_equal(got, want), mismatch_report(got, want)
    direct = to_host(pm.polymul_negacyclic_rns(da, to_dev(rep(b, batch)), qs), np.uint32)
    assert np.array_equal(direct, want), mismatch_report(direct, want)


@pytest.mark.parametrize("n,batch", [(256, 700), (1024, 300), (4096, 70)])
def test_shared_rns_many_chunks(n, batch):
    # more products than one workgroup round: several chunks per channel, ragged last chunk
    rng = np.random.Generator(np.random.PCG64(n + batch))
    qs = [3329, 7681, 12289]
    a = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(n,), dtype=np.uint64).astype(np.uint32) for q in qs], axis=0)
    da, db = to_dev(a), to_dev(b)
    got = to_host(pm.polymul_negacyclic_rns_shared(da, db, qs), np.uint32)
    want = oracle.negacyclic_rns(a, rep(b, batch), qs)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_shared_rns_large_degree():
    rng = np.random.Generator(np.random.PCG64(5))
    n, batch, qs = 32768, 2, [998244353, 65537]
    a = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(n,), dtype=np.uint64).astype(np.uint32) for q in qs], axis=0)
    got = to_host(pm.polymul_negacyclic_rns_shared(to_dev(a), to_dev(b), qs), np.uint32)
    for l, q in enumerate(qs):
        pidx = rng.integers(0, batch, size=48, dtype=np.uint64)
        jidx = rng.integers(0, n, size=48, dtype=np.uint64)
        jidx[:3] = [0, n - 1, n // 2]
        want = oracle.negacyclic_sample(a[:, l], rep(b[l], batch), q, pidx, jidx)
        g = got[pidx.astype(np.int64), l, jidx.astype(np.int64)]
        assert np.array_equal(g, want), mismatch_report(g, want)


@pytest.mark.parametrize("n", [8, 1024, 8192])
def test_shared_u64(n):
    q = inputs.GOLDILOCKS
    rng = np.random.Generator(np.random.PCG64(n + 64))
    a = rng.integers(0, q, size=(3, n), dtype=np.uint64)
    b = rng.integers(0, q, size=(n,), dtype=np.uint64)
    got = to_host(pm.polymul_negacyclic_u64_shared(to_dev(a), to_dev(b), q), np.uint64)
    want = oracle.negacyclic(a, rep(b, 3), q)
    assert np.array_equal(got, want), mismatch_report(got, want)
