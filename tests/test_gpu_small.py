"""GPU parity of the 16x16-tile kernel (v_mfma_i32_16x16x64_i8, Toeplitz side 16)
that the tile table selects with t = 16 for 64 <= n <= 512: every limb count,
ragged workgroups, RNS channels, the cyclic ring, the shared operand and the
Karatsuba sub-products that run on it, against the oracle word for word."""
import contextlib

import numpy as np
import pytest

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu

Q30 = 1068236801


@contextlib.contextmanager
def small_tiles(ns, Ls=(2, 3, 4)):
    old = {(n, L): pm.polymul_tune_get(n, L) for n in ns for L in Ls}
    for n in ns:
        for L in Ls:
            pm.polymul_tune_set(n, L, 16)
    try:
        yield
    finally:
        for (n, L), t in old.items():
            pm.polymul_tune_set(n, L, t)


def _rand(rng, shape, q):
    return rng.integers(0, q, size=shape, dtype=np.uint64).astype(np.uint32)


@pytest.mark.parametrize("n", [64, 128, 256, 512])
@pytest.mark.parametrize("q", [3329, (1 << 24) - 3, Q30, (1 << 32) - 5])
@pytest.mark.parametrize("batch", [1, 5, 37, 1100])
def test_small_tiles_match_oracle(n, q, batch):
    rng = np.random.Generator(np.random.PCG64(n * 13 + batch + q % 1000))
    a, b = _rand(rng, (batch, n), q), _rand(rng, (batch, n), q)
    with small_tiles([n]):
        got = to_host(pm.polymul_negacyclic(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.negacyclic(a, b, q)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.mark.parametrize("n", [64, 256, 512])
def test_small_tiles_edges(n):
    # non-canonical words, all q - 1, monomials, digit-window edges
    q = Q30
    rng = np.random.Generator(np.random.PCG64(n))
    a = rng.integers(0, 1 << 32, size=(6, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << 32, size=(6, n), dtype=np.uint64).astype(np.uint32)
    a[1] = q - 1
    b[1] = q - 1
    b[2] = 0
    b[2, n - 1] = 1
    b[3] = 0
    b[3, 0] = 1
    a[4] = 0x7F7F7F7F % q
    b[4] = 0x80808080 % q
    with small_tiles([n]):
        got = to_host(pm.polymul_negacyclic(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.negacyclic(a, b, q)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_small_tiles_rns_cyclic_shared():
    rng = np.random.Generator(np.random.PCG64(3))
    n, batch = 256, 19
    qs = [Q30, 12289, 7340033, 998244353]
    a = np.stack([_rand(rng, (batch, n), q) for q in qs], axis=1)
    b = np.stack([_rand(rng, (batch, n), q) for q in qs], axis=1)
    with small_tiles([n]):
        got = to_host(pm.polymul_negacyclic_rns(to_dev(a), to_dev(b), qs), np.uint32)
        cyc = to_host(pm.polymul_cyclic(to_dev(a[:, 0]), to_dev(b[:, 0]), Q30), np.uint32)
        b0 = np.ascontiguousarray(b[0])
        sh = to_host(pm.polymul_negacyclic_rns_shared(to_dev(a), to_dev(b0), qs), np.uint32)
    want = oracle.negacyclic_rns(a, b, qs)
    assert np.array_equal(got, want), mismatch_report(got, want)
    wc = oracle.cyclic(a[:, 0], b[:, 0], Q30)
    assert np.array_equal(cyc, wc), mismatch_report(cyc, wc)
    ws = oracle.negacyclic_rns(a, np.ascontiguousarray(np.broadcast_to(b0, a.shape)), qs)
    assert np.array_equal(sh, ws), mismatch_report(sh, ws)


@pytest.mark.parametrize("n,depth", [(4096, 3), (1024, 1), (2048, 3), (512, 1)])
def test_small_tiles_karatsuba_subproducts(n, depth):
    rng = np.random.Generator(np.random.PCG64(n + depth))
    qs = []
    for _ in range(3):
        qs.append(inputs.ntt_prime(rng, 30, 2 * n, exclude=qs))
    a = np.stack([_rand(rng, (6, n), q) for q in qs], axis=1)
    b = np.stack([_rand(rng, (6, n), q) for q in qs], axis=1)
    with small_tiles([n >> depth]):
        got = to_host(pm.polymul_negacyclic_rns_karatsuba(to_dev(a), to_dev(b), qs, depth), np.uint32)
    want = oracle.negacyclic_rns(a, b, qs)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.mark.parametrize("tile", [16, 32])
def test_small_tiles_in_plans(tile):
    """Grouped plans run their 64..512-degree groups on whichever tile the table
    names: 16x16-tile items of up to 16 products (ragged last item) beside 32x32
    resident groups and streamed blocks, 2, 3 and 4 limbs, three replays."""
    import torch
    rng = np.random.Generator(np.random.PCG64(9 + tile))
    specs = [(64, 3329, 33), (128, Q30, 17), (256, Q30, 70), (256, 12289, 5), (512, (1 << 24) - 3, 21),
             (512, Q30, 40), (1024, Q30, 6), (4096, Q30, 2), (16384, Q30, 1)]
    groups, refs = [], []
    for n, q, count in specs:
        a, b = _rand(rng, (count, n), q), _rand(rng, (count, n), q)
        da, db = to_dev(a), to_dev(b)
        groups.append((da, db, torch.zeros_like(da), n, q))
        refs.append((a, b, q))
    with small_tiles([64, 128, 256, 512]) if tile == 16 else contextlib.nullcontext():
        if tile == 32:
            for n in (64, 128, 256, 512):
                for L in (2, 3, 4):
                    pm.polymul_tune_set(n, L, 32)
        try:
            plan = pm.Plan(groups)
        finally:
            if tile == 32:
                for n in (64, 128, 256, 512):
                    for L in (2, 3, 4):
                        pm.polymul_tune_set(n, L, 0)
    for rep in range(3):
        for g in groups:
            g[2].zero_()
        plan.execute()
        torch.cuda.synchronize()
        for (da, db, dc, n, q), (a, b, _) in zip(groups, refs):
            got = to_host(dc, np.uint32)
            want = oracle.negacyclic(a, b, q)
            assert np.array_equal(got, want), f"tile {tile}, replay {rep}, n={n}: " + mismatch_report(got, want)
    plan.close()
