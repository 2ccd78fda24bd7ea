"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu

Q30 = 1068236801
QS = [2, 3, 17, 251, 257, 3329, 65536, 65537, 1 << 24, (1 << 24) + 1, Q30, (1 << 31) - 1,
      (1 << 31) + 6, (1 << 32) - 5, (1 << 32) - 1]
NS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]


def _rand(rng, shape, q):
    return rng.integers(0, q, size=shape, dtype=np.uint64).astype(np.uint32)


def _check(fn, a, b, q):
    want = oracle.negacyclic(a, b, q)
    got = to_host(fn(to_dev(a), to_dev(b), q), np.uint32)
    assert np.array_equal(got, want), mismatch_report(got, want)


def _batch_for(n):
    # several workgroups and a ragged last one for every tile geometry
    return 5 if n >= 2048 else 9


@pytest.mark.parametrize("n", NS)
def test_mfma_all_degrees(n):
    rng = np.random.Generator(np.random.PCG64(n))
    B = _batch_for(n)
    _check(pm.polymul_negacyclic, _rand(rng, (B, n), Q30), _rand(rng, (B, n), Q30), Q30)


@pytest.mark.parametrize("q", QS)
def test_mfma_all_moduli(q):
    rng = np.random.Generator(np.random.PCG64(q % 100003))
    for n in (256, 1024, 4096):
        B = 3
        _check(pm.polymul_negacyclic, _rand(rng, (B, n), q), _rand(rng, (B, n), q), q)


@pytest.mark.parametrize("q", [3329, Q30, (1 << 32) - 5, (1 << 31) + 6])
def test_mfma_noncanonical_words(q):
    rng = np.random.Generator(np.random.PCG64(77))
    n = 1024
    a = rng.integers(0, 1 << 32, size=(3, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << 32, size=(3, n), dtype=np.uint64).astype(np.uint32)
    _check(pm.polymul_negacyclic, a, b, q)


@pytest.mark.parametrize("q", [2, 3, 3329, Q30, (1 << 31) - 1, 1 << 31, (1 << 31) + 6, (1 << 32) - 5])
def test_mfma_word_reduction_extremes(q):
    """Input words at the top of the 32-bit range and next to multiples of q, where a
    word's quotient estimate is furthest off, through every staging path (n < 256,
    n >= 256) and both epilogue forms (q below and above 2^31)."""
    k = ((1 << 32) - 1) // q
    words = {(1 << 32) - 1, (1 << 32) - 2, (1 << 32) - q, k * q, k * q - 1, (k - 1) * q + q - 1, q, q - 1, 0}
    words = np.array(sorted(w for w in words if 0 <= w < (1 << 32)), dtype=np.uint64)
    rng = np.random.Generator(np.random.PCG64(q % 65521))
    for n in (64, 256, 1024, 4096):
        a = rng.choice(words, size=(3, n)).astype(np.uint32)
        b = rng.choice(words, size=(3, n)).astype(np.uint32)
        _check(pm.polymul_negacyclic, a, b, q)


@pytest.mark.parametrize("q", [257, 65537, Q30, (1 << 32) - 5])
def test_mfma_digit_window_edges(q):
    """Representatives at the edges of the balanced-digit window and words whose
    bytes are 0x80 (digit -128)."""
    L = 1
    while q > 256 ** L:
        L += 1
    L = max(L, 2)
    S = sum(256 ** i for i in range(L))
    thr = 127 * S
    special = sorted({0, 1, q - 1, q // 2, (q + 1) // 2, min(thr, q - 1), min(thr + 1, q - 1),
                      0x80 % q, 0x8080 % q, 0x808080 % q, 0x80808080 % q, 0x7F7F7F7F % q,
                      0xFFFFFFFF % q, 0x80000000 % q})
    rng = np.random.Generator(np.random.PCG64(q % 9973))
    for n in (64, 1024, 4096):
        a = rng.choice(np.array(special, dtype=np.uint64), size=(2, n)).astype(np.uint32)
        b = rng.choice(np.array(special, dtype=np.uint64), size=(2, n)).astype(np.uint32)
        _check(pm.polymul_negacyclic, a, b, q)
        full = np.full((1, n), q - 1, dtype=np.uint32)
        _check(pm.polymul_negacyclic, full, full, q)


@pytest.mark.parametrize("n", [256, 4096])
def test_mfma_monomials(n):
    q = Q30
    rng = np.random.Generator(np.random.PCG64(5))
    a = _rand(rng, (4, n), q)
    b = np.zeros((4, n), dtype=np.uint32)
    for r, k in enumerate((0, 1, n // 2 + 3, n - 1)):
        b[r, k] = 1
    _check(pm.polymul_negacyclic, a, b, q)


def test_mfma_repeatable():
    rng = np.random.Generator(np.random.PCG64(11))
    a, b = _rand(rng, (16, 4096), Q30), _rand(rng, (16, 4096), Q30)
    da, db = to_dev(a), to_dev(b)
    c1 = to_host(pm.polymul_negacyclic(da, db, Q30), np.uint32)
    c2 = to_host(pm.polymul_negacyclic(da, db, Q30), np.uint32)
    assert np.array_equal(c1, c2)


@pytest.mark.parametrize("n", [1, 4, 64, 256, 1024, 4096])
@pytest.mark.parametrize("q", [3329, Q30, (1 << 32) - 5])
def test_plain_kernel(n, q):
    rng = np.random.Generator(np.random.PCG64(n + 3))
    _check(pm.polymul_negacyclic_plain, _rand(rng, (3, n), q), _rand(rng, (3, n), q), q)


@pytest.mark.parametrize("q", [2, 3329, Q30, (1 << 31) - 1, (1 << 31) + 6, 2863311531, (1 << 32) - 5])
def test_plain_kernel_largest_terms(q):
    """Every term of the middle outputs is (q - 1)^2, the most a lazy sum takes
    between folds (b_k = q - 1 below n/2 and 1 above, so the wrapped operand
    q - b_(n+k) is q - 1 too), words above q, and degrees of several input chunks."""
    n = 4096
    a = np.full((2, n), q - 1, dtype=np.uint32)
    b = np.where(np.arange(n) < n // 2, q - 1, 1).astype(np.uint32)[None, :].repeat(2, axis=0)
    a[1, ::3] = np.uint32(0xFFFFFFFF)
    _check(pm.polymul_negacyclic_plain, a, b, q)
    rng = np.random.Generator(np.random.PCG64(q % 1000))
    for n in (8192, 16384):
        _check(pm.polymul_negacyclic_plain, _rand(rng, (2, n), q), _rand(rng, (2, n), q), q)


def test_rns_channels():
    w = inputs.make_workload(2, scale=3 / 256)
    got = to_host(pm.polymul_negacyclic_rns(to_dev(w.a), to_dev(w.b), w.qs), np.uint32)
    want = oracle.negacyclic_rns(w.a, w.b, w.qs)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_rns_many_channels_chunked():
    """More channels than one launch carries (chunked over moduli)."""
    rng = np.random.Generator(np.random.PCG64(21))
    n, L, B = 256, 37, 2
    qs = []
    while len(qs) < L:
        qs.append(inputs.ntt_prime(rng, 30, 2 * n, exclude=qs))
    a = np.stack([_rand(rng, (B, n), q) for q in qs], axis=1)
    b = np.stack([_rand(rng, (B, n), q) for q in qs], axis=1)
    got = to_host(pm.polymul_negacyclic_rns(to_dev(a), to_dev(b), qs), np.uint32)
    assert np.array_equal(got, oracle.negacyclic_rns(a, b, qs))


def test_workload0_full():
    w = inputs.make_workload(0)
    _check(pm.polymul_negacyclic, w.a, w.b, w.q)


def test_workload1_full():
    w = inputs.make_workload(1)
    _check(pm.polymul_negacyclic, w.a, w.b, w.q)


def test_workload3_groups_full():
    w = inputs.make_workload(3)
    for g in w.groups:
        _check(pm.polymul_negacyclic, g.a, g.b, g.q)



def test_launches_go_to_the_current_stream():
    """With no stream given, a call launches on torch's current stream of the current
    device (read as a raw handle), also when the caller has made another stream current."""
    from paper_2307_06554_amd import binding
    q = 1068236801
    rng = np.random.Generator(np.random.PCG64(77))
    a = rng.integers(0, q, size=(64, 1024), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, size=(64, 1024), dtype=np.uint64).astype(np.uint32)
    da, db = to_dev(a), to_dev(b)
    assert (binding._stream(None).value or 0) == torch.cuda.current_stream().cuda_stream
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        assert binding._stream(None).value == s.cuda_stream
        dc = pm.polymul_negacyclic(da, db, q)
    s.synchronize()
    got = to_host(dc, np.uint32)
    wv = oracle.negacyclic(a, b, q)
    assert np.array_equal(got, wv), mismatch_report(got, wv)
