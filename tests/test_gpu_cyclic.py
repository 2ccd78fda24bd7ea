"""GPU parity for the cyclic ring Z_q[x]/(x^n - 1) (same kernels, wrap sign kept)."""
import numpy as np
import pytest

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 4, 16, 64, 256, 1024, 4096, 8192, 16384])
@pytest.mark.parametrize("q", [3329, 1068236801, (1 << 32) - 5])
def test_cyclic_u32(n, q):
    rng = np.random.Generator(np.random.PCG64(n + q % 1000))
    B = 3 if n <= 8192 else 1
    a = rng.integers(0, q, size=(B, n), dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, size=(B, n), dtype=np.uint64).astype(np.uint32)
    got = to_host(pm.polymul_cyclic(to_dev(a), to_dev(b), q), np.uint32)
    want = oracle.cyclic(a, b, q)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.mark.parametrize("n", [1, 8, 64, 1024, 8192])
def test_cyclic_u64(n):
    q = inputs.GOLDILOCKS
    rng = np.random.Generator(np.random.PCG64(n))
    a = rng.integers(0, q, size=(2, n), dtype=np.uint64)
    b = rng.integers(0, q, size=(2, n), dtype=np.uint64)
    got = to_host(pm.polymul_cyclic_u64(to_dev(a), to_dev(b), q), np.uint64)
    want = oracle.cyclic(a, b, q)
    assert np.array_equal(got, want), mismatch_report(got, want)
