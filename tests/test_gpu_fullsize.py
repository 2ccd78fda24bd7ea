"""GPU parity at the workloads' full sizes: every coefficient of every product
compared with the CPU oracle (paper Sec. 2.1 coefficient form; Sec. 2.2 fold
rule and Eq. (3); Sec. 2.4 for the RNS channels), for the launch the benchmark
times and for every other route that computes the same product.

  - n = 4096, eight 30-bit RNS channels, 256 pairs (2048 limb-products): the
    direct route, the Karatsuba route at depths 1-3, the small-modulus CRT route
    and the shared-operand route (pair 0's b for every pair).
  - n = 65536, q = 2^64 - 2^32 + 1, 16 pairs: the direct streaming route and the
    64-bit Karatsuba route at depths 1-3, one product per oracle call so that a
    mismatch names its product.
The other three workloads are compared in full in test_gpu_parity.py and
test_gpu_plan.py.
"""
import numpy as np
import pytest

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w2():
    w = inputs.make_workload(2)
    return w, to_dev(w.a), to_dev(w.b)


@pytest.fixture(scope="module")
def w2_want(w2):
    w = w2[0]
    return oracle.negacyclic_rns(w.a, w.b, w.qs)


def test_workload2_direct_full(w2, w2_want):
    w, da, db = w2
    got = to_host(pm.polymul_negacyclic_rns(da, db, w.qs), np.uint32)
    assert got.shape == w2_want.shape == (256, 8, 4096)
    assert np.array_equal(got, w2_want), mismatch_report(got, w2_want)


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_workload2_karatsuba_full(w2, w2_want, depth):
    w, da, db = w2
    got = to_host(pm.polymul_negacyclic_rns_karatsuba(da, db, w.qs, depth), np.uint32)
    assert np.array_equal(got, w2_want), f"depth {depth}: " + mismatch_report(got, w2_want)


def test_workload2_crt_full(w2, w2_want):
    w, da, db = w2
    got = to_host(pm.polymul_negacyclic_rns_crt(da, db, w.qs), np.uint32)
    assert np.array_equal(got, w2_want), mismatch_report(got, w2_want)


def test_workload2_shared_operand_full(w2):
    w, da, _ = w2
    b0 = np.ascontiguousarray(w.b[0])
    got = to_host(pm.polymul_negacyclic_rns_shared(da, to_dev(b0), w.qs), np.uint32)
    want = oracle.negacyclic_rns(w.a, np.ascontiguousarray(np.broadcast_to(b0, w.a.shape)), w.qs)
    assert np.array_equal(got, want), mismatch_report(got, want)


@pytest.fixture(scope="module")
def w4_out():
    w = inputs.make_workload(4)
    da, db = to_dev(w.a), to_dev(w.b)
    direct = to_host(pm.polymul_negacyclic_u64(da, db, w.q), np.uint64)
    kara = {d: to_host(pm.polymul_negacyclic_u64_karatsuba(da, db, w.q, d), np.uint64) for d in (1, 2, 3)}
    return w, direct, kara


@pytest.mark.parametrize("p", range(16))
def test_workload4_full_product(w4_out, p):
    w, direct, kara = w4_out
    assert direct.shape == (16, 65536)
    want = oracle.negacyclic(w.a[p:p + 1], w.b[p:p + 1], w.q)
    got = direct[p:p + 1]
    assert np.array_equal(got, want), f"product {p}, direct: " + mismatch_report(got, want)
    for d, k in kara.items():
        got = k[p:p + 1]
        assert np.array_equal(got, want), f"product {p}, Karatsuba depth {d}: " + mismatch_report(got, want)
