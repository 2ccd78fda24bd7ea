"""The allocation-free Karatsuba entry point through the C ABI: word for word
the result of the entry point that takes a caller-owned workspace (and of the
oracle), on two calls in a row whose second is smaller than the first, so that
the second call runs over what the first left in the library's scratch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2307_06554_amd as pm
from paper_2307_06554_amd import binding, inputs
from gpu_util import to_dev, to_host, mismatch_report

pytestmark = pytest.mark.gpu


def rns_case(seed, batch, n, L):
    rng = np.random.Generator(np.random.PCG64(seed))
    qs = []
    for _ in range(L):
        qs.append(inputs.ntt_prime(rng, 30, 2 * n, exclude=qs))
    a = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    b = np.stack([rng.integers(0, q, size=(batch, n), dtype=np.uint64).astype(np.uint32) for q in qs], axis=1)
    return a, b, qs


def noalloc_c_abi(da, db, dc, qs, depth):
    """One call of polymul_negacyclic_rns_karatsuba_noalloc straight through ctypes."""
    batch, L, n = da.shape
    qarr = (ctypes.c_uint32 * L)(*qs)
    lib = pm.load_library()
    return lib.polymul_negacyclic_rns_karatsuba_noalloc(
        ctypes.c_void_p(da.data_ptr()), ctypes.c_void_p(db.data_ptr()), ctypes.c_void_p(dc.data_ptr()), n,
        ctypes.cast(qarr, ctypes.c_void_p), L, batch, depth,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_two_calls_second_smaller():
    # first call: n = 4096, 8 channels, 16 pairs, depth 2 (about 14 MB of scratch);
    # second: n = 1024, 3 channels, 5 pairs, depth 1
    for seed, batch, n, L, depth in ((1, 16, 4096, 8, 2), (2, 5, 1024, 3, 1)):
        a, b, qs = rns_case(seed, batch, n, L)
        need = pm.polymul_karatsuba_workspace_size(n, L, batch, depth)
        assert need <= binding.POLYMUL_NOALLOC_SCRATCH_BYTES
        da, db = to_dev(a), to_dev(b)
        dc = torch.full_like(da, -1)
        assert noalloc_c_abi(da, db, dc, qs, depth) == 0
        got = to_host(dc, np.uint32)
        ref = to_host(pm.polymul_negacyclic_rns_karatsuba(da, db, qs, depth), np.uint32)
        assert np.array_equal(got, ref), f"n={n}, depth {depth}: " + mismatch_report(got, ref)
        want = oracle.negacyclic_rns(a, b, qs)
        assert np.array_equal(got, want), f"n={n}, depth {depth}: " + mismatch_report(got, want)


def test_noalloc_depth3_and_binding():
    a, b, qs = rns_case(3, 7, 256, 2)
    da, db = to_dev(a), to_dev(b)
    got = to_host(pm.polymul_negacyclic_rns_karatsuba_noalloc(da, db, qs, 3), np.uint32)
    want = oracle.negacyclic_rns(a, b, qs)
    assert np.array_equal(got, want), mismatch_report(got, want)


def test_noalloc_rejects_calls_beyond_its_scratch():
    # the headline batch at depth 1 needs about 151 MB of workspace: refused before any launch
    n, L, batch, depth = 4096, 8, 256, 1
    assert pm.polymul_karatsuba_workspace_size(n, L, batch, depth) > binding.POLYMUL_NOALLOC_SCRATCH_BYTES
    da = torch.zeros((batch, L, n), dtype=torch.int32, device="cuda:0")
    db = torch.zeros_like(da)
    dc = torch.full_like(da, 7)
    assert noalloc_c_abi(da, db, dc, [3329] * L, depth) == 6  # POLYMUL_ESCRATCH
    torch.cuda.synchronize()
    assert bool((dc == 7).all()), "a refused call wrote its output"
    with pytest.raises(pm.PolymulError, match="ESCRATCH"):
        pm.polymul_negacyclic_rns_karatsuba_noalloc(da, db, [3329] * L, depth, out=dc)
