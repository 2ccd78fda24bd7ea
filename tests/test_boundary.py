"""The C ABI on the CPU: the library loads, exports what the header declares,
and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_2307_06554_amd as pm
from paper_2307_06554_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polymul.h")

EINVAL, EALIAS, EUNSUPPORTED = 1, 2, 3


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(polymul_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("polymul_negacyclic", "polymul_negacyclic_u64", "polymul_negacyclic_rns",
                 "polymul_negacyclic_plain", "polymul_plan_create", "polymul_plan_execute",
                 "polymul_plan_destroy", "polymul_status_string"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    lib = pm.load_library()
    for name in header_functions():
        assert hasattr(lib, name), f"libpolymul.so does not export {name}"
    assert set(header_functions()) <= set(binding._SIGNATURES), "binding misses an entry point"


def test_status_strings():
    for code, name in binding.STATUS.items():
        assert pm.polymul_status_string(code).startswith(name)
    assert "UNKNOWN" in pm.polymul_status_string(99)


# Fake, never-dereferenced device addresses: argument errors must be reported first.
A, B, C = 0x10000000, 0x20000000, 0x30000000
C_ = C


def call(name, *args):
    lib = pm.load_library()
    return getattr(lib, name)(*args)


@pytest.mark.parametrize("n", [0, 3, 6, 100, 131072, 1 << 40])
def test_bad_degree(n):
    assert call("polymul_negacyclic", A, B, C, n, 17, 1, None) == EINVAL
    assert call("polymul_negacyclic_plain", A, B, C, n, 17, 1, None) == EINVAL
    assert call("polymul_negacyclic_u64", A, B, C, n, 17, 1, None) == EINVAL


@pytest.mark.parametrize("q", [0, 1])
def test_bad_modulus(q):
    assert call("polymul_negacyclic", A, B, C, 256, q, 1, None) == EINVAL
    assert call("polymul_negacyclic_u64", A, B, C, 256, q, 1, None) == EINVAL
    assert call("polymul_negacyclic_plain", A, B, C, 256, q, 1, None) == EINVAL


def test_null_pointers():
    for args in ((None, B, C), (A, None, C), (A, B, None)):
        assert call("polymul_negacyclic", *args, 256, 17, 1, None) == EINVAL


def test_zero_batch_is_a_noop():
    assert call("polymul_negacyclic", None, None, None, 256, 17, 0, None) == 0
    assert call("polymul_negacyclic_u64", None, None, None, 256, 17, 0, None) == 0
    assert call("polymul_negacyclic_plain", None, None, None, 256, 17, 0, None) == 0


def test_aliasing_is_rejected():
    n, batch = 256, 4
    nbytes = n * batch * 4
    assert call("polymul_negacyclic", A, B, A, n, 17, batch, None) == EALIAS
    assert call("polymul_negacyclic", A, B, B + nbytes - 16, n, 17, batch, None) == EALIAS
    assert call("polymul_negacyclic", A, B, A - nbytes + 16, n, 17, batch, None) == EALIAS
    assert call("polymul_negacyclic_plain", A, B, B, n, 17, batch, None) == EALIAS
    assert call("polymul_negacyclic_u64", A, B, A + 16, n, 17, batch, None) == EALIAS


def test_misaligned_pointers():
    assert call("polymul_negacyclic", A + 4, B, C, 256, 17, 1, None) == EINVAL
    assert call("polymul_negacyclic_u64", A, B, C + 8, 256, 17, 1, None) == EINVAL


def test_size_overflow():
    assert call("polymul_negacyclic", A, B, C, 65536, 17, 1 << 50, None) == EINVAL


def test_rns_arguments():
    qs = (ctypes.c_uint32 * 2)(17, 1)
    assert call("polymul_negacyclic_rns", A, B, C, 256, ctypes.cast(qs, ctypes.c_void_p), 2, 1, None) == EINVAL
    qs = (ctypes.c_uint32 * 2)(17, 19)
    assert call("polymul_negacyclic_rns", A, B, C, 256, ctypes.cast(qs, ctypes.c_void_p), 0, 1, None) == EINVAL
    assert call("polymul_negacyclic_rns", A, B, C, 256, None, 2, 1, None) == EINVAL
    assert call("polymul_negacyclic_rns", A, B, A, 256, ctypes.cast(qs, ctypes.c_void_p), 2, 1, None) == EALIAS
    assert call("polymul_negacyclic_rns", None, None, None, 256, ctypes.cast(qs, ctypes.c_void_p), 2, 0, None) == 0


def test_plan_arguments():
    h = ctypes.c_void_p()
    assert call("polymul_plan_create", None, None, 0, 0) == EINVAL
    assert call("polymul_plan_execute", None, None) == EINVAL
    assert call("polymul_plan_destroy", None) == 0


def test_plan_group_validation():
    import ctypes as C
    from paper_2307_06554_amd.binding import _Group
    h = C.c_void_p()
    good = _Group(A, B, C_, 256, 17, 2, 4)
    for bad in (_Group(A, B, C_, 255, 17, 2, 4), _Group(A, B, C_, 256, 1, 2, 4), _Group(A, B, C_, 256, 17, 2, 3),
                _Group(A, B, C_, 256, 1 << 33, 2, 4), _Group(0, B, C_, 256, 17, 2, 4), _Group(A + 4, B, C_, 256, 17, 2, 4)):
        arr = (_Group * 2)(good, bad)
        assert call("polymul_plan_create", C.byref(h), C.cast(arr, C.c_void_p), 2, 0) == EINVAL
    arr = (_Group * 1)(_Group(A, B, A, 256, 17, 2, 4))
    assert call("polymul_plan_create", C.byref(h), C.cast(arr, C.c_void_p), 1, 0) == EALIAS
    arr = (_Group * 1)(good)
    assert call("polymul_plan_create", C.byref(h), C.cast(arr, C.c_void_p), 1, 0x80) == EINVAL
    assert h.value is None


def test_tile_table():
    for n, t in ((4096, 64), (4096, 128), (4096, 32), (1024, 64), (16, 16), (512, 16), (64, 16), (256, 32)):
        pm.polymul_tune_set(n, 4, t)
        assert pm.polymul_tune_get(n, 4) == t
        pm.polymul_tune_set(n, 4, 0)
    # built-in: 16x16 tiles for 64..512, 32x32 at 1024, a 64-side above
    assert pm.polymul_tune_get(4096, 4) == 64 and pm.polymul_tune_get(1024, 2) == 32
    assert pm.polymul_tune_get(256, 2) == 16 and pm.polymul_tune_get(512, 4) == 16 and pm.polymul_tune_get(64, 3) == 16
    for n, L, t in ((4096, 4, 48), (4096, 4, 256), (4096, 5, 64), (1000, 4, 32), (16, 4, 32), (64, 4, 128),
                    (1024, 4, 16), (32, 4, 16)):
        with pytest.raises(pm.PolymulError):
            pm.polymul_tune_set(n, L, t)


def test_binding_refuses_host_tensors():
    import torch
    with pytest.raises(TypeError):
        pm.polymul_negacyclic(torch.zeros(4, dtype=torch.int32), torch.zeros(4, dtype=torch.int32), 17)


def test_karatsuba_workspace_size():
    for n, L, batch, depth in ((4096, 8, 16, 2), (64, 1, 3, 1), (65536, 2, 1, 3), (32, 4, 2, 3)):
        words = batch * L * 3 ** depth * (n >> depth)
        assert pm.polymul_karatsuba_workspace_size(n, L, batch, depth) == 3 * 4 * words
    for n, L, depth in ((4096, 8, 4), (16, 1, 3), (100, 1, 1), (4096, 0, 1), (4096, 17, 1),
                        (131072, 1, 1), (100, 1, 0)):
        with pytest.raises(pm.PolymulError):
            pm.polymul_karatsuba_workspace_size(n, L, 1, depth)


def test_karatsuba_arguments():
    qs = (ctypes.c_uint32 * 2)(17, 19)
    qp = ctypes.cast(qs, ctypes.c_void_p)
    W = 0x40000000
    need = pm.polymul_karatsuba_workspace_size(256, 2, 1, 2)
    k = "polymul_negacyclic_rns_karatsuba"
    assert call(k, A, B, C, 256, qp, 2, 1, 2, W, need - 1, None) == EINVAL   # workspace too small
    assert call(k, A, B, C, 256, qp, 2, 1, 2, W + 4, need, None) == EINVAL   # misaligned workspace
    assert call(k, A, B, C, 256, qp, 2, 1, 2, None, need, None) == EINVAL    # no workspace
    # depth 0 resolves to the tuned depth (built-in: two levels at n = 4096), checked like an explicit one
    need0 = pm.polymul_karatsuba_workspace_size(4096, 2, 1, 0)
    assert need0 == pm.polymul_karatsuba_workspace_size(4096, 2, 1, 2)
    assert call(k, A, B, C, 4096, qp, 2, 1, 0, W, need0 - 1, None) == EINVAL
    assert call(k, A, B, C, 256, qp, 2, 1, 4, W, 1 << 30, None) == EINVAL    # depth 4
    assert call(k, A, B, C, 8, qp, 2, 1, 2, W, need, None) == EINVAL         # n / 2^depth < 4
    assert call(k, A, B, C, 256, None, 2, 1, 2, W, need, None) == EINVAL
    bad = (ctypes.c_uint32 * 2)(17, 1)
    assert call(k, A, B, C, 256, ctypes.cast(bad, ctypes.c_void_p), 2, 1, 2, W, need, None) == EINVAL
    assert call(k, A, B, A, 256, qp, 2, 1, 2, W, need, None) == EALIAS         # c overlaps a
    assert call(k, A, B, C, 256, qp, 2, 1, 2, A - 16, need, None) == EALIAS    # workspace overlaps a
    assert call(k, A, B, C, 256, qp, 2, 1, 2, C + 64, need, None) == EALIAS    # workspace overlaps c
    assert call(k, None, None, None, 256, qp, 2, 0, 2, None, 0, None) == 0     # empty batch


def test_karatsuba_noalloc_arguments():
    # the allocation-free route: the same argument checks, and a call needing more than
    # the library's scratch is refused with POLYMUL_ESCRATCH, all before any HIP call
    ESCRATCH = 6
    qs = (ctypes.c_uint32 * 8)(*([1068236801] * 8))
    qp = ctypes.cast(qs, ctypes.c_void_p)
    k = "polymul_negacyclic_rns_karatsuba_noalloc"
    assert pm.polymul_karatsuba_workspace_size(4096, 8, 256, 1) > binding.POLYMUL_NOALLOC_SCRATCH_BYTES
    assert call(k, A, B, C, 4096, qp, 8, 256, 1, None) == ESCRATCH
    assert call(k, A, B, C, 4096, qp, 8, 256, 0, None) == ESCRATCH    # depth 0: two levels here
    assert call(k, A, B, C, 4096, qp, 8, 1, 4, None) == EINVAL        # depth 4
    assert call(k, A, B, C, 8, qp, 8, 1, 2, None) == EINVAL           # n / 2^depth < 4
    assert call(k, A, B, C, 4096, None, 8, 1, 2, None) == EINVAL
    assert call(k, A, B, C, 4096, qp, 0, 1, 2, None) == EINVAL
    assert call(k, A, B, A + 64, 4096, qp, 8, 1, 2, None) == EALIAS   # c overlaps a
    assert call(k, None, None, None, 4096, qp, 8, 0, 2, None) == 0    # empty batch
    assert pm.polymul_status_string(ESCRATCH).startswith("POLYMUL_ESCRATCH")


def test_shared_operand_arguments():
    qs = (ctypes.c_uint32 * 2)(17, 19)
    qp = ctypes.cast(qs, ctypes.c_void_p)
    for name in ("polymul_negacyclic_shared", "polymul_negacyclic_u64_shared"):
        assert call(name, A, B, C, 255, 17, 4, None) == EINVAL
        assert call(name, A, B, C, 256, 1, 4, None) == EINVAL
        assert call(name, None, B, C, 256, 17, 4, None) == EINVAL
        assert call(name, A, B + 8, C, 256, 17, 4, None) == EINVAL
        assert call(name, A, B, A + 1024, 256, 17, 4, None) == EALIAS      # c overlaps a
        assert call(name, A, B, B - 16, 256, 17, 4, None) == EALIAS        # c overlaps b
        assert call(name, None, None, None, 256, 17, 0, None) == 0
    k = "polymul_negacyclic_rns_shared"
    assert call(k, A, B, C, 256, None, 2, 4, None) == EINVAL
    assert call(k, A, B, C, 256, qp, 0, 4, None) == EINVAL
    bad = (ctypes.c_uint32 * 2)(17, 0)
    assert call(k, A, B, C, 256, ctypes.cast(bad, ctypes.c_void_p), 2, 4, None) == EINVAL
    assert call(k, A, B, B + 2 * 256 * 4 - 16, 256, qp, 2, 4, None) == EALIAS  # c overlaps the end of b
    assert call(k, None, None, None, 256, qp, 2, 0, None) == 0


def test_crt_arguments():
    assert call("polymul_negacyclic_crt", A, B, C, 255, 17, 1, None) == EINVAL
    assert call("polymul_negacyclic_crt", A, B, C, 256, 1, 1, None) == EINVAL
    assert call("polymul_negacyclic_crt", A, B, A, 256, 17, 1, None) == EALIAS
    assert call("polymul_negacyclic_crt", A, B, C, 8192, 17, 1, None) == EUNSUPPORTED  # planes exceed LDS
    assert call("polymul_negacyclic_crt", None, None, None, 256, 17, 0, None) == 0
    qs = (ctypes.c_uint32 * 2)(17, 1)
    assert call("polymul_negacyclic_rns_crt", A, B, C, 256, ctypes.cast(qs, ctypes.c_void_p), 2, 1, None) == EINVAL
    out = (ctypes.c_uint32 * 11)()
    cnt = ctypes.c_uint32()
    assert call("polymul_crt_moduli", 256, 1, out, ctypes.byref(cnt)) == EINVAL
    assert call("polymul_crt_moduli", 100, 17, out, ctypes.byref(cnt)) == EINVAL
    assert call("polymul_crt_moduli", 256, 17, None, ctypes.byref(cnt)) == EINVAL
    assert call("polymul_crt_moduli", 65536, 0xFFFFFFFF, out, ctypes.byref(cnt)) == 0 and cnt.value <= 11


def test_karatsuba_u64_arguments():
    # sub-operands of a and b, the sub-products and four copies of them for K runs
    assert pm.polymul_karatsuba_u64_workspace_size(65536, 16, 2) == 7 * 8 * 16 * 9 * 16384
    with pytest.raises(pm.PolymulError):
        pm.polymul_karatsuba_u64_workspace_size(65536, 16, 4)
    W = 0x40000000
    need = pm.polymul_karatsuba_u64_workspace_size(256, 1, 1)
    k = "polymul_negacyclic_u64_karatsuba"
    assert call(k, A, B, C, 256, 17, 1, 1, W, need - 1, None) == EINVAL
    assert call(k, A, B, C, 256, 1, 1, 1, W, need, None) == EINVAL
    need3 = pm.polymul_karatsuba_u64_workspace_size(65536, 16, 3)
    assert pm.polymul_karatsuba_u64_workspace_size(65536, 16, 0) == need3  # depth 0: three levels at n = 65536
    assert call(k, A, B, C, 65536, 17, 16, 0, W, need3 - 1, None) == EINVAL
    assert call(k, A, B, A, 256, 17, 1, 1, W, need, None) == EALIAS
    assert call(k, A, B, C, 256, 17, 1, 1, B + 16, need, None) == EALIAS
    assert call(k, None, None, None, 256, 17, 0, 1, None, 0, None) == 0


def test_plan_tuning_knobs():
    assert pm.polymul_tune_param_get("plan_share_pct") == 140
    assert pm.polymul_tune_param_get("plan_stream_pct") == 125
    lib = pm.load_library()
    assert lib.polymul_tune_param_set(1, 9) == EINVAL
    assert lib.polymul_tune_param_set(1, 1001) == EINVAL
    assert lib.polymul_tune_param_set(2, 49) == EINVAL
    assert lib.polymul_tune_param_set(99, 100) == EINVAL
    assert lib.polymul_tune_param_get(1, None) == EINVAL
    assert pm.polymul_tune_param_get("u64_karatsuba_runs") == 4
    assert lib.polymul_tune_param_set(3, 3) == EINVAL
    pm.polymul_tune_param_set("plan_share_pct", 250)
    assert pm.polymul_tune_param_get("plan_share_pct") == 250
    pm.polymul_tune_param_set("plan_share_pct", 140)


def test_karatsuba_depth_table():
    # built-in choices, a tuned entry for one products bucket, and back
    assert pm.polymul_tune_get_karatsuba(4096, 2048, 4) == 2
    assert pm.polymul_tune_get_karatsuba(512, 2048, 4) == 1
    assert pm.polymul_tune_get_karatsuba(256, 2048, 4) == 0
    assert pm.polymul_tune_get_karatsuba(65536, 16, 8) == 3
    assert pm.polymul_tune_get_karatsuba(16, 16, 8) == 1
    try:
        pm.polymul_tune_set_karatsuba(4096, 2048, 4, 3)
        assert pm.polymul_tune_get_karatsuba(4096, 2048, 4) == 3
        assert pm.polymul_tune_get_karatsuba(4096, 4095, 4) == 3      # same power-of-two bucket
        assert pm.polymul_tune_get_karatsuba(4096, 4096, 4) == 2      # the next bucket is untouched
        assert pm.polymul_tune_get_karatsuba(4096, 2048, 8) == 1      # and so are 64-bit words
        assert pm.polymul_karatsuba_workspace_size(4096, 8, 256, 0) == pm.polymul_karatsuba_workspace_size(
            4096, 8, 256, 3)
        pm.polymul_tune_set_karatsuba(4096, 2048, 4, 0)
        assert pm.polymul_karatsuba_workspace_size(4096, 8, 256, 0) == 0  # direct route: no workspace
    finally:
        pm.polymul_tune_set_karatsuba(4096, 2048, 4, pm.binding.KARATSUBA_BUILTIN)
    assert pm.polymul_tune_get_karatsuba(4096, 2048, 4) == 2
    lib = pm.load_library()
    assert lib.polymul_tune_set_karatsuba(4096, 1, 4, 4) == EINVAL
    assert lib.polymul_tune_set_karatsuba(8, 1, 4, 2) == EINVAL   # n / 2^depth < 4
    assert lib.polymul_tune_set_karatsuba(4096, 0, 4, 1) == EINVAL
    assert lib.polymul_tune_set_karatsuba(4096, 1, 2, 1) == EINVAL
