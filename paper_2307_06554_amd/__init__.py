"""MI355X split-limb int8-MFMA negacyclic polynomial multiplication.

The compute path lives in ``libpolymul.so`` (HIP for gfx950, C ABI declared in
``include/polymul.h``); ``binding`` wraps it with ctypes for torch device
tensors.  Nothing here computes a product on the CPU.
"""
from .binding import (  # noqa: F401
    PolymulError,
    lib_path,
    polymul_cyclic,
    polymul_crt_moduli,
    polymul_cyclic_u64,
    load_library,
    polymul_karatsuba_u64_workspace_size,
    polymul_karatsuba_workspace_size,
    polymul_negacyclic,
    polymul_negacyclic_crt,
    polymul_negacyclic_plain,
    polymul_negacyclic_rns,
    polymul_negacyclic_rns_crt,
    polymul_negacyclic_rns_karatsuba,
    polymul_negacyclic_rns_karatsuba_noalloc,
    polymul_negacyclic_rns_shared,
    polymul_negacyclic_shared,
    polymul_negacyclic_u64_shared,
    polymul_negacyclic_u64,
    polymul_negacyclic_u64_karatsuba,
    polymul_plan_create,
    polymul_plan_destroy,
    polymul_plan_execute,
    polymul_status_string,
    polymul_tune_get,
    polymul_tune_set,
    polymul_tune_get_karatsuba,
    polymul_tune_set_karatsuba,
    polymul_tune_param_get,
    polymul_tune_param_set,
    Plan,
)
