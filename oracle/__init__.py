"""CPU oracle for exact negacyclic polynomial multiplication (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the two
share no code: the oracle is plain C (``polymul_oracle.c``) built into its own
``liboracle.so`` and wrapped here with ctypes.

Definition followed (paper Sec. 2.1 coefficient form; Sec. 2.2 fold rule and
Eq. (3)): c_j = (sum_{i<=j} a_i b_{j-i} - sum_{i>j} a_i b_{n+j-i}) mod q in
[0, q).  RNS products (Sec. 2.4) apply it channel by channel.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polymul_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose=False):
    """Compile liboracle.so with gcc (portable x86-64 code, OpenMP over outputs)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", _LIB_PATH + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u64, u32 = ctypes.c_uint64, ctypes.c_uint32
    vp = ctypes.c_void_p
    lib.oracle_negacyclic_u32.argtypes = [vp, vp, vp, u64, u32, u64]
    lib.oracle_negacyclic_u64.argtypes = [vp, vp, vp, u64, u64, u64]
    lib.oracle_negacyclic_rns_u32.argtypes = [vp, vp, vp, u64, vp, u32, u64]
    lib.oracle_negacyclic_u32_sample.argtypes = [vp, vp, u64, u32, vp, vp, u64, vp]
    lib.oracle_negacyclic_u64_sample.argtypes = [vp, vp, u64, u64, vp, vp, u64, vp]
    lib.oracle_cyclic_u32.argtypes = [vp, vp, vp, u64, u32, u64]
    lib.oracle_cyclic_u64.argtypes = [vp, vp, vp, u64, u64, u64]
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    for f in (lib.oracle_negacyclic_u32, lib.oracle_negacyclic_u64, lib.oracle_negacyclic_rns_u32,
              lib.oracle_negacyclic_u32_sample, lib.oracle_negacyclic_u64_sample, lib.oracle_cyclic_u32, lib.oracle_cyclic_u64):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(x):
    return ctypes.c_void_p(x.ctypes.data)


def _as(x, dtype):
    return np.ascontiguousarray(np.asarray(x).astype(dtype, copy=False))


def set_threads(threads):
    """OpenMP threads for the following calls (0 leaves it); returns the previous count."""
    return _load().oracle_set_threads(int(threads))


def negacyclic(a, b, q):
    """c = a*b in Z_q[x]/(x^n+1) for arrays [..., n]; uint32 words if q < 2^32, else uint64."""
    q = int(q)
    wide = q >= (1 << 32)
    dt = np.uint64 if wide else np.uint32
    a = _as(a, dt)
    b = _as(b, dt)
    if a.shape != b.shape or a.ndim < 1:
        raise ValueError("a and b must have the same shape [..., n]")
    n = a.shape[-1]
    batch = a.size // n if n else 0
    c = np.empty_like(a)
    lib = _load()
    fn = lib.oracle_negacyclic_u64 if wide else lib.oracle_negacyclic_u32
    if fn(_ptr(a), _ptr(b), _ptr(c), n, q, batch) != 0:
        raise ValueError("oracle rejected arguments (n >= 1, q >= 2)")
    return c


def cyclic(a, b, q):
    """c = a*b in Z_q[x]/(x^n-1) (Sec. 2.1's other ring); uint32 words if q < 2^32, else uint64."""
    q = int(q)
    wide = q >= (1 << 32)
    dt = np.uint64 if wide else np.uint32
    a = _as(a, dt)
    b = _as(b, dt)
    if a.shape != b.shape or a.ndim < 1:
        raise ValueError("a and b must have the same shape [..., n]")
    n = a.shape[-1]
    batch = a.size // n if n else 0
    c = np.empty_like(a)
    lib = _load()
    fn = lib.oracle_cyclic_u64 if wide else lib.oracle_cyclic_u32
    if fn(_ptr(a), _ptr(b), _ptr(c), n, q, batch) != 0:
        raise ValueError("oracle rejected arguments (n >= 1, q >= 2)")
    return c


def negacyclic_rns(a, b, qs):
    """RNS form: a, b are uint32 [batch, L, n]; channel l is reduced mod qs[l] (Sec. 2.4)."""
    qs = np.ascontiguousarray(np.asarray(qs, dtype=np.uint32))
    a = _as(a, np.uint32)
    b = _as(b, np.uint32)
    if a.shape != b.shape or a.ndim != 3 or a.shape[1] != qs.size:
        raise ValueError("a, b must be [batch, L, n] with L == len(qs)")
    batch, L, n = a.shape
    c = np.empty_like(a)
    if _load().oracle_negacyclic_rns_u32(_ptr(a), _ptr(b), _ptr(c), n, _ptr(qs), L, batch) != 0:
        raise ValueError("oracle rejected arguments")
    return c


def negacyclic_sample(a, b, q, pidx, jidx):
    """Coefficients c[pidx[s], jidx[s]] only, for a, b of shape [batch, n]."""
    q = int(q)
    wide = q >= (1 << 32)
    dt = np.uint64 if wide else np.uint32
    a = _as(a, dt)
    b = _as(b, dt)
    n = a.shape[-1]
    a = a.reshape(-1, n)
    b = b.reshape(-1, n)
    pidx = _as(pidx, np.uint64)
    jidx = _as(jidx, np.uint64)
    if pidx.shape != jidx.shape:
        raise ValueError("pidx and jidx must have the same shape")
    if pidx.size and int(pidx.max()) >= a.shape[0]:
        raise ValueError("pidx out of range")
    out = np.empty(pidx.shape, dtype=dt)
    lib = _load()
    fn = lib.oracle_negacyclic_u64_sample if wide else lib.oracle_negacyclic_u32_sample
    if fn(_ptr(a), _ptr(b), n, q, _ptr(pidx), _ptr(jidx), pidx.size, _ptr(out)) != 0:
        raise ValueError("oracle rejected arguments")
    return out
