"""ctypes binding of libpolymul.so: argument marshalling only.

Each function has the name of the C entry point it calls.  Tensors are torch
device tensors used as plain device memory (int32/uint32 for 32-bit words,
int64/uint64 for 64-bit words, reinterpreted bit for bit); the call is queued
on torch's current stream.  Every step of the product runs in the library's
HIP kernels; there is no CPU fallback: a missing library raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libpolymul.so"
_lib = None

STATUS = {0: "POLYMUL_OK", 1: "POLYMUL_EINVAL", 2: "POLYMUL_EALIAS", 3: "POLYMUL_EUNSUPPORTED",
          4: "POLYMUL_ENOMEM", 5: "POLYMUL_EDEVICE", 6: "POLYMUL_ESCRATCH"}
POLYMUL_NOALLOC_SCRATCH_BYTES = 64 << 20
POLYMUL_PLAN_NO_GRAPH = 1

# name -> (restype, argtypes) exactly as declared in include/polymul.h
_vp, _u32, _u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
_SIGNATURES = {
    "polymul_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "polymul_negacyclic": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u32, _u64, _vp]),
    "polymul_negacyclic_u64": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u64, _u64, _vp]),
    "polymul_negacyclic_rns": (ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _u32, _u64, _vp]),
    "polymul_negacyclic_plain": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u32, _u64, _vp]),
    "polymul_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), _vp, _u32, _u32]),
    "polymul_plan_execute": (ctypes.c_int, [_vp, _vp]),
    "polymul_plan_destroy": (ctypes.c_int, [_vp]),
    "polymul_cyclic": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u32, _u64, _vp]),
    "polymul_cyclic_u64": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u64, _u64, _vp]),
    "polymul_tune_set": (ctypes.c_int, [_u64, _u32, _u32]),
    "polymul_negacyclic_crt": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u32, _u64, _vp]),
    "polymul_negacyclic_rns_crt": (ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _u32, _u64, _vp]),
    "polymul_crt_moduli": (ctypes.c_int, [_u64, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_u32)]),
    "polymul_negacyclic_shared": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u32, _u64, _vp]),
    "polymul_negacyclic_rns_shared": (ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _u32, _u64, _vp]),
    "polymul_negacyclic_u64_shared": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u64, _u64, _vp]),
    "polymul_karatsuba_u64_workspace_size": (ctypes.c_int, [_u64, _u64, _u32, ctypes.POINTER(_u64)]),
    "polymul_negacyclic_u64_karatsuba": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u64, _u64, _u32, _vp, _u64, _vp]),
    "polymul_karatsuba_workspace_size": (ctypes.c_int, [_u64, _u32, _u64, _u32, ctypes.POINTER(_u64)]),
    "polymul_negacyclic_rns_karatsuba": (ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _u32, _u64, _u32, _vp, _u64,
                                                        _vp]),
    "polymul_tune_get": (ctypes.c_int, [_u64, _u32, ctypes.POINTER(_u32)]),
    "polymul_negacyclic_rns_karatsuba_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _u32, _u64, _u32, _vp]),
    "polymul_tune_param_set": (ctypes.c_int, [_u32, _u64]),
    "polymul_tune_param_get": (ctypes.c_int, [_u32, ctypes.POINTER(_u64)]),
    "polymul_tune_set_karatsuba": (ctypes.c_int, [_u64, _u64, _u32, _u32]),
    "polymul_tune_get_karatsuba": (ctypes.c_int, [_u64, _u64, _u32, ctypes.POINTER(_u32)]),
}
TUNE_PARAMS = {"plan_share_pct": 1, "plan_stream_pct": 2, "u64_karatsuba_runs": 3}
KARATSUBA_BUILTIN = 0xFF


class PolymulError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class _Group(ctypes.Structure):
    _fields_ = [("a", _vp), ("b", _vp), ("c", _vp), ("n", _u64), ("q", _u64), ("count", _u64),
                ("elem_bytes", _u32)]


def lib_path():
    return os.path.join(_HERE, _LIB_NAME)


def load_library():
    """Load libpolymul.so (built in-tree by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its HIP runtime must be the one the library binds to, so that
    # the library's launches and torch's memory and streams share one runtime
    import torch  # noqa: F401
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def polymul_status_string(status):
    return load_library().polymul_status_string(int(status)).decode()


def _check(status, where):
    if status != 0:
        raise PolymulError(status, where)


def _stream(stream):
    """The HIP stream to launch on: `stream`, else torch's current stream on the current
    device (read as a raw handle: building a torch Stream object costs ~3 us a call)."""
    import torch
    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            dev = getattr(torch._C, "_cuda_getDevice", torch.cuda.current_device)
            return ctypes.c_void_p(raw(dev()))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


_INT_WORDS = {}  # bytes per word -> the integer dtypes of that width


def _int_dtypes(nbytes):
    if nbytes not in _INT_WORDS:
        import torch
        cands = [getattr(torch, n, None) for n in ("int8", "uint8", "int16", "uint16", "int32", "uint32",
                                                   "int64", "uint64")]
        _INT_WORDS[nbytes] = frozenset(d for d in cands if d is not None and d.itemsize == nbytes)
    return _INT_WORDS[nbytes]


def _words(t, nbytes, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype not in _int_dtypes(nbytes):
        raise TypeError(f"{name} must hold {8 * nbytes}-bit integer words")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _result(out, like, nbytes, name="out"):
    """`out` checked against the result it must hold (the shape of `like`, words of
    `nbytes` bytes), or a new tensor like `like`.  The C ABI carries no buffer
    sizes, so an undersized output would be written past its end: refuse it here."""
    import torch
    if out is None:
        return torch.empty_like(like)
    if not isinstance(out, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if tuple(out.shape) != tuple(like.shape):
        raise ValueError(f"{name} has shape {tuple(out.shape)}, the result needs {tuple(like.shape)}")
    if out.dtype not in _int_dtypes(nbytes):
        raise ValueError(f"{name} must hold {8 * nbytes}-bit integer words")
    return out


def _pair(a, b):
    """a and b of one shape [..., n]; returns (n, batch)."""
    if a.shape != b.shape or a.dim() < 1:
        raise ValueError("a and b must have the same shape [..., n]")
    n = a.shape[-1]
    return n, (a.numel() // n if n else 0)


def _rns_shape(a, b, qs):
    """a and b of one shape [batch, L, n] with one modulus per channel; returns (batch, L, n)."""
    if a.shape != b.shape or a.dim() != 3:
        raise ValueError("a and b must be [batch, L, n]")
    batch, L, n = a.shape
    if len(qs) != L:
        raise ValueError("need one modulus per channel")
    return batch, L, n


def polymul_negacyclic(a, b, q, out=None, stream=None):
    """c = a*b in Z_q[x]/(x^n+1) for 32-bit words [..., n], q < 2^32 (int8-MFMA path)."""
    n, batch = _pair(a, b)
    c = _result(out, a, 4)
    st = load_library().polymul_negacyclic(_words(a, 4, "a"), _words(b, 4, "b"), _words(c, 4, "out"),
                                          n, int(q), batch, _stream(stream))
    _check(st, "polymul_negacyclic")
    return c


def polymul_negacyclic_plain(a, b, q, out=None, stream=None):
    """Same product with the plain integer schoolbook kernel (baseline)."""
    n, batch = _pair(a, b)
    c = _result(out, a, 4)
    st = load_library().polymul_negacyclic_plain(_words(a, 4, "a"), _words(b, 4, "b"), _words(c, 4, "out"),
                                                n, int(q), batch, _stream(stream))
    _check(st, "polymul_negacyclic_plain")
    return c


def polymul_negacyclic_u64(a, b, q, out=None, stream=None):
    """c = a*b in Z_q[x]/(x^n+1) for 64-bit words [..., n], q < 2^64."""
    n, batch = _pair(a, b)
    c = _result(out, a, 8)
    st = load_library().polymul_negacyclic_u64(_words(a, 8, "a"), _words(b, 8, "b"), _words(c, 8, "out"),
                                              n, int(q), batch, _stream(stream))
    _check(st, "polymul_negacyclic_u64")
    return c


def _binary(name, a, b, q, out, stream, nbytes):
    n, batch = _pair(a, b)
    c = _result(out, a, nbytes)
    st = getattr(load_library(), name)(_words(a, nbytes, "a"), _words(b, nbytes, "b"), _words(c, nbytes, "out"),
                                       n, int(q), batch, _stream(stream))
    _check(st, name)
    return c


def polymul_cyclic(a, b, q, out=None, stream=None):
    """c = a*b in Z_q[x]/(x^n-1) for 32-bit words [..., n], q < 2^32."""
    return _binary("polymul_cyclic", a, b, q, out, stream, 4)


def polymul_cyclic_u64(a, b, q, out=None, stream=None):
    """c = a*b in Z_q[x]/(x^n-1) for 64-bit words [..., n], q < 2^64."""
    return _binary("polymul_cyclic_u64", a, b, q, out, stream, 8)


def polymul_negacyclic_rns(a, b, qs, out=None, stream=None):
    """RNS form: a, b are 32-bit words [batch, L, n]; channel l is taken mod qs[l]."""
    batch, L, n = _rns_shape(a, b, qs)
    c = _result(out, a, 4)
    qarr = (ctypes.c_uint32 * L)(*[int(x) for x in qs])
    st = load_library().polymul_negacyclic_rns(_words(a, 4, "a"), _words(b, 4, "b"), _words(c, 4, "out"),
                                              n, ctypes.cast(qarr, ctypes.c_void_p), L, batch, _stream(stream))
    _check(st, "polymul_negacyclic_rns")
    return c


def polymul_negacyclic_crt(a, b, q, out=None, stream=None):
    """c = a*b in Z_q[x]/(x^n+1) through small-modulus residues and the CRT (32-bit words, n <= 4096)."""
    return _binary("polymul_negacyclic_crt", a, b, q, out, stream, 4)


def polymul_negacyclic_rns_crt(a, b, qs, out=None, stream=None):
    """RNS form [batch, L, n] of polymul_negacyclic_crt; channel l is taken mod qs[l]."""
    batch, L, n = _rns_shape(a, b, qs)
    c = _result(out, a, 4)
    qarr = (ctypes.c_uint32 * L)(*[int(x) for x in qs])
    st = load_library().polymul_negacyclic_rns_crt(_words(a, 4, "a"), _words(b, 4, "b"), _words(c, 4, "out"),
                                                  n, ctypes.cast(qarr, ctypes.c_void_p), L, batch, _stream(stream))
    _check(st, "polymul_negacyclic_rns_crt")
    return c


def polymul_crt_moduli(n, q):
    """The small co-prime moduli polymul_negacyclic_crt uses for (n, q), largest first."""
    arr = (ctypes.c_uint32 * 11)()
    cnt = ctypes.c_uint32()
    _check(load_library().polymul_crt_moduli(int(n), int(q), arr, ctypes.byref(cnt)), "polymul_crt_moduli")
    return [int(arr[i]) for i in range(cnt.value)]


def _shared(name, a, b, q, out, stream, nbytes):
    if a.dim() < 1 or b.dim() != 1 or b.shape[0] != a.shape[-1]:
        raise ValueError("a must be [..., n] and b [n]")
    n = a.shape[-1]
    batch = a.numel() // n if n else 0
    c = _result(out, a, nbytes)
    st = getattr(load_library(), name)(_words(a, nbytes, "a"), _words(b, nbytes, "b"), _words(c, nbytes, "out"),
                                       n, int(q), batch, _stream(stream))
    _check(st, name)
    return c


def polymul_negacyclic_shared(a, b, q, out=None, stream=None):
    """c[i] = a[i] * b in Z_q[x]/(x^n+1): a is [..., n], b one [n] polynomial (32-bit words)."""
    return _shared("polymul_negacyclic_shared", a, b, q, out, stream, 4)


def polymul_negacyclic_u64_shared(a, b, q, out=None, stream=None):
    """As polymul_negacyclic_shared for 64-bit words, q < 2^64."""
    return _shared("polymul_negacyclic_u64_shared", a, b, q, out, stream, 8)


def polymul_negacyclic_rns_shared(a, b, qs, out=None, stream=None):
    """RNS form with one b per channel: a is [batch, L, n], b is [L, n]."""
    if a.dim() != 3 or b.dim() != 2 or b.shape != a.shape[1:]:
        raise ValueError("a must be [batch, L, n] and b [L, n]")
    batch, L, n = a.shape
    if len(qs) != L:
        raise ValueError("need one modulus per channel")
    c = _result(out, a, 4)
    qarr = (ctypes.c_uint32 * L)(*[int(x) for x in qs])
    st = load_library().polymul_negacyclic_rns_shared(_words(a, 4, "a"), _words(b, 4, "b"), _words(c, 4, "out"),
                                                     n, ctypes.cast(qarr, ctypes.c_void_p), L, batch,
                                                     _stream(stream))
    _check(st, "polymul_negacyclic_rns_shared")
    return c


def polymul_karatsuba_workspace_size(n, L, batch, depth):
    """Bytes of device workspace polymul_negacyclic_rns_karatsuba needs."""
    out = ctypes.c_uint64()
    _check(load_library().polymul_karatsuba_workspace_size(int(n), int(L), int(batch), int(depth),
                                                           ctypes.byref(out)), "polymul_karatsuba_workspace_size")
    return out.value


def polymul_negacyclic_rns_karatsuba(a, b, qs, depth, workspace=None, out=None, stream=None):
    """polymul_negacyclic_rns through `depth` Karatsuba levels.  workspace: a device
    tensor of at least polymul_karatsuba_workspace_size bytes (allocated here if None)."""
    import torch
    batch, L, n = _rns_shape(a, b, qs)
    c = _result(out, a, 4)
    need = polymul_karatsuba_workspace_size(n, L, batch, depth)
    if workspace is None:
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=a.device)
    ws_bytes = workspace.numel() * workspace.element_size()  # depth 0 may need none
    qarr = (ctypes.c_uint32 * L)(*[int(x) for x in qs])
    st = load_library().polymul_negacyclic_rns_karatsuba(
        _words(a, 4, "a"), _words(b, 4, "b"), _words(c, 4, "out"), n, ctypes.cast(qarr, ctypes.c_void_p), L,
        batch, int(depth), ctypes.c_void_p(workspace.data_ptr()), ws_bytes, _stream(stream))
    _check(st, "polymul_negacyclic_rns_karatsuba")
    return c


def polymul_negacyclic_rns_karatsuba_noalloc(a, b, qs, depth, out=None, stream=None):
    """polymul_negacyclic_rns_karatsuba with the library's own per-GPU scratch as the
    workspace (no allocation in the call; calls on one GPU must not overlap)."""
    batch, L, n = _rns_shape(a, b, qs)
    c = _result(out, a, 4)
    qarr = (ctypes.c_uint32 * L)(*[int(x) for x in qs])
    st = load_library().polymul_negacyclic_rns_karatsuba_noalloc(
        _words(a, 4, "a"), _words(b, 4, "b"), _words(c, 4, "out"), n, ctypes.cast(qarr, ctypes.c_void_p), L,
        batch, int(depth), _stream(stream))
    _check(st, "polymul_negacyclic_rns_karatsuba_noalloc")
    return c


def polymul_karatsuba_u64_workspace_size(n, batch, depth):
    """Bytes of device workspace polymul_negacyclic_u64_karatsuba needs."""
    out = ctypes.c_uint64()
    _check(load_library().polymul_karatsuba_u64_workspace_size(int(n), int(batch), int(depth), ctypes.byref(out)),
           "polymul_karatsuba_u64_workspace_size")
    return out.value


def polymul_negacyclic_u64_karatsuba(a, b, q, depth, workspace=None, out=None, stream=None):
    """polymul_negacyclic_u64 through `depth` Karatsuba levels (64-bit words [..., n])."""
    import torch
    n, batch = _pair(a, b)
    c = _result(out, a, 8)
    need = polymul_karatsuba_u64_workspace_size(n, batch, depth)
    if workspace is None:
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=a.device)
    st = load_library().polymul_negacyclic_u64_karatsuba(
        _words(a, 8, "a"), _words(b, 8, "b"), _words(c, 8, "out"), n, int(q), batch, int(depth),
        ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(), _stream(stream))
    _check(st, "polymul_negacyclic_u64_karatsuba")
    return c


def polymul_plan_create(groups, flags=0):
    """groups: list of (a, b, c, n, q) device tensors [count, n] (32- or 64-bit words).
    Returns an opaque plan handle (ctypes c_void_p)."""
    arr = (_Group * max(1, len(groups)))()
    for i, (a, b, c, n, q) in enumerate(groups):
        eb = a.element_size()
        if eb not in (4, 8):
            raise ValueError(f"group {i}: words must be 32 or 64 bits")
        if int(n) < 1 or a.numel() % int(n):
            raise ValueError(f"group {i}: a does not hold whole polynomials of degree bound {n}")
        if b.shape != a.shape or c.shape != a.shape:
            raise ValueError(f"group {i}: a, b and c must have the same shape")
        if b.element_size() != eb or c.element_size() != eb:
            raise ValueError(f"group {i}: a, b and c must hold words of the same size")
        count = a.numel() // n
        arr[i] = _Group(_words(a, eb, "a").value, _words(b, eb, "b").value, _words(c, eb, "c").value,
                        int(n), int(q), int(count), eb)
    handle = ctypes.c_void_p()
    st = load_library().polymul_plan_create(ctypes.byref(handle), ctypes.cast(arr, ctypes.c_void_p),
                                           len(groups), int(flags))
    _check(st, "polymul_plan_create")
    return handle


def polymul_plan_execute(plan, stream=None):
    _check(load_library().polymul_plan_execute(plan, _stream(stream)), "polymul_plan_execute")


def polymul_plan_destroy(plan):
    _check(load_library().polymul_plan_destroy(plan), "polymul_plan_destroy")


def polymul_tune_set(n, L, t):
    """Set the Toeplitz tile side of the resident 32-bit path for (n, L); 0 = built-in."""
    _check(load_library().polymul_tune_set(int(n), int(L), int(t)), "polymul_tune_set")


def polymul_tune_param_set(name, value):
    """Set a plan scheduling knob by name (see TUNE_PARAMS)."""
    _check(load_library().polymul_tune_param_set(TUNE_PARAMS[name], int(value)), "polymul_tune_param_set")


def polymul_tune_param_get(name):
    out = ctypes.c_uint64()
    _check(load_library().polymul_tune_param_get(TUNE_PARAMS[name], ctypes.byref(out)), "polymul_tune_param_get")
    return out.value


def polymul_tune_set_karatsuba(n, products, elem_bytes, depth):
    """Karatsuba depth that depth 0 resolves to for (n, products) and word size; 0xFF = built-in."""
    _check(load_library().polymul_tune_set_karatsuba(int(n), int(products), int(elem_bytes), int(depth)),
           "polymul_tune_set_karatsuba")


def polymul_tune_get_karatsuba(n, products, elem_bytes):
    out = ctypes.c_uint32()
    _check(load_library().polymul_tune_get_karatsuba(int(n), int(products), int(elem_bytes), ctypes.byref(out)),
           "polymul_tune_get_karatsuba")
    return out.value


def polymul_tune_get(n, L):
    out = ctypes.c_uint32()
    _check(load_library().polymul_tune_get(int(n), int(L), ctypes.byref(out)), "polymul_tune_get")
    return out.value


class Plan:
    """Owning wrapper: keeps the tensors alive as long as the plan."""

    def __init__(self, groups, flags=0):
        self._groups = list(groups)
        self.handle = polymul_plan_create(self._groups, flags)

    def execute(self, stream=None):
        polymul_plan_execute(self.handle, stream)

    def close(self):
        if self.handle is not None and self.handle.value:
            polymul_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
