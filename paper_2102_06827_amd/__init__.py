"""Python binding of libcomet: permuted tensor contractions on MI355X (gfx950).

Argument marshalling only: every step of a contraction runs in the HIP
kernels of libcomet.so, reached through its C ABI (include/comet.h).  There is
no CPU fallback: if the library is missing or cannot load, every call raises.

    import torch, paper_2102_06827_amd as comet
    C = comet.contract("abij=acik*cbkj", A, B)                 # C = A * B
    comet.contract("abij=acik*bkcj", A, B, C, beta=1.0)         # C += A * B

The contraction is the one of Section 2 of the COMET paper (arXiv
2102.06827), with the alpha scaling of its ta.tc operation and the "=", "+=",
"-=" forms of its operation grammar (beta = 0, 1, 1 with -alpha).
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

__all__ = [
    "CometError", "contract", "permute", "analyze", "Plan", "Batch", "ContractFn", "contract_ad",
    "set_split_slices", "set_int8_slices", "autotune", "lib", "library_path", "COMPUTE", "PATH",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcomet.so")

COMPUTE = {"default": 0, "f64": 1, "f32": 2, "split_bf16": 3, "split_bf16x3": 4, "split_fp16x2": 5,
           "split_int8": 6}
PATH = {"auto": 0, "gett": 1, "ttgt": 2}
_DTYPE = {torch.float64: 0, torch.float32: 1}
STATUS = {0: "OK", 1: "INVALID_SPEC", 2: "INVALID_SHAPE", 3: "INVALID_STRIDE", 4: "NULL_POINTER",
          5: "UNSUPPORTED", 6: "WORKSPACE", 7: "HIP", 8: "INTERNAL"}

# exported symbols of include/comet.h
SYMBOLS = [
    "comet_contract", "comet_plan_create", "comet_plan_create_ex", "comet_plan_workspace_size",
    "comet_plan_execute", "comet_plan_destroy", "comet_plan_describe", "comet_analyze",
    "comet_plan_execute_noalloc",
    "comet_batch_create", "comet_batch_workspace_size", "comet_batch_execute", "comet_batch_destroy",
    "comet_batch_describe",
    "comet_permute", "comet_fill", "comet_chain_plan", "comet_contract_chain", "comet_autotune", "comet_set_split_slices", "comet_set_int8_slices", "comet_last_error",
    "comet_version",
]


class CometError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code
        self.name = STATUS.get(code, str(code))


class _Problem(ctypes.Structure):
    _fields_ = [
        ("spec", ctypes.c_char_p),
        ("extents", ctypes.POINTER(ctypes.c_int64)),
        ("strides_A", ctypes.POINTER(ctypes.c_int64)),
        ("strides_B", ctypes.POINTER(ctypes.c_int64)),
        ("strides_C", ctypes.POINTER(ctypes.c_int64)),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("A", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
        ("C", ctypes.c_void_p),
    ]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libcomet (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libcomet.so is not built (run paper_2102_06827_amd/build.py or "
                               "__graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64P = ctypes.POINTER(ctypes.c_int64)
        D = ctypes.c_double
        I = ctypes.c_int
        S = ctypes.c_char_p
        L.comet_contract.argtypes = [S, I64P, I, I, D, P, I64P, P, I64P, D, P, I64P, P]
        L.comet_plan_create.argtypes = [ctypes.POINTER(P), S, I64P, I64P, I64P, I64P, I, I]
        L.comet_plan_create_ex.argtypes = [ctypes.POINTER(P), S, I64P, I64P, I64P, I64P, I, I, I]
        L.comet_plan_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.comet_plan_execute.argtypes = [P, D, P, P, D, P, P, ctypes.c_size_t, P]
        L.comet_plan_destroy.argtypes = [P]
        L.comet_plan_execute_noalloc.argtypes = [P, D, P, P, D, P, P]
        L.comet_plan_describe.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        L.comet_analyze.argtypes = [S, I64P, I64P, I64P, I64P, I, I, I, ctypes.c_char_p, ctypes.c_size_t]
        L.comet_batch_create.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(_Problem), I, I]
        L.comet_batch_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.comet_batch_execute.argtypes = [P, P, ctypes.c_size_t, P]
        L.comet_batch_destroy.argtypes = [P]
        L.comet_batch_describe.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        L.comet_permute.argtypes = [S, I64P, I, D, P, I64P, D, P, I64P, P]
        L.comet_fill.argtypes = [I, I64P, I, D, P, I64P, P]
        L.comet_chain_plan.argtypes = [S, I64P, ctypes.c_char_p, ctypes.c_size_t]
        L.comet_contract_chain.argtypes = [S, I64P, I, I, D, I, ctypes.POINTER(P), ctypes.POINTER(I64P), D, P,
                                           I64P, P]
        L.comet_autotune.argtypes = [S, I]
        L.comet_set_split_slices.argtypes = [I]
        L.comet_set_int8_slices.argtypes = [I]
        L.comet_last_error.restype = ctypes.c_char_p
        L.comet_version.restype = ctypes.c_char_p
        for name in SYMBOLS:
            f = getattr(L, name)
            if name not in ("comet_last_error", "comet_version"):
                f.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise CometError(rc, lib().comet_last_error().decode())


def _i64(seq):
    if seq is None:
        return None
    seq = list(seq)
    return (ctypes.c_int64 * max(1, len(seq)))(*seq)


def split_spec(spec: str):
    s = "".join(spec.split())
    lhs, rhs = s.split("=")
    a, b = rhs.split("*")
    return lhs, a, b


def _labels_in_order(c, a, b):
    seen = []
    for ch in c + a + b:
        if ch not in seen:
            seen.append(ch)
    return seen


def extents_of(spec, A_shape, B_shape):
    """Extents in comet order (first appearance scanning C, A, B) from the input shapes."""
    c, a, b = split_spec(spec)
    ext = {}
    for labs, shp in ((a, A_shape), (b, B_shape)):
        if len(labs) != len(shp):
            raise ValueError("rank of %r does not match shape %s" % (labs, tuple(shp)))
        for ch, n in zip(labs, shp):
            if ch in ext and ext[ch] != n:
                raise ValueError("extent mismatch for label %r: %d vs %d" % (ch, ext[ch], n))
            ext[ch] = int(n)
    missing = [ch for ch in c if ch not in ext]
    if missing:
        raise ValueError("labels %s of C appear in neither input" % missing)
    return [ext[ch] for ch in _labels_in_order(c, a, b)], tuple(ext[ch] for ch in c)


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(*ts):
    dt = ts[0].dtype
    for t in ts:
        if t.dtype != dt:
            raise TypeError("A, B and C must share one dtype (got %s)" % [x.dtype for x in ts])
        if not t.is_cuda:
            raise TypeError("tensors must be on the GPU (device memory); there is no CPU path")
    if dt not in _DTYPE:
        raise TypeError("dtype %s not supported (float64 or float32)" % dt)
    return _DTYPE[dt]


# Marshalled call arguments of comet_contract by (spec, shapes, strides):
# repeated calls on same-shaped tensors skip the label bookkeeping.
_ARGS_CACHE = {}
_ARGS_CACHE_MAX = 256


def _contract_args(spec, A, B, C):
    key = (spec, tuple(A.shape), A.stride(), tuple(B.shape), B.stride(), None if C is None else (tuple(C.shape), C.stride()))
    hit = _ARGS_CACHE.get(key)
    if hit is not None:
        return hit
    ext, cshape = extents_of(spec, A.shape, B.shape)
    if C is not None and tuple(C.shape) != cshape:
        raise ValueError("C shape %s != %s" % (tuple(C.shape), cshape))
    val = (spec.encode(), _i64(ext), cshape, _i64(A.stride()), _i64(B.stride()),
           None if C is None else _i64(C.stride()))
    if len(_ARGS_CACHE) >= _ARGS_CACHE_MAX:
        _ARGS_CACHE.clear()
    _ARGS_CACHE[key] = val
    return val


def contract(spec, A, B, C=None, alpha=1.0, beta=0.0, compute="default", stream=None):
    """C = alpha * contract(A, B) + beta * C  (C allocated when None).

    A, B (and C) are CUDA/HIP torch tensors of one dtype, any strides >= 0.
    """
    spec_b, ext, cshape, sa, sb, sc = _contract_args(spec, A, B, C)
    if C is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs C")
        C = torch.empty(cshape, dtype=A.dtype, device=A.device)
        sc = _i64(C.stride())
    dt = _dtype_code(A, B, C)
    rc = lib().comet_contract(spec_b, ext, dt, COMPUTE[compute], float(alpha),
                              ctypes.c_void_p(A.data_ptr()), sa,
                              ctypes.c_void_p(B.data_ptr()), sb, float(beta),
                              ctypes.c_void_p(C.data_ptr()), sc, _stream_handle(stream))
    _check(rc)
    return C


def permute(spec, x, out=None, alpha=1.0, beta=0.0, stream=None):
    """out = alpha * x with labels permuted ("ji=ij") + beta * out."""
    s = "".join(spec.split())
    lo, li = s.split("=")
    if len(li) != x.dim():
        raise ValueError("rank mismatch")
    ext_in = dict(zip(li, x.shape))
    ext = [int(ext_in[ch]) for ch in lo]
    if out is None:
        out = torch.empty(tuple(ext), dtype=x.dtype, device=x.device)
    dt = _dtype_code(x, out)
    rc = lib().comet_permute(s.encode(), _i64(ext), dt, float(alpha), ctypes.c_void_p(x.data_ptr()),
                             _i64(x.stride()), float(beta), ctypes.c_void_p(out.data_ptr()),
                             _i64(out.stride()), _stream_handle(stream))
    _check(rc)
    return out


def _chain_parts(spec):
    s = "".join(spec.split())
    out, rhs = s.split("=")
    return out, rhs.split("*")


def chain_labels(spec):
    """Distinct labels of a chain spec in order of first appearance (C, then A1..An)."""
    out, ops = _chain_parts(spec)
    seen = []
    for t in [out] + ops:
        for ch in t:
            if ch not in seen:
                seen.append(ch)
    return seen


def chain_plan(spec, extents):
    """Host-only: the grouping of a multi-operand chain with the fewest
    operations.  extents: dict label -> extent, or a list in chain_labels order."""
    if isinstance(extents, dict):
        extents = [extents[ch] for ch in chain_labels(spec)]
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().comet_chain_plan(spec.encode(), _i64(extents), buf, len(buf)))
    return json.loads(buf.value.decode())


def contract_chain(spec, tensors, C=None, alpha=1.0, beta=0.0, compute="default", stream=None):
    """C = alpha * (A1 * ... * An) + beta * C for spec "C=A1*...*An", in the
    order with the fewest operations (intermediates held by the library)."""
    out, ops = _chain_parts(spec)
    if len(ops) != len(tensors):
        raise ValueError("spec has %d operands, %d tensors given" % (len(ops), len(tensors)))
    ext = {}
    for labels, t in zip(ops, tensors):
        if len(labels) != t.dim():
            raise ValueError("rank mismatch for operand " + labels)
        for ch, e in zip(labels, t.shape):
            if ext.setdefault(ch, int(e)) != int(e):
                raise ValueError("extent mismatch for label " + ch)
    if C is None:
        C = torch.empty(tuple(ext[ch] for ch in out), dtype=tensors[0].dtype, device=tensors[0].device)
    dt = _dtype_code(*(list(tensors) + [C]))
    n = len(tensors)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in tensors])
    strs = [_i64(t.stride()) for t in tensors]
    sarr = (ctypes.POINTER(ctypes.c_int64) * n)(*[ctypes.cast(x, ctypes.POINTER(ctypes.c_int64)) for x in strs])
    rc = lib().comet_contract_chain(spec.encode(), _i64([ext[ch] for ch in chain_labels(spec)]), dt,
                                    COMPUTE[compute], float(alpha), n, ptrs, sarr, float(beta),
                                    ctypes.c_void_p(C.data_ptr()), _i64(C.stride()), _stream_handle(stream))
    _check(rc)
    return C


def fill(x, value, stream=None):
    """Set every element of the tensor x (any strides) to value; returns x."""
    dt = _dtype_code(x, x)
    rc = lib().comet_fill(x.dim(), _i64(list(x.shape)), dt, float(value), ctypes.c_void_p(x.data_ptr()),
                          _i64(list(x.stride())), _stream_handle(stream))
    _check(rc)
    return x


def analyze(spec, extents, strides_A=None, strides_B=None, strides_C=None, dtype="f64", compute="default",
            path="auto"):
    """Host-only planning (no device needed): returns the planner's decisions as a dict."""
    buf = ctypes.create_string_buffer(1 << 16)
    dt = {"f64": 0, "f32": 1}[dtype]
    rc = lib().comet_analyze(spec.encode(), _i64(extents), _i64(strides_A), _i64(strides_B), _i64(strides_C),
                             dt, COMPUTE[compute], PATH[path], buf, len(buf))
    _check(rc)
    return json.loads(buf.value.decode())


def analyze_status(spec, extents, strides_A=None, strides_B=None, strides_C=None, dtype=0, compute=0, path=0):
    """The raw status code of comet_analyze (for validation tests)."""
    buf = ctypes.create_string_buffer(1 << 16)
    return lib().comet_analyze(None if spec is None else spec.encode(), _i64(extents), _i64(strides_A),
                               _i64(strides_B), _i64(strides_C), dtype, compute, path, buf, len(buf))


def set_split_slices(S: int):
    _check(lib().comet_set_split_slices(int(S)))


def set_int8_slices(S: int):
    _check(lib().comet_set_int8_slices(int(S)))


def autotune(cache_path=None, mode=1):
    _check(lib().comet_autotune(None if cache_path is None else cache_path.encode(), int(mode)))


class Plan:
    """A planned contraction for fixed shapes/strides (capturable execute)."""

    def __init__(self, spec, A_like, B_like, C_like=None, compute="default", path="auto"):
        ext, cshape = extents_of(spec, A_like.shape, B_like.shape)
        self.spec = spec
        self.cshape = cshape
        self.dtype = A_like.dtype
        dt = _DTYPE[A_like.dtype]
        sc = None if C_like is None else C_like.stride()
        self._h = ctypes.c_void_p()
        _check(lib().comet_plan_create_ex(ctypes.byref(self._h), spec.encode(), _i64(ext), _i64(A_like.stride()),
                                          _i64(B_like.stride()), _i64(sc), dt, COMPUTE[compute], PATH[path]))
        n = ctypes.c_size_t()
        _check(lib().comet_plan_workspace_size(self._h, ctypes.byref(n)))
        self.workspace_bytes = n.value
        self._ws = None

    def describe(self):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().comet_plan_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def workspace(self, device):
        if self.workspace_bytes and (self._ws is None or self._ws.device != device):
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        return self._ws

    def __call__(self, A, B, C=None, alpha=1.0, beta=0.0, workspace=None, stream=None):
        if C is None:
            C = torch.empty(self.cshape, dtype=A.dtype, device=A.device)
        _dtype_code(A, B, C)
        ws = workspace if workspace is not None else self.workspace(A.device)
        wp = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
        wn = ws.numel() * ws.element_size() if ws is not None else 0
        _check(lib().comet_plan_execute(self._h, float(alpha), ctypes.c_void_p(A.data_ptr()),
                                        ctypes.c_void_p(B.data_ptr()), float(beta),
                                        ctypes.c_void_p(C.data_ptr()), wp, wn, _stream_handle(stream)))
        return C

    def execute_noalloc(self, A, B, C, alpha=1.0, beta=0.0, stream=None):
        """The same contraction with the library's static device buffer as
        workspace: nothing is allocated (C must be given)."""
        _dtype_code(A, B, C)
        _check(lib().comet_plan_execute_noalloc(self._h, float(alpha), ctypes.c_void_p(A.data_ptr()),
                                                ctypes.c_void_p(B.data_ptr()), float(beta),
                                                ctypes.c_void_p(C.data_ptr()), _stream_handle(stream)))
        return C

    def __del__(self):
        try:
            if self._h:
                lib().comet_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


class Batch:
    """Many independent contractions executed by one persistent launch."""

    def __init__(self, problems, dtype=torch.float32, compute="default"):
        """problems: list of dicts with spec, A, B, C, alpha (1.0), beta (0.0)."""
        self._keep = []
        arr = (_Problem * len(problems))()
        for i, pr in enumerate(problems):
            A, B, C = pr["A"], pr["B"], pr["C"]
            ext, cshape = extents_of(pr["spec"], A.shape, B.shape)
            if tuple(C.shape) != cshape:
                raise ValueError("problem %d: C shape %s != %s" % (i, tuple(C.shape), cshape))
            _dtype_code(A, B, C)
            spec_b = pr["spec"].encode()
            e, sa, sb, sc = _i64(ext), _i64(A.stride()), _i64(B.stride()), _i64(C.stride())
            self._keep += [spec_b, e, sa, sb, sc]
            arr[i] = _Problem(spec_b, e, sa, sb, sc, float(pr.get("alpha", 1.0)), float(pr.get("beta", 0.0)),
                              A.data_ptr(), B.data_ptr(), C.data_ptr())
        self._h = ctypes.c_void_p()
        _check(lib().comet_batch_create(ctypes.byref(self._h), len(problems), arr, _DTYPE[dtype], COMPUTE[compute]))
        n = ctypes.c_size_t()
        _check(lib().comet_batch_workspace_size(self._h, ctypes.byref(n)))
        self.workspace_bytes = n.value
        self._ws = None

    def __call__(self, device=None, stream=None, workspace=None):
        ws = workspace
        if ws is None and self.workspace_bytes:
            if self._ws is None:
                self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device or "cuda")
            ws = self._ws
        wp = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
        wn = ws.numel() if ws is not None else 0
        _check(lib().comet_batch_execute(self._h, wp, wn, _stream_handle(stream)))

    def describe(self):
        buf = ctypes.create_string_buffer(1 << 12)
        _check(lib().comet_batch_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def __del__(self):
        try:
            if self._h:
                lib().comet_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass


from .autograd import ContractFn, contract_ad  # noqa: E402
