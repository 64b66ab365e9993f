"""CPU FP64 oracle for the binary tensor contraction (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does; the
two share no code.  The arithmetic lives in ``oracle.c`` (plain nested loops,
double precision, no FMA contraction); this module only marshals numpy arrays
into it and derives the gradient specs.

What is computed: the contraction of Section 2 (the summation over the indices
shared by both inputs), scaled by alpha as in the ta.tc operation of
Section 5, plus beta times the previous output (the "=", "+=", "-=" forms of
the Fig. 2 operation grammar).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ERRORS = {1: "invalid spec", 2: "invalid shape", 4: "null pointer", 5: "point out of range"}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = bind(ctypes.CDLL(_LIB))
    return _lib


def bind(lib):
    """Declare the C signatures on a loaded liboracle (also used on rebuilt copies)."""
    P = ctypes.c_void_p
    D = ctypes.c_double
    I64 = ctypes.c_int64
    lib.oracle_contract.argtypes = [ctypes.c_char_p, D, P, P, P, P, P, P, D, P, P, P, ctypes.c_int]
    lib.oracle_contract.restype = ctypes.c_int
    lib.oracle_contract_points.argtypes = [ctypes.c_char_p, D, P, P, P, P, P, P, D, P, P, P,
                                           I64, P, P, ctypes.c_int]
    lib.oracle_contract_points.restype = ctypes.c_int
    lib.oracle_bruteforce.argtypes = [ctypes.c_char_p, D, P, P, P, P, P, P, D, P, P, P, P]
    lib.oracle_bruteforce.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def split_spec(spec: str):
    """'abij=acik*cbkj' -> ('abij', 'acik', 'cbkj'), blanks removed."""
    s = "".join(spec.split())
    lhs, rhs = s.split("=")
    a, b = rhs.split("*")
    return lhs, a, b


def output_shape(spec: str, A: np.ndarray, B: np.ndarray):
    c, a, b = split_spec(spec)
    ext = {}
    for labels, arr in ((a, A), (b, B)):
        for ch, n in zip(labels, arr.shape):
            ext[ch] = n
    return tuple(ext[ch] for ch in c)


class OracleError(RuntimeError):
    pass


def _as_f64(x):
    """Widen to float64 exactly, keeping a strided layout (element strides >= 0)."""
    x = np.asarray(x)
    if any(s < 0 for s in x.strides):
        x = np.ascontiguousarray(x)
    if x.dtype != np.float64:
        x = x.astype(np.float64, order="K")
    return x


def _meta(x):
    dims = np.ascontiguousarray(np.array(x.shape, dtype=np.int64).reshape(-1))
    strides = np.ascontiguousarray(np.array([s // 8 for s in x.strides], dtype=np.int64).reshape(-1))
    return dims, strides


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _check(rc):
    if rc != 0:
        raise OracleError(ERRORS.get(rc, "error %d" % rc))


def contract(spec, A, B, C0=None, alpha=1.0, beta=0.0, nthreads=0):
    """C = alpha * contract(A, B) + beta * C0, in FP64, as a new dense array."""
    A = _as_f64(A)
    B = _as_f64(B)
    shape = output_shape(spec, A, B)
    if beta != 0.0:
        if C0 is None:
            raise ValueError("beta != 0 needs C0")
        C = np.array(np.asarray(C0, dtype=np.float64), dtype=np.float64, order="C", copy=True)
        if C.shape != shape:
            raise ValueError("C0 shape %s != %s" % (C.shape, shape))
    else:
        C = np.zeros(shape, dtype=np.float64)
    dA, sA = _meta(A)
    dB, sB = _meta(B)
    dC, sC = _meta(C)
    lib = _load()
    rc = lib.oracle_contract(spec.encode(), float(alpha), _ptr(A), _ptr(dA), _ptr(sA),
                             _ptr(B), _ptr(dB), _ptr(sB), float(beta),
                             _ptr(C), _ptr(dC), _ptr(sC), int(nthreads))
    _check(rc)
    return C


def contract_points(spec, A, B, points, C0=None, alpha=1.0, beta=0.0, nthreads=0):
    """alpha*sum + beta*C0 at the given output multi-indices (rows of `points`)."""
    A = _as_f64(A)
    B = _as_f64(B)
    shape = output_shape(spec, A, B)
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int64).reshape(-1, len(shape)))
    out = np.empty(pts.shape[0], dtype=np.float64)
    if beta != 0.0:
        C = _as_f64(C0)
        if C.shape != shape:
            raise ValueError("C0 shape %s != %s" % (C.shape, shape))
    else:
        C = np.zeros((0,), dtype=np.float64)
    dA, sA = _meta(A)
    dB, sB = _meta(B)
    dC = np.array(shape, dtype=np.int64).reshape(-1)
    sC = (np.array([s // 8 for s in C.strides], dtype=np.int64) if beta != 0.0
          else np.zeros(len(shape), dtype=np.int64)).reshape(-1)
    dC = np.ascontiguousarray(dC)
    sC = np.ascontiguousarray(sC)
    lib = _load()
    rc = lib.oracle_contract_points(spec.encode(), float(alpha), _ptr(A), _ptr(dA), _ptr(sA),
                                    _ptr(B), _ptr(dB), _ptr(sB), float(beta),
                                    _ptr(C) if beta != 0.0 else None, _ptr(dC), _ptr(sC),
                                    int(pts.shape[0]), _ptr(pts), _ptr(out), int(nthreads))
    _check(rc)
    return out


def bruteforce(spec, A, B, C0=None, alpha=1.0, beta=0.0):
    """Same result by one odometer over every label tuple (tiny inputs only)."""
    A = _as_f64(A)
    B = _as_f64(B)
    shape = output_shape(spec, A, B)
    if beta != 0.0:
        C = np.array(np.asarray(C0, dtype=np.float64), dtype=np.float64, order="C", copy=True)
    else:
        C = np.zeros(shape, dtype=np.float64)
    acc = np.zeros(max(1, int(np.prod(shape, dtype=np.int64))), dtype=np.float64)
    dA, sA = _meta(A)
    dB, sB = _meta(B)
    dC, sC = _meta(C)
    lib = _load()
    rc = lib.oracle_bruteforce(spec.encode(), float(alpha), _ptr(A), _ptr(dA), _ptr(sA),
                               _ptr(B), _ptr(dB), _ptr(sB), float(beta),
                               _ptr(C), _ptr(dC), _ptr(sC), _ptr(acc))
    _check(rc)
    return C


def grad_specs(spec):
    """Specs of the two input gradients of C = alpha*A*B + beta*C0.

    With L = <dC, C>, dL/dA[..] = alpha * sum over B's free labels of
    dC[..] * B[..]: a contraction whose output carries A's labels and whose
    inputs are dC and B.  Likewise for B.
    """
    c, a, b = split_spec(spec)
    return "%s=%s*%s" % (a, c, b), "%s=%s*%s" % (b, a, c)


def grad(spec, A, B, dC, alpha=1.0, beta=0.0, nthreads=0):
    """(dA, dB, dC0) of L = sum(dC * C) for C = alpha*contract(A,B) + beta*C0."""
    sa, sb = grad_specs(spec)
    dA = contract(sa, dC, B, alpha=alpha, nthreads=nthreads)
    dB = contract(sb, A, dC, alpha=alpha, nthreads=nthreads)
    dC0 = float(beta) * np.asarray(dC, dtype=np.float64)
    return dA, dB, dC0


def relerr(x, ref):
    """Relative Frobenius error ||x - ref|| / ||ref||, accumulated in long double."""
    x = np.asarray(x, dtype=np.longdouble).ravel()
    r = np.asarray(ref, dtype=np.longdouble).ravel()
    num = np.sqrt(np.sum((x - r) ** 2))
    den = np.sqrt(np.sum(r ** 2))
    if den == 0:
        return float(num)
    return float(num / den)
