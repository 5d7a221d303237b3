"""CPU oracle for the count sketch Kaczmarz (CSK) method -- test infrastructure.

Plain, slow, sequential FP64 code in ``csk_oracle.c`` (see its header for what
each function follows in the paper), wrapped here with ctypes and NumPy.  Only
the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product library never does, and this package never touches
the product library.
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK = 0
NOT_CONVERGED = 1
ERR_INVALID_ARG = 2
ERR_NONFINITE = 6
ERR_DEGENERATE = 7

STOP_REL_ERR = 0
STOP_REL_RESID = 1

_lib = None

_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    lib.orc_splitmix64_mix.restype = _u64
    lib.orc_splitmix64_mix.argtypes = [_u64]
    lib.orc_splitmix64_stream.argtypes = [_u64, _i64, _p]
    lib.orc_hash.argtypes = [_u64, _i64, _i64, _p, _p]
    lib.orc_bucket_sort.argtypes = [_p, _i64, _i64, _p, _p]
    lib.orc_sketch_dense_f64.argtypes = [_p, _i64, _i64, _i64, _p, _i64, _i64, _i64, _u64, _p, _i64, _p, _i64]
    lib.orc_sketch_dense_f32.argtypes = lib.orc_sketch_dense_f64.argtypes
    lib.orc_sketch_csr_f32.argtypes = [_p, _p, _p, _i64, _i64, _p, _i64, _u64, _p, _i64, _p]
    lib.orc_sketch_residual_csr.argtypes = [_p, _p, _p, _i64, _p, _p, _i64, _u64, _p]
    for name in ("orc_round_f64_to_f32", "orc_round_f64_to_bf16", "orc_round_f64_to_f16",
                 "orc_round_f32_to_bf16", "orc_round_f32_to_f16"):
        getattr(lib, name).argtypes = [_p, _p, _i64]
    lib.orc_row_norms2.argtypes = [_p, _i64, _i64, _i64, _p]
    lib.orc_mwrk.restype = ctypes.c_int
    lib.orc_mwrk.argtypes = [_p, _i64, _i64, _i64, _p, _p, _p, ctypes.c_double, _i64, ctypes.c_int,
                             _p, _p, _p, _p, _p]
    lib.orc_rgrk.restype = ctypes.c_int
    lib.orc_rgrk.argtypes = [_p, _i64, _i64, _i64, _p, _p, _p, ctypes.c_double, _i64, ctypes.c_int,
                             ctypes.c_double, _u64, _p, _p, _p, _p, _p]
    lib.orc_rk.restype = ctypes.c_int
    lib.orc_rk.argtypes = [_p, _i64, _i64, _i64, _p, _p, _p, ctypes.c_double, _i64, _u64,
                           _p, _p, _p, _p, _p]
    lib.orc_uniform_stream.argtypes = [_u64, _i64, _i64, _p]
    lib.orc_set_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads(1)
    _lib = lib
    return lib


def set_threads(t: int) -> int:
    """Threads for the sketch's bucket ranges and the loop's residual rows
    (bitwise the single-thread results); returns the count in effect."""
    return int(_load().orc_set_threads(int(t)))


class threads:
    """Context manager: run the oracle on t threads, then go back to one."""

    def __init__(self, t: int):
        self.t = t

    def __enter__(self):
        return set_threads(self.t)

    def __exit__(self, *exc):
        set_threads(1)
        return False


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def splitmix64_mix(z: int) -> int:
    return int(_load().orc_splitmix64_mix(z & (2**64 - 1)))


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, np.uint64)
    _load().orc_splitmix64_stream(seed, count, _ptr(out))
    return out


def hash_rows(seed: int, m: int, d: int):
    """(bucket u32[m], sign i8[m]) of Definition 1 for rows 0..m-1."""
    bucket = np.empty(m, np.uint32)
    sign = np.empty(m, np.int8)
    _load().orc_hash(seed, m, d, _ptr(bucket), _ptr(sign))
    return bucket, sign


def bucket_sort(bucket: np.ndarray, d: int):
    """Stable counting sort: (perm u32[m], ptr u32[d+1])."""
    bucket = _c(bucket, np.uint32)
    m = bucket.shape[0]
    perm = np.empty(m, np.uint32)
    ptr = np.empty(d + 1, np.uint32)
    _load().orc_bucket_sort(_ptr(bucket), m, d, _ptr(perm), _ptr(ptr))
    return perm, ptr


def sketch_dense(A: np.ndarray, b, d: int, seed: int):
    """(At f64[d,n], bt f64[d] or [d,nrhs]) = (S A, S b), Algorithm 1 Initialize.

    A is FP64 or FP32 (widened exactly); b is FP64, a vector or an m x nrhs
    matrix, or None."""
    lib = _load()
    if A.dtype == np.float32:
        A = _c(A, np.float32)
        fn = lib.orc_sketch_dense_f32
    else:
        A = _c(A, np.float64)
        fn = lib.orc_sketch_dense_f64
    m, n = A.shape
    At = np.empty((d, n), np.float64)
    Bt = None
    vec = False
    if b is not None:
        B = _c(b, np.float64)
        if B.ndim == 1:
            vec = True
            B = B.reshape(m, 1)
        nrhs = B.shape[1]
        Bt = np.empty((d, nrhs), np.float64)
        fn(_ptr(A), m, n, n, _ptr(B), nrhs, nrhs, d, seed, _ptr(At), n, _ptr(Bt), nrhs)
    else:
        fn(_ptr(A), m, n, n, None, 0, 1, d, seed, _ptr(At), n, None, 1)
    if Bt is not None and vec:
        Bt = Bt.reshape(d)
    return At, Bt


def sketch_csr(row_ptr, col, val, m: int, n: int, b, d: int, seed: int):
    """Dense FP64 (At, bt) from a CSR A with FP32 values."""
    row_ptr = _c(row_ptr, np.int64)
    col = _c(col, np.int32)
    val = _c(val, np.float32)
    At = np.empty((d, n), np.float64)
    bt = np.empty(d, np.float64) if b is not None else None
    bb = _c(b, np.float64) if b is not None else None
    _load().orc_sketch_csr_f32(_ptr(row_ptr), _ptr(col), _ptr(val), m, n, _ptr(bb), d, seed,
                               _ptr(At), n, _ptr(bt))
    return At, bt


def sketch_residual_csr(row_ptr, col, val, m: int, b, x, d: int, seed: int):
    """S (b - A x) for a CSR A with FP32 values (orc_sketch_residual_csr)."""
    row_ptr = _c(row_ptr, np.int64)
    col = _c(col, np.int32)
    val = _c(val, np.float32)
    bb = _c(b, np.float64)
    xx = _c(x, np.float64)
    r = np.empty(d, np.float64)
    _load().orc_sketch_residual_csr(_ptr(row_ptr), _ptr(col), _ptr(val), m, _ptr(bb), _ptr(xx), d, seed, _ptr(r))
    return r


def round_f64_to_f32(a):
    a = _c(a, np.float64)
    out = np.empty(a.shape, np.float32)
    _load().orc_round_f64_to_f32(_ptr(a), _ptr(out), a.size)
    return out


def round_f64_to_bf16_bits(a):
    a = _c(a, np.float64)
    out = np.empty(a.shape, np.uint16)
    _load().orc_round_f64_to_bf16(_ptr(a), _ptr(out), a.size)
    return out


def round_f64_to_f16_bits(a):
    a = _c(a, np.float64)
    out = np.empty(a.shape, np.uint16)
    _load().orc_round_f64_to_f16(_ptr(a), _ptr(out), a.size)
    return out


def round_f32_to_bf16_bits(a):
    a = _c(a, np.float32)
    out = np.empty(a.shape, np.uint16)
    _load().orc_round_f32_to_bf16(_ptr(a), _ptr(out), a.size)
    return out


def round_f32_to_f16_bits(a):
    a = _c(a, np.float32)
    out = np.empty(a.shape, np.uint16)
    _load().orc_round_f32_to_f16(_ptr(a), _ptr(out), a.size)
    return out


def row_norms2(At):
    At = _c(At, np.float64)
    d, n = At.shape
    nu2 = np.empty(d, np.float64)
    _load().orc_row_norms2(_ptr(At), d, n, n, _ptr(nu2))
    return nu2


class MwrkResult:
    def __init__(self, x, iters, status, idx=None, err2=None, r=None):
        self.x = x
        self.iters = iters
        self.status = status
        self.idx = idx
        self.err2 = err2
        self.r = r


def mwrk(At, bt, *, x0=None, xref=None, tol=1e-10, maxit=100000, stop_mode=None, trace=False):
    """The loop of Algorithm 1 on (At, bt); see orc_mwrk in csk_oracle.c."""
    At = _c(At, np.float64)
    bt = _c(bt, np.float64)
    d, n = At.shape
    if stop_mode is None:
        stop_mode = STOP_REL_ERR if xref is not None else STOP_REL_RESID
    x = np.empty(n, np.float64)
    iters = np.zeros(1, np.int64)
    x0c = _c(x0, np.float64) if x0 is not None else None
    xrc = _c(xref, np.float64) if xref is not None else None
    tidx = terr = tr = None
    if trace:
        tidx = np.full(maxit + 1, -1, np.int64)
        terr = np.full(maxit + 1, np.nan, np.float64)
        tr = np.full(maxit + 1, np.nan, np.float64)
    st = _load().orc_mwrk(_ptr(At), d, n, n, _ptr(bt), _ptr(x0c), _ptr(xrc), float(tol), int(maxit),
                          int(stop_mode), _ptr(x), _ptr(iters), _ptr(tidx), _ptr(terr), _ptr(tr))
    k = int(iters[0])
    if trace:
        return MwrkResult(x, k, st, tidx[:k], terr[:k + 1], tr[:k])
    return MwrkResult(x, k, st)


def _traces(trace, maxit):
    if not trace:
        return None, None, None
    return (np.full(maxit + 1, -1, np.int64), np.full(maxit + 1, np.nan, np.float64),
            np.full(maxit + 1, np.nan, np.float64))


def rgrk(At, bt, *, theta, sel_seed, x0=None, xref=None, tol=1e-10, maxit=100000, stop_mode=None,
         trace=False):
    """Relaxed greedy randomized Kaczmarz (theta = 1/2: greedy randomized
    Kaczmarz); see orc_rgrk in csk_oracle.c."""
    At = _c(At, np.float64)
    bt = _c(bt, np.float64)
    d, n = At.shape
    if stop_mode is None:
        stop_mode = STOP_REL_ERR if xref is not None else STOP_REL_RESID
    x = np.empty(n, np.float64)
    iters = np.zeros(1, np.int64)
    x0c = _c(x0, np.float64) if x0 is not None else None
    xrc = _c(xref, np.float64) if xref is not None else None
    tidx, terr, tr = _traces(trace, maxit)
    st = _load().orc_rgrk(_ptr(At), d, n, n, _ptr(bt), _ptr(x0c), _ptr(xrc), float(tol), int(maxit),
                          int(stop_mode), float(theta), int(sel_seed) & (2**64 - 1), _ptr(x), _ptr(iters),
                          _ptr(tidx), _ptr(terr), _ptr(tr))
    k = int(iters[0])
    if trace:
        return MwrkResult(x, k, st, tidx[:k], terr[:k + 1], tr[:k])
    return MwrkResult(x, k, st)


def rk(At, bt, *, sel_seed, xref, x0=None, tol=1e-10, maxit=100000, trace=False):
    """Randomized Kaczmarz (relative-error stop only); see orc_rk."""
    At = _c(At, np.float64)
    bt = _c(bt, np.float64)
    d, n = At.shape
    x = np.empty(n, np.float64)
    iters = np.zeros(1, np.int64)
    x0c = _c(x0, np.float64) if x0 is not None else None
    xrc = _c(xref, np.float64)
    tidx, terr, tr = _traces(trace, maxit)
    st = _load().orc_rk(_ptr(At), d, n, n, _ptr(bt), _ptr(x0c), _ptr(xrc), float(tol), int(maxit),
                        int(sel_seed) & (2**64 - 1), _ptr(x), _ptr(iters), _ptr(tidx), _ptr(terr), _ptr(tr))
    k = int(iters[0])
    if trace:
        return MwrkResult(x, k, st, tidx[:k], terr[:k + 1], tr[:k])
    return MwrkResult(x, k, st)


def uniforms(sel_seed: int, first: int, count: int) -> np.ndarray:
    """Uniforms first .. first+count-1 of the selection stream (orc_uniform)."""
    out = np.empty(count, np.float64)
    _load().orc_uniform_stream(int(sel_seed) & (2**64 - 1), first, count, _ptr(out))
    return out


def csk(A, b, d, seed, *, x0=None, xref=None, tol=1e-10, maxit=100000, stop_mode=None):
    """Algorithm 1 end to end: sketch, then the MWRK loop on the sketch."""
    At, bt = sketch_dense(A, b, d, seed)
    return mwrk(At, bt, x0=x0, xref=xref, tol=tol, maxit=maxit, stop_mode=stop_mode)
