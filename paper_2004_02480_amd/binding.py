"""Python binding of libcsk (count sketch Kaczmarz on AMD MI355X).

Thin layer over the C ABI in ``include/csk.h``: the functions below carry the
same names as the C entry points, take PyTorch tensors (device memory) and
the current HIP stream, allocate outputs and workspace with PyTorch, and
raise :class:`CskError` on a failing status.  All arithmetic of the method
runs in the HIP kernels of ``libcsk.so``; there is no fallback path.

Method (Zhang & Li, arXiv 2004.02480, Algorithm 1): sketch ``At = S A``,
``bt = S b`` with the count sketch of Definition 1, then run the maximal
weighted residual Kaczmarz loop on ``(At, bt)``.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _abi
from ._abi import (CSK_BF16, CSK_CANCELLED, CSK_ERR_DEGENERATE, CSK_ERR_DEVICE,  # noqa: F401
                   CSK_ERR_INVALID_ARG, CSK_ERR_NONFINITE, CSK_ERR_UNSUPPORTED,
                   CSK_ERR_WORKSPACE, CSK_F16, CSK_F32, CSK_F64, CSK_NOT_CONVERGED, CSK_OK,
                   CSK_STOP_REL_ERR, CSK_STOP_REL_RESID)

_lib = _abi.load()

__all__ = ["CskError", "SketchOut", "SolveResult", "csk_hash", "csk_sketch", "csk_sketch_csr", "csk_solve_csr_refresh",
           "csk_solve", "csk_solve_noalloc", "csk_solve_batched", "csk_solve_batched_sketches", "csk_solve_mrhs", "csk_tune_solve",
           "csk_tune_mrhs", "csk_tune_batched", "csk_tune_save", "csk_tune_load",
           "csk_tune_lookup", "csk_tune_clear", "csk_status_string", "lib"]

lib = _lib

_TORCH_TO_CSK = {torch.float64: CSK_F64, torch.float32: CSK_F32,
                 torch.float16: CSK_F16, torch.bfloat16: CSK_BF16}
_CSK_TO_TORCH = {v: k for k, v in _TORCH_TO_CSK.items()}


class CskError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.csk_last_error().decode(errors="replace")
        super().__init__(f"{where}: {csk_status_string(status)}" + (f" ({msg})" if msg else ""))


def csk_status_string(status: int) -> str:
    return _lib.csk_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != CSK_OK:
        raise CskError(status, where)


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device) -> torch.Tensor:
    buf = torch.empty(int(nbytes) + 512, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + int(nbytes) + 256]


def _padded_rows(d: int, n: int, dtype: torch.dtype, device) -> torch.Tensor:
    """A d x n view of a buffer whose rows are padded to whole 16-byte
    vectors: the solve reads such rows with vector loads, where unpadded
    rows of a width that is not a multiple of 16 bytes fall back to scalar
    loads (several times slower)."""
    per = 16 // torch.tensor([], dtype=dtype).element_size()
    ld = (n + per - 1) // per * per
    return torch.empty((d, ld), dtype=dtype, device=device)[:, :n]


def _ld(t: Optional[torch.Tensor], n: int) -> int:
    return t.stride(0) if t is not None else n


def _need_cuda(t: torch.Tensor, name: str):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise ValueError(f"{name} must be a device tensor")


def _rowmajor(t: torch.Tensor, name: str) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D tensor with unit column stride")
    return t.stride(0)


def csk_hash(seed: int, m: int, d: int, *, device="cuda", stream=None):
    """(bucket, sign): h(i) as int32 (values < d) and D_ii as int8, Definition 1."""
    bucket = torch.empty(m, dtype=torch.int32, device=device)
    sign = torch.empty(m, dtype=torch.int8, device=device)
    _check(_lib.csk_hash(ctypes.c_uint64(seed & (2**64 - 1)), m, d, _ptr(bucket), _ptr(sign),
                         _stream(stream)), "csk_hash")
    return bucket, sign


@dataclass
class SketchOut:
    At64: Optional[torch.Tensor]
    At_lp: Optional[torch.Tensor]
    bt: Optional[torch.Tensor]
    nu2: torch.Tensor
    perm: Optional[torch.Tensor]
    ptr: Optional[torch.Tensor]


def csk_sketch(A: torch.Tensor, b: Optional[torch.Tensor], d: int, seed: int, *,
               lp_dtype: Optional[torch.dtype] = None, want_f64: bool = True,
               want_perm: bool = False, out: Optional[SketchOut] = None,
               workspace: Optional[torch.Tensor] = None, stream=None) -> SketchOut:
    """At = S A and bt = S b (Algorithm 1, Initialize).

    A: m x n, float64 or float32, row-major.  b: m (vector) or m x nrhs,
    float64, or None.  lp_dtype: also return the low-precision copy.
    out: a SketchOut of the same shapes to write into (no allocation);
    workspace: a uint8 tensor of at least csk_sketch_workspace_size bytes,
    256-byte aligned."""
    _need_cuda(A, "A")
    if A.dtype not in (torch.float64, torch.float32):
        raise ValueError("A must be float64 or float32")
    lda = _rowmajor(A, "A")
    m, n = A.shape
    dev = A.device
    if out is not None:
        At64, At_lp, nu2, perm, ptr = out.At64, out.At_lp, out.nu2, out.perm, out.ptr
        if (At64 is None and At_lp is None) or nu2 is None:
            raise ValueError("out needs nu2 and At64 or At_lp")
        if lp_dtype is None and At_lp is not None:
            lp_dtype = At_lp.dtype
    else:
        At64 = _padded_rows(d, n, torch.float64, dev) if want_f64 else None
        At_lp = _padded_rows(d, n, lp_dtype, dev) if lp_dtype is not None else None
        nu2 = torch.empty(d, dtype=torch.float64, device=dev)
        perm = torch.empty(m, dtype=torch.int32, device=dev) if want_perm else None
        ptr = torch.empty(d + 1, dtype=torch.int32, device=dev) if want_perm else None
    if At64 is None and At_lp is None:
        raise ValueError("nothing to compute")
    B = bt = None
    nrhs, ldb, ldbt = 0, 1, 1
    if b is not None:
        _need_cuda(b, "b")
        if b.dtype != torch.float64:
            raise ValueError("b must be float64")
        if b.dim() == 1:
            B = b.contiguous()
            nrhs, ldb = 1, 1
            bt = out.bt if out is not None else torch.empty(d, dtype=torch.float64, device=dev)
            ldbt = 1
        else:
            B = b
            nrhs = b.shape[1]
            ldb = _rowmajor(b, "b")
            bt = out.bt if out is not None else torch.empty((d, nrhs), dtype=torch.float64, device=dev)
            ldbt = nrhs
        if bt is None:
            raise ValueError("out needs bt when b is given")
    if workspace is not None:
        ws = workspace
    else:
        nbytes = ctypes.c_size_t(0)
        _check(_lib.csk_sketch_workspace_size(m, n, d, nrhs, ctypes.byref(nbytes)), "csk_sketch_workspace_size")
        ws = _workspace(nbytes.value, dev)
    lp_code = _TORCH_TO_CSK[lp_dtype] if lp_dtype is not None else CSK_F64
    _check(_lib.csk_sketch(_ptr(A), _TORCH_TO_CSK[A.dtype], m, n, lda, _ptr(B), nrhs, ldb, d,
                           ctypes.c_uint64(seed & (2**64 - 1)),
                           _ptr(At64), _ld(At64, n), _ptr(At_lp), lp_code, _ld(At_lp, n), _ptr(bt), ldbt, _ptr(nu2),
                           _ptr(perm), _ptr(ptr), _ptr(ws), ws.numel(), _stream(stream)), "csk_sketch")
    return SketchOut(At64, At_lp, bt, nu2, perm, ptr)


def csk_sketch_csr(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n: int,
                   b: Optional[torch.Tensor], d: int, seed: int, *,
                   lp_dtype: Optional[torch.dtype] = None, want_f64: bool = True,
                   stream=None) -> SketchOut:
    """Dense (At, bt) from a CSR A (int64 row_ptr, int32 col, float32 val)."""
    for t, nm in ((row_ptr, "row_ptr"), (col, "col"), (val, "val")):
        _need_cuda(t, nm)
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or val.dtype != torch.float32:
        raise ValueError("row_ptr int64, col int32, val float32 expected")
    m = row_ptr.numel() - 1
    nnz = col.numel()
    dev = row_ptr.device
    At64 = _padded_rows(d, n, torch.float64, dev) if want_f64 else None
    At_lp = _padded_rows(d, n, lp_dtype, dev) if lp_dtype is not None else None
    nu2 = torch.empty(d, dtype=torch.float64, device=dev)
    bt = torch.empty(d, dtype=torch.float64, device=dev) if b is not None else None
    nbytes = ctypes.c_size_t(0)
    _check(_lib.csk_sketch_csr_workspace_size(m, n, d, ctypes.byref(nbytes)), "csk_sketch_csr_workspace_size")
    ws = _workspace(nbytes.value, dev)
    lp_code = _TORCH_TO_CSK[lp_dtype] if lp_dtype is not None else CSK_F64
    _check(_lib.csk_sketch_csr(_ptr(row_ptr), _ptr(col), _ptr(val), m, n, nnz,
                               _ptr(b.contiguous() if b is not None else None), d,
                               ctypes.c_uint64(seed & (2**64 - 1)), _ptr(At64), _ld(At64, n), _ptr(At_lp), lp_code,
                               _ld(At_lp, n),
                               _ptr(bt), _ptr(nu2), _ptr(ws), ws.numel(), _stream(stream)), "csk_sketch_csr")
    return SketchOut(At64, At_lp, bt, nu2, None, None)


@dataclass
class CsrSketchOut:
    row_ptr: torch.Tensor   # d + 1 int64
    col: torch.Tensor       # nnz(At) int32 (a view of the first row_ptr[d] entries)
    val: torch.Tensor       # nnz(At) float64
    bt: Optional[torch.Tensor]
    nu2: torch.Tensor
    nnz: int


def csk_sketch_csr_sparse(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n: int,
                          b: Optional[torch.Tensor], d: int, seed: int, *, stream=None) -> CsrSketchOut:
    """At = S A as a CSR matrix from a CSR A (Algorithm 1, Initialize).

    Synchronizes the stream once to read nnz(At)."""
    for t, nm in ((row_ptr, "row_ptr"), (col, "col"), (val, "val")):
        _need_cuda(t, nm)
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or val.dtype != torch.float32:
        raise ValueError("row_ptr int64, col int32, val float32 expected")
    m = row_ptr.numel() - 1
    nnz = col.numel()
    dev = row_ptr.device
    at_rp = torch.empty(d + 1, dtype=torch.int64, device=dev)
    at_col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    at_val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
    nu2 = torch.empty(d, dtype=torch.float64, device=dev)
    bt = torch.empty(d, dtype=torch.float64, device=dev) if b is not None else None
    nbytes = ctypes.c_size_t(0)
    _check(_lib.csk_sketch_csr_sparse_workspace_size(m, n, d, ctypes.byref(nbytes)),
           "csk_sketch_csr_sparse_workspace_size")
    ws = _workspace(nbytes.value, dev)
    _check(_lib.csk_sketch_csr_sparse(_ptr(row_ptr), _ptr(col), _ptr(val), m, n, nnz,
                                      _ptr(b.contiguous() if b is not None else None), d,
                                      ctypes.c_uint64(seed & (2**64 - 1)), _ptr(at_rp), _ptr(at_col), _ptr(at_val),
                                      _ptr(bt), _ptr(nu2), _ptr(ws), ws.numel(), _stream(stream)),
           "csk_sketch_csr_sparse")
    nnz_at = int(at_rp[d].item())
    return CsrSketchOut(at_rp, at_col[:nnz_at], at_val[:nnz_at], bt, nu2, nnz_at)


def csk_solve_csr(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n: int, bt: torch.Tensor, *,
                  nu2: Optional[torch.Tensor] = None, x0: Optional[torch.Tensor] = None,
                  x_ref: Optional[torch.Tensor] = None, tol: float = 1e-10, maxit: int = 100000,
                  stop_mode: Optional[int] = None, cancel: Optional[int] = None, check_every: int = 256,
                  grid: int = 0, single_wg: int = -1, out: Optional[torch.Tensor] = None,
                  result: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                  trace_idx: Optional[torch.Tensor] = None, sync: bool = True, stream=None):
    """MWRK (Algorithm 1, loop) on a CSR At (int64 row_ptr, int32 col, float64 val), FP64.

    trace_idx: optional int64 device tensor of at least maxit entries that
    receives the row projected at each iteration.
    Returns a SolveResult when sync=True, else (x, raw_result_tensor)."""
    for t, nm in ((row_ptr, "row_ptr"), (col, "col"), (val, "val"), (bt, "bt")):
        _need_cuda(t, nm)
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or val.dtype != torch.float64:
        raise ValueError("row_ptr int64, col int32, val float64 expected")
    d = row_ptr.numel() - 1
    nnz = col.numel()
    if val.numel() != nnz:
        raise ValueError("col and val lengths differ")
    if stop_mode is None:
        stop_mode = CSK_STOP_REL_ERR if x_ref is not None else CSK_STOP_REL_RESID
    dev = row_ptr.device
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=dev)
    res = result if result is not None else torch.zeros(_abi.RESULT_BYTES, dtype=torch.uint8, device=dev)
    if workspace is None:
        nbytes = ctypes.c_size_t(0)
        _check(_lib.csk_solve_csr_workspace_size(d, n, nnz, ctypes.byref(nbytes)), "csk_solve_csr_workspace_size")
        workspace = _workspace(nbytes.value, dev)
    o = _opts(tol, maxit, stop_mode, 0, x_ref, cancel, check_every, grid, single_wg, trace_idx)
    _check(_lib.csk_solve_csr(_ptr(row_ptr), _ptr(col), _ptr(val), d, n, nnz, _ptr(bt), _ptr(nu2), _ptr(x0),
                              _ptr(x), ctypes.byref(o), _ptr(res), _ptr(workspace), workspace.numel(),
                              _stream(stream)), "csk_solve_csr")
    if not sync:
        return x, res
    (stream or torch.cuda.current_stream()).synchronize()
    it, st, fb, meas, nref = parse_results(res)[0]
    return SolveResult(x, it, st, fb, meas, nref)


@dataclass
class SolveResult:
    x: torch.Tensor
    iters: int
    status: int
    fp64_fallback: int
    final_measure: float
    refreshes: int

    @property
    def status_name(self) -> str:
        return csk_status_string(self.status)


def parse_results(raw: torch.Tensor) -> List[tuple]:
    """Decode csk_solve_result records (device or host uint8 tensor)."""
    host = raw.cpu().numpy()
    out = []
    import numpy as np
    for k in range(host.size // _abi.RESULT_BYTES):
        rec = host[k * _abi.RESULT_BYTES:(k + 1) * _abi.RESULT_BYTES]
        iters = int(np.frombuffer(rec[0:8].tobytes(), np.int64)[0])
        status, fb = (int(v) for v in np.frombuffer(rec[8:16].tobytes(), np.int32))
        meas = float(np.frombuffer(rec[16:24].tobytes(), np.float64)[0])
        nref = int(np.frombuffer(rec[24:32].tobytes(), np.int64)[0])
        out.append((iters, status, fb, meas, nref))
    return out


def _opts(tol, maxit, stop_mode, refresh_every, x_ref, cancel, check_every, grid, single_wg, trace_idx=None):
    if trace_idx is not None:
        _need_cuda(trace_idx, "trace_idx")
        if trace_idx.dtype != torch.int64 or not trace_idx.is_contiguous() or trace_idx.numel() < int(maxit):
            raise ValueError("trace_idx must be a contiguous int64 device tensor of at least maxit entries")
    o = _abi.SolveOpts()
    o.tol = float(tol)
    o.maxit = int(maxit)
    o.stop_mode = int(stop_mode)
    o.refresh_every = int(refresh_every)
    o.x_ref = None if x_ref is None else x_ref.data_ptr()
    o.cancel = None if cancel is None else int(cancel)
    o.check_every = int(check_every)
    o.grid = int(grid)
    o.block = 0
    o.single_wg = int(single_wg)
    o.trace_idx = None if trace_idx is None else trace_idx.data_ptr()
    return o


def csk_solve(At: torch.Tensor, bt: torch.Tensor, *, At64: Optional[torch.Tensor] = None,
              nu2: Optional[torch.Tensor] = None, x0: Optional[torch.Tensor] = None,
              x_ref: Optional[torch.Tensor] = None, tol: float = 1e-10, maxit: int = 100000,
              stop_mode: Optional[int] = None, refresh_every: int = 64, cancel: Optional[int] = None,
              check_every: int = 256, grid: int = 0, single_wg: int = -1,
              out: Optional[torch.Tensor] = None, result: Optional[torch.Tensor] = None,
              workspace: Optional[torch.Tensor] = None, trace_idx: Optional[torch.Tensor] = None,
              sync: bool = True, stream=None):
    """MWRK on (At, bt) (Algorithm 1, loop).

    At: d x n float64 (plain) or float32/float16/bfloat16 (mixed, At64 required).
    trace_idx: optional int64 device tensor of at least maxit entries that
    receives the row projected at each iteration.
    Returns a SolveResult when sync=True, else (x, raw_result_tensor)."""
    _need_cuda(At, "At")
    ldat = _rowmajor(At, "At")
    d, n = At.shape
    at_code = _TORCH_TO_CSK[At.dtype]
    ldat64 = ldat
    if At64 is not None:
        ldat64 = _rowmajor(At64, "At64")
    if stop_mode is None:
        stop_mode = CSK_STOP_REL_ERR if x_ref is not None else CSK_STOP_REL_RESID
    dev = At.device
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=dev)
    res = result if result is not None else torch.zeros(_abi.RESULT_BYTES, dtype=torch.uint8, device=dev)
    if workspace is None:
        nbytes = ctypes.c_size_t(0)
        _check(_lib.csk_solve_workspace_size(d, n, at_code, ctypes.byref(nbytes)), "csk_solve_workspace_size")
        workspace = _workspace(nbytes.value, dev)
    o = _opts(tol, maxit, stop_mode, refresh_every, x_ref, cancel, check_every, grid, single_wg, trace_idx)
    _check(_lib.csk_solve(_ptr(At), at_code, ldat, _ptr(At64), ldat64, d, n, _ptr(bt), _ptr(nu2), _ptr(x0),
                          _ptr(x), ctypes.byref(o), _ptr(res), _ptr(workspace), workspace.numel(),
                          _stream(stream)), "csk_solve")
    if not sync:
        return x, res
    (stream or torch.cuda.current_stream()).synchronize()
    it, st, fb, meas, nref = parse_results(res)[0]
    return SolveResult(x, it, st, fb, meas, nref)


def csk_solve_csr_refresh(At: torch.Tensor, bt: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor,
                          val: torch.Tensor, b: torch.Tensor, seed: int, *, At64: torch.Tensor,
                          nu2: Optional[torch.Tensor] = None, x0: Optional[torch.Tensor] = None,
                          x_ref: Optional[torch.Tensor] = None, tol: float = 1e-10, maxit: int = 100000,
                          stop_mode: Optional[int] = None, refresh_every: int = 64, cancel: Optional[int] = None,
                          check_every: int = 256, grid: int = 0, single_wg: int = -1,
                          out: Optional[torch.Tensor] = None, result: Optional[torch.Tensor] = None,
                          workspace: Optional[torch.Tensor] = None, trace_idx: Optional[torch.Tensor] = None,
                          sync: bool = True, stream=None):
    """Mixed-precision MWRK on the sketch of a CSR matrix with each refresh
    residual formed as S (b - A x) from the CSR A (row_ptr int64, col int32,
    val float32, b float64; seed of the sketch) instead of bt - At64 x.
    At: d x n float32/float16/bfloat16; At64 the FP64 sketch (projections and
    the FP64 fallback).  Returns as csk_solve."""
    _need_cuda(At, "At")
    ldat = _rowmajor(At, "At")
    ldat64 = _rowmajor(At64, "At64")
    d, n = At.shape
    m = row_ptr.numel() - 1
    at_code = _TORCH_TO_CSK[At.dtype]
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or val.dtype != torch.float32 \
            or b.dtype != torch.float64:
        raise TypeError("row_ptr int64, col int32, val float32 and b float64 expected")
    if stop_mode is None:
        stop_mode = CSK_STOP_REL_ERR if x_ref is not None else CSK_STOP_REL_RESID
    dev = At.device
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=dev)
    res = result if result is not None else torch.zeros(_abi.RESULT_BYTES, dtype=torch.uint8, device=dev)
    if workspace is None:
        nbytes = ctypes.c_size_t(0)
        _check(_lib.csk_solve_csr_refresh_workspace_size(m, d, n, ctypes.byref(nbytes)),
               "csk_solve_csr_refresh_workspace_size")
        workspace = _workspace(nbytes.value, dev)
    o = _opts(tol, maxit, stop_mode, refresh_every, x_ref, cancel, check_every, grid, single_wg, trace_idx)
    _check(_lib.csk_solve_csr_refresh(_ptr(At), at_code, ldat, _ptr(At64), ldat64, d, n, _ptr(row_ptr), _ptr(col),
                                      _ptr(val), m, _ptr(b), seed, _ptr(bt), _ptr(nu2), _ptr(x0), _ptr(x),
                                      ctypes.byref(o), _ptr(res), _ptr(workspace), workspace.numel(),
                                      _stream(stream)), "csk_solve_csr_refresh")
    if not sync:
        return x, res
    (stream or torch.cuda.current_stream()).synchronize()
    it, st, fb, meas, nref = parse_results(res)[0]
    return SolveResult(x, it, st, fb, meas, nref)


def csk_solve_noalloc(At: torch.Tensor, bt: torch.Tensor, *, At64: Optional[torch.Tensor] = None,
                      nu2: Optional[torch.Tensor] = None, x0: Optional[torch.Tensor] = None,
                      x_ref: Optional[torch.Tensor] = None, tol: float = 1e-10, maxit: int = 100000,
                      stop_mode: Optional[int] = None, refresh_every: int = 64, cancel: Optional[int] = None,
                      check_every: int = 256, grid: int = 0, single_wg: int = -1,
                      out: torch.Tensor, result: torch.Tensor, trace_idx: Optional[torch.Tensor] = None,
                      stream=None):
    """csk_solve with its workspace taken from the library's static scratch:
    the caller passes the output x and the raw result buffer, and nothing is
    allocated (no workspace argument).  Returns (x, raw_result_tensor)
    without synchronizing."""
    _need_cuda(At, "At")
    ldat = _rowmajor(At, "At")
    d, n = At.shape
    at_code = _TORCH_TO_CSK[At.dtype]
    ldat64 = _rowmajor(At64, "At64") if At64 is not None else ldat
    if stop_mode is None:
        stop_mode = CSK_STOP_REL_ERR if x_ref is not None else CSK_STOP_REL_RESID
    o = _opts(tol, maxit, stop_mode, refresh_every, x_ref, cancel, check_every, grid, single_wg, trace_idx)
    _check(_lib.csk_solve_noalloc(_ptr(At), at_code, ldat, _ptr(At64), ldat64, d, n, _ptr(bt), _ptr(nu2),
                                  _ptr(x0), _ptr(out), ctypes.byref(o), _ptr(result), _stream(stream)),
           "csk_solve_noalloc")
    return out, result


def _solve_fp64_select(name, At, bt, extra, nu2, x0, x_ref, tol, maxit, stop_mode, cancel, check_every, grid,
                       single_wg, out, result, workspace, sync, stream, trace_idx=None):
    _need_cuda(At, "At")
    if At.dtype != torch.float64:
        raise ValueError("the randomized selection rules run on the FP64 sketch")
    ldat = _rowmajor(At, "At")
    d, n = At.shape
    dev = At.device
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=dev)
    res = result if result is not None else torch.zeros(_abi.RESULT_BYTES, dtype=torch.uint8, device=dev)
    if workspace is None:
        nbytes = ctypes.c_size_t(0)
        _check(getattr(_lib, name + "_workspace_size")(d, n, ctypes.byref(nbytes)), name + "_workspace_size")
        workspace = _workspace(nbytes.value, dev)
    o = _opts(tol, maxit, stop_mode, 0, x_ref, cancel, check_every, grid, single_wg, trace_idx)
    _check(getattr(_lib, name)(_ptr(At), ldat, d, n, _ptr(bt), _ptr(nu2), _ptr(x0), _ptr(x), *extra,
                               ctypes.byref(o), _ptr(res), _ptr(workspace), workspace.numel(), _stream(stream)),
           name)
    if not sync:
        return x, res
    (stream or torch.cuda.current_stream()).synchronize()
    it, st, fb, meas, nref = parse_results(res)[0]
    return SolveResult(x, it, st, fb, meas, nref)


def csk_solve_rgrk(At: torch.Tensor, bt: torch.Tensor, *, theta: float = 0.5, sel_seed: int = 0,
                   nu2: Optional[torch.Tensor] = None, x0: Optional[torch.Tensor] = None,
                   x_ref: Optional[torch.Tensor] = None, tol: float = 1e-10, maxit: int = 100000,
                   stop_mode: Optional[int] = None, cancel: Optional[int] = None, check_every: int = 256,
                   grid: int = 0, single_wg: int = -1, out: Optional[torch.Tensor] = None,
                   result: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                   trace_idx: Optional[torch.Tensor] = None, sync: bool = True, stream=None):
    """The loop on the FP64 (At, bt) with the relaxed greedy randomized rule
    (theta = 1/2: greedy randomized Kaczmarz; theta = 1: the greedy rule).

    Returns a SolveResult when sync=True, else (x, raw_result_tensor)."""
    if stop_mode is None:
        stop_mode = CSK_STOP_REL_ERR if x_ref is not None else CSK_STOP_REL_RESID
    return _solve_fp64_select("csk_solve_rgrk", At, bt, (float(theta), int(sel_seed) & (2**64 - 1)), nu2, x0,
                              x_ref, tol, maxit, stop_mode, cancel, check_every, grid, single_wg, out, result,
                              workspace, sync, stream, trace_idx)


def csk_solve_rk(At: torch.Tensor, bt: torch.Tensor, *, x_ref: torch.Tensor, sel_seed: int = 0,
                 nu2: Optional[torch.Tensor] = None, x0: Optional[torch.Tensor] = None, tol: float = 1e-10,
                 maxit: int = 1000000, cancel: Optional[int] = None, check_every: int = 256,
                 out: Optional[torch.Tensor] = None, result: Optional[torch.Tensor] = None,
                 workspace: Optional[torch.Tensor] = None, trace_idx: Optional[torch.Tensor] = None,
                 sync: bool = True, stream=None):
    """Randomized Kaczmarz on the FP64 (At, bt), stopped on the relative
    error against x_ref.  Returns a SolveResult when sync=True, else
    (x, raw_result_tensor)."""
    return _solve_fp64_select("csk_solve_rk", At, bt, (int(sel_seed) & (2**64 - 1),), nu2, x0, x_ref, tol, maxit,
                              CSK_STOP_REL_ERR, cancel, check_every, 0, -1, out, result, workspace, sync, stream,
                              trace_idx)


class Pipeline:
    """Algorithm 1 (sketch, then the loop) captured once into a HIP graph by
    csk_pipeline_capture; launch() replays it.  Holds every buffer the graph
    reads or writes: refill A, b, x0 and x_ref in place between launches."""

    def __init__(self, handle, keep, x, result, sketch):
        self._h = handle
        self._keep = keep
        self.x = x
        self.result = result
        self.sketch = sketch

    def launch(self, stream=None):
        if self._h is None:
            raise CskError(CSK_ERR_INVALID_ARG, "pipeline destroyed")
        _check(_lib.csk_pipeline_launch(self._h, _stream(stream)), "csk_pipeline_launch")

    def results(self) -> "SolveResult":
        torch.cuda.synchronize()
        it, st, fb, meas, nref = parse_results(self.result)[0]
        return SolveResult(self.x, it, st, fb, meas, nref)

    def close(self):
        if self._h is not None:
            _check(_lib.csk_pipeline_destroy(self._h), "csk_pipeline_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def csk_pipeline_capture(A: torch.Tensor, b: torch.Tensor, d: int, seed: int, *,
                         lp_dtype: Optional[torch.dtype] = None, x0: Optional[torch.Tensor] = None,
                         x_ref: Optional[torch.Tensor] = None, tol: float = 1e-10, maxit: int = 100000,
                         stop_mode: Optional[int] = None, refresh_every: int = 64, grid: int = 0,
                         single_wg: int = -1, capture_stream=None) -> Pipeline:
    """Capture csk_sketch then csk_solve (mixed precision when lp_dtype is
    given) into one HIP graph through the C ABI; returns a Pipeline."""
    _need_cuda(A, "A")
    _need_cuda(b, "b")
    if A.dtype not in (torch.float64, torch.float32) or b.dtype != torch.float64 or b.dim() != 1:
        raise ValueError("A float64/float32 (m x n), b float64 (m) expected")
    lda = _rowmajor(A, "A")
    m, n = A.shape
    dev = A.device
    At64 = _padded_rows(d, n, torch.float64, dev)
    At_lp = _padded_rows(d, n, lp_dtype, dev) if lp_dtype is not None else None
    bt = torch.empty(d, dtype=torch.float64, device=dev)
    nu2 = torch.empty(d, dtype=torch.float64, device=dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    res = torch.zeros(_abi.RESULT_BYTES, dtype=torch.uint8, device=dev)
    a_code = _TORCH_TO_CSK[A.dtype]
    lp_code = _TORCH_TO_CSK[lp_dtype] if lp_dtype is not None else CSK_F64
    nb = ctypes.c_size_t(0)
    _check(_lib.csk_sketch_workspace_size(m, n, d, 1, ctypes.byref(nb)), "csk_sketch_workspace_size")
    ws_sk = _workspace(nb.value, dev)
    _check(_lib.csk_solve_workspace_size(d, n, lp_code, ctypes.byref(nb)), "csk_solve_workspace_size")
    ws_so = _workspace(nb.value, dev)
    if stop_mode is None:
        stop_mode = CSK_STOP_REL_ERR if x_ref is not None else CSK_STOP_REL_RESID
    o = _opts(tol, maxit, stop_mode, refresh_every, x_ref, None, 256, grid, single_wg)
    cs = capture_stream if capture_stream is not None else torch.cuda.Stream(device=dev)
    cs.wait_stream(torch.cuda.current_stream(dev))
    h = ctypes.c_void_p()
    _check(_lib.csk_pipeline_capture(_ptr(A), a_code, m, n, lda, _ptr(b), d, int(seed) & (2**64 - 1), _ptr(At64),
                                     At64.stride(0), _ptr(At_lp), lp_code, _ld(At_lp, n), _ptr(bt), _ptr(nu2),
                                     _ptr(x0), _ptr(x), ctypes.byref(o), _ptr(res), _ptr(ws_sk), ws_sk.numel(),
                                     _ptr(ws_so), ws_so.numel(), ctypes.c_void_p(cs.cuda_stream), ctypes.byref(h)),
           "csk_pipeline_capture")
    keep = (A, b, x0, x_ref, ws_sk, ws_so, cs)
    return Pipeline(h, keep, x, res, SketchOut(At64, At_lp, bt, nu2, None, None))


def _batched_descs(systems: Sequence[dict]):
    """(descriptor array, outputs x, tensors to keep alive, A's dtype code)."""
    nsys = len(systems)
    a_dtype = systems[0]["A"].dtype
    descs = (_abi.SystemDesc * nsys)()
    xs = []
    keep = []
    for s, sysd in enumerate(systems):
        A = sysd["A"]
        if A.dtype != a_dtype:
            raise ValueError("all systems must share A's dtype")
        _need_cuda(A, "A")
        lda = _rowmajor(A, "A")
        m, n = A.shape
        b = sysd["b"].contiguous()
        xr = sysd.get("x_ref")
        x = torch.empty(n, dtype=torch.float64, device=A.device)
        xs.append(x)
        keep += [A, b, xr]
        dsc = descs[s]
        dsc.A = A.data_ptr()
        dsc.b = b.data_ptr()
        dsc.x_ref = None if xr is None else xr.data_ptr()
        dsc.x = x.data_ptr()
        dsc.m, dsc.n, dsc.lda, dsc.d = m, n, lda, int(sysd["d"])
        dsc.seed = int(sysd["seed"]) & (2**64 - 1)
    return descs, xs, keep, _TORCH_TO_CSK[a_dtype]


def csk_solve_batched(systems: Sequence[dict], *, lp_dtype: torch.dtype = torch.float32, tol: float = 1e-8,
                      maxit: int = 200000, refresh_every: int = 64, sync: bool = True, stream=None):
    """Sketch and solve many independent systems in one pass.

    Each system is a dict with A (m x n, float32 or float64), b (m float64),
    d, seed and optional x_ref (n float64).  Returns (xs, results)."""
    nsys = len(systems)
    descs, xs, keep, a_code = _batched_descs(systems)
    dev = systems[0]["A"].device
    lp_code = _TORCH_TO_CSK[lp_dtype]
    nbytes = ctypes.c_size_t(0)
    _check(_lib.csk_solve_batched_workspace_size(descs, nsys, a_code, lp_code, ctypes.byref(nbytes)),
           "csk_solve_batched_workspace_size")
    ws = _workspace(nbytes.value, dev)
    res = torch.zeros(_abi.RESULT_BYTES * nsys, dtype=torch.uint8, device=dev)
    o = _opts(tol, maxit, CSK_STOP_REL_ERR, refresh_every, None, None, 256, 0, -1)
    _check(_lib.csk_solve_batched(descs, nsys, a_code, lp_code, ctypes.byref(o), _ptr(res), _ptr(ws),
                                  ws.numel(), _stream(stream)), "csk_solve_batched")
    if not sync:
        return xs, res, ws
    (stream or torch.cuda.current_stream()).synchronize()
    return xs, parse_results(res)


def _report(r) -> dict:
    return dict(choice=r.choice, default_choice=r.default_choice, us=r.us, default_us=r.default_us,
                candidates=r.candidates)


def csk_tune_batched(systems: Sequence[dict], *, lp_dtype: torch.dtype = torch.float32, tol: float = 1e-8,
                     maxit: int = 200000, refresh_every: int = 64, stream=None) -> dict:
    """Runs the batched solve once per plan variant, caches the fastest for
    these shapes and returns the report (choice, default_choice, us,
    default_us in microseconds per call, candidates)."""
    nsys = len(systems)
    descs, xs, keep, a_code = _batched_descs(systems)
    dev = systems[0]["A"].device
    lp_code = _TORCH_TO_CSK[lp_dtype]
    nbytes = ctypes.c_size_t(0)
    _check(_lib.csk_solve_batched_workspace_size(descs, nsys, a_code, lp_code, ctypes.byref(nbytes)),
           "csk_solve_batched_workspace_size")
    ws = _workspace(nbytes.value, dev)
    res = torch.zeros(_abi.RESULT_BYTES * nsys, dtype=torch.uint8, device=dev)
    o = _opts(tol, maxit, CSK_STOP_REL_ERR, refresh_every, None, None, 256, 0, -1)
    rep = _abi.TuneReport()
    _check(_lib.csk_tune_batched(descs, nsys, a_code, lp_code, ctypes.byref(o), _ptr(res), ctypes.byref(rep),
                                 _ptr(ws), ws.numel(), _stream(stream)), "csk_tune_batched")
    return _report(rep)


def csk_solve_batched_sketches(systems: Sequence[dict], ws: torch.Tensor, *,
                               lp_dtype: torch.dtype = torch.float32) -> List[SketchOut]:
    """Views of the per-system sketches csk_solve_batched wrote into its
    workspace `ws` (the third value it returns with sync=False): At64 and
    At_lp as d x n views of their padded rows, bt and nu2.  Valid once the
    call's work has finished and while ws is alive."""
    nsys = len(systems)
    a_dtype = systems[0]["A"].dtype
    descs = (_abi.SystemDesc * nsys)()
    for k, sysd in enumerate(systems):
        m, n = sysd["A"].shape
        dsc = descs[k]
        dsc.m, dsc.n, dsc.lda, dsc.d = m, n, _rowmajor(sysd["A"], "A"), int(sysd["d"])
        dsc.A = dsc.b = dsc.x = 1  # sizes only: the layout query reads no buffer
    out = []
    for k, sysd in enumerate(systems):
        loc = _abi.BatchedSketchLoc()
        _check(_lib.csk_solve_batched_sketch_loc(descs, nsys, _TORCH_TO_CSK[a_dtype], _TORCH_TO_CSK[lp_dtype], k,
                                                 ctypes.byref(loc)), "csk_solve_batched_sketch_loc")
        d, n = int(sysd["d"]), sysd["A"].shape[1]

        def view(off, dtype, count):
            es = torch.tensor([], dtype=dtype).element_size()
            return ws[off:off + count * es].view(dtype)

        at64 = view(loc.at64, torch.float64, d * loc.ld64).view(d, loc.ld64)[:, :n]
        at_lp = None
        if loc.at_lp >= 0:
            at_lp = view(loc.at_lp, lp_dtype, d * loc.ld_lp).view(d, loc.ld_lp)[:, :n]
        out.append(SketchOut(at64, at_lp, view(loc.bt, torch.float64, d), view(loc.nu2, torch.float64, d), None,
                             None))
    return out


def csk_solve_mrhs(At_lp: torch.Tensor, At64: torch.Tensor, Bt: torch.Tensor, nu2: torch.Tensor, *,
                   X0: Optional[torch.Tensor] = None, Xref: Optional[torch.Tensor] = None,
                   tol: float = 1e-8, maxit: int = 200000, refresh_every: int = 64,
                   stop_mode: Optional[int] = None, sync: bool = True, stream=None):
    """Solve At X[:, j] = Bt[:, j] for every column j (shared sketch)."""
    _need_cuda(At_lp, "At_lp")
    d, n = At_lp.shape
    nrhs = Bt.shape[1]
    dev = At_lp.device
    if stop_mode is None:
        stop_mode = CSK_STOP_REL_ERR if Xref is not None else CSK_STOP_REL_RESID
    X = torch.empty((n, nrhs), dtype=torch.float64, device=dev)
    nbytes = ctypes.c_size_t(0)
    _check(_lib.csk_solve_mrhs_workspace_size(d, n, nrhs, ctypes.byref(nbytes)), "csk_solve_mrhs_workspace_size")
    ws = _workspace(nbytes.value, dev)
    res = torch.zeros(_abi.RESULT_BYTES * nrhs, dtype=torch.uint8, device=dev)
    o = _opts(tol, maxit, stop_mode, refresh_every, None, None, 256, 0, -1)
    _check(_lib.csk_solve_mrhs(_ptr(At_lp), _TORCH_TO_CSK[At_lp.dtype], _rowmajor(At_lp, "At_lp"), _ptr(At64),
                               _rowmajor(At64, "At64"), d, n, _ptr(Bt), nrhs, _rowmajor(Bt, "Bt"), _ptr(nu2),
                               _ptr(X0), _ptr(X), nrhs, _ptr(Xref), nrhs if Xref is not None else 0,
                               ctypes.byref(o), _ptr(res), _ptr(ws), ws.numel(), _stream(stream)),
           "csk_solve_mrhs")
    if not sync:
        return X, res
    (stream or torch.cuda.current_stream()).synchronize()
    return X, parse_results(res)


def csk_tune_solve(At: torch.Tensor, bt: torch.Tensor, *, At64: Optional[torch.Tensor] = None,
                   nu2: Optional[torch.Tensor] = None, trial_iters: int = 200, stream=None) -> dict:
    """Times the persistent solve's candidate launch shapes on (At, bt) and
    caches the fastest for later default-shaped csk_solve calls of the same
    shape (synchronizes the stream).  Returns the chosen entry."""
    _need_cuda(At, "At")
    ldat = _rowmajor(At, "At")
    d, n = At.shape
    at_code = _TORCH_TO_CSK[At.dtype]
    ldat64 = ldat if At64 is None else _rowmajor(At64, "At64")
    nbytes = ctypes.c_size_t(0)
    _check(_lib.csk_tune_solve_workspace_size(d, n, at_code, ctypes.byref(nbytes)), "csk_tune_solve_workspace_size")
    ws = _workspace(nbytes.value, At.device)
    best = _abi.TuneEntry()
    _check(_lib.csk_tune_solve(_ptr(At), at_code, ldat, _ptr(At64), ldat64, d, n, _ptr(bt), _ptr(nu2),
                               int(trial_iters), ctypes.byref(best), _ptr(ws), ws.numel(), _stream(stream)),
           "csk_tune_solve")
    return dict(grid=best.grid, lanes_per_row=best.lanes_per_row, us_per_iter=best.us_per_iter)


def csk_tune_mrhs(At_lp: torch.Tensor, At64: torch.Tensor, Bt: torch.Tensor, nu2: torch.Tensor, *,
                  trial_iters: int = 200, stream=None) -> dict:
    """Times the multi-RHS solve's row-tile counts on this system, caches
    the fastest for its shape and returns the report (choice and
    default_choice in 16-row tiles per workgroup, us and default_us per
    iteration, candidates)."""
    _need_cuda(At_lp, "At_lp")
    d, n = At_lp.shape
    nrhs = Bt.shape[1]
    nbytes = ctypes.c_size_t(0)
    _check(_lib.csk_tune_mrhs_workspace_size(d, n, nrhs, ctypes.byref(nbytes)), "csk_tune_mrhs_workspace_size")
    ws = _workspace(nbytes.value, At_lp.device)
    rep = _abi.TuneReport()
    _check(_lib.csk_tune_mrhs(_ptr(At_lp), _TORCH_TO_CSK[At_lp.dtype], _rowmajor(At_lp, "At_lp"), _ptr(At64),
                              _rowmajor(At64, "At64"), d, n, _ptr(Bt), nrhs, _rowmajor(Bt, "Bt"), _ptr(nu2),
                              int(trial_iters), ctypes.byref(rep), _ptr(ws), ws.numel(), _stream(stream)),
           "csk_tune_mrhs")
    return _report(rep)


def csk_tune_save(path: str) -> None:
    """Writes every tuned choice of this process to `path`."""
    _check(_lib.csk_tune_save(os.fsencode(path)), "csk_tune_save")


def csk_tune_load(path: str) -> int:
    """Merges the tuned choices in `path` (a file written by csk_tune_save
    with this library version); returns the count read, -1 for none."""
    k = ctypes.c_int32(0)
    _check(_lib.csk_tune_load(os.fsencode(path), ctypes.byref(k)), "csk_tune_load")
    return int(k.value)


def csk_tune_lookup(d: int, n: int, dtype: torch.dtype, vector_rows: bool = True) -> dict:
    """The cached launch shape for (d, n, dtype) on the current device
    (grid 0: none)."""
    e = _abi.TuneEntry()
    _check(_lib.csk_tune_lookup(d, n, _TORCH_TO_CSK[dtype], 1 if vector_rows else 0, ctypes.byref(e)),
           "csk_tune_lookup")
    return dict(grid=e.grid, lanes_per_row=e.lanes_per_row, us_per_iter=e.us_per_iter)


def csk_tune_clear() -> None:
    """Empties the cache of tuned launch shapes."""
    _lib.csk_tune_clear()
