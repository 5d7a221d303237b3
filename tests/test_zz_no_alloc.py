"""csk_solve_noalloc (the solve whose workspace is the library's static
scratch) against csk_solve with a caller workspace, through the C ABI.

Both run the same kernels with the same launch shape, so x, the iteration
count, the status and the final stop measure must agree bit for bit.  Two
calls in a row share the scratch: a large grid-path solve (nu2 computed into
the scratch, mixed precision with its FP64 refresh residual there too), then
a smaller one, so leftovers of the first call must not leak into the second.
A solve whose workspace exceeds the scratch is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2004_02480_amd import _abi
from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
P = ctypes.c_void_p


def _ptr(t):
    return None if t is None else P(t.data_ptr())


def _opts(x_ref, tol, maxit, grid=0, single_wg=-1):
    o = _abi.SolveOpts()
    o.tol = tol
    o.maxit = maxit
    o.stop_mode = _abi.CSK_STOP_REL_ERR
    o.refresh_every = 64
    o.x_ref = x_ref.data_ptr()
    o.cancel = None
    o.check_every = 256
    o.grid = grid
    o.block = 0
    o.single_wg = single_wg
    o.trace_idx = None
    return o


def _results(raw):
    b = raw.cpu().numpy().tobytes()
    return (np.frombuffer(b[0:8], np.int64)[0], np.frombuffer(b[8:12], np.int32)[0],
            np.frombuffer(b[16:24], np.float64)[0])


def _both(lib, At, at_code, At64, bt, nu2, x_ref, n, d, o):
    """(x, result) of csk_solve with its own workspace, then of csk_solve_noalloc."""
    ldat = At.stride(0)
    ld64 = At64.stride(0) if At64 is not None else ldat
    nb = ctypes.c_size_t(0)
    assert lib.csk_solve_workspace_size(d, n, at_code, ctypes.byref(nb)) == _abi.CSK_OK
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=DEV)
    ws = ws[(-ws.data_ptr()) % 256:]
    x1 = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    r1 = torch.zeros(_abi.RESULT_BYTES, dtype=torch.uint8, device=DEV)
    st = lib.csk_solve(_ptr(At), at_code, ldat, _ptr(At64), ld64, d, n, _ptr(bt), _ptr(nu2), None, _ptr(x1),
                       ctypes.byref(o), _ptr(r1), _ptr(ws), ws.numel(), None)
    assert st == _abi.CSK_OK, lib.csk_last_error()
    x2 = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    r2 = torch.zeros(_abi.RESULT_BYTES, dtype=torch.uint8, device=DEV)
    st = lib.csk_solve_noalloc(_ptr(At), at_code, ldat, _ptr(At64), ld64, d, n, _ptr(bt), _ptr(nu2), None,
                               _ptr(x2), ctypes.byref(o), _ptr(r2), None)
    assert st == _abi.CSK_OK, lib.csk_last_error()
    torch.cuda.synchronize()
    return (x1.cpu().numpy(), _results(r1)), (x2.cpu().numpy(), _results(r2))


def _check_same(a, b, x_star, tol):
    (x1, (it1, st1, m1)), (x2, (it2, st2, m2)) = a, b
    assert st1 == _abi.CSK_OK and st2 == _abi.CSK_OK, (st1, st2)
    assert it1 == it2 and m1.tobytes() == m2.tobytes(), ((it1, m1), (it2, m2))
    assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))
    assert np.linalg.norm(x2 - x_star) / np.linalg.norm(x_star) <= tol


@pytest.mark.parametrize("lp", [None, torch.bfloat16])
def test_noalloc_matches_csk_solve_large_then_small(gpu, lp):
    lib = gpu.lib
    # first call: a grid-path solve over 64 workgroups, nu2 computed in the scratch
    s = W.gaussian(40000, 200, seed=71, dtype=torch.float32 if lp is not None else torch.float64, device=DEV)
    sk = gpu.csk_sketch(s.A, s.b, 6000, 72, lp_dtype=lp)
    torch.cuda.synchronize()
    At, code = (sk.At_lp, _abi.CSK_BF16) if lp is not None else (sk.At64, _abi.CSK_F64)
    o = _opts(s.x_star, 1e-10, 100000, grid=64, single_wg=0)
    a, b = _both(lib, At, code, sk.At64, sk.bt, None, s.x_star, 200, 6000, o)
    _check_same(a, b, s.x_star.cpu().numpy(), 1e-10)
    # second call, smaller: one workgroup, given norms
    s2 = W.gaussian(2000, 50, seed=73, device=DEV)
    sk2 = gpu.csk_sketch(s2.A, s2.b, 500, 74)
    torch.cuda.synchronize()
    o2 = _opts(s2.x_star, 1e-10, 100000)
    a, b = _both(lib, sk2.At64, _abi.CSK_F64, None, sk2.bt, sk2.nu2, s2.x_star, 50, 500, o2)
    _check_same(a, b, s2.x_star.cpu().numpy(), 1e-10)


def test_noalloc_second_smaller_grid_call_reuses_scratch(gpu):
    """Two grid-path calls in a row on the same scratch: the exchange records
    of the first (more workgroups, later iteration tags) must not be taken
    for the second's."""
    lib = gpu.lib
    for (m, n, d, seed, grid) in ((60000, 300, 9000, 81, 128), (20000, 120, 3000, 83, 16)):
        s = W.gaussian(m, n, seed=seed, device=DEV)
        sk = gpu.csk_sketch(s.A, s.b, d, seed + 1)
        torch.cuda.synchronize()
        o = _opts(s.x_star, 1e-10, 100000, grid=grid, single_wg=0)
        a, b = _both(lib, sk.At64, _abi.CSK_F64, None, sk.bt, None, s.x_star, n, d, o)
        _check_same(a, b, s.x_star.cpu().numpy(), 1e-10)


def test_noalloc_refuses_a_workspace_beyond_the_scratch(gpu):
    """d = 600000 rows need 9.6 MB of workspace: refused before any launch
    (the pointers are never dereferenced)."""
    lib = gpu.lib
    d, n = 600000, 16
    fake = P(256)
    xr = torch.zeros(n, dtype=torch.float64, device=DEV)
    o = _opts(xr, 1e-10, 10)
    st = lib.csk_solve_noalloc(fake, _abi.CSK_F64, n, None, n, d, n, fake, None, None, fake,
                               ctypes.byref(o), fake, None)
    assert st == _abi.CSK_ERR_WORKSPACE
    assert b"scratch" in lib.csk_last_error()
