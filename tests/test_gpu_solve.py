"""GPU parity of the MWRK loop (Algorithm 1, loop; Section 3 stopping rule).

Floating-point residuals are summed in a different order than the oracle's,
so trajectories are compared step by step while no near-tie intervenes: the
rows selected in iterations 0..K-1 equal the oracle's bit for bit, and the
iterate after K steps agrees with the oracle's element by element to 1e-12 of
its norm.  Converged solutions agree with x* to the requested tolerance and
with the oracle's converged solution to twice it.  The mixed-precision loop
starts with an exact FP64 refresh, so its first step equals the oracle's
FP64 step; its converged solution is held to the same bounds.  Status paths,
determinism and resume are checked directly."""
import os

import numpy as np
import pytest
import torch

from _compare import assert_iterate_close, assert_trace_equal, new_trace
from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def relerr(x, xs):
    x = x.cpu().numpy() if torch.is_tensor(x) else x
    xs = xs.cpu().numpy() if torch.is_tensor(xs) else xs
    return np.linalg.norm(x - xs) / np.linalg.norm(xs)


def sketched(gpu, s, d, seed, lp=None):
    out = gpu.csk_sketch(s.A, s.b, d, seed, lp_dtype=lp)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("path", ["single", "grid"])
def test_oracle_size_converges_and_matches_oracle(gpu, orc, path):
    c = W.config("oracle_small")
    s = W.gaussian(c["m"], c["n"], c["seed"], device=DEV)
    sk = sketched(gpu, s, c["d"], c["sketch_seed"])
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=8)
    r = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10, maxit=100000, **kw)
    assert r.status == gpu.CSK_OK, r.status_name
    assert relerr(r.x, s.x_star) <= 1e-10
    o = orc.csk(s.A.cpu().numpy(), s.b.cpu().numpy(), c["d"], c["sketch_seed"], xref=s.x_star.cpu().numpy(),
                tol=1e-10, maxit=100000)
    assert relerr(r.x, o.x) <= 3e-10
    assert abs(r.iters - o.iters) <= max(5, 0.1 * o.iters), (r.iters, o.iters)


@pytest.mark.parametrize("path,K", [("single", 1), ("single", 7), ("single", 60), ("grid", 1), ("grid", 7),
                                    ("grid", 60)])
def test_iterates_match_oracle_step_by_step(gpu, orc, path, K):
    s = W.gaussian(12000, 90, seed=21, device=DEV)
    sk = sketched(gpu, s, 1100, 22)
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=16)
    tr = new_trace(K)
    r = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=K, trace_idx=tr, **kw)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == K
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), 1100, 22)
    o = orc.mwrk(At, bt, xref=s.x_star.cpu().numpy(), tol=0.0, maxit=K, trace=True)
    assert_trace_equal(tr, o.idx)
    assert_iterate_close(r.x, o.x)


@pytest.mark.parametrize("grid", [5, 13, 22, 255])
def test_exchange_with_a_short_last_record_group(gpu, orc, grid):
    # the grid exchange interleaves the records of four workgroups; with a
    # grid that is not a multiple of four the last group is shorter (one,
    # one, two and three records here) and must still map every word once
    s = W.gaussian(12000, 90, seed=21, device=DEV)
    sk = sketched(gpu, s, 1100, 22)
    K = 40
    tr = new_trace(K)
    r = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=K, trace_idx=tr, single_wg=0,
                      grid=grid)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == K
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), 1100, 22)
    o = orc.mwrk(At, bt, xref=s.x_star.cpu().numpy(), tol=0.0, maxit=K, trace=True)
    assert_trace_equal(tr, o.idx, f"grid={grid}")
    assert_iterate_close(r.x, o.x, what=f"grid={grid}")


@pytest.mark.parametrize("path,m,n,d,grid", [("single", 8000, 60, 1500, 1), ("grid", 60000, 90, 9000, 8),
                                              ("grid", 40000, 1000, 20000, 16)])
def test_alternating_walk_iterates_match_oracle(gpu, orc, path, m, n, d, grid):
    # shapes whose workgroups stream rows past the LDS-resident ones, with one
    # or two segments per row and lane groups of unequal row counts: the odd
    # iterations walk those rows backwards
    s = W.gaussian(m, n, seed=m + n, device=DEV)
    sk = sketched(gpu, s, d, 5)
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=grid)
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), d, 5)
    for K in (1, 2, 25):
        tr = new_trace(K)
        r = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=K, trace_idx=tr, **kw)
        assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == K
        o = orc.mwrk(At, bt, xref=s.x_star.cpu().numpy(), tol=0.0, maxit=K, trace=True)
        assert_trace_equal(tr, o.idx, f"{path} K={K}")
        assert_iterate_close(r.x, o.x, what=f"{path} K={K}")


def test_full_size_dense_coherent(gpu, orc):
    # the benchmark workload end to end: every output checked against x*
    # (any size) and the first iterates against the oracle
    c = W.config("dense_coherent")
    s = W.uniform01(c["m"], c["n"], c["seed"], device=DEV)
    sk = sketched(gpu, s, c["d"], c["sketch_seed"])
    tr = new_trace(3)
    r3 = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=3, trace_idx=tr)
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), c["d"], c["sketch_seed"])
    o3 = orc.mwrk(At, bt, xref=s.x_star.cpu().numpy(), tol=0.0, maxit=3, trace=True)
    assert_trace_equal(tr, o3.idx)
    assert_iterate_close(r3.x, o3.x)
    r = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=c["tol"], maxit=c["maxit"])
    assert r.status == gpu.CSK_OK, r.status_name
    assert relerr(r.x, s.x_star) <= 1e-10
    print(f"dense_coherent iterations {r.iters}")


def oracle_threads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.mark.parametrize("path", ["single", "grid"])
@pytest.mark.parametrize("n", [200, 203])  # whole 16-byte vectors, and a masked tail
@pytest.mark.parametrize("lp", [torch.bfloat16, torch.float16, torch.float32])
def test_mixed_precision_matches_oracle(gpu, orc, lp, n, path):
    # the mixed loop's iteration 0 is an exact FP64 refresh: the same row and
    # the same step as the oracle's FP64 loop; the converged solution lies
    # within twice the tolerance of the oracle's FP64 solution
    s = W.row_scaled(60000, n, seed=31, device=DEV)
    sk = sketched(gpu, s, 2000, 32, lp=lp)
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=16)
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), 2000, 32)
    xs = s.x_star.cpu().numpy()
    tr = new_trace(1)
    r1 = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=1, trace_idx=tr,
                       **kw)
    o1 = orc.mwrk(At, bt, xref=xs, tol=0.0, maxit=1, trace=True)
    assert r1.iters == 1 and r1.refreshes == 1
    assert_trace_equal(tr, o1.idx)
    assert_iterate_close(r1.x, o1.x)
    tol = 1e-10
    r = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=tol, maxit=200000, **kw)
    o = orc.mwrk(At, bt, xref=xs, tol=tol, maxit=200000)
    assert r.status == gpu.CSK_OK and o.status == orc.OK, (r.status_name, o.status)
    assert relerr(r.x, xs) <= tol
    assert np.linalg.norm(r.x.cpu().numpy() - o.x) <= 2 * tol * np.linalg.norm(xs)
    assert r.iters <= 1.5 * o.iters + 64, (r.iters, o.iters)
    print(f"mixed {lp} n={n} {path}: iterations {r.iters} (oracle FP64 {o.iters}), "
          f"|x - x_oracle|/|x*| = {np.linalg.norm(r.x.cpu().numpy() - o.x) / np.linalg.norm(xs):.2e}")


@pytest.mark.parametrize("n", [200, 203])  # whole 16-byte vectors, and a masked tail
@pytest.mark.parametrize("lp", [torch.bfloat16, torch.float16, torch.float32])
def test_mixed_precision_reaches_1e10(gpu, lp, n):
    s = W.row_scaled(60000, n, seed=31, device=DEV)
    sk = sketched(gpu, s, 2000, 32, lp=lp)
    r64 = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10, maxit=200000)
    r = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10, maxit=200000)
    assert r64.status == gpu.CSK_OK and r.status == gpu.CSK_OK, (r64.status_name, r.status_name)
    assert relerr(r.x, s.x_star) <= 1e-10
    assert r.iters <= 1.5 * r64.iters + 64, (r.iters, r64.iters)
    assert r.refreshes >= r.iters // 64


@pytest.mark.parametrize("path", ["single", "grid"])
def test_residual_stopping_rule(gpu, path):
    s = W.gaussian(20000, 60, seed=41, device=DEV)
    sk = sketched(gpu, s, 1200, 42)
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=12)
    r = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, tol=1e-9, maxit=100000, stop_mode=gpu.CSK_STOP_REL_RESID, **kw)
    assert r.status == gpu.CSK_OK
    res = (sk.bt - sk.At64 @ r.x).norm() / sk.bt.norm()
    assert res.item() <= 1e-9 * (1 + 1e-6)
    rb = gpu.csk_solve(sk.At_lp if sk.At_lp is not None else sk.At64.float(), sk.bt, At64=sk.At64, nu2=sk.nu2,
                       tol=1e-9, maxit=100000, stop_mode=gpu.CSK_STOP_REL_RESID, **kw)
    assert rb.status == gpu.CSK_OK
    res = (sk.bt - sk.At64 @ rb.x).norm() / sk.bt.norm()
    assert res.item() <= 1e-9 * (1 + 1e-6)


@pytest.mark.parametrize("path", ["single", "grid"])
def test_status_paths(gpu, path):
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=4)
    n = 8
    z = torch.zeros((40, n), dtype=torch.float64, device=DEV)
    xr = torch.ones(n, dtype=torch.float64, device=DEV)
    r = gpu.csk_solve(z, torch.zeros(40, dtype=torch.float64, device=DEV), x_ref=xr, tol=1e-10, maxit=10, **kw)
    assert r.status == gpu.CSK_ERR_DEGENERATE and r.iters == 0
    A = torch.eye(n, dtype=torch.float64, device=DEV).repeat(5, 1)
    bt = A @ xr
    bt[3] = float("nan")
    r = gpu.csk_solve(A, bt, x_ref=xr, tol=1e-10, maxit=10, **kw)
    assert r.status == gpu.CSK_ERR_NONFINITE
    s = W.gaussian(500, 10, seed=1, device=DEV)
    r = gpu.csk_solve(s.A, s.b, x_ref=s.x_star, tol=1e-14, maxit=3, **kw)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == 3
    # a solve that starts at the solution stops before any projection
    r = gpu.csk_solve(s.A, s.b, x0=s.x_star, x_ref=s.x_star, tol=1e-10, maxit=3, **kw)
    assert r.status == gpu.CSK_OK and r.iters == 0


def test_cancel_word(gpu):
    # host-mapped pinned word set before the launch: the solve stops at its
    # first poll with CSK_CANCELLED (no kernel waits on the host)
    flag = torch.ones(1, dtype=torch.int32).pin_memory()
    s = W.gaussian(4000, 30, seed=2, device=DEV)
    for kw in (dict(single_wg=1), dict(single_wg=0, grid=4)):
        r = gpu.csk_solve(s.A, s.b, x_ref=s.x_star, tol=1e-12, maxit=1000, cancel=flag.data_ptr(), **kw)
        assert r.status == gpu.CSK_CANCELLED and r.iters == 0
    flag.zero_()
    r = gpu.csk_solve(s.A, s.b, x_ref=s.x_star, tol=1e-12, maxit=100000, cancel=flag.data_ptr())
    assert r.status == gpu.CSK_OK


@pytest.mark.parametrize("path", ["single", "grid"])
def test_deterministic_and_resumable(gpu, path):
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=32)
    s = W.gaussian(40000, 150, seed=51, device=DEV)
    sk = sketched(gpu, s, 3000, 52)
    a = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=300, **kw)
    b = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=300, **kw)
    assert torch.equal(a.x, b.x)
    h = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=120, **kw)
    c = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x0=h.x.clone(), x_ref=s.x_star, tol=0.0, maxit=180, **kw)
    assert torch.equal(a.x, c.x)


def test_nu2_computed_when_absent(gpu):
    s = W.gaussian(8000, 64, seed=61, device=DEV)
    sk = sketched(gpu, s, 700, 62)
    a = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10)
    b = gpu.csk_solve(sk.At64, sk.bt, x_ref=s.x_star, tol=1e-10)
    assert a.status == b.status == gpu.CSK_OK
    assert relerr(b.x, s.x_star) <= 1e-10


_ROW_SCALED = {}


def row_scaled_oracle(orc, s, c):
    """The oracle's sketch, first step and converged FP64 solution of the
    full row-scaled workload (computed once per session, on the host cores;
    bitwise the single-thread oracle)."""
    if not _ROW_SCALED:
        xs = s.x_star.cpu().numpy()
        with orc.threads(oracle_threads()):
            At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), c["d"], c["sketch_seed"])
            o1 = orc.mwrk(At, bt, xref=xs, tol=0.0, maxit=1, trace=True)
            o = orc.mwrk(At, bt, xref=xs, tol=c["tol"], maxit=c["maxit"])
        _ROW_SCALED.update(o1=o1, o=o)
    return _ROW_SCALED["o1"], _ROW_SCALED["o"]


@pytest.mark.parametrize("lp", [torch.bfloat16, torch.float16, torch.float32])
def test_mixed_full_size_row_scaled(gpu, orc, lp):
    # rows scaled over four decades: the FP16 operand copy of x - x_ref is
    # rescaled at every refresh; every low-precision format reaches 1e-10
    # without the FP64 fallback, in about the FP64 loop's iteration count;
    # the first step equals the oracle's and the solution lies within twice
    # the tolerance of the oracle's FP64 solution
    c = W.config("row_scaled")
    s = W.row_scaled(c["m"], c["n"], c["seed"], device=DEV)
    sk = sketched(gpu, s, c["d"], c["sketch_seed"], lp=lp)
    o1, o = row_scaled_oracle(orc, s, c)
    tr = new_trace(1)
    r1 = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=1, trace_idx=tr)
    assert_trace_equal(tr, o1.idx)
    assert_iterate_close(r1.x, o1.x)
    r = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=c["tol"], maxit=c["maxit"])
    assert r.status == gpu.CSK_OK, r.status_name
    assert relerr(r.x, s.x_star) <= c["tol"]
    assert r.fp64_fallback == 0
    assert r.iters <= 6400, r.iters
    xs = s.x_star.cpu().numpy()
    assert o.status == orc.OK
    dif = np.linalg.norm(r.x.cpu().numpy() - o.x) / np.linalg.norm(xs)
    assert dif <= 2 * c["tol"]
    print(f"row_scaled {lp} iterations {r.iters} (oracle FP64 {o.iters}) refreshes {r.refreshes} "
          f"fallback {r.fp64_fallback} |x - x_oracle|/|x*| = {dif:.2e}")
