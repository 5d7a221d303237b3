"""GPU parity of the randomized selection rules on the FP64 sketch: the
relaxed greedy randomized rule (theta = 1/2: greedy randomized Kaczmarz;
theta = 1: Algorithm 1's greedy rule) and randomized Kaczmarz.

Both sides draw the same uniforms (the selection stream of the seed), so the
rows drawn are the same as long as no draw sits within rounding of a
boundary: the relaxed greedy rule's keys and working-set test read residuals
summed in another order than the oracle's, and randomized Kaczmarz's
cumulative norms start from squared norms summed in another order.  The rows
drawn in iterations 0..K-1 are compared bit for bit with the oracle's, the
iterate after K steps element by element to 1e-12 of its norm, converged
solutions against x* and the oracle's."""
import numpy as np
import pytest
import torch

from _compare import assert_iterate_close, assert_trace_equal, new_trace
from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _relerr(x, xs):
    return np.linalg.norm(x - xs) / np.linalg.norm(xs)


def _setup(gpu, orc, m, n, d, seed, sketch_seed):
    s = W.gaussian(m, n, seed, device=DEV)
    sk = gpu.csk_sketch(s.A, s.b, d, sketch_seed)
    torch.cuda.synchronize()
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), d, sketch_seed)
    return s, sk, At, bt


@pytest.mark.parametrize("theta", [0.5, 0.8, 1.0])
@pytest.mark.parametrize("path,K", [("single", 1), ("single", 40), ("grid", 1), ("grid", 9), ("grid", 70)])
def test_rgrk_iterates_match_oracle(gpu, orc, theta, path, K):
    s, sk, At, bt = _setup(gpu, orc, 20000, 150, 1900, 61, 62)
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=24)
    tr = new_trace(K)
    r = gpu.csk_solve_rgrk(sk.At64, sk.bt, theta=theta, sel_seed=77, nu2=sk.nu2, x_ref=s.x_star, tol=0.0,
                           maxit=K, trace_idx=tr, **kw)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == K
    o = orc.rgrk(At, bt, theta=theta, sel_seed=77, xref=s.x_star.cpu().numpy(), tol=0.0, maxit=K, trace=True)
    assert_trace_equal(tr, o.idx)
    assert_iterate_close(r.x, o.x)


@pytest.mark.parametrize("path", ["single", "grid"])
def test_rgrk_theta_one_is_the_greedy_solve(gpu, orc, path):
    # the same residuals, the same best row, the same step: bitwise csk_solve
    s, sk, At, bt = _setup(gpu, orc, 20000, 150, 1900, 63, 64)
    kw = dict(single_wg=1) if path == "single" else dict(single_wg=0, grid=24)
    a = gpu.csk_solve_rgrk(sk.At64, sk.bt, theta=1.0, sel_seed=5, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10,
                           maxit=100000, **kw)
    b = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10, maxit=100000, **kw)
    assert a.status == b.status == gpu.CSK_OK
    assert a.iters == b.iters
    assert torch.equal(a.x, b.x)


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_rgrk_converges_and_matches_oracle(gpu, orc, theta):
    s, sk, At, bt = _setup(gpu, orc, 20000, 120, 1600, 65, 66)
    xs = s.x_star.cpu().numpy()
    r = gpu.csk_solve_rgrk(sk.At64, sk.bt, theta=theta, sel_seed=9, x_ref=s.x_star, tol=1e-10, maxit=200000)
    assert r.status == gpu.CSK_OK
    assert _relerr(r.x.cpu().numpy(), xs) <= 1e-10
    o = orc.rgrk(At, bt, theta=theta, sel_seed=9, xref=xs, tol=1e-10, maxit=200000)
    assert o.status == 0
    assert np.linalg.norm(r.x.cpu().numpy() - o.x) <= 3e-10 * np.linalg.norm(xs)
    # the same draws while no near-boundary row intervenes: counts agree closely
    assert abs(r.iters - o.iters) <= max(5, 0.1 * o.iters), (r.iters, o.iters)


def test_rgrk_grid_shape_and_residual_mode(gpu, orc):
    s, sk, At, bt = _setup(gpu, orc, 30000, 200, 2500, 67, 68)
    xs = s.x_star.cpu().numpy()
    ta, tb = new_trace(50), new_trace(50)
    xa = gpu.csk_solve_rgrk(sk.At64, sk.bt, sel_seed=3, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=50, grid=8,
                            trace_idx=ta).x
    xb = gpu.csk_solve_rgrk(sk.At64, sk.bt, sel_seed=3, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=50, grid=40,
                            trace_idx=tb).x
    assert torch.equal(ta, tb)
    assert_iterate_close(xa, xb)
    # residual stop, norms computed by the library
    r = gpu.csk_solve_rgrk(sk.At64, sk.bt, sel_seed=3, tol=1e-9, maxit=200000, stop_mode=gpu.CSK_STOP_REL_RESID,
                           single_wg=0)
    assert r.status == gpu.CSK_OK
    x = r.x.cpu().numpy()
    assert np.linalg.norm(bt - At @ x) <= 1e-9 * np.linalg.norm(bt) * (1 + 1e-6)
    # determinism: same seed and shape, same bits
    r2 = gpu.csk_solve_rgrk(sk.At64, sk.bt, sel_seed=3, tol=1e-9, maxit=200000, stop_mode=gpu.CSK_STOP_REL_RESID,
                            single_wg=0)
    assert torch.equal(r.x, r2.x) and r.iters == r2.iters


def test_rgrk_full_size_first_steps_and_convergence(gpu, orc):
    # the headline workload (A 200000 x 1000 uniform entries, d = 20000) with
    # the greedy randomized rule: the first iterates against the oracle, then
    # the solve to 1e-10
    c = W.config("dense_coherent")
    s = W.uniform01(c["m"], c["n"], c["seed"], device=DEV)
    sk = gpu.csk_sketch(s.A, s.b, c["d"], c["sketch_seed"])
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), c["d"], c["sketch_seed"])
    xs = s.x_star.cpu().numpy()
    tr = new_trace(4)
    r = gpu.csk_solve_rgrk(sk.At64, sk.bt, theta=0.5, sel_seed=1, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=4,
                           trace_idx=tr)
    o = orc.rgrk(At, bt, theta=0.5, sel_seed=1, xref=xs, tol=0.0, maxit=4, trace=True)
    assert_trace_equal(tr, o.idx)
    assert_iterate_close(r.x, o.x)
    r = gpu.csk_solve_rgrk(sk.At64, sk.bt, theta=0.5, sel_seed=1, nu2=sk.nu2, x_ref=s.x_star, tol=c["tol"],
                           maxit=10 * c["maxit"])
    assert r.status == gpu.CSK_OK, r.status_name
    assert _relerr(r.x.cpu().numpy(), xs) <= c["tol"]
    print(f"greedy randomized iterations {r.iters}")


@pytest.mark.parametrize("n,K", [(150, 1), (150, 700), (150, 1500), (1100, 1100), (37, 2000)])
def test_rk_iterates_match_oracle(gpu, orc, n, K):
    # K crosses the 512-iteration draw batches; n = 1100 gives three columns
    # per thread with a ragged tail
    s, sk, At, bt = _setup(gpu, orc, 12 * n + 500, n, 6 * n + 50, 70 + n, 71)
    tr = new_trace(K)
    r = gpu.csk_solve_rk(sk.At64, sk.bt, sel_seed=8, nu2=sk.nu2, x_ref=s.x_star, tol=0.0, maxit=K, trace_idx=tr)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == K
    o = orc.rk(At, bt, sel_seed=8, xref=s.x_star.cpu().numpy(), tol=0.0, maxit=K, trace=True)
    assert_trace_equal(tr, o.idx)
    assert_iterate_close(r.x, o.x)


@pytest.mark.parametrize("n", [900, 3000, 8192])
def test_rk_wide_rows_match_oracle(gpu, orc, n):
    # 2, 8 and 16 columns per thread (ring depths 4, 2 and 1), on a plain
    # random system (the rule takes any matrix); 600 steps cross a draw batch
    d, K = 1500, 600
    g = torch.Generator().manual_seed(n)
    A = torch.randn(d, n, dtype=torch.float64, generator=g)
    xs = torch.randn(n, dtype=torch.float64, generator=g)
    b = A @ xs
    An, bn, xn = A.numpy(), b.numpy(), xs.numpy()
    tr = new_trace(K)
    r = gpu.csk_solve_rk(A.to(DEV), b.to(DEV), sel_seed=12, x_ref=xs.to(DEV), tol=0.0, maxit=K, trace_idx=tr)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == K
    o = orc.rk(An, bn, sel_seed=12, xref=xn, tol=0.0, maxit=K, trace=True)
    assert_trace_equal(tr, o.idx)
    assert_iterate_close(r.x, o.x)


def test_rk_converges_with_library_norms_and_x0(gpu, orc):
    s, sk, At, bt = _setup(gpu, orc, 8000, 60, 900, 81, 82)
    xs = s.x_star.cpu().numpy()
    x0 = torch.randn(60, dtype=torch.float64, generator=torch.Generator().manual_seed(2)).to(DEV)
    r = gpu.csk_solve_rk(sk.At64, sk.bt, sel_seed=4, x0=x0, x_ref=s.x_star, tol=1e-8, maxit=2000000)
    assert r.status == gpu.CSK_OK
    assert _relerr(r.x.cpu().numpy(), xs) <= 1e-8
    o = orc.rk(At, bt, sel_seed=4, x0=x0.cpu().numpy(), xref=xs, tol=1e-8, maxit=2000000)
    assert o.status == 0
    assert abs(r.iters - o.iters) <= max(5, 0.02 * o.iters), (r.iters, o.iters)


def test_select_status_paths(gpu):
    Z = torch.zeros(6, 3, dtype=torch.float64, device=DEV)
    one6 = torch.ones(6, dtype=torch.float64, device=DEV)
    one3 = torch.ones(3, dtype=torch.float64, device=DEV)
    assert gpu.csk_solve_rgrk(Z, one6, x_ref=one3, tol=1e-10, maxit=10).status == gpu.CSK_ERR_DEGENERATE
    assert gpu.csk_solve_rk(Z, one6, x_ref=one3, tol=1e-10, maxit=10).status == gpu.CSK_ERR_DEGENERATE
    # rows far from orthogonal: three projections do not reach x* exactly
    A = torch.tensor([[1.0, 0.3, 0.1], [0.2, 2.0, 0.7], [0.4, 0.6, 0.5], [1.0, 1.0, 1.0]], dtype=torch.float64,
                     device=DEV)
    xs = torch.tensor([1.0, -2.0, 3.0], dtype=torch.float64, device=DEV)
    b = A @ xs
    r = gpu.csk_solve_rgrk(A, b, x_ref=xs, tol=0.0, maxit=3)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == 3
    r = gpu.csk_solve_rk(A, b, x_ref=xs, tol=0.0, maxit=3)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == 3
    r = gpu.csk_solve_rk(A, b, x_ref=xs, tol=1e-12, maxit=100000)
    assert r.status == gpu.CSK_OK
    # maxit 0: x0 returned untouched, the stop measure of x0 reported
    r = gpu.csk_solve_rk(A, b, x_ref=xs, tol=0.0, maxit=0)
    assert r.status == gpu.CSK_NOT_CONVERGED and r.iters == 0 and torch.count_nonzero(r.x) == 0
    with pytest.raises(gpu.CskError):
        gpu.csk_solve_rgrk(A, b, theta=2.0, x_ref=xs)
    # a NaN in the right-hand side reaches a weighted residual; a NaN norm
    # makes the row distribution undefined
    bn = b.clone()
    bn[1] = float("nan")
    assert gpu.csk_solve_rgrk(A, bn, x_ref=xs, tol=1e-12, maxit=100).status == gpu.CSK_ERR_NONFINITE
    for single in (0, 1):
        r = gpu.csk_solve_rgrk(A, bn, x_ref=xs, tol=1e-12, maxit=100, single_wg=single)
        assert r.status == gpu.CSK_ERR_NONFINITE
    nun = (A * A).sum(1)
    nun[2] = float("nan")
    assert gpu.csk_solve_rk(A, b, nu2=nun, x_ref=xs, tol=1e-12, maxit=100).status == gpu.CSK_ERR_NONFINITE
    # one workgroup cannot keep the residuals of 30000 rows in LDS: refused
    # before launch, with a message; the grid path takes the same system
    big = torch.randn(30000, 8, dtype=torch.float64, device=DEV)
    bb = big @ xs.new_ones(8)
    with pytest.raises(gpu.CskError) as ei:
        gpu.csk_solve_rgrk(big, bb, x_ref=xs.new_ones(8), tol=1e-8, maxit=100, single_wg=1)
    assert ei.value.status == gpu.CSK_ERR_UNSUPPORTED
    assert "LDS" in str(ei.value)
    r = gpu.csk_solve_rgrk(big, bb, x_ref=xs.new_ones(8), tol=1e-8, maxit=100000, single_wg=0)
    assert r.status == gpu.CSK_OK
