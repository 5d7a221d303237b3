"""GPU parity of the mixed-precision loop on the sketch of a CSR matrix whose
refresh residual is S (b - A x) from the CSR A (csk_solve_csr_refresh), in
place of bt - At64 x.

With a refresh every iteration every residual the loop selects from is the
exact one, so its selected rows for iterations 0..K-1 equal the FP64
oracle's (Algorithm 1's loop on the oracle's sketch) bit for bit and the
iterate after K steps agrees element by element to 1e-12 of its norm.  With
the default window the converged solution is checked against x* and the
oracle's, and the iteration count against the refresh from At64."""
import numpy as np
import pytest
import torch

from _compare import assert_iterate_close, assert_trace_equal, new_trace
from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _system(gpu, orc, m, n, dens, d, seed, lp=torch.float32):
    s = W.sparse_csr(m, n, dens, seed=seed)
    rp, col, val, b = (torch.from_numpy(a).to(DEV) for a in (s.row_ptr, s.col, s.val, s.b))
    sk = gpu.csk_sketch_csr(rp, col, val, n, b, d, seed + 7, lp_dtype=lp)
    torch.cuda.synchronize()
    At, bt = orc.sketch_csr(s.row_ptr, s.col, s.val, m, n, s.b, d, seed + 7)
    return s, (rp, col, val, b), sk, At, bt


@pytest.mark.parametrize("lp,single_wg", [(torch.float32, 0), (torch.bfloat16, 0), (torch.float32, 1)])
def test_csr_refresh_every_iteration_follows_oracle(gpu, orc, lp, single_wg):
    m, n, dens, d, seed, K = 20000, 300, 0.01, 1500, 41, 60
    s, (rp, col, val, b), sk, At, bt = _system(gpu, orc, m, n, dens, d, seed, lp)
    xs = torch.from_numpy(s.x_star).to(DEV)
    trace = new_trace(K)
    r = gpu.csk_solve_csr_refresh(sk.At_lp, sk.bt, rp, col, val, b, seed + 7, At64=sk.At64, nu2=sk.nu2,
                                  x_ref=xs, tol=0.0, maxit=K, refresh_every=1, single_wg=single_wg,
                                  trace_idx=trace)
    o = orc.mwrk(At, bt, xref=s.x_star, tol=0.0, maxit=K, trace=True)
    assert r.iters == K == o.iters
    assert r.refreshes == K + 1 or r.refreshes == K
    assert_trace_equal(trace, o.idx)
    assert_iterate_close(r.x, o.x)


def test_csr_refresh_converges_like_the_refresh_from_at64(gpu, orc):
    m, n, dens, d, seed = 40000, 500, 0.006, 3000, 43
    s, (rp, col, val, b), sk, At, bt = _system(gpu, orc, m, n, dens, d, seed)
    xs = torch.from_numpy(s.x_star).to(DEV)
    tol = 1e-8
    ra = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=xs, tol=tol, maxit=200000)
    rc = gpu.csk_solve_csr_refresh(sk.At_lp, sk.bt, rp, col, val, b, seed + 7, At64=sk.At64, nu2=sk.nu2,
                                   x_ref=xs, tol=tol, maxit=200000)
    assert ra.status == gpu.CSK_OK and rc.status == gpu.CSK_OK
    assert abs(rc.iters - ra.iters) <= 0.02 * ra.iters + 2, (rc.iters, ra.iters)
    xstar = s.x_star
    rel = np.linalg.norm(rc.x.cpu().numpy() - xstar) / np.linalg.norm(xstar)
    assert rel <= tol
    o = orc.mwrk(At, bt, xref=xstar, tol=tol, maxit=200000)
    assert np.linalg.norm(rc.x.cpu().numpy() - o.x) <= 2 * tol * np.linalg.norm(xstar)


def test_csr_refresh_rejects_fp64_and_missing_arrays(gpu, orc):
    s, (rp, col, val, b), sk, At, bt = _system(gpu, orc, 2000, 100, 0.02, 200, 45)
    with pytest.raises(gpu.CskError):
        gpu.csk_solve_csr_refresh(sk.At64, sk.bt, rp, col, val, b, 52, At64=sk.At64, maxit=5)
    with pytest.raises(TypeError):
        gpu.csk_solve_csr_refresh(sk.At_lp, sk.bt, rp, col.long(), val, b, 52, At64=sk.At64, maxit=5)
