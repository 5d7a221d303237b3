"""GPU parity of the multi-right-hand-side form: the loop of Algorithm 1 run
for every column of Bt on one shared sketch, with the residuals formed on the
matrix cores.  Every column's solution meets the tolerance against its x* and
agrees with the oracle's single-column solution."""
import numpy as np
import pytest
import torch

from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup(m, n, nrhs, d, seed, sketch_seed, lp=torch.bfloat16):
    import paper_2004_02480_amd as P
    s = W.multi_rhs(m, n, nrhs, seed, device=DEV)
    sk = P.csk_sketch(s.A, s.B, d, sketch_seed, lp_dtype=lp)
    torch.cuda.synchronize()
    return s, sk


@pytest.mark.parametrize("lp", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("m,n,nrhs,d", [(20000, 60, 24, 1500), (12000, 33, 130, 900), (30000, 100, 7, 2600)])
def test_mrhs_matches_oracle(gpu, orc, lp, m, n, nrhs, d):
    s, sk = setup(m, n, nrhs, d, seed=m + nrhs, sketch_seed=5, lp=lp)
    X, res = gpu.csk_solve_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, Xref=s.X_star, tol=1e-8, maxit=200000)
    Xs = s.X_star.cpu().numpy()
    Xg = X.cpu().numpy()
    At, Bt = orc.sketch_dense(s.A.cpu().numpy(), s.B.cpu().numpy(), d, 5)
    for j in range(nrhs):
        it, st, fb, meas, nref = res[j]
        assert st == gpu.CSK_OK, (j, st)
        assert np.linalg.norm(Xg[:, j] - Xs[:, j]) <= 1e-8 * np.linalg.norm(Xs[:, j]), j
        if j % max(1, nrhs // 5) == 0:
            o = orc.mwrk(At, Bt[:, j], xref=Xs[:, j], tol=1e-8, maxit=200000)
            assert o.status == 0
            assert np.linalg.norm(Xg[:, j] - o.x) <= 2e-8 * np.linalg.norm(Xs[:, j])
            # 16-bit residual products between exact refreshes pick slightly
            # different rows; the iteration count of this schedule is not
            # pinned to the FP64 loop's, only bounded by it
            assert it <= 2 * o.iters + 64, (j, it, o.iters)


def test_mrhs_first_iterates_match_oracle(gpu, orc):
    # before the first refresh the residual is exact (R_ref), so the first
    # step of every column is the oracle's first step
    s, sk = setup(8000, 40, 20, 700, seed=3, sketch_seed=4)
    X, res = gpu.csk_solve_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, Xref=s.X_star, tol=0.0, maxit=1)
    At, Bt = orc.sketch_dense(s.A.cpu().numpy(), s.B.cpu().numpy(), 700, 4)
    for j in range(20):
        assert res[j][1] == gpu.CSK_NOT_CONVERGED and res[j][0] == 1
        o = orc.mwrk(At, Bt[:, j], xref=s.X_star[:, j].cpu().numpy(), tol=0.0, maxit=1)
        np.testing.assert_allclose(X[:, j].cpu().numpy(), o.x, rtol=0, atol=1e-12 * np.linalg.norm(o.x))


def test_mrhs_residual_mode_and_determinism(gpu):
    s, sk = setup(15000, 50, 40, 1200, seed=8, sketch_seed=9)
    X1, r1 = gpu.csk_solve_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, tol=1e-9, maxit=200000,
                                stop_mode=gpu.CSK_STOP_REL_RESID)
    X2, r2 = gpu.csk_solve_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, tol=1e-9, maxit=200000,
                                stop_mode=gpu.CSK_STOP_REL_RESID)
    assert torch.equal(X1, X2) and r1 == r2
    R = sk.bt - sk.At64 @ X1
    rel = R.norm(dim=0) / sk.bt.norm(dim=0)
    assert all(r[1] == gpu.CSK_OK for r in r1)
    assert rel.max().item() <= 1e-9 * (1 + 1e-6)


def test_mrhs_full_size(gpu):
    # A 200000 x 500 FP32 Gaussian, 256 right-hand sides, d = 10000, BF16
    # residual products with FP64 refresh, tol 1e-8 per column
    c = W.config("multi_rhs")
    s, sk = setup(c["m"], c["n"], c["nrhs"], c["d"], c["seed"], c["sketch_seed"])
    X, res = gpu.csk_solve_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, Xref=s.X_star, tol=c["tol"], maxit=c["maxit"])
    err = ((X - s.X_star).norm(dim=0) / s.X_star.norm(dim=0)).max().item()
    assert all(r[1] == gpu.CSK_OK for r in res)
    assert err <= 1e-8
    print(f"multi_rhs max iterations {max(r[0] for r in res)}")


@pytest.mark.parametrize("lp", [torch.bfloat16, torch.float16])
def test_mrhs_wide_rows_two_barrier_form(gpu, orc, lp):
    """Rows longer than 512 columns take the two-barrier form (Delta shared
    through device memory); same bounds as the register-Delta form."""
    m, n, nrhs, d = 30000, 700, 9, 3000
    s, sk = setup(m, n, nrhs, d, seed=17, sketch_seed=18, lp=lp)
    X, res = gpu.csk_solve_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, Xref=s.X_star, tol=1e-8, maxit=200000)
    Xs = s.X_star.cpu().numpy()
    Xg = X.cpu().numpy()
    At, Bt = orc.sketch_dense(s.A.cpu().numpy(), s.B.cpu().numpy(), d, 18)
    for j in (0, nrhs - 1):
        assert res[j][1] == gpu.CSK_OK, (j, res[j])
        assert np.linalg.norm(Xg[:, j] - Xs[:, j]) <= 1e-8 * np.linalg.norm(Xs[:, j])
        with orc.threads(8):
            o = orc.mwrk(At, Bt[:, j], xref=Xs[:, j], tol=1e-8, maxit=200000)
        assert np.linalg.norm(Xg[:, j] - o.x) <= 2e-8 * np.linalg.norm(Xs[:, j])
