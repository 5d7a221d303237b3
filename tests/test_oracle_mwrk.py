"""Pins of the oracle's MWRK loop (Algorithm 1, loop; Section 3 stopping rule)
against the identities and bounds of the convergence proof (Theorem 2),
closed-form special cases, and the iteration counts printed in Table 1."""
import numpy as np
import pytest

from test_golden_table1 import load_table1

import oracle as O


def consistent(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    xs = rng.standard_normal(n)
    return A, xs, A @ xs


def test_per_step_error_identity_and_greedy_bounds(orc):
    # Proof of Theorem 2 (consistent system, e_k = x_k - x*):
    #   ||e_{k+1}||^2 = ||e_k||^2 - r_{i_k}^2 / ||At^(i_k)||^2            (exact step)
    #   r_{i_k}^2 / ||At^(i_k)||^2 >= ||At e_k||^2 / ||At||_F^2           (greedy choice)
    #   ||e_{k+1}||^2 <= ||e_k||^2 - ||At e_k||^2 / (n ||At||_2^2)
    A, xs, b = consistent(3000, 30, 1)
    At, bt = orc.sketch_dense(A, b, 400, 2)
    # make the sketched system exactly consistent with xs so e_k is exact
    bt = At @ xs
    K = 60
    r = orc.mwrk(At, bt, xref=xs, tol=0.0, maxit=K, trace=True)
    assert r.status == O.NOT_CONVERGED and r.iters == K
    nu2 = orc.row_norms2(At)
    fro2 = np.sum(At * At)
    spec2 = np.linalg.norm(At, 2) ** 2
    x = np.zeros(30)
    for k in range(K):
        e = x - xs
        e2 = e @ e
        assert abs(r.err2[k] - e2) <= 1e-12 * (xs @ xs)
        i = r.idx[k]
        step = r.r[k] ** 2 / nu2[i]
        assert abs(r.err2[k + 1] - (r.err2[k] - step)) <= 1e-10 * r.err2[k]
        Ae2 = np.sum((At @ e) ** 2)
        assert step >= Ae2 / fro2 * (1 - 1e-9)
        assert r.err2[k + 1] <= r.err2[k] - Ae2 / (30 * spec2) + 1e-10 * r.err2[k]
        # the chosen row maximizes |r_i| / ||At^(i)|| (brute force)
        res = bt - At @ x
        w = np.full(res.shape, -np.inf)
        nz = nu2 > 0  # empty buckets are never selected
        w[nz] = np.abs(res[nz]) / np.sqrt(nu2[nz])
        assert i == int(np.argmax(w))
        x = x + res[i] / nu2[i] * At[i]
    # error is monotone
    assert np.all(np.diff(r.err2) <= 1e-12 * r.err2[0])


def test_diagonal_closed_form(orc):
    # At = diag(2^k_i): the weighted residuals are |x*_i - x_i|, so the rows
    # are taken in decreasing |x*_i| (lowest index on ties) and each step sets
    # x_i = x*_i exactly; after n steps x = x* bitwise.
    n = 12
    rng = np.random.default_rng(4)
    a = 2.0 ** rng.integers(-5, 6, n)
    xs = rng.standard_normal(n)
    xs[7] = xs[2]  # a tie: index 2 must come first
    At = np.diag(a)
    bt = a * xs
    r = orc.mwrk(At, bt, xref=xs, tol=0.0, maxit=n, trace=True)
    np.testing.assert_array_equal(r.x, xs)
    expect = sorted(range(n), key=lambda i: (-abs(xs[i]), i))
    np.testing.assert_array_equal(r.idx, expect)
    r2 = orc.mwrk(At, bt, xref=xs, tol=0.0, maxit=n + 5)
    assert r2.status == O.OK and r2.iters == n


def test_orthogonal_rows_converge_in_n_steps(orc):
    # Rows of a scaled Hadamard matrix are orthogonal: each projection fixes
    # one coordinate of the row basis without disturbing the others.
    from scipy.linalg import hadamard
    n = 16
    H = hadamard(n).astype(np.float64) * 0.25
    xs = np.random.default_rng(5).standard_normal(n)
    r = orc.mwrk(H, H @ xs, xref=xs, tol=1e-14, maxit=100)
    assert r.status == O.OK and r.iters <= n
    assert len(set(orc.mwrk(H, H @ xs, xref=xs, tol=0, maxit=n, trace=True).idx)) == n


def test_single_column_one_step(orc):
    At = np.array([[2.0], [-3.0], [0.5]])
    xs = np.array([1.25])
    r = orc.mwrk(At, At[:, 0] * xs, xref=xs, tol=1e-15, maxit=10)
    assert r.status == O.OK and r.iters == 1
    np.testing.assert_array_equal(r.x, xs)


def test_power_of_two_row_scaling_bitwise_invariant(orc):
    # Scaling (At^(i), bt_i) by 2^k changes neither the weighted residuals nor
    # the projections in floating point.
    A, xs, b = consistent(2000, 20, 6)
    At, bt = orc.sketch_dense(A, b, 200, 7)
    s = 2.0 ** np.random.default_rng(7).integers(-20, 21, 200)
    r1 = orc.mwrk(At, bt, xref=xs, tol=0, maxit=150, trace=True)
    r2 = orc.mwrk(At * s[:, None], bt * s, xref=xs, tol=0, maxit=150, trace=True)
    np.testing.assert_array_equal(r1.idx, r2.idx)
    np.testing.assert_array_equal(r1.x, r2.x)


def test_resume_is_bitwise(orc):
    # x_{k+1} depends only on x_k: K1 + K2 iterations equal K1 then K2 from
    # the saved iterate.
    A, xs, b = consistent(2000, 25, 8)
    At, bt = orc.sketch_dense(A, b, 300, 9)
    full = orc.mwrk(At, bt, xref=xs, tol=0, maxit=70)
    a = orc.mwrk(At, bt, xref=xs, tol=0, maxit=30)
    c = orc.mwrk(At, bt, x0=a.x, xref=xs, tol=0, maxit=40)
    np.testing.assert_array_equal(full.x, c.x)


def test_status_paths(orc):
    At = np.zeros((5, 3))
    r = orc.mwrk(At, np.zeros(5), xref=np.ones(3), tol=1e-10, maxit=10)
    assert r.status == O.ERR_DEGENERATE and r.iters == 0
    At = np.eye(3)
    bt = np.array([1.0, np.nan, 2.0])
    r = orc.mwrk(At, bt, xref=np.ones(3), tol=1e-10, maxit=10)
    assert r.status == O.ERR_NONFINITE
    A, xs, b = consistent(500, 10, 10)
    r = orc.mwrk(A, b, xref=xs, tol=1e-12, maxit=3)
    assert r.status == O.NOT_CONVERGED and r.iters == 3
    # zero rows (empty buckets) are never selected
    At = np.vstack([np.zeros((4, 3)), np.eye(3)])
    r = orc.mwrk(At, np.concatenate([np.zeros(4), [1.0, 2.0, 3.0]]), xref=np.array([1.0, 2.0, 3.0]),
                 tol=0, maxit=3, trace=True)
    assert set(r.idx) == {4, 5, 6}
    # residual stopping rule
    r = orc.mwrk(A, b, tol=1e-9, maxit=100000, stop_mode=O.STOP_REL_RESID)
    assert r.status == O.OK
    assert np.linalg.norm(b - A @ r.x) <= 1e-9 * np.linalg.norm(b)


def test_oracle_size_csk_reaches_1e10(orc):
    # Section 3's protocol at the oracle-size shape: A 2000 x 50 N(0,1),
    # b = A x*, d = 500, x0 = 0.
    A, xs, b = consistent(2000, 50, 1)
    r = orc.csk(A, b, 500, 101, xref=xs, tol=1e-10, maxit=100000)
    assert r.status == O.OK
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= 1e-10
    assert 150 < r.iters < 600


@pytest.mark.slow
@pytest.mark.parametrize("n,trials", [(50, 8), (100, 3)])
def test_table1_iteration_counts(orc, n, trials):
    # Table 1, m = 300000: randn A and x*, b = A x*, d = n^2, x0 = 0, stop at
    # RES = ||x - x*||^2/||x*||^2 <= 1e-6 (tol 1e-3 on the unsquared error).
    m = 300000
    row = [r for r in load_table1() if (r["m"], r["n"]) == (m, n)][0]
    csk_it, mwrk_it = row["csk_it"], row["mwrk_it"]
    its, mits = [], []
    for t in range(trials):
        rng = np.random.default_rng(10000 + t)
        A = rng.standard_normal((m, n))
        xs = rng.standard_normal(n)
        b = A @ xs
        its.append(orc.csk(A, b, n * n, 20000 + t, xref=xs, tol=1e-3, maxit=20000).iters)
        if t < 2:
            mits.append(orc.mwrk(A, b, xref=xs, tol=1e-3, maxit=20000).iters)
    assert abs(np.mean(its) - csk_it) <= 3.0, its
    assert abs(np.mean(mits) - mwrk_it) <= 2.5, mits
