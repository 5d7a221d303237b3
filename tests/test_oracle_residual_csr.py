"""Pins of the oracle's sketched residual of a CSR system, S (b - A x)
(Definition 1's S applied to the residual; the exact residual that the mixed
precision loop on the sketch of a sparse A refreshes from)."""
import numpy as np
import pytest

from paper_2004_02480_amd import workloads as W


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle._load()
    return oracle


def _dense(s):
    A = np.zeros((s.m, s.n))
    rows = np.repeat(np.arange(s.m), np.diff(s.row_ptr))
    A[rows, s.col] = s.val.astype(np.float64)
    return A


def test_residual_csr_matches_explicit_sketch_matrix(orc):
    # brute force on a tiny system: S = Phi D as an explicit d x m matrix
    # from the hash (bucket h(i), sign D_ii), times b - A x
    s = W.sparse_csr(40, 7, 0.3, seed=5)
    d, seed = 6, 11
    x = np.random.default_rng(1).standard_normal(s.n)
    bucket, sign = orc.hash_rows(seed, s.m, d)
    S = np.zeros((d, s.m))
    S[bucket, np.arange(s.m)] = sign
    want = S @ (s.b - _dense(s) @ x)
    got = orc.sketch_residual_csr(s.row_ptr, s.col, s.val, s.m, s.b, x, d, seed)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_residual_csr_at_zero_is_the_sketched_b_bitwise(orc):
    # x = 0: every y_i is b_i exactly, and the signed sums run in the same
    # ascending row order as the sketch's b~
    s = W.sparse_csr(3000, 200, 0.01, seed=3)
    d, seed = 150, 29
    _, bt = orc.sketch_csr(s.row_ptr, s.col, s.val, s.m, s.n, s.b, d, seed)
    got = orc.sketch_residual_csr(s.row_ptr, s.col, s.val, s.m, s.b, np.zeros(s.n), d, seed)
    np.testing.assert_array_equal(got, bt)


def test_residual_csr_equals_sketched_residual(orc):
    # S linear: S (b - A x) = S b - (S A) x up to rounding
    s = W.sparse_csr(5000, 300, 0.02, seed=7)
    d, seed = 400, 17
    At, bt = orc.sketch_csr(s.row_ptr, s.col, s.val, s.m, s.n, s.b, d, seed)
    x = np.random.default_rng(2).standard_normal(s.n)
    got = orc.sketch_residual_csr(s.row_ptr, s.col, s.val, s.m, s.b, x, d, seed)
    want = bt - At @ x
    scale = np.abs(bt).max() + np.abs(At).max() * np.abs(x).sum()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * scale)
    # at the consistent system's solution the residual vanishes (to rounding)
    r0 = orc.sketch_residual_csr(s.row_ptr, s.col, s.val, s.m, s.b, s.x_star, d, seed)
    assert np.abs(r0).max() <= 1e-12 * scale
