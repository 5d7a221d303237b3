"""Pins of the oracle's hash and sketch (Definition 1; Algorithm 1, Initialize)
against facts that do not depend on the oracle itself: the matrix product
with an explicit S = Phi D, invariants of the count sketch, the closed-form
mean and variance of ||S y||^2, library sorts and the distribution the
paper asks for."""
import numpy as np
import pytest
from scipy import stats


def dense_S(bucket, sign, d):
    """Definition 1 written out: Phi[h(i), i] = 1, D = diag(sign), S = Phi D."""
    m = bucket.shape[0]
    Phi = np.zeros((d, m))
    Phi[bucket.astype(np.int64), np.arange(m)] = 1.0
    D = np.diag(sign.astype(np.float64))
    return Phi @ D


def test_counter_form_is_the_splitmix64_stream(orc):
    # h and D for row i come from the (i+1)-th output of a SplitMix64
    # generator seeded with `seed`; the stream routine advances a state
    # sequentially, the hash indexes it directly.
    seed, m, d = 0xDEADBEEF, 4096, 1 << 20
    stream = orc.splitmix64_stream(seed, m)
    bucket, sign = orc.hash_rows(seed, m, d)
    hi = (stream >> np.uint64(32)).astype(object)
    expect_bucket = np.array([(int(h) * d) >> 32 for h in hi], dtype=np.uint32)
    np.testing.assert_array_equal(bucket, expect_bucket)
    np.testing.assert_array_equal(sign, np.where(stream & np.uint64(1), -1, 1).astype(np.int8))


def test_bucket_is_floor_of_uniform_times_d(orc):
    # h(i) = floor(u_i * d) with u_i = (w >> 32) / 2^32 uniform on [0, 1).
    seed = 7
    for d in (1, 2, 3, 500, 20000, 2**31 - 1):
        stream = orc.splitmix64_stream(seed, 2000)
        bucket, _ = orc.hash_rows(seed, 2000, d)
        u = (stream >> np.uint64(32)).astype(np.float64) / 2.0**32
        np.testing.assert_array_equal(bucket, np.floor(u * d).astype(np.uint32))
        assert bucket.max() < d


def test_buckets_uniform_and_signs_balanced(orc):
    # Definition 1: h(i) = j with probability 1/d; D_ii = +-1 with prob 1/2,
    # independently.
    m, d = 1_000_000, 1000
    bucket, sign = orc.hash_rows(12345, m, d)
    counts = np.bincount(bucket, minlength=d)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4, (chi2, p)
    npos = int((sign == 1).sum())
    assert abs(npos - m / 2) < 5 * np.sqrt(m / 4)
    # sign independent of bucket parity classes
    tab = np.zeros((2, 10))
    np.add.at(tab, ((sign == 1).astype(int), bucket % 10), 1)
    _, p2, _, _ = stats.chi2_contingency(tab)
    assert p2 > 1e-4


def test_bucket_sort_matches_stable_argsort(orc):
    for m, d in [(1, 1), (17, 5), (2000, 500), (5000, 7), (300, 1000)]:
        bucket, _ = orc.hash_rows(99 + m, m, d)
        perm, ptr = orc.bucket_sort(bucket, d)
        np.testing.assert_array_equal(perm, np.argsort(bucket, kind="stable").astype(np.uint32))
        np.testing.assert_array_equal(ptr, np.concatenate([[0], np.cumsum(np.bincount(bucket, minlength=d))]))
        assert ptr[-1] == m


@pytest.mark.parametrize("m,n,d", [(64, 8, 16), (40, 3, 40), (50, 5, 1), (10, 4, 64)])
def test_sketch_equals_dense_product_integer_exact(orc, m, n, d):
    # With small integer entries every sum is exact, so S A computed as a
    # matrix product must agree bit for bit with the scatter form.
    rng = np.random.default_rng(m * 1000 + d)
    A = rng.integers(-9, 10, size=(m, n)).astype(np.float64)
    b = rng.integers(-9, 10, size=m).astype(np.float64)
    seed = 31 + d
    At, bt = orc.sketch_dense(A, b, d, seed)
    bucket, sign = orc.hash_rows(seed, m, d)
    S = dense_S(bucket, sign, d)
    np.testing.assert_array_equal(At, S @ A)
    np.testing.assert_array_equal(bt, S @ b)


def test_sketch_equals_dense_product_float(orc):
    rng = np.random.default_rng(5)
    m, n, d = 3000, 20, 300
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    At, bt = orc.sketch_dense(A, b, d, 77)
    bucket, sign = orc.hash_rows(77, m, d)
    S = dense_S(bucket, sign, d)
    np.testing.assert_allclose(At, S @ A, rtol=0, atol=1e-13)
    np.testing.assert_allclose(bt, S @ b, rtol=0, atol=1e-13)


def test_sketch_sum_is_in_ascending_row_order(orc):
    # Entries chosen so that the FP64 result depends on the summation order:
    # 1e16 + 1 - 1e16 in row order gives 0 (1 is absorbed), other orders 1.
    m, d, seed = 3, 1, 0
    _, sign = orc.hash_rows(seed, m, d)
    # A_i = s_i * v_i, so the signed terms s_i A_i are v = (1e16, 1, -1e16)
    A = (np.array([1e16, 1.0, -1e16]) * sign).reshape(m, 1).astype(np.float64)
    At, _ = orc.sketch_dense(A, None, d, seed)
    assert At[0, 0] == (1e16 + 1.0) - 1e16 == 0.0


def test_column_sums_and_SSt(orc):
    # 1^T (S A) = (S^T 1)^T A = sign^T A exactly (integer data), and
    # S S^T = diag(bucket counts).
    rng = np.random.default_rng(3)
    m, n, d = 5000, 6, 257
    A = rng.integers(-100, 101, size=(m, n)).astype(np.float64)
    seed = 4242
    At, _ = orc.sketch_dense(A, None, d, seed)
    bucket, sign = orc.hash_rows(seed, m, d)
    np.testing.assert_array_equal(At.sum(axis=0), sign.astype(np.float64) @ A)
    S = dense_S(bucket, sign, d)
    np.testing.assert_array_equal(S @ S.T, np.diag(np.bincount(bucket, minlength=d).astype(np.float64)))


def test_norm_unbiased_with_closed_form_variance(orc):
    # E ||S y||^2 = ||y||^2 and Var = (2/d)(||y||^4 - sum y_i^4) for a count
    # sketch with independent buckets and signs; 2000 seeds at the oracle-size
    # shape (m = 2000, d = 500).
    rng = np.random.default_rng(11)
    m, n, d = 2000, 50, 500
    A = rng.standard_normal((m, n))
    x = rng.standard_normal(n)
    y = A @ x
    vals = np.empty(2000)
    for s in range(2000):
        _, yt = orc.sketch_dense(A[:, :1], y, d, s)
        vals[s] = yt @ yt
    ny2 = y @ y
    var = 2.0 / d * (ny2**2 - np.sum(y**4))
    se = np.sqrt(var / vals.size)
    assert abs(vals.mean() - ny2) < 5 * se
    assert abs(vals.var(ddof=1) / var - 1.0) < 0.15


def test_subspace_embedding_tightens_with_d(orc):
    # Lemma 1: singular values of S A stay within (1 +- eps) of those of A,
    # with eps shrinking as d grows (d = O(n^2 / (delta eps^2))).
    rng = np.random.default_rng(8)
    m, n = 20000, 10
    A = rng.standard_normal((m, n))
    sA = np.linalg.svd(A, compute_uv=False)
    devs = []
    for d in (200, 2000, 10000):
        At, _ = orc.sketch_dense(A, None, d, 1000 + d)
        s = np.linalg.svd(At, compute_uv=False)
        devs.append(np.max(np.abs(s / sA - 1.0)))
    assert devs[0] > devs[1] > devs[2]
    assert devs[2] < 0.1


def test_fp32_input_widened_exactly(orc):
    rng = np.random.default_rng(9)
    A32 = rng.standard_normal((700, 13)).astype(np.float32)
    b = rng.standard_normal(700)
    At32, bt32 = orc.sketch_dense(A32, b, 90, 5)
    At64, bt64 = orc.sketch_dense(A32.astype(np.float64), b, 90, 5)
    np.testing.assert_array_equal(At32, At64)
    np.testing.assert_array_equal(bt32, bt64)


def test_multi_rhs_columns_sketch_independently(orc):
    rng = np.random.default_rng(10)
    m, n, d, r = 900, 7, 60, 5
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, r))
    _, Bt = orc.sketch_dense(A, B, d, 12)
    for j in range(r):
        _, bt = orc.sketch_dense(A, B[:, j], d, 12)
        np.testing.assert_array_equal(Bt[:, j], bt)


def test_csr_sketch_equals_dense_sketch_bitwise(orc):
    from paper_2004_02480_amd import workloads as W
    s = W.sparse_csr(3000, 400, 0.01, seed=21)
    A = W.csr_to_dense(s)
    At_d, bt_d = orc.sketch_dense(A, s.b, 150, 33)
    At_s, bt_s = orc.sketch_csr(s.row_ptr, s.col, s.val, s.m, s.n, s.b, 150, 33)
    np.testing.assert_array_equal(At_s, At_d)
    np.testing.assert_array_equal(bt_s, bt_d)
    # the generator's contract: rows non-empty, columns distinct and sorted
    assert np.all(np.diff(s.row_ptr) >= 1)
    for i in range(0, 3000, 97):
        c = s.col[s.row_ptr[i]:s.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_row_norms(orc):
    # Pythagorean rows and scaled unit rows have exact squared norms; the
    # total equals the Frobenius norm.
    At = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 0.0], [0.0, -2.0**-3, 0.0], [5.0, 12.0, 84.0]])
    np.testing.assert_array_equal(orc.row_norms2(At), [25.0, 0.0, 2.0**-6, 7225.0])
    rng = np.random.default_rng(1)
    B = rng.standard_normal((100, 37))
    assert abs(orc.row_norms2(B).sum() - np.linalg.norm(B, "fro")**2) < 1e-12 * B.size
