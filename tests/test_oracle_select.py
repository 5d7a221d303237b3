"""Pins of the oracle's randomized selection rules: relaxed greedy randomized
Kaczmarz (theta = 1/2: greedy randomized Kaczmarz) and randomized Kaczmarz,
the members of the family that the introduction places Algorithm 1's loop in
and that Section 3's figure compares it with.

What fixes them without the oracle's own arithmetic:
  * theta = 1 makes the working set the rows of maximal weighted residual, so
    the trajectory is Algorithm 1's loop (orc_mwrk), bit for bit;
  * the distribution of the first draw, against the working set and the
    probabilities recomputed here from the published definition (the
    eps_k form, not the oracle's rewritten threshold), by a chi-square test;
  * randomized Kaczmarz draws independently of x with probability
    ||A_i||^2 / ||A||_F^2, so the frequencies along one long run pin it;
  * every step is an orthogonal projection on a consistent system, so
    ||e_{k+1}||^2 = ||e_k||^2 - r_{i_k}^2 / ||A_{i_k}||^2 whatever row is drawn;
  * Section 3's figure: the maximal weighted residual rule needs the fewest
    iterations, then greedy randomized, then randomized Kaczmarz."""
import numpy as np
import pytest
from scipy import stats

import oracle as O


def _system(d, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, n))
    xs = rng.standard_normal(n)
    return A, A @ xs, xs


@pytest.mark.parametrize("seed", [1, 2])
def test_theta_one_is_the_greedy_loop(seed):
    A, b, xs = _system(300, 15, seed)
    m = O.mwrk(A, b, xref=xs, tol=1e-12, maxit=5000, trace=True)
    for sel in (0, 977):
        r = O.rgrk(A, b, theta=1.0, sel_seed=sel, xref=xs, tol=1e-12, maxit=5000, trace=True)
        assert r.status == O.OK and r.iters == m.iters
        np.testing.assert_array_equal(r.idx, m.idx)
        np.testing.assert_array_equal(r.x, m.x)


def _working_set(A, b, x, theta):
    """The published definition: rows with |r_i|^2 >= eps ||r||^2 ||A_i||^2,
    eps = theta max_i(|r_i|^2/||A_i||^2)/||r||^2 + (1 - theta)/||A||_F^2."""
    r = b - A @ x
    nu2 = np.einsum("ij,ij->i", A, A)
    R = r @ r
    eps = theta * np.max(r * r / nu2) / R + (1 - theta) / nu2.sum()
    lhs = r * r
    rhs = eps * R * nu2
    # the test systems keep every row well away from the boundary
    assert np.min(np.abs(lhs - rhs) / np.maximum(lhs, rhs)) > 1e-6
    return lhs >= rhs, r


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.8])
def test_first_draw_distribution(theta):
    rng = np.random.default_rng(11)
    A = rng.standard_normal((12, 4)) * rng.uniform(0.5, 2.0, size=(12, 1))
    b = rng.standard_normal(12)
    x0 = rng.standard_normal(4)
    member, r = _working_set(A, b, x0, theta)
    p = np.where(member, r * r, 0.0)
    p /= p.sum()
    trials = 20000
    counts = np.zeros(12, np.int64)
    for s in range(trials):
        res = O.rgrk(A, b, theta=theta, sel_seed=1000003 * s + 7, x0=x0, tol=0.0, maxit=1,
                     stop_mode=O.STOP_REL_RESID, trace=True)
        assert res.iters == 1
        counts[res.idx[0]] += 1
    assert counts[~member].sum() == 0, (theta, counts)
    obs = counts[member]
    exp = p[member] * trials
    if obs.size > 1:
        assert stats.chisquare(obs, exp).pvalue > 1e-4, (theta, obs, exp)


def test_rk_frequencies_follow_row_norms():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((10, 3)) * rng.uniform(0.3, 3.0, size=(10, 1))
    A[4] = 0.0  # an empty row (as an empty bucket of the sketch) is never drawn
    xs = rng.standard_normal(3)
    b = A @ xs + 0.1 * rng.standard_normal(10)  # inconsistent: the run never stops early
    K = 60000
    res = O.rk(A, b, sel_seed=21, xref=xs, tol=0.0, maxit=K, trace=True)
    assert res.iters == K
    counts = np.bincount(res.idx, minlength=10)
    nu2 = np.einsum("ij,ij->i", A, A)
    assert counts[4] == 0
    keep = nu2 > 0
    assert stats.chisquare(counts[keep], nu2[keep] / nu2.sum() * K).pvalue > 1e-4


def test_uniforms_are_uniform_and_inside_the_interval():
    u = O.uniforms(3, 0, 200000)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    g = u * 2.0**52 - 0.5  # the top 52 bits of each word: integers
    assert np.array_equal(g, np.floor(g))
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # exponential clocks built from them
    e = -np.log(u)
    assert abs(e.mean() - 1.0) < 5 * 1.0 / np.sqrt(u.size)


@pytest.mark.parametrize("rule", ["rgrk0", "grk", "rk"])
def test_each_step_is_an_orthogonal_projection(rule):
    A, b, xs = _system(200, 12, 9)
    nu2 = np.einsum("ij,ij->i", A, A)
    K = 150
    if rule == "rk":
        res = O.rk(A, b, sel_seed=4, xref=xs, tol=0.0, maxit=K, trace=True)
    else:
        res = O.rgrk(A, b, theta=0.0 if rule == "rgrk0" else 0.5, sel_seed=4, xref=xs, tol=0.0, maxit=K,
                     trace=True)
    assert res.iters == K
    drop = res.r ** 2 / nu2[res.idx]
    np.testing.assert_allclose(res.err2[1:], res.err2[:-1] - drop, rtol=0, atol=1e-11 * res.err2[0])
    assert np.all(np.diff(res.err2) <= 1e-13 * res.err2[0])


def test_section3_iteration_order():
    # fewest iterations for the greedy rule, then greedy randomized, then
    # randomized Kaczmarz (means over seeded systems)
    its = {"mwrk": [], "grk": [], "rk": []}
    for s in range(4):
        A, b, xs = _system(2000, 40, 100 + s)
        its["mwrk"].append(O.mwrk(A, b, xref=xs, tol=1e-6, maxit=200000).iters)
        its["grk"].append(O.rgrk(A, b, theta=0.5, sel_seed=s, xref=xs, tol=1e-6, maxit=200000).iters)
        its["rk"].append(O.rk(A, b, sel_seed=s, xref=xs, tol=1e-6, maxit=200000).iters)
    m = {k: np.mean(v) for k, v in its.items()}
    assert m["mwrk"] < m["grk"] < m["rk"], its


def test_converge_degenerate_and_invalid():
    A, b, xs = _system(500, 20, 3)
    for th in (0.0, 0.5, 1.0):
        r = O.rgrk(A, b, theta=th, sel_seed=1, xref=xs, tol=1e-10, maxit=100000)
        assert r.status == O.OK
        assert np.linalg.norm(r.x - xs) <= 1e-10 * np.linalg.norm(xs) * (1 + 1e-9)
    r = O.rk(A, b, sel_seed=1, xref=xs, tol=1e-10, maxit=1000000)
    assert r.status == O.OK
    # residual stop for the greedy randomized rule
    r = O.rgrk(A, b, theta=0.5, sel_seed=2, tol=1e-9, maxit=100000, stop_mode=O.STOP_REL_RESID)
    assert r.status == O.OK and np.linalg.norm(b - A @ r.x) <= 1e-9 * np.linalg.norm(b) * (1 + 1e-9)
    Z = np.zeros((6, 3))
    assert O.rgrk(Z, np.ones(6), theta=0.5, sel_seed=1, xref=np.ones(3), tol=1e-10, maxit=5).status == \
        O.ERR_DEGENERATE
    assert O.rk(Z, np.ones(6), sel_seed=1, xref=np.ones(3), tol=1e-10, maxit=5).status == O.ERR_DEGENERATE
    assert O.rgrk(A, b, theta=1.5, sel_seed=1, xref=xs, maxit=5).status == O.ERR_INVALID_ARG
    assert O.rgrk(A, b, theta=-0.1, sel_seed=1, xref=xs, maxit=5).status == O.ERR_INVALID_ARG
