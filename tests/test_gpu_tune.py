"""The launch-shape tuner of the persistent solve: it times candidate shapes
on a real system, caches the fastest, and a default-shaped solve of the same
shape then uses it and still meets the tolerance against x* and the oracle."""
import numpy as np
import pytest
import torch

from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_tune_then_solve(gpu, orc):
    gpu.csk_tune_clear()
    s = W.gaussian(60000, 300, seed=31, device=DEV)
    sk = gpu.csk_sketch(s.A, s.b, 6000, 32)
    best = gpu.csk_tune_solve(sk.At64, sk.bt, nu2=sk.nu2, trial_iters=50)
    assert best["grid"] >= 1 and best["lanes_per_row"] in (4, 16, 64) and best["us_per_iter"] > 0
    assert gpu.csk_tune_lookup(6000, 300, torch.float64) == best
    r = gpu.csk_solve(sk.At64, sk.bt, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10, maxit=200000)
    assert r.status == gpu.CSK_OK
    xs = s.x_star.cpu().numpy()
    assert np.linalg.norm(r.x.cpu().numpy() - xs) <= 1e-10 * np.linalg.norm(xs)
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), 6000, 32)
    o = orc.mwrk(At, bt, xref=xs, tol=1e-10, maxit=200000)
    assert o.status == 0
    assert np.linalg.norm(r.x.cpu().numpy() - o.x) <= 2e-10 * np.linalg.norm(xs)
    gpu.csk_tune_clear()
    assert gpu.csk_tune_lookup(6000, 300, torch.float64)["grid"] == 0


def test_tune_mixed_precision_entry(gpu):
    gpu.csk_tune_clear()
    s = W.row_scaled(40000, 200, seed=33, device=DEV)
    sk = gpu.csk_sketch(s.A, s.b, 4000, 34, lp_dtype=torch.bfloat16)
    best = gpu.csk_tune_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, trial_iters=40)
    assert gpu.csk_tune_lookup(4000, 200, torch.bfloat16) == best
    r = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10, maxit=400000)
    assert r.status == gpu.CSK_OK
    gpu.csk_tune_clear()


def test_tune_mrhs_then_solve(gpu, orc):
    """The multi-RHS tuner times the row-tile counts, caches the fastest, and
    a later solve of that shape (which uses it) still meets the tolerance
    per column and agrees with the oracle's single-column solution."""
    gpu.csk_tune_clear()
    s = W.multi_rhs(30000, 120, 40, 41, device=DEV)
    sk = gpu.csk_sketch(s.A, s.B, 2500, 42, lp_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    rep = gpu.csk_tune_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, trial_iters=60)
    assert rep["candidates"] >= 1 and rep["choice"] >= rep["default_choice"] >= 1
    assert rep["us"] > 0 and rep["us"] <= rep["default_us"]
    X, res = gpu.csk_solve_mrhs(sk.At_lp, sk.At64, sk.bt, sk.nu2, Xref=s.X_star, tol=1e-8, maxit=200000)
    Xs = s.X_star.cpu().numpy()
    Xg = X.cpu().numpy()
    assert all(r[1] == gpu.CSK_OK for r in res)
    At, Bt = orc.sketch_dense(s.A.cpu().numpy(), s.B.cpu().numpy(), 2500, 42)
    for j in (0, 39):
        assert np.linalg.norm(Xg[:, j] - Xs[:, j]) <= 1e-8 * np.linalg.norm(Xs[:, j])
        o = orc.mwrk(At, Bt[:, j], xref=Xs[:, j], tol=1e-8, maxit=200000)
        assert np.linalg.norm(Xg[:, j] - o.x) <= 2e-8 * np.linalg.norm(Xs[:, j])
    gpu.csk_tune_clear()


def test_tune_batched_then_solve(gpu):
    """The batched tuner runs every plan variant (each a full, converged
    solve), caches the fastest for these shapes, and a later call uses it."""
    gpu.csk_tune_clear()
    shapes, _ = W.batched_shapes(24, 5100, 15100, m_range=(2000, 12000), n_range=(20, 150))
    systems = []
    for sh in shapes:
        s = W.gaussian(sh.m, sh.n, sh.seed, dtype=torch.float32, device=DEV)
        systems.append(dict(A=s.A, b=s.b, d=sh.d, seed=sh.sketch_seed, x_ref=s.x_star))
    torch.cuda.synchronize()
    rep = gpu.csk_tune_batched(systems, lp_dtype=torch.float32, tol=1e-8)
    assert rep["candidates"] == 5 and 0 <= rep["choice"] <= 4 and rep["default_choice"] == 0
    assert 0 < rep["us"] <= rep["default_us"]
    xs, res = gpu.csk_solve_batched(systems, lp_dtype=torch.float32, tol=1e-8)
    for x, sd, r in zip(xs, systems, res):
        assert r[1] == gpu.CSK_OK
        assert ((x - sd["x_ref"]).norm() / sd["x_ref"].norm()).item() <= 1e-8
    gpu.csk_tune_clear()


def test_tune_cache_file_round_trip(gpu, tmp_path):
    """Tuned choices survive a save / clear / load round trip and are used
    again (the lookup after loading equals the tuned entry)."""
    gpu.csk_tune_clear()
    s = W.gaussian(40000, 200, seed=35, device=DEV)
    sk = gpu.csk_sketch(s.A, s.b, 4000, 36)
    best = gpu.csk_tune_solve(sk.At64, sk.bt, nu2=sk.nu2, trial_iters=30)
    path = str(tmp_path / "csk_tune.txt")
    gpu.csk_tune_save(path)
    gpu.csk_tune_clear()
    assert gpu.csk_tune_lookup(4000, 200, torch.float64)["grid"] == 0
    assert gpu.csk_tune_load(path) == 1
    got = gpu.csk_tune_lookup(4000, 200, torch.float64)
    assert got["grid"] == best["grid"] and got["lanes_per_row"] == best["lanes_per_row"]
    assert abs(got["us_per_iter"] - best["us_per_iter"]) <= 1e-6 * best["us_per_iter"]
    gpu.csk_tune_clear()
