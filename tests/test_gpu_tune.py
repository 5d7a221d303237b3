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
