"""GPU parity of the batched form: many independent systems, each sketched
with its own seed and solved by its own MWRK loop, in one pass.  The
sketches the batched call builds for its solves (read from its workspace)
are bit-exact with the oracle's, zero padding included; every solution meets
the tolerance against x* and lies within twice it of the oracle's FP64
solution."""
import math

import numpy as np
import pytest
import torch

from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def make_batch(shapes, dtype):
    systems = []
    for sh in shapes:
        s = W.gaussian(sh.m, sh.n, sh.seed, dtype=dtype, device=DEV)
        systems.append(dict(A=s.A, b=s.b, d=sh.d, seed=sh.sketch_seed, x_ref=s.x_star))
    return systems


@pytest.mark.parametrize("a_dtype,lp", [(torch.float32, torch.float32), (torch.float64, torch.float64),
                                        (torch.float32, torch.bfloat16)])
def test_batched_small_matches_oracle(gpu, orc, a_dtype, lp):
    shapes, _ = W.batched_shapes(24, base_seed=700, sketch_base=900, m_range=(1000, 9000), n_range=(20, 120))
    systems = make_batch(shapes, a_dtype)
    xs, res = gpu.csk_solve_batched(systems, lp_dtype=lp, tol=1e-8, maxit=400000)
    for k, (sysd, x, r) in enumerate(zip(systems, xs, res)):
        it, st, fb, meas, nref = r
        assert st == gpu.CSK_OK, (k, st)
        xr = sysd["x_ref"].cpu().numpy()
        xg = x.cpu().numpy()
        assert np.linalg.norm(xg - xr) <= 1e-8 * np.linalg.norm(xr), k
        o = orc.csk(sysd["A"].cpu().numpy(), sysd["b"].cpu().numpy(), sysd["d"], sysd["seed"], xref=xr, tol=1e-8,
                    maxit=400000)
        assert o.status == 0
        assert np.linalg.norm(xg - o.x) <= 2e-8 * np.linalg.norm(xr), k


@pytest.mark.parametrize("a_dtype,lp", [(torch.float32, torch.bfloat16), (torch.float64, torch.float64),
                                        (torch.float32, torch.float16), (torch.float32, torch.float32)])
def test_batched_sketch_bitexact(gpu, orc, a_dtype, lp):
    # uneven systems, some with d > m / 10 and odd n (ragged rows padded with
    # zeros to the library's row length), sketched together in one pipeline:
    # every system's At64, its low-precision copy and bt equal the oracle's
    shapes, _ = W.batched_shapes(20, base_seed=300, sketch_base=400, m_range=(1000, 30000), n_range=(20, 300))
    systems = make_batch(shapes, a_dtype)
    xs, raw, ws = gpu.csk_solve_batched(systems, lp_dtype=lp, tol=1e-8, maxit=5, sync=False)
    torch.cuda.synchronize()
    views = gpu.csk_solve_batched_sketches(systems, ws, lp_dtype=lp)
    for k, (sysd, v) in enumerate(zip(systems, views)):
        At, bt = orc.sketch_dense(sysd["A"].cpu().numpy(), sysd["b"].cpu().numpy(), sysd["d"], sysd["seed"])
        np.testing.assert_array_equal(v.At64.cpu().numpy(), At, err_msg=f"system {k}")
        np.testing.assert_array_equal(v.bt.cpu().numpy(), bt, err_msg=f"system {k}")
        np.testing.assert_allclose(v.nu2.cpu().numpy(), orc.row_norms2(At), rtol=1e-13, atol=0)
        n = sysd["A"].shape[1]
        full64 = v.At64.as_strided((v.At64.shape[0], v.At64.stride(0)), (v.At64.stride(0), 1))
        assert torch.count_nonzero(full64[:, n:]).item() == 0, k
        if v.At_lp is not None:
            if lp == torch.float32:
                np.testing.assert_array_equal(v.At_lp.cpu().numpy().view(np.uint32),
                                              orc.round_f64_to_f32(At).view(np.uint32), err_msg=f"system {k}")
            else:
                bits = v.At_lp.contiguous().view(torch.int16).cpu().numpy().view(np.uint16)
                want = orc.round_f64_to_bf16_bits(At) if lp == torch.bfloat16 else orc.round_f64_to_f16_bits(At)
                np.testing.assert_array_equal(bits, want, err_msg=f"system {k}")
            fl = v.At_lp.as_strided((v.At_lp.shape[0], v.At_lp.stride(0)), (v.At_lp.stride(0), 1))
            assert torch.count_nonzero(fl[:, n:]).item() == 0, k
    del ws


def test_batched_single_system_equals_plain_path(gpu):
    # one system through the batched entry point against sketch + solve
    s = W.gaussian(6000, 80, seed=3, dtype=torch.float32, device=DEV)
    xs, res = gpu.csk_solve_batched([dict(A=s.A, b=s.b, d=600, seed=9, x_ref=s.x_star)], lp_dtype=torch.float32,
                                    tol=1e-8)
    sk = gpu.csk_sketch(s.A, s.b, 600, 9, lp_dtype=torch.float32)
    r = gpu.csk_solve(sk.At_lp, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=1e-8, single_wg=1)
    assert res[0][1] == gpu.CSK_OK and r.status == gpu.CSK_OK
    # the two paths may split rows over different lane counts (FP32 partial
    # sums in another order), so trajectories agree to rounding, not bitwise
    assert abs(res[0][0] - r.iters) <= 0.1 * r.iters + 5
    assert ((xs[0] - r.x).norm() / s.x_star.norm()).item() <= 2e-8


def test_batched_residual_mode_without_reference(gpu):
    shapes, _ = W.batched_shapes(8, base_seed=11, sketch_base=12, m_range=(2000, 5000), n_range=(20, 60))
    systems = make_batch(shapes, torch.float32)
    for sysd in systems:
        sysd["x_ref"] = None
    xs, res = gpu.csk_solve_batched(systems, lp_dtype=torch.float32, tol=1e-9)
    for sysd, x, r in zip(systems, xs, res):
        assert r[1] == gpu.CSK_OK
        A = sysd["A"].double()
        sk = gpu.csk_sketch(sysd["A"], sysd["b"], sysd["d"], sysd["seed"])
        torch.cuda.synchronize()
        rel = (sk.bt - sk.At64 @ x).norm() / sk.bt.norm()
        assert rel.item() <= 1e-9 * (1 + 1e-6)
        del A


@pytest.mark.parametrize("lp", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
def test_batched_deterministic(gpu, lp):
    # systems from the full recipe's range, some long enough to be split over
    # several workgroups: two runs give the same bits whatever workgroup
    # claims which work item
    shapes, _ = W.batched_shapes(48, base_seed=21, sketch_base=22)
    systems = make_batch(shapes, torch.float32)
    xa, ra = gpu.csk_solve_batched(systems, lp_dtype=lp, tol=1e-8)
    xb, rb = gpu.csk_solve_batched(systems, lp_dtype=lp, tol=1e-8)
    assert ra == rb
    for a, b in zip(xa, xb):
        assert torch.equal(a, b)
    assert all(r[1] == gpu.CSK_OK for r in ra)


def test_batched_shapes_recipe():
    shapes, redraws = W.batched_shapes(512)
    assert len(shapes) == 512
    for sh in shapes:
        assert 1000 <= sh.m <= 50000 and 20 <= sh.n <= 500
        assert sh.d == math.ceil(sh.m / 10) and sh.d >= 2 * sh.n
    assert redraws >= 0
