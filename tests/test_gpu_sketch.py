"""GPU parity of the sketch (Definition 1; Algorithm 1, Initialize) against the
CPU oracle: hash, signs, bucket permutation and offsets, the FP64 sketch and
its low-precision copies are bit-exact; squared row norms agree to FP64
rounding.  Called through the C ABI (via the ctypes binding)."""
import numpy as np
import pytest
import torch

from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _bits16(t):
    return t.view(torch.int16).cpu().numpy().view(np.uint16)


@pytest.mark.parametrize("m,d,seed", [(2000, 500, 101), (200000, 20000, 102), (1000, 1, 5),
                                      (5000, 2**31 - 1, 7), (1_000_003, 50000, 104)])
def test_hash_bitexact(gpu, orc, m, d, seed):
    bucket, sign = gpu.csk_hash(seed, m, d, device=DEV)
    ob, os_ = orc.hash_rows(seed, m, d)
    np.testing.assert_array_equal(bucket.cpu().numpy().view(np.uint32), ob)
    np.testing.assert_array_equal(sign.cpu().numpy(), os_)


def test_hash_equals_published_splitmix64_outputs(gpu):
    # the library's hash against the generator's published first outputs
    # (tests/golden/splitmix64.json), independently of the oracle
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")) as f:
        vecs = json.load(f)["vectors"]
    for v in vecs:
        words = [int(h, 16) for h in v["outputs_hex"]] if "outputs_hex" in v else [int(w) for w in v["outputs"]]
        for d in (2, 20000, 2**31 - 1):
            bucket, sign = gpu.csk_hash(int(v["seed"]), len(words), d, device=DEV)
            assert [int(x) for x in bucket.cpu().numpy().view(np.uint32)] == [((w >> 32) * d) >> 32 for w in words]
            assert [int(x) for x in sign.cpu().numpy()] == [-1 if (w & 1) else 1 for w in words]


def _check_sketch(gpu, orc, A, b, d, seed, lp=None):
    out = gpu.csk_sketch(A, b, d, seed, lp_dtype=lp, want_perm=True)
    torch.cuda.synchronize()
    An = A.cpu().numpy()
    bn = None if b is None else b.cpu().numpy()
    At, bt = orc.sketch_dense(An, bn, d, seed)
    np.testing.assert_array_equal(out.At64.cpu().numpy(), At)
    if b is not None:
        np.testing.assert_array_equal(out.bt.cpu().numpy(), bt)
    bucket, _ = orc.hash_rows(seed, A.shape[0], d)
    perm, ptr = orc.bucket_sort(bucket, d)
    np.testing.assert_array_equal(out.perm.cpu().numpy().view(np.uint32), perm)
    np.testing.assert_array_equal(out.ptr.cpu().numpy().view(np.uint32), ptr)
    nu2 = orc.row_norms2(At)
    np.testing.assert_allclose(out.nu2.cpu().numpy(), nu2, rtol=1e-13, atol=0)
    if lp is not None:
        got = out.At_lp
        if lp == torch.float32:
            np.testing.assert_array_equal(got.cpu().numpy().view(np.uint32), orc.round_f64_to_f32(At).view(np.uint32))
        elif lp == torch.bfloat16:
            np.testing.assert_array_equal(_bits16(got), orc.round_f64_to_bf16_bits(At))
        else:
            np.testing.assert_array_equal(_bits16(got), orc.round_f64_to_f16_bits(At))
    return out


@pytest.mark.parametrize("m,n,d", [
    (2000, 50, 500),      # oracle-size shape
    (1, 1, 1),            # smallest
    (37, 5, 100),         # d > m: many empty buckets
    (5000, 3, 1),         # one bucket longer than the LDS sort capacity
    (3000, 1001, 64),     # odd n: ragged vector tails, two column chunks
    (4000, 600, 333),     # several chunks, ragged
])
def test_sketch_f64_bitexact(gpu, orc, m, n, d):
    s = W.gaussian(m, n, seed=m + n, device=DEV)
    _check_sketch(gpu, orc, s.A, s.b, d, seed=1000 + d)


def test_sketch_strided_rows(gpu, orc):
    s = W.gaussian(3000, 130, seed=3, device=DEV)
    Abig = torch.zeros((3000, 136), dtype=torch.float64, device=DEV)
    Abig[:, :130] = s.A
    A = Abig[:, :130]
    assert A.stride(0) == 136
    _check_sketch(gpu, orc, A, s.b, 211, seed=4)


@pytest.mark.parametrize("lp", [torch.float32, torch.bfloat16, torch.float16])
def test_sketch_f32_input_lowprec_bitexact(gpu, orc, lp):
    s = W.row_scaled(20000, 203, seed=5, device=DEV)
    _check_sketch(gpu, orc, s.A, s.b, 1500, seed=6, lp=lp)


def test_sketch_multi_rhs_bitexact(gpu, orc):
    s = W.multi_rhs(6000, 40, 34, seed=7, device=DEV)
    out = gpu.csk_sketch(s.A, s.B, 400, 8, lp_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    At, Bt = orc.sketch_dense(s.A.cpu().numpy(), s.B.cpu().numpy(), 400, 8)
    np.testing.assert_array_equal(out.At64.cpu().numpy(), At)
    np.testing.assert_array_equal(out.bt.cpu().numpy(), Bt)
    np.testing.assert_array_equal(_bits16(out.At_lp), orc.round_f64_to_bf16_bits(At))


def test_sketch_dense_coherent_full_size_bitexact(gpu, orc):
    # the benchmark workload: A 200000 x 1000 U[0,1) FP64, d = 20000
    c = W.config("dense_coherent")
    s = W.uniform01(c["m"], c["n"], c["seed"], device=DEV)
    out = gpu.csk_sketch(s.A, s.b, c["d"], c["sketch_seed"])
    torch.cuda.synchronize()
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), c["d"], c["sketch_seed"])
    np.testing.assert_array_equal(out.At64.cpu().numpy(), At)
    np.testing.assert_array_equal(out.bt.cpu().numpy(), bt)


def test_sketch_row_scaled_full_size_bitexact(gpu, orc):
    c = W.config("row_scaled")
    s = W.row_scaled(c["m"], c["n"], c["seed"], device=DEV)
    out = gpu.csk_sketch(s.A, s.b, c["d"], c["sketch_seed"], lp_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    At, bt = orc.sketch_dense(s.A.cpu().numpy(), s.b.cpu().numpy(), c["d"], c["sketch_seed"])
    np.testing.assert_array_equal(out.At64.cpu().numpy(), At)
    np.testing.assert_array_equal(out.bt.cpu().numpy(), bt)
    np.testing.assert_array_equal(_bits16(out.At_lp), orc.round_f64_to_bf16_bits(At))


# (6000, 3000, 0.02, 600): about 600 stored entries per bucket, so some
# buckets fit the ranked-run kernel's 512-entry staging and the rest go
# through the queue to the accumulator-row kernel; (20000, 2000, 0.01, 40):
# 500 rows per bucket, every bucket queued
@pytest.mark.parametrize("m,n,dens,d", [(3000, 400, 0.01, 150), (20000, 3000, 0.002, 700), (50, 9000, 0.01, 10),
                                        (6000, 3000, 0.02, 600), (20000, 2000, 0.01, 40)])
def test_sketch_csr_bitexact(gpu, orc, m, n, dens, d):
    s = W.sparse_csr(m, n, dens, seed=m)
    rp = torch.from_numpy(s.row_ptr).to(DEV)
    col = torch.from_numpy(s.col).to(DEV)
    val = torch.from_numpy(s.val).to(DEV)
    b = torch.from_numpy(s.b).to(DEV)
    out = gpu.csk_sketch_csr(rp, col, val, n, b, d, 17, lp_dtype=torch.float32)
    torch.cuda.synchronize()
    At, bt = orc.sketch_csr(s.row_ptr, s.col, s.val, m, n, s.b, d, 17)
    np.testing.assert_array_equal(out.At64.cpu().numpy(), At)
    np.testing.assert_array_equal(out.bt.cpu().numpy(), bt)
    np.testing.assert_array_equal(out.At_lp.cpu().numpy().view(np.uint32), orc.round_f64_to_f32(At).view(np.uint32))
    np.testing.assert_allclose(out.nu2.cpu().numpy(), orc.row_norms2(At), rtol=1e-13, atol=0)


def test_sketch_csr_full_size_sampled(gpu, orc):
    # A 1e6 x 5000 at 0.1% density, d = 50000: full sketch on the GPU, the
    # oracle's dense FP64 result compared on a sample of 400 rows (FP32 copy,
    # bt and nu2 compared in full).
    c = W.config("sparse_csr")
    s = W.sparse_csr(c["m"], c["n"], c["density"], c["seed"])
    rp = torch.from_numpy(s.row_ptr).to(DEV)
    col = torch.from_numpy(s.col).to(DEV)
    val = torch.from_numpy(s.val).to(DEV)
    b = torch.from_numpy(s.b).to(DEV)
    out = gpu.csk_sketch_csr(rp, col, val, c["n"], b, c["d"], c["sketch_seed"], lp_dtype=torch.float32,
                             want_f64=False)
    torch.cuda.synchronize()
    At, bt = orc.sketch_csr(s.row_ptr, s.col, s.val, s.m, s.n, s.b, c["d"], c["sketch_seed"])
    rows = np.random.default_rng(0).choice(c["d"], 400, replace=False)
    got = out.At_lp[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint32), orc.round_f64_to_f32(At[rows]).view(np.uint32))
    np.testing.assert_array_equal(out.bt.cpu().numpy(), bt)
    np.testing.assert_allclose(out.nu2.cpu().numpy(), orc.row_norms2(At), rtol=1e-13, atol=0)


def test_sketch_deterministic(gpu):
    s = W.gaussian(30000, 77, seed=9, device=DEV)
    a = gpu.csk_sketch(s.A, s.b, 900, 3, want_perm=True)
    b = gpu.csk_sketch(s.A, s.b, 900, 3, want_perm=True)
    torch.cuda.synchronize()
    assert torch.equal(a.At64, b.At64) and torch.equal(a.perm, b.perm) and torch.equal(a.nu2, b.nu2)
