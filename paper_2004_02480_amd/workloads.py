"""Seeded synthetic inputs shaped like the paper's workloads.

Input generation only -- none of the method's arithmetic lives here.  Both the
HIP path and the CPU oracle receive the same arrays from these generators.

Section 3 of the paper draws A and x* with a standard normal generator and
sets b = A x* (a consistent system), starting from x0 = 0.  The configurations
below follow that recipe with the distributions named for each workload:

  oracle_small   A 2000 x 50 N(0,1) FP64, d = 500                  (seed 1, sketch 101)
  dense_coherent A 200000 x 1000 U[0,1) FP64, d = 20000            (seed 2, sketch 102)
  row_scaled     A 500000 x 1000 FP32 N(0,1) * 10^U[-2,2] per row,
                 d = 10000                                          (seed 3, sketch 103)
  sparse_csr     A 1e6 x 5000 CSR, density 0.1%, every row non-empty,
                 FP32 N(0,1) values, d = 50000                      (seed 4, sketch 104)
  batched        512 systems, m ~ U{1000..50000}, n ~ U{20..500},
                 d = ceil(m/10) (redrawn until d >= 2n), FP32 N(0,1) (seed 5000+s, sketch 15000+s)
  multi_rhs      A 200000 x 500 FP32 N(0,1), 256 right-hand sides,
                 d = 10000                                          (seed 6, sketch 106)
  table1         A m x n N(0,1) FP64, d = n^2 (Section 3, Table 1)  (seed 10000+t, sketch 20000+t)
  figure         A 200000 x 200 N(0,1) FP64, d = n^2 = 40000 (Section 3's figure:
                 RK, GRK and MWRK on A, CSK on the sketch)          (seed 11000+t, sketch 21000+t,
                                                                     selection 31000+t)

b is always formed in FP64 from the exact (already rounded) entries of A, so
the system stays consistent to FP64 rounding even when A is stored in FP32.
Dense generators use PyTorch's generator on the requested device (Philox on
the GPU, so a 1.6 GB matrix takes milliseconds); the CSR generator uses
NumPy's PCG64 on the host.
"""
import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

CONFIGS = {
    "oracle_small": dict(m=2000, n=50, d=500, seed=1, sketch_seed=101, tol=1e-10, maxit=100000),
    "dense_coherent": dict(m=200000, n=1000, d=20000, seed=2, sketch_seed=102, tol=1e-10, maxit=200000),
    "row_scaled": dict(m=500000, n=1000, d=10000, seed=3, sketch_seed=103, tol=1e-10, maxit=200000),
    "sparse_csr": dict(m=1000000, n=5000, d=50000, density=1e-3, seed=4, sketch_seed=104, tol=1e-8,
                       maxit=2000000),
    "batched": dict(nsys=512, seed=5000, sketch_seed=15000, tol=1e-8, maxit=400000),
    "multi_rhs": dict(m=200000, n=500, nrhs=256, d=10000, seed=6, sketch_seed=106, tol=1e-8, maxit=400000),
    # Section 3's experiment: N(0,1) A and x*, d = n^2, x0 = 0, stop at
    # RES = ||x - x*||^2 / ||x*||^2 <= 1e-6 (tol 1e-3 on the plain relative
    # error) or 20000 iterations; trial t uses seeds seed + t, sketch_seed + t
    "table1": dict(ms=(300000, 400000, 500000, 600000, 700000), ns=(50, 100, 150), seed=10000,
                   sketch_seed=20000, tol=1e-3, maxit=20000),
    # Section 3's figure: the four methods on A 200000 x 200 with the same
    # stopping rule as Table 1
    "figure": dict(m=200000, n=200, d=40000, seed=11000, sketch_seed=21000, sel_seed=31000, tol=1e-3,
                   maxit=200000),
}


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


@dataclass
class DenseSystem:
    A: torch.Tensor
    x_star: torch.Tensor
    b: torch.Tensor


def _rhs(A: torch.Tensor, xs: torch.Tensor) -> torch.Tensor:
    """b = A x* in FP64 from the exact entries of A."""
    return (A.to(torch.float64) @ xs).contiguous()


def gaussian(m: int, n: int, seed: int, *, dtype=torch.float64, device="cpu") -> DenseSystem:
    g = _gen(seed, device)
    A = torch.randn((m, n), generator=g, dtype=torch.float64, device=device).to(dtype)
    xs = torch.randn(n, generator=g, dtype=torch.float64, device=device)
    return DenseSystem(A, xs, _rhs(A, xs))


def uniform01(m: int, n: int, seed: int, *, device="cpu") -> DenseSystem:
    """Entries i.i.d. U[0,1): highly coherent rows (all share the mean 1/2)."""
    g = _gen(seed, device)
    A = torch.rand((m, n), generator=g, dtype=torch.float64, device=device)
    xs = torch.randn(n, generator=g, dtype=torch.float64, device=device)
    return DenseSystem(A, xs, _rhs(A, xs))


def row_scaled(m: int, n: int, seed: int, *, device="cpu") -> DenseSystem:
    """FP32 N(0,1) rows scaled by 10^U[-2,2] (row norms spread over 4 decades)."""
    g = _gen(seed, device)
    A = torch.randn((m, n), generator=g, dtype=torch.float64, device=device)
    scale = torch.pow(10.0, torch.rand(m, generator=g, dtype=torch.float64, device=device) * 4.0 - 2.0)
    A = (A * scale[:, None]).to(torch.float32)
    xs = torch.randn(n, generator=g, dtype=torch.float64, device=device)
    return DenseSystem(A, xs, _rhs(A, xs))


@dataclass
class CsrSystem:
    row_ptr: np.ndarray   # int64, m+1
    col: np.ndarray       # int32, nnz (sorted and distinct within a row)
    val: np.ndarray       # float32, nnz
    x_star: np.ndarray    # float64, n
    b: np.ndarray         # float64, m
    m: int
    n: int


def sparse_csr(m: int, n: int, density: float, seed: int) -> CsrSystem:
    """CSR A: per-row count ~ Binomial(n, density) conditioned on >= 1, distinct
    uniform columns, FP32 N(0,1) values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cnt = rng.binomial(n, density, size=m)
    while True:
        zero = np.flatnonzero(cnt == 0)
        if zero.size == 0:
            break
        cnt[zero] = rng.binomial(n, density, size=zero.size)
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(cnt, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    rows = np.repeat(np.arange(m, dtype=np.int64), cnt)
    col = rng.integers(0, n, size=nnz, dtype=np.int64)
    while True:
        key = rows * n + col
        order = np.argsort(key, kind="stable")
        col = col[order]
        key = key[order]
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            break
        col[dup] = rng.integers(0, n, size=dup.size, dtype=np.int64)
    val = rng.standard_normal(nnz).astype(np.float32)
    xs = rng.standard_normal(n)
    prod = val.astype(np.float64) * xs[col]
    b = np.add.reduceat(prod, row_ptr[:-1]) if nnz else np.zeros(m)
    return CsrSystem(row_ptr, col.astype(np.int32), val, xs, b, m, n)


def csr_to_dense(s: CsrSystem) -> np.ndarray:
    A = np.zeros((s.m, s.n), np.float32)
    rows = np.repeat(np.arange(s.m), np.diff(s.row_ptr))
    A[rows, s.col] = s.val
    return A


@dataclass
class BatchShape:
    m: int
    n: int
    d: int
    seed: int
    sketch_seed: int


def batched_shapes(nsys: int = 512, base_seed: int = 5000, sketch_base: int = 15000,
                   m_range=(1000, 50000), n_range=(20, 500), ratio: int = 10) -> (List[BatchShape], int):
    """Uneven systems: m ~ U{m_range}, n ~ U{n_range}, d = ceil(m/ratio),
    redrawn while d < 2n so every sketched system is overdetermined.
    Returns (shapes, number of redraws)."""
    rng = np.random.Generator(np.random.PCG64(base_seed))
    out = []
    redraws = 0
    for s in range(nsys):
        while True:
            m = int(rng.integers(m_range[0], m_range[1] + 1))
            n = int(rng.integers(n_range[0], n_range[1] + 1))
            d = int(math.ceil(m / ratio))
            if d >= 2 * n:
                break
            redraws += 1
        out.append(BatchShape(m, n, d, base_seed + s, sketch_base + s))
    return out, redraws


@dataclass
class MultiRhsSystem:
    A: torch.Tensor       # m x n float32
    X_star: torch.Tensor  # n x nrhs float64
    B: torch.Tensor       # m x nrhs float64


def multi_rhs(m: int, n: int, nrhs: int, seed: int, *, device="cpu") -> MultiRhsSystem:
    g = _gen(seed, device)
    A = torch.randn((m, n), generator=g, dtype=torch.float64, device=device).to(torch.float32)
    Xs = torch.randn((n, nrhs), generator=g, dtype=torch.float64, device=device)
    B = (A.to(torch.float64) @ Xs).contiguous()
    return MultiRhsSystem(A, Xs, B)


def config(name: str, **over) -> dict:
    c = dict(CONFIGS[name])
    c.update(over)
    return c
