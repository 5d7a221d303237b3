"""Comparisons shared by the GPU parity tests (imported by test modules).

Iterates of the GPU loop and of the oracle differ only in the rounding of
the residual sums (another summation order), so they are compared element by
element to a bound of 1e-12 of the iterate's norm; the rows the two loops
select (Algorithm 1's i_k) are compared bit for bit."""
import numpy as np
import torch


def host(v):
    return v.detach().cpu().numpy() if torch.is_tensor(v) else np.asarray(v)


def assert_iterate_close(x_gpu, x_orc, rel=1e-12, what=""):
    """Every entry of x_gpu within rel * ||x_orc||_2 of x_orc's."""
    xg, xo = host(x_gpu), host(x_orc)
    assert xg.shape == xo.shape, (xg.shape, xo.shape)
    np.testing.assert_allclose(xg, xo, rtol=0.0, atol=rel * max(np.linalg.norm(xo), 1e-300), err_msg=what)


def assert_trace_equal(trace_gpu, idx_orc, what=""):
    """The GPU's selected rows for iterations 0..K-1 equal the oracle's."""
    tg = host(trace_gpu)[:len(idx_orc)]
    np.testing.assert_array_equal(tg, host(idx_orc).astype(np.int64), err_msg=what)


def new_trace(maxit, device="cuda:0"):
    return torch.full((max(int(maxit), 1),), -1, dtype=torch.int64, device=device)
