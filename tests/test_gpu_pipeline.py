"""Algorithm 1 (sketch, then the loop) captured into a HIP graph through the
C ABI (csk_pipeline_capture) and replayed (csk_pipeline_launch).

Every replay must equal, bit for bit, the eager calls on the same inputs: the
graph holds the same kernels with the same arguments.  Between replays the
program does eager work of its own, synchronizes, and swaps the other
system's values into the captured input buffers, so a replay that did
nothing, or read state left by the previous one, fails."""
import pytest
import torch

from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = {
    "single": dict(m=4000, n=50, d=500, kw=dict(single_wg=1)),
    "grid": dict(m=60000, n=200, d=6000, kw=dict(single_wg=0)),
}


@pytest.mark.parametrize("lp", [None, torch.bfloat16], ids=["f64", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_pipeline_replays_match_eager(gpu, case, lp):
    c = CASES[case]
    s1 = W.gaussian(c["m"], c["n"], 17, device=DEV)
    s2 = W.gaussian(c["m"], c["n"], 18, device=DEV)
    refs = []
    for s in (s1, s2):
        sk = gpu.csk_sketch(s.A, s.b, c["d"], 9, lp_dtype=lp)
        At = sk.At64 if lp is None else sk.At_lp
        r = gpu.csk_solve(At, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=s.x_star, tol=1e-10, maxit=100000, **c["kw"])
        assert r.status == gpu.CSK_OK, (case, r.status_name)
        refs.append((r.x.clone(), r.iters, r.status, sk.bt.clone()))
    assert not torch.equal(refs[0][0], refs[1][0])

    A = s1.A.clone()
    b = s1.b.clone()
    xs = s1.x_star.clone()
    p = gpu.csk_pipeline_capture(A, b, c["d"], 9, lp_dtype=lp, x_ref=xs, tol=1e-10, maxit=100000, **c["kw"])
    torch.cuda.synchronize()
    for rep, which in enumerate((0, 1, 1, 0, 1)):
        src = (s1, s2)[which]
        A.copy_(src.A)
        b.copy_(src.b)
        xs.copy_(src.x_star)
        p.launch()
        r = p.results()
        x_ref, iters, status, bt_ref = refs[which]
        assert torch.equal(r.x, x_ref), (case, rep)
        assert (r.iters, r.status) == (iters, status), (case, rep)
        assert torch.equal(p.sketch.bt, bt_ref), (case, rep)
        y = torch.randn(4096, device=DEV)
        assert torch.isfinite((y @ y).cpu())
    p.close()
    p.close()  # idempotent


def test_pipeline_capture_errors_leave_no_capture(gpu):
    s = W.gaussian(2000, 40, 3, device=DEV)
    xs = s.x_star
    # maxit < 0 is rejected before the capture starts; d = 0 inside it (the
    # capture is ended and nothing recorded); both leave the stream usable
    with pytest.raises(gpu.CskError):
        gpu.csk_pipeline_capture(s.A, s.b, 300, 1, x_ref=xs, maxit=-1)
    st = torch.cuda.Stream()
    with pytest.raises(gpu.CskError):
        gpu.csk_pipeline_capture(s.A, s.b, 0, 1, x_ref=xs, capture_stream=st)
    with torch.cuda.stream(st):
        z = torch.ones(8, device=DEV) * 2
    torch.cuda.synchronize()
    assert float(z.sum()) == 16.0
    p = gpu.csk_pipeline_capture(s.A, s.b, 300, 1, x_ref=xs, tol=1e-10, maxit=100000, capture_stream=st)
    p.launch()
    assert p.results().status == gpu.CSK_OK
