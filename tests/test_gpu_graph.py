"""The whole path, sketch (Algorithm 1, Initialize) then loop (Algorithm 1,
loop), captured once into a HIP graph and replayed.

Each replay is checked against the eager result of the same inputs, bit for
bit: the graph holds the same kernels with the same arguments, so nothing may
differ.  Between replays the program does eager work of its own, synchronizes,
and swaps a second system into the captured input buffers, so a replay that
silently did nothing, or read stale state left by the previous one, fails."""
import pytest
import torch

from paper_2004_02480_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = {
    # single workgroup: the system fits one CU
    "single": dict(m=4000, n=50, d=500, kw=dict(single_wg=1)),
    # cooperative grid over every CU
    "grid": dict(m=60000, n=200, d=6000, kw=dict(single_wg=0)),
}


def _path(gpu, A, b, x_star, d, lp, kw):
    sk = gpu.csk_sketch(A, b, d, 8, lp_dtype=lp)
    At = sk.At64 if lp is None else sk.At_lp
    return gpu.csk_solve(At, sk.bt, At64=sk.At64, nu2=sk.nu2, x_ref=x_star, tol=1e-10, maxit=100000,
                         sync=False, **kw)


@pytest.mark.parametrize("lp", [None, torch.bfloat16], ids=["f64", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_captured_sketch_and_solve_replays_match_eager(gpu, case, lp):
    c = CASES[case]
    s1 = W.gaussian(c["m"], c["n"], 7, device=DEV)
    s2 = W.gaussian(c["m"], c["n"], 8, device=DEV)
    refs = []
    for s in (s1, s2):
        x, raw = _path(gpu, s.A, s.b, s.x_star, c["d"], lp, c["kw"])
        torch.cuda.synchronize()
        r = gpu.parse_results(raw)[0]
        assert r[1] == gpu.CSK_OK, (case, r)
        refs.append((x.clone(), r))
    assert not torch.equal(refs[0][0], refs[1][0])

    # static buffers that the graph reads
    A = s1.A.clone()
    b = s1.b.clone()
    xs = s1.x_star.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _path(gpu, A, b, xs, c["d"], lp, c["kw"])
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        x_g, raw_g = _path(gpu, A, b, xs, c["d"], lp, c["kw"])

    for rep, which in enumerate((0, 1, 0, 1, 0)):
        src = (s1, s2)[which]
        A.copy_(src.A)
        b.copy_(src.b)
        xs.copy_(src.x_star)
        g.replay()
        torch.cuda.synchronize()
        x_ref, r_ref = refs[which]
        assert torch.equal(x_g, x_ref), (case, rep)
        assert gpu.parse_results(raw_g)[0] == r_ref, (case, rep)
        # eager work of the program's own between replays
        y = torch.randn(4096, device=DEV)
        assert torch.isfinite((y @ y).cpu())
