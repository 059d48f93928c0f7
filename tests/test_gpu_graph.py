"""Solves captured in a graph: fftfem_solve issues only kernel launches on the
caller's stream (no allocation, no memset, no host synchronisation), so a
caller can capture it.  Each case captures one solve with torch's graph
capture, replays it three times with eager work and synchronisations in
between (the output cleared before each replay), and checks every replay
against the eager solve bit for bit, and the eager solve against the
oracle."""
import numpy as np
import pytest

from oracle import solve as osolve
from paper_1701_03967_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1701_03967_amd import fftfem
    fftfem.lib()
    return fftfem


CASES = [
    # K, n, precision, algorithm, nrhs, oracle tolerance
    ((24, 40), 3, "fp64", "a", 1, 1e-12),
    ((24, 40), 3, "fp64", "b", 2, 1e-12),
    ((20, 16), 4, "fp32_refine", "a", 1, 1e-10),
    ((6, 8, 10), 2, "fp64", "a", 1, 1e-12),
    ((2048,), 5, "fp64", "a", 2, 1e-11),   # long line: four-step passes
    ((1031,), 3, "fp64", "a", 1, 1e-11),   # long line: Bluestein passes
]


@pytest.mark.parametrize("K,n,prec,alg,nrhs,tol", CASES)
def test_captured_solve_replays(fm, K, n, prec, alg, nrhs, tol):
    say("graph", K, n, prec, alg, nrhs)
    N = len(K)
    kw = dict(max_iter=4, tol=1e-13) if prec == "fp32_refine" else {}
    p = fm.Plan(K, n, (1.0,) * N, 0.7, precision=prec, algorithm=alg, nrhs=nrhs, **kw)
    shape = ((nrhs,) if nrhs > 1 else ()) + p.shape
    f_host = inputs.draw_rhs(list(p.shape), 2000 + sum(K) + n, "normal", nrhs=nrhs)
    f = torch.from_numpy(f_host).cuda()
    u_eager = p.solve(f)
    torch.cuda.synchronize()
    ref = u_eager.cpu().numpy().copy()
    # the eager solve against the oracle (small cases only)
    if int(np.prod(p.shape)) <= 40000 or N == 1 and K[0] <= 2048:
        for r in range(nrhs):
            fr = f_host[r] if nrhs > 1 else f_host
            ur = ref[r] if nrhs > 1 else ref
            if N == 1 and K[0] > 1024:
                continue  # long lines: against the oracle in test_gpu_long
            want = osolve.solve(fr, n, K, (1.0,) * N, 0.7)
            assert np.linalg.norm(ur - want) / np.linalg.norm(want) < tol
    # capture on a side stream, as torch requires
    u = torch.empty(shape, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        p.solve(f, u)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.solve(f, u)
    for rep in range(3):
        u.fill_(float(rep + 1))
        scratch = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        got = u.cpu().numpy()
        assert np.array_equal(got, ref), (rep, float(np.abs(got - ref).max()))
    del g
