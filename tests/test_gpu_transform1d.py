"""GPU parity of the 1D FC_n and F_n transforms (Sect. 3, Theorem 2) at the
kinds of element counts of the transform microbenchmark: powers of two,
primes and composites (the latter two through the chirp-z DFTs), n = 5.
Forward: (y, s)/||s||_C against the oracle's eigenvectors of Theorem 1;
inverse of the forward: C^{-1} y (completeness), checked by applying the
oracle's element-wise mass operator."""
import numpy as np
import pytest

from oracle import fem1d, transforms
from oracle.element import element_matrices
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("K", [31, 48, 64, 61])
def test_forward_matches_theorem1_eigenvectors(fm, K):
    n = 5
    say("fc_n", n, K)
    y = inputs.draw_rhs([n * K - 1], 700 + K, "normal")
    _, S, norms2 = transforms.basis(n, K, 20)
    want = (S.T @ y) / np.sqrt(norms2)
    p = fm.Plan((K,), n, (1.0,), 0.0)
    got = p.debug_transform(0, +1, torch.from_numpy(y).cuda()).cpu().numpy()
    for c in range(n - 1):  # k = 0 eigenvectors: free sign
        if got[c] * want[c] < 0:
            got[c] = -got[c]
    assert np.allclose(got, want, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("K", [127, 200, 509, 600, 1000, 1021, 1024])
def test_round_trip_large_K(fm, K):
    n = 5
    say("round trip", n, K)
    # 9 lines along axis 1 of a 2D plan (axis 0: K0 = 2, M0 = 9)
    p = fm.Plan((2, K), n, (1.0, 1.0), 0.0)
    M0 = p.shape[0]
    y = inputs.draw_rhs([M0, n * K - 1], 800 + K, "normal")
    yt = torch.from_numpy(y).cuda()
    c = p.debug_transform(1, +1, yt)
    back = p.debug_transform(1, -1, c).cpu().numpy()
    _, C = element_matrices(n)
    assert rel(fem1d.apply_elementwise(C, back, 1), y) < 1e-12


@pytest.mark.parametrize("K", [7, 14, 21, 49, 243, 343, 625, 720, 729, 875, 1008])
def test_mixed_radix_round_trip_and_solve(fm, K):
    """Element counts with prime factors 2, 3, 5, 7 only (the mixed-radix
    Stockham stages, including radix-7 and long radix-3/5 chains): the 1D
    round trip, and a 2D solve against the oracle where it is cheap."""
    n = 3
    say("mixed radix", n, K)
    p = fm.Plan((2, K), n, (1.0, 1.0), 0.0)
    y = inputs.draw_rhs(list(p.shape), 900 + K, "normal")
    yt = torch.from_numpy(y).cuda()
    back = p.debug_transform(1, -1, p.debug_transform(1, +1, yt)).cpu().numpy()
    _, C = element_matrices(n)
    assert rel(fem1d.apply_elementwise(C, back, 1), y) < 1e-12
    if K <= 243:
        from oracle import solve as osolve
        f = inputs.draw_rhs([n * 5 - 1, n * K - 1], 950 + K, "normal")
        for precision, tol in (("fp64", 1e-11), ("fp32_refine", 1e-10)):
            kw = dict(max_iter=4, tol=1e-13) if precision == "fp32_refine" else {}
            u = fm.Plan((5, K), n, (1.0, 0.5), 1.0, precision=precision, **kw).solve(torch.from_numpy(f).cuda())
            torch.cuda.synchronize()
            assert rel(u.cpu().numpy(), osolve.solve(f, n, (5, K), (1.0, 0.5), 1.0)) < tol, precision
