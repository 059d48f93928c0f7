"""GPU parity of the expansion in the tensor eigenbasis (Sect. 3, Theorem 2:
direct FC_n transform of loads; item 3, the direct F_n transform of grid
values) and its synthesis, against the oracle: the 1D coefficients equal
(C w, s)/||s|| for Theorem 1's eigenvectors; in N-D the round trip is the
identity, Parseval holds in the C-norm, and the load coefficients of A w are
the value coefficients of w times the denominators."""
import numpy as np
import pytest

from oracle import solve as osolve
from oracle import timestep, transforms
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


@pytest.mark.parametrize("n,K", [(3, 8), (5, 12), (2, 16)])
def test_values_coefficients_1d_match_theorem1(fm, n, K):
    w = inputs.draw_rhs([n * K - 1], 1000 + K, "normal")
    _, S, norms2 = transforms.basis(n, K, 20)
    Cw = timestep.mass_apply(w, n, (K,))
    want = (S.T @ Cw) / np.sqrt(norms2)
    got = fm.Plan((K,), n, (1.0,), 0.0).coefficients(torch.from_numpy(w).cuda()).cpu().numpy()
    for c in range(n - 1):  # k = 0 eigenvectors: free sign
        if got[c] * want[c] < 0:
            got[c] = -got[c]
    assert np.allclose(got, want, atol=1e-12 * np.abs(want).max())


CASES = [((16, 12), (3, 3), 1), ((24, 10), (2, 5), 2), ((6, 5, 8), (2, 3, 2), 1), ((64, 48), (9, 4), 1)]


@pytest.mark.parametrize("K,ns,nrhs", CASES)
def test_nd_round_trip_parseval_and_diagonal(fm, K, ns, nrhs):
    N = len(K)
    diff, react = (1.0, 0.5, 2.0)[:N], 0.3
    shape = tuple(m * k - 1 for m, k in zip(ns, K))
    say("coefficients", K, ns, nrhs)
    p = fm.Plan(K, ns, diff, react, nrhs=nrhs)
    w = inputs.draw_rhs(shape, seed=1100 + sum(K), nrhs=nrhs)
    full = ((nrhs,) if nrhs > 1 else ()) + shape
    wt = torch.from_numpy(np.ascontiguousarray(w.reshape(full))).cuda()
    c = p.coefficients(wt)
    back = p.synthesize(c)
    torch.cuda.synchronize()
    assert rel(back.cpu().numpy(), w.reshape(full)) < 1e-12
    ws = w.reshape((nrhs,) + shape)
    cs = c.cpu().numpy().reshape((nrhs,) + shape)
    # denominators in the spectral order of every axis (plan tables)
    den = np.full(shape, react)
    coef = osolve.coefficients(K, diff)
    for d in range(N):
        lam, _ = p.tables(d)
        sh = [1] * N
        sh[d] = shape[d]
        den = den + (coef[d] * lam).reshape(sh)
    for r in range(nrhs):
        # Parseval in the C-norm: sum c^2 = w . C w
        wCw = float(np.sum(ws[r] * timestep.mass_apply(ws[r], ns, K)))
        assert abs(float(np.sum(cs[r] ** 2)) - wCw) <= 1e-12 * abs(wCw)
        # load coefficients of A w = denominators x value coefficients of w
        Aw = osolve.apply_A(ws[r], ns, K, diff, react)
        cA = p.coefficients(torch.from_numpy(np.ascontiguousarray(
            np.broadcast_to(Aw, full) if nrhs == 1 else np.stack([Aw] * nrhs))).cuda(), kind="loads")
        torch.cuda.synchronize()
        cA = cA.cpu().numpy().reshape((nrhs,) + shape)[0]
        assert rel(cA, den * cs[r]) < 1e-11
