"""GPU parity of the long-line transforms: one-axis plans whose element count
K exceeds one LDS tile (1024 < K <= 2^20), n = 5: powers of two (four-step
DFT passes) and other K, odd and even, primes among them (Bluestein's
chirp-z over a power-of-two length L >= 2K - 1, up to L = 2^21).

- forward FC_n (Sect. 3, Theorem 2): sampled coefficients (y, s)/||s||_C
  against the oracle's eigenvectors of Theorem 1 (the norm taken as s.Ccal s
  with the oracle's element-wise mass operator);
- inverse of the forward: C^{-1} y (completeness, Theorem 2), checked with the
  oracle's mass operator, on two lines at once and in place;
- the 1D solve (Sect. 4 with N = 1): against the interpolant of a sine whose
  load the oracle integrates element by element (the FEM error of order
  h^(n+1) is far below rounding at these K), and against a sparse direct solve
  of the oracle-assembled matrices where that is accurate;
- NaN in the load reported through the statistics.
"""
import numpy as np
import pytest

from oracle import eigen1d, fem1d, loads
from oracle.element import element_matrices
from paper_1701_03967_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N5 = 5
KS = [1 << 11, 1 << 12, 1 << 16, 1 << 20]
# not powers of two: odd composite, primes, even composites, the largest
# prime below 2^20 (L = 2^21)
KS_OTHER = [1025, 1031, 2308, 4099, 60695, 65537, 319564, 1048573]


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1701_03967_amd import fftfem
    fftfem.lib()
    return fftfem


_plans = {}


def plan(fm, K, diff=1.0, react=0.0, X=1.0, nrhs=1):
    """Plans are costly to build at K = 2^20 (host tables of 2^20 pencils):
    one per configuration for the whole module."""
    key = (K, diff, react, X, nrhs)
    if key not in _plans:
        say("plan", key)
        _plans[key] = fm.Plan((K,), N5, (diff,), react, X=(X,), nrhs=nrhs)
    return _plans[key]


def coef_index(n, k, l):
    return l - 1 if k == 0 else n - 1 + (k - 1) * n + (l - 1)


SAMPLES = {
    1 << 11: [(0, 1), (0, 4), (1, 1), (1, 5), (2, 3), (333, 2), (1024, 1), (1024, 5), (1025, 4), (2047, 5)],
    1 << 12: [(1, 2), (2047, 1), (2048, 3), (2049, 5), (4095, 4)],
    1 << 16: [(1, 1), (40000, 5)],
    1025: [(0, 2), (0, 3), (1, 1), (512, 4), (513, 5), (1024, 2)],
    1031: [(1, 5), (515, 1), (516, 3), (1030, 4)],
    2308: [(1, 3), (1154, 2), (1155, 5), (2307, 1)],
    65537: [(32768, 2), (65536, 5)],
}


@pytest.mark.parametrize("K", sorted(SAMPLES))
def test_long_forward_matches_theorem1_eigenvectors(fm, K):
    n = N5
    say("long forward", n, K)
    y = inputs.draw_rhs([n * K - 1], 1700 + K % 997, "normal")
    p = plan(fm, K)
    got = p.debug_transform(0, +1, torch.from_numpy(y).cuda()).cpu().numpy()
    _, C = element_matrices(n)
    tol = 1e-13 * np.linalg.norm(y)
    for k, l in SAMPLES[K]:
        _, s = eigen1d.eigvec(n, K, k, l, dps=20)
        want = float(y @ s) / np.sqrt(float(s @ fem1d.apply_elementwise(C, s, 0)))
        g = got[coef_index(n, k, l)]
        if k == 0 and g * want < 0:  # k = 0 eigenvectors: free sign
            g = -g
        assert abs(g - want) <= tol, (k, l, g, want)


@pytest.mark.parametrize("K", KS + KS_OTHER)
def test_long_round_trip(fm, K):
    n = N5
    say("long round trip", n, K)
    p = plan(fm, K, nrhs=2)
    y = inputs.draw_rhs([2, n * K - 1], 1800 + K % 991, "normal")
    yt = torch.from_numpy(y).cuda()
    c = p.debug_transform(0, +1, yt)
    back = p.debug_transform(0, -1, c, out=c).cpu().numpy()  # inverse in place
    _, C = element_matrices(n)
    for r in range(2):
        Cb = fem1d.apply_elementwise(C, back[r], 0)
        assert np.linalg.norm(Cb - y[r]) / np.linalg.norm(y[r]) < 1e-12, r


@pytest.mark.parametrize("K,diff,react,X", [
    (1 << 11, 1.0, 0.0, 1.0), (1 << 12, 0.7, 2.5, 3.0), (1 << 16, 1.3, 0.4, 2.0), (1 << 20, 1.0, 0.0, 1.0),
    (1025, 0.7, 2.5, 3.0), (4099, 1.0, 0.0, 1.0), (319564, 1.0, 0.0, 1.0), (1048573, 1.0, 0.0, 1.0)])
def test_long_solve_sine(fm, K, diff, react, X):
    """Two right-hand sides at once: the loads of sin(m pi x / X), m = 1, 3."""
    n = N5
    say("long solve sine", n, K, diff, react, X)
    p = plan(fm, K, diff, react, X, nrhs=2)
    f = np.empty((2, n * K - 1))
    want = np.empty_like(f)
    for r, m in enumerate((1, 3)):
        ue, fe = loads.sin_product((m,), (diff,), react, X=[X])
        f[r] = loads.load_vector_1d(fe, n, K, X=X)
        want[r] = loads.interpolate(ue, n, (K,), X=[X])
    u = p.solve(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    err = np.abs(u.cpu().numpy() - want).max(axis=1)
    assert (err < 1e-12).all(), err
    st = p.stats()
    assert st["converged"] and st["stop"] == "none", st


@pytest.mark.parametrize("K", [1 << 11, 1031, 2308])
def test_long_solve_matches_sparse_direct(fm, K):
    """Random load: the sparse LU solve alone is only accurate to about
    cond(A) eps (1e-8 here), so it is refined with the residual of the
    oracle's element-wise operator in extended precision, as the oracle's
    own solve does."""
    import scipy.sparse.linalg as spla
    from oracle import solve as osolve
    n, diff, react = N5, 1.0, 0.5
    say("long solve sparse", n, K)
    A, C = fem1d.assemble(n, K, dense=False)
    f = inputs.draw_rhs([n * K - 1], 1900, "normal")
    lu = spla.splu((diff * 4.0 * K * K * A + react * C).tocsc())
    ref = lu.solve(f)
    for _ in range(3):
        r = f - osolve.apply_A(ref, n, (K,), (diff,), react, extended=True)
        ref = ref + lu.solve(r.astype(np.float64))
    u = plan(fm, K, diff, react).solve(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-11


@pytest.mark.parametrize("K", [1 << 11, 1031])
def test_long_solve_reports_nonfinite(fm, K):
    n = N5
    say("long solve nan", n, K)
    p = plan(fm, K, nrhs=2)
    f = inputs.draw_rhs([2, n * K - 1], 1901, "normal")
    f[1, 77] = np.nan
    u = p.solve(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    assert np.isfinite(u[0].cpu().numpy()).all()
    st = p.stats()
    assert not st["converged"] and st["stop"] == "nonfinite", st
    # the same plan solves finite loads again with clean statistics
    f[1, 77] = 0.0
    p.solve(torch.from_numpy(f).cuda())
    assert p.stats()["converged"]


@pytest.mark.parametrize("K", [1 << 16, 60695])
def test_long_coefficients_synthesize_apply(fm, K):
    """The other entry points on a long-line plan: expansion coefficients of
    loads are the forward transform, synthesis the inverse, coefficients of
    synthesized values return the coefficients (Theorem 2, item 3), and the
    operator apply matches the oracle's element-wise operator."""
    from oracle import solve as osolve
    n, diff, react = N5, 1.3, 0.4
    say("long coefficients", n, K)
    p = plan(fm, K, diff, react, 2.0, nrhs=2)
    y = inputs.draw_rhs([2, n * K - 1], 1902, "normal")
    yt = torch.from_numpy(y).cuda()
    c = p.coefficients(yt, kind="loads")
    assert torch.equal(c, p.debug_transform(0, +1, yt))
    w = p.synthesize(c)
    assert torch.equal(w, p.debug_transform(0, -1, c))
    c2 = p.coefficients(w, kind="values")
    assert (torch.linalg.norm(c2 - c) / torch.linalg.norm(c)).item() < 1e-12
    Au = p.apply_A(yt).cpu().numpy()
    for r in range(2):
        ref = osolve.apply_A(y[r], n, (K,), (diff,), react, X=(2.0,))
        assert np.linalg.norm(Au[r] - ref) / np.linalg.norm(ref) < 1e-13, r


def refined_sparse_solve(n, K, diff, react, f):
    """The oracle-assembled system solved by sparse LU and refined with the
    oracle's extended-precision element-wise residual."""
    import scipy.sparse.linalg as spla
    from oracle import solve as osolve
    A, C = fem1d.assemble(n, K, dense=False)
    lu = spla.splu((diff * 4.0 * K * K * A + react * C).tocsc())
    ref = lu.solve(f)
    for _ in range(3):
        r = f - osolve.apply_A(ref, n, (K,), (diff,), react, extended=True)
        ref = ref + lu.solve(r.astype(np.float64))
    return ref


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 7, 8, 9])
@pytest.mark.parametrize("K", [1 << 11, 1537])
def test_long_other_orders(fm, n, K):
    """Every element order of the long-line kernels (n = 1 has no bubbles;
    even n an unpaired last bubble channel), a power of two and an odd K:
    the round trip against the oracle's mass operator and the solve of a
    random load against the refined sparse solve."""
    say("long orders", n, K)
    p = fm.Plan((K,), n, (1.0,), 0.3, nrhs=1)
    y = inputs.draw_rhs([n * K - 1], 1910 + n, "normal")
    yt = torch.from_numpy(y).cuda()
    back = p.debug_transform(0, -1, p.debug_transform(0, +1, yt)).cpu().numpy()
    _, C = element_matrices(n)
    assert np.linalg.norm(fem1d.apply_elementwise(C, back, 0) - y) / np.linalg.norm(y) < 1e-12
    u = p.solve(yt).cpu().numpy()
    ref = refined_sparse_solve(n, K, 1.0, 0.3, y)
    # the reference's own accuracy: its extended-precision residual (2^-64)
    # loses the stiffness cancellation factor of about (nK)^2
    tol = max(1e-11, 2.0 ** -62 * (n * K) ** 2)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < tol


# --- two axes, both longer than a tile (axis 1 directly, axis 0 through the
# transposed array) ---------------------------------------------------------

_plans2 = {}


def plan2(fm, K, n, diff=(1.0, 1.0), react=0.0, X=(1.0, 1.0), nrhs=1):
    key = (K, n, diff, react, X, nrhs)
    if key not in _plans2:
        say("plan 2d", key)
        _plans2[key] = fm.Plan(K, n, diff, react, X=X, nrhs=nrhs)
    return _plans2[key]


def test_long2d_solve_sine(fm):
    """-div(diff grad u) + react u = f on (0, 1) x (0, 2) with
    u = sin(pi x) sin(2 pi y / 2): the load is the product of the oracle's 1D
    element-by-element loads (the tensor Gauss rule factorizes), times the
    eigenvalue lam; the FEM error of order h^6 is far below rounding."""
    K, n, diff, react, X = (1100, 1030), 5, (1.0, 0.6), 0.5, (1.0, 2.0)
    say("long 2d sine", K, n)
    p = plan2(fm, K, n, diff, react, X)
    m = (1, 2)
    lam = sum(d * (mm * np.pi / x) ** 2 for d, mm, x in zip(diff, m, X)) + react
    l0 = loads.load_vector_1d(lambda x: np.sin(m[0] * np.pi * x / X[0]), n, K[0], X=X[0])
    l1 = loads.load_vector_1d(lambda y: np.sin(m[1] * np.pi * y / X[1]), n, K[1], X=X[1])
    f = lam * np.outer(l0, l1)
    ue, _ = loads.sin_product(m, diff, react, X=list(X))
    want = loads.interpolate(ue, n, K, X=list(X))
    u = p.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.abs(u - want).max() < 1e-11
    assert p.stats()["converged"]


def test_long2d_transforms_and_apply(fm):
    """Expansion coefficients of loads are the forward transforms along axis
    1 then axis 0 (same kernels, bit for bit); synthesis inverts the
    coefficients of values (Theorem 2, item 3); the operator apply matches
    the oracle's element-wise operator; two right-hand sides."""
    from oracle import solve as osolve
    K, n, diff, react = (1100, 1030), 2, (1.0, 1.3), 0.4
    say("long 2d transforms", K, n)
    p = plan2(fm, K, n, diff, react, nrhs=2)
    y = inputs.draw_rhs(list(p.shape), 1920, "normal", nrhs=2)
    yt = torch.from_numpy(y).cuda()
    c = p.coefficients(yt, kind="loads")
    c2 = p.debug_transform(0, +1, p.debug_transform(1, +1, yt))
    assert torch.equal(c, c2)
    w = p.synthesize(c)
    back = p.coefficients(w, kind="values")
    assert (torch.linalg.norm(back - c) / torch.linalg.norm(c)).item() < 1e-12
    Au = p.apply_A(yt).cpu().numpy()
    for r in range(2):
        ref = osolve.apply_A(y[r], n, K, diff, react)
        assert np.linalg.norm(Au[r] - ref) / np.linalg.norm(ref) < 1e-13, r
    # A u = f for the solve of a smooth u's load: the solve inverts the apply
    xs = [np.linspace(0, 1, m + 2)[1:-1] for m in p.shape]
    u0 = np.outer(np.sin(np.pi * xs[0]) * (1 + xs[0]), np.sin(3 * np.pi * xs[1]))
    f0 = osolve.apply_A(u0, n, K, diff, react, extended=True).astype(np.float64)
    p1 = plan2(fm, K, n, diff, react)
    u = p1.solve(torch.from_numpy(np.ascontiguousarray(f0)).cuda()).cpu().numpy()
    assert np.linalg.norm(u - u0) / np.linalg.norm(u0) < 1e-10


def test_long2d_reports_nonfinite(fm):
    K, n = (1100, 1030), 2
    say("long 2d nan", K, n)
    p = plan2(fm, K, n, nrhs=2)
    f = inputs.draw_rhs(list(p.shape), 1921, "normal", nrhs=2)
    f[1, 5, 7] = np.nan
    u = p.solve(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    assert np.isfinite(u[0].cpu().numpy()).all()
    st = p.stats()
    assert not st["converged"] and st["stop"] == "nonfinite", st
    f[1, 5, 7] = 0.0
    p.solve(torch.from_numpy(f).cuda())
    assert p.stats()["converged"]


@pytest.mark.parametrize("K,n,nrhs,chunk", [((2308,), 5, 3, 2), ((1100, 1030), 3, 2, 333)])
def test_long_chunked_lines_match_whole(fm, monkeypatch, K, n, nrhs, chunk):
    """Work arrays smaller than an axis' lines (FFTFEM_LONG_CHUNK lines per
    pass, the last chunk ragged) give the same solve, coefficients and
    synthesis bit for bit (the kernels see the same lines in the same order),
    and still report a NaN in one right-hand side."""
    say("long chunked", K, n, nrhs, chunk)
    N = len(K)
    whole = fm.Plan(K, n, (1.0,) * N, 0.3, nrhs=nrhs)
    monkeypatch.setenv("FFTFEM_LONG_CHUNK", str(chunk))
    part = fm.Plan(K, n, (1.0,) * N, 0.3, nrhs=nrhs)
    monkeypatch.delenv("FFTFEM_LONG_CHUNK")
    assert part.workspace_bytes() < whole.workspace_bytes()
    f = inputs.draw_rhs(list(whole.shape), 1930 + N, "normal", nrhs=nrhs)
    ft = torch.from_numpy(f).cuda()
    assert torch.equal(part.solve(ft), whole.solve(ft))
    c = whole.coefficients(ft, kind="loads")
    assert torch.equal(part.coefficients(ft, kind="loads"), c)
    assert torch.equal(part.synthesize(c), whole.synthesize(c))
    f[nrhs - 1].flat[77] = np.nan
    u = part.solve(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    assert np.isfinite(u[0].cpu().numpy()).all()
    assert part.stats()["stop"] == "nonfinite"


def test_long2d_solve_sine_fills_hbm(fm):
    """The largest two-axis case that fits one MI355X: n = 9, K = 11000 per
    axis, 9.8e9 unknowns (78.4 GB per float64 array; f, u and the plan's
    transposed copy take 235 GB, the work arrays 16 GB in chunks of lines).
    u = sin(pi x) sin(pi y) on the unit square: the load is lam times the
    outer product of the oracle's 1D loads, the expected values the outer
    product of the 1D interpolants (FEM error of order h^10, far below
    rounding); compared in blocks of rows on the device."""
    import gc
    K, n = 11000, 9
    say("long 2d fills hbm", K, n)
    gc.collect()  # plans of earlier tests that nothing references any more
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < 256 * 2 ** 30:
        pytest.skip(f"needs about 252 GB of free device memory, {free / 2 ** 30:.0f} GiB free of {total / 2 ** 30:.0f}")
    lam = 2 * np.pi ** 2
    l1 = loads.load_vector_1d(lambda x: np.sin(np.pi * x), n, K)
    i1 = loads.interpolate(lambda x: np.sin(np.pi * x), n, (K,))
    p = fm.Plan((K, K), n, (1.0, 1.0), 0.0)
    lt = torch.from_numpy(l1).cuda()
    it = torch.from_numpy(np.ascontiguousarray(i1)).cuda()
    f = torch.outer(lt * lam, lt)
    u = p.solve(f)
    del f
    torch.cuda.synchronize()
    st = p.stats()
    assert st["converged"] and st["stop"] == "none", st
    M = u.shape[0]
    err = 0.0
    for r0 in range(0, M, 4096):
        r1 = min(M, r0 + 4096)
        err = max(err, (u[r0:r1] - torch.outer(it[r0:r1], it)).abs().max().item())
    say("long 2d fills hbm: max error", err)
    assert err < 1e-11
    del u, p
    torch.cuda.empty_cache()


@pytest.mark.parametrize("K,n", [((1030, 20), 2), ((24, 1100), 3), ((1025, 12), (3, 2))])
def test_long2d_one_long_axis(fm, K, n):
    """Two axes of which only one is longer than a tile: the multi-pass
    transforms on that axis, the LDS line passes on the other (axis 0 on the
    transposed copy, with the axis-1 denominators per line).  Solves of two
    random loads against the oracle's eigen solve, expansion coefficients and
    synthesis (Theorem 2), the operator apply (one order: the fused pass;
    two orders: the two-pass form) and NaN reporting."""
    from oracle import solve as osolve
    say("long 2d one long axis", K, n)
    diff, react = (1.0, 0.7), 0.3
    p = fm.Plan(K, n, diff, react, nrhs=2)
    f = inputs.draw_rhs(list(p.shape), 1940 + K[0] + K[1], "normal", nrhs=2)
    ft = torch.from_numpy(f).cuda()
    u = p.solve(ft).cpu().numpy()
    want = osolve.solve(f, n, K, diff, react)
    for r in range(2):
        assert np.linalg.norm(u[r] - want[r]) / np.linalg.norm(want[r]) < 1e-11, r
    assert p.stats()["converged"]
    c = p.coefficients(ft, kind="loads")
    assert torch.equal(c, p.debug_transform(0, +1, p.debug_transform(1, +1, ft)))
    w = p.synthesize(c)
    back = p.coefficients(w, kind="values")
    assert (torch.linalg.norm(back - c) / torch.linalg.norm(c)).item() < 1e-12
    Au = p.apply_A(ft).cpu().numpy()
    for r in range(2):
        ref = osolve.apply_A(f[r], n, K, diff, react)
        assert np.linalg.norm(Au[r] - ref) / np.linalg.norm(ref) < 1e-13, r
    f[1, 3, 5] = np.nan
    u = p.solve(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    assert np.isfinite(u[0].cpu().numpy()).all()
    assert p.stats()["stop"] == "nonfinite"
