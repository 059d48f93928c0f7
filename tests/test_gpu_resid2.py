"""The fused 2D operator pass (one kernel over both axes) and the fused
plane pass of the 3D operator (axes 1 and 2 in one kernel, then the axis-0
pass) against the oracle: the double-double apply y = A u within about one float64 ulp per
entry of the oracle's extended-precision (or exact rational) apply, for
every element order, chunkings of axis 0 that leave partial chunks, column
counts that are not multiples of the 64-column tile, tiny meshes and a
non-zero reaction; the same values as the two-pass apply
(FFTFEM_RESID2=0) to that accuracy; and float32 + refinement solves (whose
first residual is the double-double pass and later ones the plain float64
pass r - A c) against the oracle's solve at 1e-10."""
import numpy as np
import pytest

from oracle import fem1d, solve as osolve
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


def smooth(n, K):
    u = np.ones(())
    for d, k in enumerate(K):
        x = fem1d.dof_positions(n, k)
        u = np.multiply.outer(u, np.sin((d + 1) * np.pi * x))
    return u


CASES = [
    (1, (8, 40), (1.0, 1.0), 0.0),
    (2, (2, 2), (1.0, 1.0), 0.0),
    (2, (33, 70), (1.0, 2.0), 0.5),
    (3, (17, 29), (0.5, 1.0), 10.0),
    (4, (40, 16), (1.0, 0.25), 0.0),
    (5, (9, 13), (1.0, 1.0), 1.0),
    (6, (21, 11), (2.0, 1.0), 0.0),
    (7, (5, 19), (1.0, 3.0), 100.0),
    (8, (12, 8), (1.0, 1.0), 0.0),
    (9, (64, 32), (1.0, 1.0), 0.0),
    (9, (3, 7), (1.0, 0.5), 2.0),
]


@pytest.mark.parametrize("kind", ["smooth", "normal"])
@pytest.mark.parametrize("n,K,diff,react", CASES)
def test_fused_apply_vs_oracle(fm, monkeypatch, n, K, diff, react, kind):
    say("fused apply", n, K, diff, react, kind)
    shape = [n * k - 1 for k in K]
    u = smooth(n, K) if kind == "smooth" else inputs.draw_rhs(shape, 2100 + n, "normal")
    # reference: the oracle's exact rational apply (meshes up to 20000
    # dofs), else its x87 extended apply, whose own error (up to ~2^-64 per
    # operation times the partial sums, over the ~(n+1)^2 products of each
    # entry, measured 9e-10 on terms of ~5e6) exceeds one float64 ulp where
    # the terms cancel: bounded then by 2^-56 (n+1)^2 times a bound on the
    # terms' size
    p = fm.Plan(K, n, diff, react)
    y = p.apply_A(torch.from_numpy(np.ascontiguousarray(u)).cuda()).cpu().numpy()
    if u.size <= 20000:
        y_ref = osolve.apply_A_exact(u, n, K, diff, react)
        tol_abs = 1e-24 * float(np.abs(y_ref).max())
    else:
        y_ref = osolve.apply_A(u, n, K, diff, react, extended=True).astype(np.float64)
        coef = osolve.coefficients(K, diff)
        terms = float(np.abs(u).max()) * (n + 1) ** 2 * (sum(coef) * 4 + abs(react))
        tol_abs = 2.0 ** -56 * (n + 1) ** 2 * terms
    err = np.abs(y - y_ref)
    bound = 2.3e-16 * np.abs(y_ref) + tol_abs
    assert np.all(err <= bound), float((err / (np.abs(y_ref) + 1e-300)).max())
    # the two-pass double-double apply: both within about half an ulp of the
    # exact value
    monkeypatch.setenv("FFTFEM_RESID2", "0")
    y2 = p.apply_A(torch.from_numpy(np.ascontiguousarray(u)).cuda()).cpu().numpy()
    d = np.abs(y - y2)
    assert np.all(d <= 4.5e-16 * np.abs(y2) + 1e-22 * float(np.abs(y2).max())), float(d.max())


@pytest.mark.parametrize("n,K,kind", [(9, (8, 16), "smooth"), (4, (16, 12), "normal")])
def test_fused_apply_exact(fm, n, K, kind):
    """Against exact rational arithmetic (small meshes)."""
    say("fused apply exact", n, K, kind)
    diff, react = (1.0, 0.75), 0.5
    shape = [n * k - 1 for k in K]
    u = smooth(n, K) if kind == "smooth" else inputs.draw_rhs(shape, 2200 + n, "normal")
    y_ex = osolve.apply_A_exact(u, n, K, diff, react)
    y = fm.Plan(K, n, diff, react).apply_A(torch.from_numpy(np.ascontiguousarray(u)).cuda()).cpu().numpy()
    err = np.abs(y - y_ex)
    assert np.all(err <= 2.3e-16 * np.abs(y_ex) + 1e-24 * np.abs(y_ex).max())


@pytest.mark.parametrize("n,K,diff,react,kind", [
    (9, (256, 128), (1.0, 1.0), 0.0, "uniform"),
    (4, (100, 52), (1.0, 0.25), 0.0, "normal"),
    (3, (33, 70), (2.0, 1.0), 1000.0, "normal"),
    (1, (64, 200), (1.0, 1.0), 0.0, "uniform"),
])
def test_refine_with_fused_residuals(fm, monkeypatch, n, K, diff, react, kind):
    say("refine fused", n, K, diff, react, kind)
    f = inputs.draw_rhs([n * k - 1 for k in K], 2300 + n, kind)
    u_ref = osolve.solve(f, n, K, diff, react)
    fd = torch.from_numpy(f).cuda()
    p = fm.Plan(K, n, diff, react, precision="fp32_refine", max_iter=6, tol=1e-13)
    u = p.solve(fd).cpu().numpy()
    st = p.stats()
    say("  ", st)
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-10
    monkeypatch.setenv("FFTFEM_RESID2", "0")
    u2 = p.solve(fd).cpu().numpy()
    st2 = p.stats()
    say("  two-pass", st2)
    assert np.linalg.norm(u2 - u_ref) / np.linalg.norm(u_ref) < 1e-10


CASES3 = [
    (2, (3, 8, 12), (1.0, 2.0, 0.5), 0.0),
    (3, (4, 5, 7), (0.5, 1.0, 2.0), 3.0),
    ((2, 4, 4), (5, 6, 3), (1.0, 1.0, 1.0), 0.0),
    (9, (2, 3, 2), (1.0, 0.5, 2.0), 1.0),
    (5, (3, 4, 9), (1.0, 1.0, 1.0), 100.0),
]


@pytest.mark.parametrize("kind", ["smooth", "normal"])
@pytest.mark.parametrize("n,K,diff,react", CASES3)
def test_fused3d_apply_exact(fm, monkeypatch, n, K, diff, react, kind):
    """3D operator apply with the plane pass: every entry within about one
    ulp of exact rational arithmetic, and equal to the three-pass apply to
    that accuracy (axis 0 may have another order than axes 1 and 2)."""
    say("fused 3D apply", n, K, diff, react, kind)
    ns = osolve.orders(n, 3)
    shape = [m * k - 1 for m, k in zip(ns, K)]
    if kind == "smooth":
        u = np.ones(())
        for d, (m, k) in enumerate(zip(ns, K)):
            x = fem1d.dof_positions(m, k)
            u = np.multiply.outer(u, np.sin((d + 1) * np.pi * x))
    else:
        u = inputs.draw_rhs(shape, 2400 + sum(ns), "normal")
    y_ex = osolve.apply_A_exact(u, ns, K, diff, react)
    p = fm.Plan(K, n, diff, react)
    ud = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    y = p.apply_A(ud).cpu().numpy()
    err = np.abs(y - y_ex)
    assert np.all(err <= 2.3e-16 * np.abs(y_ex) + 1e-24 * np.abs(y_ex).max()), \
        float((err / (np.abs(y_ex) + 1e-300)).max())
    monkeypatch.setenv("FFTFEM_RESID2", "0")
    y2 = p.apply_A(ud).cpu().numpy()
    d = np.abs(y - y2)
    assert np.all(d <= 4.5e-16 * np.abs(y2) + 1e-22 * float(np.abs(y2).max())), float(d.max())


@pytest.mark.parametrize("n,K,diff,react,kind", [
    (9, (8, 12, 16), (1.0, 2.0, 0.5), 0.0, "normal"),
    (3, (20, 17, 33), (1.0, 1.0, 1.0), 0.0, "uniform"),
    ((4, 2, 2), (16, 40, 24), (1.0, 0.5, 2.0), 1000.0, "normal"),
])
def test_refine_3d_with_fused_residuals(fm, monkeypatch, n, K, diff, react, kind):
    say("refine fused 3D", n, K, diff, react, kind)
    ns = osolve.orders(n, 3)
    f = inputs.draw_rhs([m * k - 1 for m, k in zip(ns, K)], 2500 + sum(ns), kind)
    u_ref = osolve.solve(f, n, K, diff, react)
    fd = torch.from_numpy(f).cuda()
    p = fm.Plan(K, n, diff, react, precision="fp32_refine", max_iter=6, tol=1e-13)
    u = p.solve(fd).cpu().numpy()
    say("  ", p.stats())
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-10
    monkeypatch.setenv("FFTFEM_RESID2", "0")
    u2 = p.solve(fd).cpu().numpy()
    assert np.linalg.norm(u2 - u_ref) / np.linalg.norm(u_ref) < 1e-10
