"""Pins of the oracle's non-homogeneous Dirichlet reduction (Sect. 4 remark:
a modified load): polynomials of the FEM space with non-zero boundary values
are reproduced exactly, zero boundary data leave the load unchanged, and the
reduction agrees with a dense solve of the interior rows of the full
extended system."""
import numpy as np
import pytest

from oracle import dirichlet, loads, solve
from oracle.fem1d import dof_positions


def ext_grid(n, K):
    return [np.arange(m * k + 1) / (m * k) for m, k in zip(n, K)]


def poly_case(N):
    """u* of degree <= 3 per variable, non-zero on the boundary, and
    f = -sum_d diff_d u*_{x_d x_d} + react u*."""
    cs = [(1.0, 1.0, 2.0, 0.0), (3.0, -1.0, 0.0, 1.0), (0.5, 2.0, -1.0, 1.5)][:N]
    P = [np.polynomial.Polynomial(c) for c in cs]
    diff = (1.0, 0.5, 2.0)[:N]
    react = 2.0

    def u(*xs):
        out = 1.0
        for p, x in zip(P, xs):
            out = out * p(x)
        return out

    def f(*xs):
        tot = react * u(*xs)
        for d in range(N):
            term = -diff[d] * P[d].deriv(2)(xs[d])
            for e in range(N):
                if e != d:
                    term = term * P[e](xs[e])
            tot = tot + term
        return tot

    return u, f, diff, react


@pytest.mark.parametrize("N,n,K", [(1, 3, (4,)), (1, 1, (5,)), (2, 3, (3, 4)), (2, (4, 3), (2, 3)),
                                   (3, 3, (2, 3, 2))])
def test_polynomial_reproduced(N, n, K):
    """u* in the FEM space (degree <= n per variable; n = 1 with a linear u*)
    is the discrete solution: the Gauss load integrates f phi exactly."""
    ns = solve.orders(n, N)
    u, f, diff, react = poly_case(N)
    if min(ns) == 1:
        def u(*xs):  # noqa: F811 - linear in every variable for n = 1
            out = 1.0
            for a, x in zip((2.0, -1.0, 0.5), xs):
                out = out * (1.0 + a * x)
            return out
        react = 0.0

        def f(*xs):  # noqa: F811
            return 0.0 * xs[0]
    fh = loads.load_vector(f, max(ns), K) if len(set(ns)) == 1 else None
    if fh is None:
        # per-axis orders: the tensor load built axis by axis
        mats, grids = [], []
        for m, k in zip(ns, K):
            B, xq = loads.quad_matrix(m, k)
            mats.append(B)
            grids.append(xq)
        F = f(*np.meshgrid(*grids, indexing="ij"))
        for d, B in enumerate(mats):
            F = solve.mode_product(B, F, d)
        fh = F
    b = u(*np.meshgrid(*ext_grid(ns, K), indexing="ij"))
    got = dirichlet.solve_dirichlet(b, fh, ns, K, diff, react)
    assert np.abs(got - b).max() <= 1e-11 * np.abs(b).max()


def test_zero_boundary_keeps_the_load():
    n, K = 3, (3, 4)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((n * K[0] + 1, n * K[1] + 1))
    b[0, :] = b[-1, :] = 0.0
    b[:, 0] = b[:, -1] = 0.0
    f = rng.standard_normal((n * K[0] - 1, n * K[1] - 1))
    assert np.array_equal(dirichlet.lifted_load(b, f, n, K, (1.0, 2.0), 0.5), f)


def test_matches_dense_extended_system():
    """Interior rows of the full Kronecker-assembled extended matrix, solved
    densely with the boundary values moved to the right-hand side."""
    n, K, diff, react = 2, (3, 2), (1.0, 0.7), 1.5
    rng = np.random.default_rng(6)
    E = [n * k + 1 for k in K]
    b = rng.standard_normal(E)
    f = rng.standard_normal([e - 2 for e in E])
    coef = solve.coefficients(K, diff)
    (A0, C0), (A1, C1) = [dirichlet.assemble_ext(n, k) for k in K]
    Afull = coef[0] * np.kron(A0, C1) + coef[1] * np.kron(C0, A1) + react * np.kron(C0, C1)
    inner = np.zeros(E, dtype=bool)
    inner[1:-1, 1:-1] = True
    I = inner.ravel()
    rhs = f.ravel() - Afull[np.ix_(I, ~I)] @ b.ravel()[~I]
    uI = np.linalg.solve(Afull[np.ix_(I, I)], rhs)
    got = dirichlet.solve_dirichlet(b, f, n, K, diff, react)
    assert np.allclose(got[1:-1, 1:-1].ravel(), uI, rtol=1e-11, atol=1e-12)
    assert np.array_equal(got[~inner], b[~inner])
