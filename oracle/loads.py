"""Loads and errors for manufactured solutions (test infrastructure only).

Sect. 5: the load f^h is computed with the (n+1)-point Gauss formula in each
coordinate on every element (tensor product), and the error is measured in
the uniform norm over the mesh points of S_K^(n) (nodes and the interior
bubble points, i.e. every degree of freedom).

f^h_i = prod_d (2/h_d) int f phi_i.  On one element the factor 2/h_d cancels
the Jacobian h_d/2 of the map from [-1, 1], so along one axis
f^h_g = sum_{elements e containing g} sum_q w_q f(x_{e,q}) e_{i(g,e)}(xi_q).
"""
from __future__ import annotations

from typing import Callable, Sequence

import numpy as np

from .element import lagrange_basis
from .fem1d import dof_positions
from .solve import mode_product


def _poly_eval(p, x):
    c = np.array([float(a) for a in p])
    return np.polynomial.polynomial.polyval(x, c)


def quad_matrix(n: int, K: int, X: float = 1.0, npts: int = None):
    """(B, xq): B[g, q] maps values at the quadrature points xq to f^h_g."""
    npts = n + 1 if npts is None else npts
    xi, w = np.polynomial.legendre.leggauss(npts)
    basis = lagrange_basis(n)
    vals = np.array([_poly_eval(basis[i], xi) for i in range(n + 1)])  # (n+1, npts)
    h = X / K
    M = n * K - 1
    Q = K * npts
    B = np.zeros((M, Q))
    xq = np.zeros(Q)
    for e in range(1, K + 1):
        x0 = (e - 1) * h
        xq[(e - 1) * npts:e * npts] = x0 + (xi + 1) * h / 2
        for i in range(n + 1):
            g = (e - 1) * n - 1 + i
            if 0 <= g < M:
                B[g, (e - 1) * npts:e * npts] += w * vals[i]
    return B, xq


def load_vector(fun: Callable, n: int, K: Sequence[int], X=None, npts: int = None) -> np.ndarray:
    """f^h for a function f(x_1, ..., x_N) evaluated on the Gauss grid."""
    X = [1.0] * len(K) if X is None else list(X)
    mats, grids = [], []
    for k, x in zip(K, X):
        B, xq = quad_matrix(n, k, x, npts)
        mats.append(B)
        grids.append(xq)
    F = fun(*np.meshgrid(*grids, indexing="ij"))
    for d, B in enumerate(mats):
        F = mode_product(B, F, d)
    return F


def load_vector_1d(fun: Callable, n: int, K: int, X: float = 1.0, npts: int = None) -> np.ndarray:
    """f^h of one axis, element by element (the sum over elements of the
    module docstring written out without the dense M x (K npts) matrix of
    ``quad_matrix``), for long lines."""
    npts = n + 1 if npts is None else npts
    xi, w = np.polynomial.legendre.leggauss(npts)
    basis = lagrange_basis(n)
    vals = np.array([_poly_eval(basis[i], xi) for i in range(n + 1)])  # (n+1, npts)
    h = X / K
    x0 = np.arange(K, dtype=np.float64) * h
    xq = x0[:, None] + (xi[None, :] + 1) * h / 2  # (K, npts)
    local = fun(xq) @ (w[None, :] * vals).T  # (K, n+1): sum_q w_q f(x_eq) e_i(xi_q)
    M = n * K - 1
    out = np.zeros(M + 2)  # slots -1 and M (the boundary nodes) at both ends
    for i in range(n + 1):
        out[i:i + n * K:n] += local[:, i]  # global dof (e - 1) n - 1 + i, shifted by one
    return out[1:M + 1]


def interpolate(fun: Callable, n: int, K: Sequence[int], X=None) -> np.ndarray:
    """Values of f at all dof points (the vector of S_K^(n) of f)."""
    X = [1.0] * len(K) if X is None else list(X)
    grids = [dof_positions(n, k, x) for k, x in zip(K, X)]
    return fun(*np.meshgrid(*grids, indexing="ij"))


def max_error(u: np.ndarray, exact: Callable, n: int, K: Sequence[int], X=None) -> float:
    """Uniform norm of u - exact over all dof points (Sect. 5)."""
    return float(np.abs(u - interpolate(exact, n, K, X)).max())


def l2_error(u: np.ndarray, exact: Callable, n: int, K: Sequence[int], X=None,
             npts: int = None) -> float:
    """Continuous L2 error of the FEM function with coefficients u.

    Evaluated with an npts-point Gauss rule per element per axis (default n+2).
    """
    X = [1.0] * len(K) if X is None else list(X)
    npts = n + 2 if npts is None else npts
    xi, w = np.polynomial.legendre.leggauss(npts)
    basis = lagrange_basis(n)
    vals = np.array([_poly_eval(basis[i], xi) for i in range(n + 1)])
    evals, grids, weights = [], [], []
    for k, x in zip(K, X):
        h = x / k
        M = n * k - 1
        E = np.zeros((k * npts, M))
        xq = np.zeros(k * npts)
        for e in range(1, k + 1):
            xq[(e - 1) * npts:e * npts] = (e - 1) * h + (xi + 1) * h / 2
            for i in range(n + 1):
                g = (e - 1) * n - 1 + i
                if 0 <= g < M:
                    E[(e - 1) * npts:e * npts, g] = vals[i]
        evals.append(E)
        grids.append(xq)
        weights.append(np.tile(w * h / 2, k))
    U = u
    for d, E in enumerate(evals):
        U = mode_product(E, U, d)
    err2 = (U - exact(*np.meshgrid(*grids, indexing="ij"))) ** 2
    for d, wd in enumerate(weights):
        err2 = np.tensordot(wd, err2, axes=([0], [0]))
    return float(np.sqrt(err2))


# --- manufactured solutions of Sect. 5 and of the benchmark workloads -------

def paper_2d():
    """u = sin(2 pi x1) sin(3 pi x2) cosh(sqrt2 x1 - x2) and f = -Lap u + u."""
    import sympy as s
    x1, x2 = s.symbols("x1 x2")
    u = s.sin(2 * s.pi * x1) * s.sin(3 * s.pi * x2) * s.cosh(s.sqrt(2) * x1 - x2)
    f = -s.diff(u, x1, 2) - s.diff(u, x2, 2) + u
    return s.lambdify((x1, x2), u, "numpy"), s.lambdify((x1, x2), f, "numpy")


def paper_3d():
    """u = sin(2pi x1) sin(3pi x2) sin(4pi x3) cosh(sqrt2 x1 - x2 + x3/sqrt3), f = -Lap u + u."""
    import sympy as s
    x1, x2, x3 = s.symbols("x1 x2 x3")
    u = (s.sin(2 * s.pi * x1) * s.sin(3 * s.pi * x2) * s.sin(4 * s.pi * x3)
         * s.cosh(s.sqrt(2) * x1 - x2 + x3 / s.sqrt(3)))
    f = -s.diff(u, x1, 2) - s.diff(u, x2, 2) - s.diff(u, x3, 2) + u
    return s.lambdify((x1, x2, x3), u, "numpy"), s.lambdify((x1, x2, x3), f, "numpy")


def sin_product(freqs: Sequence[int], diff: Sequence[float], react: float = 0.0, X=None):
    """u = prod_d sin(m_d pi x_d / X_d), which vanishes on the boundary of the
    box (0, X_1) x ... x (0, X_N) (Sect. 4), and
    f = -sum_d diff[d] d^2u/dx_d^2 + react u = (sum_d diff[d] (m_d pi / X_d)^2 + react) u."""
    X = [1.0] * len(freqs) if X is None else list(X)
    lam = sum(dd * (m * np.pi / x) ** 2 for dd, m, x in zip(diff, freqs, X)) + react

    def u(*xs):
        out = 1.0
        for m, x, xl in zip(freqs, xs, X):
            out = out * np.sin(m * np.pi * x / xl)
        return out

    def f(*xs):
        return lam * u(*xs)

    return u, f
