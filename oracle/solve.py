"""The N-D problem and its solution by plain definitions (test infrastructure only).

Sect. 4: the FEM system on (0,X_1) x ... x (0,X_N) with homogeneous Dirichlet
conditions is, in the scaled form (generalized here to per-axis diffusion
coefficients diff[d] and a reaction coefficient react),

    ( sum_d diff[d] 4 h_d^{-2} C_1 x..x A_d x..x C_N + react C_1 x..x C_N ) u = f,

h_d = X_d / K_d, with f the FEM average of the load,
f_i = prod_d (2/h_d) int f phi_i.  The operator is symmetric positive
definite whenever every denominator react + sum_d diff[d] 4 h_d^{-2} lam_d is
positive, so u is unique.

``solve`` computes u = A^{-1} f with no fast transforms: per axis the dense
generalized eigendecomposition Acal_d S_d = Ccal_d S_d Lam_d (S_d^T Ccal_d S_d = I,
SciPy/LAPACK), then u = (x S_d) [ ((x S_d^T) f) / (react + sum_d diff[d] 4 h_d^-2 Lam_d) ]
with the Kronecker factors applied as mode products; then float64 iterative
refinement with the residual computed by the element-by-element operator
(``apply_A``) from the exact element matrices in extended precision, because
a dense float64 eigensolver loses relative accuracy on the smallest
eigenvalues at large K and a float64 residual stalls near cond(A) * eps.  ``solve_cholesky`` assembles the full
N-D matrix (tiny meshes only) and solves by Cholesky.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import scipy.linalg

from .element import element_matrices, element_matrices_ld
from .fem1d import apply_elementwise, assemble, dense_eigen


def orders(n, N: int):
    """Per-axis element orders n = (n_1, ..., n_N) (Sect. 4 builds the space
    as a tensor product of 1D spaces of orders n_i); an int means the same
    order on every axis."""
    if isinstance(n, (int, np.integer)):
        return [int(n)] * N
    ns = [int(x) for x in n]
    if len(ns) != N:
        raise ValueError("one element order per axis")
    return ns


def _h(K, X):
    X = [1.0] * len(K) if X is None else list(X)
    return [x / k for x, k in zip(X, K)]


def coefficients(K: Sequence[int], diff: Sequence[float], X=None):
    """diff[d] * 4 / h_d^2 for every axis."""
    return [dd * 4.0 / (h * h) for dd, h in zip(diff, _h(K, X))]


def mode_product(B: np.ndarray, u: np.ndarray, axis: int) -> np.ndarray:
    """Apply the matrix B along ``axis`` of u."""
    return np.moveaxis(np.tensordot(B, u, axes=([1], [axis])), 0, axis)


def apply_A(u: np.ndarray, n, K: Sequence[int], diff: Sequence[float], react: float,
            X=None, extended: bool = False) -> np.ndarray:
    """y = A u, by element-wise 1D operators along each axis.

    float64 by default; with ``extended`` the element matrices and all
    arithmetic are x87 extended precision (np.longdouble) and the result is
    returned in that precision.
    """
    N = len(K)
    if extended:
        mats = [element_matrices_ld(m) for m in orders(n, N)]
        u = u.astype(np.longdouble)
    else:
        mats = [element_matrices(m) for m in orders(n, N)]
    coef = coefficients(K, diff, X)
    y = np.zeros_like(u)
    for d in range(N):
        t = u
        for e in range(N):
            t = apply_elementwise(mats[e][0] if e == d else mats[e][1], t, e)
        y += coef[d] * t
    if react != 0.0:
        t = u
        for e in range(N):
            t = apply_elementwise(mats[e][1], t, e)
        y += react * t
    return y


def apply_A_exact(u: np.ndarray, n, K: Sequence[int], diff: Sequence[float], react: float,
                  X=None) -> np.ndarray:
    """y = A u in exact rational arithmetic, returned correctly rounded to float64.

    The float64 entries of u, diff, react and X are taken at their exact
    binary values; the element matrices are the exact rationals of Sect. 2;
    every product and sum is a Python Fraction.  Slow (object arrays): small
    inputs only.  The reference for float64 results of an operator whose
    stiffness rows cancel by a factor ~(nK)^2 on smooth inputs.
    """
    from fractions import Fraction
    from .element import element_matrices_exact
    N = len(K)
    mats = []
    for m in orders(n, N):
        Ae, Ce = element_matrices_exact(m)
        mats.append((np.array(Ae, dtype=object), np.array(Ce, dtype=object)))
    Xs = [1.0] * N if X is None else list(X)
    coef = [Fraction(diff[d]) * 4 * (Fraction(K[d]) / Fraction(Xs[d])) ** 2 for d in range(N)]
    uq = np.vectorize(Fraction, otypes=[object])(np.asarray(u, dtype=np.float64))
    y = np.zeros(uq.shape, dtype=object)
    for d in range(N):
        t = uq
        for e in range(N):
            t = apply_elementwise(mats[e][0] if e == d else mats[e][1], t, e)
        y = y + coef[d] * t
    if react != 0.0:
        t = uq
        for e in range(N):
            t = apply_elementwise(mats[e][1], t, e)
        y = y + Fraction(react) * t
    return np.vectorize(float, otypes=[np.float64])(y)


class EigenSolver:
    """u = A^{-1} f by per-axis dense eigendecomposition, plus refinement."""

    def __init__(self, n, K: Sequence[int], diff: Sequence[float], react: float, X=None):
        self.n, self.K, self.diff, self.react, self.X = n, tuple(K), tuple(diff), react, X
        cache = {}
        self.lam, self.S = [], []
        for m, k in zip(orders(n, len(self.K)), self.K):
            if (m, k) not in cache:
                cache[(m, k)] = dense_eigen(m, k)
            lam, S = cache[(m, k)]
            self.lam.append(lam)
            self.S.append(S)
        coef = coefficients(self.K, self.diff, X)
        den = np.full([len(l) for l in self.lam], float(react))
        for d, lam in enumerate(self.lam):
            shape = [1] * len(self.K)
            shape[d] = len(lam)
            den = den + (coef[d] * lam).reshape(shape)
        self.den = den

    def apply_inverse(self, f: np.ndarray) -> np.ndarray:
        t = f
        for d, S in enumerate(self.S):
            t = mode_product(S.T, t, d)
        t = t / self.den
        for d, S in enumerate(self.S):
            t = mode_product(S, t, d)
        return t

    def residual(self, f, u):
        """f - A u with the exact element matrices, in extended precision.

        A float64 residual (element matrices rounded to float64, float64
        sums) limits refinement to about cond(A) * eps and also solves a
        slightly different operator; the extended residual converges to the
        float64 rounding of the exact discrete solution.
        """
        r = f.astype(np.longdouble) - apply_A(u, self.n, self.K, self.diff, self.react, self.X,
                                              extended=True)
        return r.astype(np.float64)

    def solve(self, f: np.ndarray, max_refine: int = 6, history=None) -> np.ndarray:
        """Dense-eigen solve, then refinement while the corrections contract."""
        u = self.apply_inverse(f)
        prev = np.inf
        for _ in range(max_refine):
            du = self.apply_inverse(self.residual(f, u))
            ndu = float(np.linalg.norm(du))
            if history is not None:
                history.append(ndu / max(float(np.linalg.norm(u)), 1e-300))
            if not ndu < prev:
                break
            u = u + du
            prev = ndu
            if ndu <= 1e-16 * np.linalg.norm(u):
                break
        return u


def solve(f: np.ndarray, n, K: Sequence[int], diff: Sequence[float], react: float,
          X=None, max_refine: int = 6) -> np.ndarray:
    """u = A^{-1} f (float64, with refinement).  f may carry a leading RHS axis."""
    s = EigenSolver(n, K, diff, react, X)
    if f.ndim == len(K) + 1:
        return np.stack([s.solve(fi, max_refine) for fi in f])
    return s.solve(f, max_refine)


def assemble_full(n, K: Sequence[int], diff: Sequence[float], react: float, X=None):
    """The full N-D matrix via Kronecker products (tiny meshes only)."""
    N = len(K)
    ns = orders(n, N)
    ops = [assemble(m, k) for m, k in zip(ns, K)]
    coef = coefficients(K, diff, X)
    size = int(np.prod([m * k - 1 for m, k in zip(ns, K)]))
    Afull = np.zeros((size, size))
    for d in range(N):
        T = np.ones((1, 1))
        for e in range(N):
            T = np.kron(T, ops[e][0] if e == d else ops[e][1])
        Afull += coef[d] * T
    if react != 0.0:
        T = np.ones((1, 1))
        for e in range(N):
            T = np.kron(T, ops[e][1])
        Afull += react * T
    return Afull


def solve_cholesky(f: np.ndarray, n, K: Sequence[int], diff: Sequence[float], react: float,
                   X=None) -> np.ndarray:
    """u = A^{-1} f by dense Cholesky of the assembled N-D matrix."""
    Afull = assemble_full(n, K, diff, react, X)
    c = scipy.linalg.cho_factor(Afull)
    return scipy.linalg.cho_solve(c, f.reshape(-1)).reshape(f.shape)
