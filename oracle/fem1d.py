"""Global 1D scaled operators (test infrastructure only).

Sect. 2: the scaled stiffness and mass operators of the nth-order FEM on a
uniform mesh of K elements, acting on S_K^(n) (dimension M = nK - 1), are the
sums over elements of the reference matrices A and C placed on the element's
n+1 local degrees of freedom; they do not depend on h, and the true
stiffness/mass differ by the factors 2/h and h/2.

Positional layout: global index g = 0..M-1 is the dof at x = (g+1) h / n.
Element e (1..K) owns the consecutive global positions (e-1)n - 1 + i,
i = 0..n; positions -1 and nK - 1 are the Dirichlet boundary nodes and are
dropped.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from .element import element_matrices


def dof_count(n: int, K: int) -> int:
    return n * K - 1


def assemble(n: int, K: int, dense: bool = True):
    """(Acal, Ccal): the M x M global scaled stiffness and mass operators."""
    A, C = element_matrices(n)
    M = dof_count(n, K)
    rows, cols, va, vc = [], [], [], []
    for e in range(1, K + 1):
        base = (e - 1) * n - 1
        for i in range(n + 1):
            gi = base + i
            if gi < 0 or gi >= M:
                continue
            for j in range(n + 1):
                gj = base + j
                if gj < 0 or gj >= M:
                    continue
                rows.append(gi)
                cols.append(gj)
                va.append(A[i, j])
                vc.append(C[i, j])
    Acal = sp.coo_matrix((va, (rows, cols)), shape=(M, M)).tocsr()
    Ccal = sp.coo_matrix((vc, (rows, cols)), shape=(M, M)).tocsr()
    if dense:
        return Acal.toarray(), Ccal.toarray()
    return Acal, Ccal


def dof_positions(n: int, K: int, X: float = 1.0) -> np.ndarray:
    """Coordinates of the M dofs: x_g = (g + 1) h / n."""
    h = X / K
    return (np.arange(dof_count(n, K)) + 1) * h / n


def is_node(n: int, K: int) -> np.ndarray:
    g = np.arange(dof_count(n, K))
    return (g + 1) % n == 0


def dense_eigen(n: int, K: int):
    """Generalized symmetric eigendecomposition Acal S = Ccal S diag(lam).

    Returns (lam ascending, S) with S^T Ccal S = I (LAPACK sygvd via SciPy).
    The eigenvalues are the scaled ones; the true 1D eigenvalues of -u'' are
    4 h^{-2} lam.
    """
    Acal, Ccal = assemble(n, K)
    lam, S = scipy.linalg.eigh(Acal, Ccal)
    return lam, S


def apply_elementwise(X: np.ndarray, u: np.ndarray, axis: int) -> np.ndarray:
    """y = Xcal u along ``axis`` where Xcal = sum_e P_e^T X P_e.

    Written as the plain element-by-element sum: pad the boundary nodes back
    in, gather each element's n+1 local values, multiply by the element
    matrix, and scatter-add.  Works on arrays of any rank.
    """
    n = X.shape[0] - 1
    u = np.moveaxis(u, axis, -1)
    M = u.shape[-1]
    if (M + 1) % n:
        raise ValueError("axis length must be n*K - 1")
    K = (M + 1) // n
    pad = np.zeros(u.shape[:-1] + (K * n + 1,), dtype=u.dtype)
    pad[..., 1:M + 1] = u
    # local values of element e (0-based): pad[e*n + i], i = 0..n
    loc = np.empty(u.shape[:-1] + (K, n + 1), dtype=u.dtype)
    body = pad[..., :K * n].reshape(u.shape[:-1] + (K, n))
    loc[..., :n] = body
    loc[..., n] = pad[..., n::n]
    yl = loc @ X.T
    ypad = np.zeros_like(pad)
    ypad[..., :K * n] += yl[..., :n].reshape(u.shape[:-1] + (K * n,))
    ypad[..., n::n] += yl[..., n]
    y = ypad[..., 1:M + 1]
    return np.moveaxis(y, -1, axis)
