"""Non-homogeneous Dirichlet data by a modified load (test infrastructure only).

Sect. 4 remarks that u = b on the boundary reduces to the homogeneous
system with f^h modified by an approximation b^h of b.  Written out: with
the dofs of the closed box (every axis extended by its two boundary points,
E_d = n_d K_d + 1 points at x = g h_d / n_d, g = 0 .. E_d - 1), the FEM
equations of the interior dofs read

    A_II u_I + A_IB b_B = f^h,

so u_I solves the homogeneous system with the load f^h - A_IB b_B, where
A_IB b_B is the interior part of the extended operator applied to b with its
interior values set to zero.  The extended operator is the same tensor sum
as in the scaled global system of Sect. 4, built from the 1D scaled stiffness and mass
assembled over all n K + 1 points (no rows or columns dropped).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .element import element_matrices
from .solve import coefficients, mode_product, orders
from . import solve as osolve


def assemble_ext(n: int, K: int):
    """(A, C): the (nK+1) x (nK+1) scaled stiffness and mass over every point
    of [0, X], element e (0-based) owning points e n .. e n + n."""
    Ae, Ce = element_matrices(n)
    E = n * K + 1
    A = np.zeros((E, E))
    C = np.zeros((E, E))
    for e in range(K):
        s = e * n
        A[s:s + n + 1, s:s + n + 1] += Ae
        C[s:s + n + 1, s:s + n + 1] += Ce
    return A, C


def boundary_only(b: np.ndarray) -> np.ndarray:
    """b with every interior value (all indices in 1 .. E_d - 2) set to zero."""
    out = b.copy()
    out[tuple(slice(1, -1) for _ in range(b.ndim))] = 0.0
    return out


def lifted_load(b: np.ndarray, f: np.ndarray, n, K: Sequence[int], diff: Sequence[float], react: float,
                X=None) -> np.ndarray:
    """f^h - A_IB b_B: b on the extended grid (only its boundary values are
    used), f on the interior grid."""
    N = len(K)
    ns = orders(n, N)
    coef = coefficients(K, diff, X)
    mats = [assemble_ext(m, k) for m, k in zip(ns, K)]
    bt = boundary_only(b)
    y = np.zeros_like(f)
    for t in range(N + 1):
        v = bt
        for d in range(N):
            A, C = mats[d]
            v = mode_product((A if d == t else C)[1:-1, :], v, d)
        y = y + (coef[t] if t < N else react) * v
    return f - y


def solve_dirichlet(b: np.ndarray, f: np.ndarray, n, K: Sequence[int], diff: Sequence[float], react: float,
                    X=None) -> np.ndarray:
    """The solution on the extended grid: b on the boundary, the interior
    solved from the lifted load."""
    u = b.copy()
    u[tuple(slice(1, -1) for _ in range(b.ndim))] = osolve.solve(
        lifted_load(b, f, n, K, diff, react, X), n, K, diff, react, X)
    return u
