"""Implicit time stepping of the semi-discrete heat equation by plain
definitions (test infrastructure only: only tests and the benchmark's CPU
baseline use this package).

Sect. 4 remarks that implicit time discretizations of heat-type equations
lead at every time level to a system of the form solved by the method.  With
the scaled FEM operators of Sect. 4 and the mass matrix
C = C_1 x ... x C_N, the implicit Euler method with step tau for

    C du/dt + A_diff u = F,   A_diff = sum_d diff[d] 4 h_d^-2 C_1 x..x A_d x..x C_N,

reads (A_diff + react C) u^{m+1} = F + react C u^m with react = 1/tau: each
step is one mass apply and one solve of the system with reaction react.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import solve as osolve


def mass_apply(u: np.ndarray, n: int, K: Sequence[int], X=None) -> np.ndarray:
    """C u with C = C_1 x ... x C_N (extended precision, rounded to float64)."""
    zero = [0.0] * len(K)
    return np.asarray(osolve.apply_A(u, n, K, zero, 1.0, X, extended=True), dtype=np.float64)


def implicit_euler(u0: np.ndarray, F: Optional[np.ndarray], n: int, K: Sequence[int], diff: Sequence[float],
                   react: float, nsteps: int, X=None) -> np.ndarray:
    """u^nsteps of the implicit Euler steps above from u^0 = u0 (F None: zero load)."""
    if react <= 0:
        raise ValueError("react = 1/tau must be positive")
    u = np.array(u0, dtype=np.float64)
    for _ in range(nsteps):
        rhs = react * mass_apply(u, n, K, X)
        if F is not None:
            rhs = rhs + F
        u = osolve.solve(rhs, n, K, diff, react, X)
    return u
