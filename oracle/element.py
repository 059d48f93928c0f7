"""Reference-element matrices, computed exactly.  (Test infrastructure only.)

Sect. 2 of the paper: on sigma_0 = [-1, 1] take the Lagrange basis
{e_l}_{l=0..n} of P_n with e_l(-1 + 2k/n) = delta_kl (equispaced nodes), and

    A_kl = int e_k'(x) e_l'(x) dx,      C_kl = int e_k(x) e_l(x) dx.

Everything here is exact rational arithmetic (``fractions.Fraction``); a
float64 copy is rounded once at the end.  The 3x3 block split of A and C
(corner scalars, border vectors, interior (n-1)x(n-1) blocks) and the flip P
with its even/odd subspaces are the paper's, in the notation A00, A0n, a, A~.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from typing import List, Tuple

import numpy as np

Poly = List[Fraction]  # coefficients, lowest degree first


def _pmul(p: Poly, q: Poly) -> Poly:
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        if a:
            for j, b in enumerate(q):
                out[i + j] += a * b
    return out


def _pderiv(p: Poly) -> Poly:
    if len(p) == 1:
        return [Fraction(0)]
    return [Fraction(i) * p[i] for i in range(1, len(p))]


def _pint_sym(p: Poly) -> Fraction:
    """Exact integral of a polynomial over [-1, 1]."""
    s = Fraction(0)
    for i, a in enumerate(p):
        if i % 2 == 0:
            s += a * Fraction(2, i + 1)
    return s


def lagrange_basis(n: int) -> List[Poly]:
    """e_l, l = 0..n, with e_l(-1 + 2k/n) = delta_kl."""
    nodes = [Fraction(-1) + Fraction(2 * k, n) for k in range(n + 1)]
    basis = []
    for l in range(n + 1):
        p: Poly = [Fraction(1)]
        for m in range(n + 1):
            if m != l:
                d = nodes[l] - nodes[m]
                p = _pmul(p, [-nodes[m] / d, Fraction(1) / d])
        basis.append(p)
    return basis


@lru_cache(maxsize=None)
def element_matrices_exact(n: int) -> Tuple[Tuple[Tuple[Fraction, ...], ...], Tuple[Tuple[Fraction, ...], ...]]:
    """(A, C) on [-1, 1] as exact rationals, (n+1) x (n+1)."""
    if n < 1:
        raise ValueError("n >= 1 required")
    e = lagrange_basis(n)
    de = [_pderiv(p) for p in e]
    A = tuple(tuple(_pint_sym(_pmul(de[k], de[l])) for l in range(n + 1)) for k in range(n + 1))
    C = tuple(tuple(_pint_sym(_pmul(e[k], e[l])) for l in range(n + 1)) for k in range(n + 1))
    return A, C


def element_matrices(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """(A, C) rounded once to float64."""
    A, C = element_matrices_exact(n)
    return (np.array([[float(x) for x in r] for r in A]),
            np.array([[float(x) for x in r] for r in C]))


def element_matrices_ld(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """(A, C) rounded once from the exact rationals to x87 extended precision
    (np.longdouble, 64-bit mantissa), for extended-precision residuals."""
    import mpmath as mp

    A, C = element_matrices_exact(n)

    def conv(x: Fraction):
        with mp.workdps(40):
            return np.longdouble(mp.nstr(mp.mpf(x.numerator) / x.denominator, 30))

    return (np.array([[conv(x) for x in r] for r in A], dtype=np.longdouble),
            np.array([[conv(x) for x in r] for r in C], dtype=np.longdouble))


def blocks(X: np.ndarray):
    """The 3x3 block form of Sect. 2: corner X00, X0n, border x, interior X~.

    x = (X_{l0})_{l=1..n-1}; by bisymmetry X_nn = X00 and the right border is
    the flip of x.
    """
    n = X.shape[0] - 1
    return X[0, 0], X[0, n], X[1:n, 0].copy(), X[1:n, 1:n].copy()


def flip(n: int) -> np.ndarray:
    """P with (Pp)_l = p_{n-l}, l = 1..n-1 (Sect. 2)."""
    return np.fliplr(np.eye(n - 1))


def bubble_eigen(n: int):
    """Eigenpairs of A~ e = lambda C~ e (the interior element problem, Sect. 2).

    Returns (lam0 ascending, E) with E[:, l] = e^(l), scaled C~ e . e = 1 and
    the sign fixed so that the largest-magnitude component is positive.
    """
    import scipy.linalg

    A, C = element_matrices(n)
    _, _, _, At = blocks(A)
    _, _, _, Ct = blocks(C)
    lam, E = scipy.linalg.eigh(At, Ct)
    for l in range(E.shape[1]):
        i = int(np.argmax(np.abs(E[:, l])))
        if E[i, l] < 0:
            E[:, l] = -E[:, l]
    return lam, E
