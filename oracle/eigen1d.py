"""1D FEM eigenpairs in the paper's own form (test infrastructure only).

Sect. 3, Theorem 1: the spectrum of Acal v = lambda Ccal v on S_K^(n) is the
interior element spectrum S~_n (eigenvectors supported on bubbles only) plus,
for every k = 1..K-1, the n roots lambda_k^(l) of the secular equation of
Sect. 3 written with theta_k = cos(pi k / K) and the bubble eigenpairs
(lambda_0^(l), e^(l)) of Sect. 2 (scaled C~ e.e = 1).  The eigenvectors are

    s_0^(l): nodes 0, bubbles (-P)^{j-1} e^(l),
    s_k^(l): nodes sin(pi k j / K), bubbles p sin(pi k (j-1)/K) + (Pp) sin(pi k j/K),

with p = p_k^(l) solving (A~ - lambda C~) p = -(a - lambda c).

Everything is done in mpmath at ``dps`` decimal digits (40 by default), from
the exact rational element matrices, so it serves as a high-precision check
of float64 results.  The roots are found as the roots of the degree-n
polynomial obtained by clearing the denominators of the secular equation.
"""
from __future__ import annotations

from functools import lru_cache
from typing import List, Tuple

import mpmath as mp
import numpy as np

from .element import element_matrices_exact


def _mpmat(X):
    return mp.matrix([[mp.mpf(x.numerator) / x.denominator for x in row] for row in X])


@lru_cache(maxsize=None)
def element_data(n: int, dps: int = 40):
    """Blocks of A, C and the bubble eigenpairs, as mpmath objects.

    Returns a dict with a0, an, a (vector a_l = A_{l0}), ac (right border,
    A_{l n}), At (A~), and the same for C, plus lam0 (ascending) and the
    list of e^(l) vectors (C~ e.e = 1, largest component positive).
    """
    with mp.workdps(dps):
        Ae, Ce = element_matrices_exact(n)
        A, C = _mpmat(Ae), _mpmat(Ce)
        d = {}
        for name, X in (("a", A), ("c", C)):
            d[name + "0"] = X[0, 0]
            d[name + "n"] = X[0, n]
            d[name] = [X[l, 0] for l in range(1, n)]
            d[name + "check"] = [X[l, n] for l in range(1, n)]
            d[name + "T"] = mp.matrix([[X[i, j] for j in range(1, n)] for i in range(1, n)])
        if n >= 2:
            L = mp.cholesky(d["cT"])
            Li = mp.inverse(L)
            H = Li * d["aT"] * Li.T
            H = (H + H.T) / 2
            w, V = mp.eigsy(H)
            order = sorted(range(n - 1), key=lambda i: w[i])
            lam0, evecs = [], []
            for i in order:
                v = Li.T * V[:, i]
                v = v / mp.sqrt((v.T * d["cT"] * v)[0])
                big = max(range(n - 1), key=lambda r: abs(v[r]))
                if v[big] < 0:
                    v = -v
                lam0.append(w[i])
                evecs.append(v)
            d["lam0"] = lam0
            d["e"] = evecs
        else:
            d["lam0"] = []
            d["e"] = []
        return d


def _polymul(p, q):
    out = [mp.mpf(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _polyadd(p, q):
    m = max(len(p), len(q))
    p = p + [mp.mpf(0)] * (m - len(p))
    q = q + [mp.mpf(0)] * (m - len(q))
    return [a + b for a, b in zip(p, q)]


def secular_roots(n: int, K: int, k: int, dps: int = 40) -> List[mp.mpf]:
    """The n roots lambda_k^(l), ascending, of the secular equation of Sect. 3.

    With theta = cos(pi k/K) the equation reads
      a0 - lam c0 + sum_l (a^(l) - lam c^(l))^2 / (lam - lam0^(l))
        = -theta (an - lam cn + sum_l (a^(l)' - lam c^(l)')(a^(l) - lam c^(l)) / (lam - lam0^(l)))
    where a^(l) = a.e^(l) and a^(l)' = (Pa).e^(l).  Multiplying through by
    prod_m (lam - lam0^(m)) gives a polynomial of degree n whose roots are
    returned.
    """
    d = element_data(n, dps)
    with mp.workdps(dps):
        theta = mp.cos(mp.pi * k / K)
        lam0 = d["lam0"]
        e = d["e"]
        av = mp.matrix(d["a"])
        cv = mp.matrix(d["c"])
        avc = mp.matrix(d["acheck"])
        cvc = mp.matrix(d["ccheck"])
        al = [(av.T * el)[0] for el in e]
        cl = [(cv.T * el)[0] for el in e]
        alc = [(avc.T * el)[0] for el in e]
        clc = [(cvc.T * el)[0] for el in e]
        # polynomials in lam, lowest degree first
        full = [mp.mpf(1)]
        for m in lam0:
            full = _polymul(full, [-m, mp.mpf(1)])
        poly = _polymul([d["a0"] + theta * d["an"], -(d["c0"] + theta * d["cn"])], full)
        for l in range(n - 1):
            others = [mp.mpf(1)]
            for m in range(n - 1):
                if m != l:
                    others = _polymul(others, [-lam0[m], mp.mpf(1)])
            num = _polyadd(_polymul([al[l], -cl[l]], [al[l], -cl[l]]),
                           [theta * x for x in _polymul([alc[l], -clc[l]], [al[l], -cl[l]])])
            poly = _polyadd(poly, _polymul(num, others))
        while len(poly) > 1 and abs(poly[-1]) < mp.mpf(10) ** (-dps + 5):
            poly.pop()
        roots = mp.polyroots(list(reversed(poly)), maxsteps=400, extraprec=4 * dps)
        roots = sorted((mp.re(r) for r in roots))
        return roots


def p_vector(n: int, lam, dps: int = 40):
    """p solving (A~ - lam C~) p = -(a - lam c)  (Sect. 3, Theorem 1, item 3)."""
    d = element_data(n, dps)
    with mp.workdps(dps):
        G = d["aT"] - lam * d["cT"]
        g = mp.matrix(d["a"]) - lam * mp.matrix(d["c"])
        return mp.lu_solve(G, -g)


def eigvec(n: int, K: int, k: int, l: int, dps: int = 40) -> Tuple[mp.mpf, np.ndarray]:
    """(lambda, s) for s = s_k^(l) of Theorem 1 in the positional layout.

    k = 0: l = 1..n-1 (bubble-only vectors); k = 1..K-1: l = 1..n.
    The vector is returned in float64; the eigenvalue as mpf.
    """
    d = element_data(n, dps)
    M = n * K - 1
    s = np.zeros(M)
    with mp.workdps(dps):
        if k == 0:
            lam = d["lam0"][l - 1]
            e = d["e"][l - 1]
            for j in range(1, K + 1):
                # (-P)^{j-1} e
                v = [e[i] for i in range(n - 1)]
                for _ in range(j - 1):
                    v = [-v[n - 2 - i] for i in range(n - 1)]
                for i in range(n - 1):
                    s[(j - 1) * n + i] = float(v[i])
            return lam, s
        lam = secular_roots(n, K, k, dps)[l - 1]
        p = p_vector(n, lam, dps)
        for j in range(1, K):
            s[j * n - 1] = float(mp.sin(mp.pi * k * j / K))
        for j in range(1, K + 1):
            a = mp.sin(mp.pi * k * (j - 1) / K)
            b = mp.sin(mp.pi * k * j / K)
            for i in range(n - 1):
                s[(j - 1) * n + i] = float(p[i] * a + p[n - 2 - i] * b)
        return lam, s


def norm_sq_formula(n: int, K: int, k: int, l: int, dps: int = 40):
    """||s_k^(l)||_C^2 by the closed form of Theorem 2, item 2.

    k >= 1: K { c0 + (C~p + 2c).p + theta_k [cn + (C~p + 2c).(Pp)] };
    k = 0:  K.
    """
    if k == 0:
        return mp.mpf(K)
    d = element_data(n, dps)
    with mp.workdps(dps):
        lam = secular_roots(n, K, k, dps)[l - 1]
        p = p_vector(n, lam, dps)
        pc = mp.matrix([p[n - 2 - i] for i in range(n - 1)])
        q = d["cT"] * p + 2 * mp.matrix(d["c"])
        theta = mp.cos(mp.pi * k / K)
        return K * (d["c0"] + (q.T * p)[0] + theta * (d["cn"] + (q.T * pc)[0]))


def all_eigenpairs(n: int, K: int, dps: int = 30):
    """All nK - 1 eigenpairs (lam, s, k, l) of Theorem 1 (small K only)."""
    out = []
    for l in range(1, n):
        lam, s = eigvec(n, K, 0, l, dps)
        out.append((lam, s, 0, l))
    for k in range(1, K):
        roots = secular_roots(n, K, k, dps)
        for l in range(1, n + 1):
            lam, s = eigvec(n, K, k, l, dps)
            out.append((lam, s, k, l))
    return out
