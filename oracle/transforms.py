"""Direct FC_n and inverse F_n transforms by definition (test infrastructure only).

Sect. 3 defines, for y, w in S_K^(n):

* the expansion w = sum_{l} w_{0l} s_0^(l) + sum_{k>=1} sum_l w_{kl} s_k^(l)
  (inverse F_n: coefficients -> vector), and
* the expansion y = sum ytilde_{kl} Ccal s_k^(l) with
  ytilde_{kl} = (y, s_k^(l)) / ||s_k^(l)||_C^2   (direct FC_n, Theorem 2).

Here both are evaluated as plain O(M^2) sums against the explicit
eigenvectors of Theorem 1 (``eigen1d``).  Theorem 2's sine/cosine-sum
formulas are also written out (``fc_by_formula``, ``f_inverse_by_formula``)
so that tests can check them against the definitions.

Coefficient order ("spectral layout"): k = 0 with l = 1..n-1, then
k = 1..K-1 with l = 1..n, i.e. index l-1 for k = 0 and n-1+(k-1)n+(l-1)
for k >= 1.  The l's of one k are in ascending eigenvalue order.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

from .eigen1d import all_eigenpairs, element_data, norm_sq_formula, p_vector, secular_roots
from .fem1d import assemble


def basis(n: int, K: int, dps: int = 30):
    """(lam, S, norms2): columns of S are the s_k^(l) in spectral order."""
    pairs = all_eigenpairs(n, K, dps)
    lam = np.array([float(p[0]) for p in pairs])
    S = np.stack([p[1] for p in pairs], axis=1)
    _, C = assemble(n, K)
    norms2 = np.einsum("ij,ik,kj->j", S, C, S)
    return lam, S, norms2


def fc_forward(y: np.ndarray, n: int, K: int, dps: int = 30) -> np.ndarray:
    """ytilde = (y, s)/||s||_C^2 for every eigenvector (Theorem 2, item 2)."""
    _, S, norms2 = basis(n, K, dps)
    return (S.T @ y) / norms2


def f_inverse(w: np.ndarray, n: int, K: int, dps: int = 30) -> np.ndarray:
    """w = sum_{kl} w_kl s_k^(l) (the inverse F_n transform of Sect. 3)."""
    _, S, _ = basis(n, K, dps)
    return S @ w


def _split(n, y):
    """Nodes y_j (j=1..K-1) and bubble vectors y_{j-1/2} (j=1..K) of a line."""
    K = (len(y) + 1) // n
    nodes = np.array([y[j * n - 1] for j in range(1, K)])
    bub = np.array([y[(j - 1) * n:(j - 1) * n + n - 1] for j in range(1, K + 1)])
    return K, nodes, bub


def fc_by_formula(y: np.ndarray, n: int, K: int, dps: int = 30) -> np.ndarray:
    """Theorem 2, item 2, evaluated literally with sine sums.

    (y, s_k^(l)) = sum_j y_j sin(pi k j/K)
                   + p_e . sum_j (y_{j-1/2} + y_{j+1/2})_e sin(pi k j/K)
                   + p_o . sum_j (y_{j+1/2} - y_{j-1/2})_o sin(pi k j/K),
    and for k = 0: ((sum_j (-P)^{j-1} y_{j-1/2}) . e^(l)) / K.
    """
    K_, nodes, bub = _split(n, y)
    assert K_ == K
    d = element_data(n, dps)
    out = []
    # k = 0
    acc = np.zeros(n - 1)
    for j in range(1, K + 1):
        v = bub[j - 1].copy()
        for _ in range(j - 1):
            v = -v[::-1]
        acc += v
    for l in range(n - 1):
        e = np.array([float(x) for x in d["e"][l]])
        out.append(acc @ e / K)
    for k in range(1, K):
        jj = np.arange(1, K)
        sk = np.sin(np.pi * k * jj / K)
        Yn = nodes @ sk
        plus = bub[:-1] + bub[1:]            # y_{j-1/2} + y_{j+1/2}, j = 1..K-1
        minus = bub[1:] - bub[:-1]           # y_{j+1/2} - y_{j-1/2}
        Zp = sk @ plus
        Zm = sk @ minus
        Zp_e = 0.5 * (Zp + Zp[::-1])
        Zm_o = 0.5 * (Zm - Zm[::-1])
        for l, lam in enumerate(secular_roots(n, K, k, dps)):
            p = np.array([float(x) for x in p_vector(n, lam, dps)])
            p_e = 0.5 * (p + p[::-1])
            p_o = 0.5 * (p - p[::-1])
            num = Yn + p_e @ Zp_e + p_o @ Zm_o
            out.append(num / float(norm_sq_formula(n, K, k, l + 1, dps)))
    return np.array(out)


def f_inverse_by_formula(w: np.ndarray, n: int, K: int, dps: int = 30) -> np.ndarray:
    """Theorem 2, item 1, evaluated literally.

    nodes:   w_j = sum_k (sum_l w_kl) sin(pi k j / K),
    bubbles: w_{j-1/2} = (-P)^{j-1} sum_l w_0l e^(l)
             + 2 sum_k d_{k,e} cos(pi k/2K) sin(pi k (j-1/2)/K)
             - 2 sum_k d_{k,o} sin(pi k/2K) cos(pi k (j-1/2)/K),
    with d_k = sum_l w_kl p_k^(l).
    """
    d = element_data(n, dps)
    M = n * K - 1
    out = np.zeros(M)
    w0 = w[:n - 1]
    wk = w[n - 1:].reshape(K - 1, n)
    e0 = sum(w0[l] * np.array([float(x) for x in d["e"][l]]) for l in range(n - 1)) \
        if n > 1 else np.zeros(0)
    dk = np.zeros((K - 1, n - 1))
    for k in range(1, K):
        for l, lam in enumerate(secular_roots(n, K, k, dps)):
            p = np.array([float(x) for x in p_vector(n, lam, dps)])
            dk[k - 1] += wk[k - 1, l] * p
    de = 0.5 * (dk + dk[:, ::-1])
    do = 0.5 * (dk - dk[:, ::-1])
    ks = np.arange(1, K)
    for j in range(1, K):
        out[j * n - 1] = wk.sum(axis=1) @ np.sin(np.pi * ks * j / K)
    for j in range(1, K + 1):
        v = e0.copy()
        for _ in range(j - 1):
            v = -v[::-1]
        v = v + 2 * (np.cos(np.pi * ks / (2 * K)) * np.sin(np.pi * ks * (j - 0.5) / K)) @ de \
              - 2 * (np.sin(np.pi * ks / (2 * K)) * np.cos(np.pi * ks * (j - 0.5) / K)) @ do
        out[(j - 1) * n:(j - 1) * n + n - 1] = v
    return out
