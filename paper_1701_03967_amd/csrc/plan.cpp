// Host plan builder: the 1D eigenstructure of the nth-order FEM operators.
//
// Sect. 3, Theorem 1 of the paper: the eigenvectors of A v = lambda C v on
// S_K^(n) with k >= 1 have nodal part sin(pi k j / K) and bubble part
// p sin(pi k (j-1)/K) + (Pp) sin(pi k j / K); splitting p into even and odd
// parts (Sect. 2) and using the sum-to-product identity of the proof of
// Theorem 2 turns the bubble part into
//   2 cos(psi) p_e sin(pi k (j-1/2)/K) - 2 sin(psi) p_o cos(pi k (j-1/2)/K),
// psi = pi k / (2K).  Hence, for fixed k, every eigenvector lies in the
// n-dimensional span of the "channel" vectors (nodal sine, even-channel
// sines at element centres, odd-channel cosines at element centres).  This
// module projects A and C onto that span in closed form (the sums over
// elements of products of shifted sines reduce to K/2 times cosines/sines of
// the phase differences), and solves the n x n symmetric-definite pencil
// (Cholesky + cyclic Jacobi) for C-orthonormal eigenvectors.  The k = 0
// (bubble-only) block is the same construction with the alternating and the
// constant patterns of Theorem 1, item 2.
//
// All arithmetic is 113-bit (__float128): at K = 1024, n = 9 the smallest
// eigenvalue (~2.4e-6) shares a pencil with entries ~1e3, and float64 would
// lose about eight digits of it.  Results are rounded to float64 once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "fftfem_internal.h"

namespace fftfem {
namespace {

typedef __float128 q;

const q kPi = 3.14159265358979323846264338327950288Q;

q qabs(q x) { return x < 0 ? -x : x; }

q qsqrt(q x) {
  if (x <= 0) return 0;
  q r = (q)std::sqrt((double)x);
  for (int i = 0; i < 3; ++i) r = (r + x / r) / 2;
  return r;
}

// sin and cos of pi * t for t in [0, 1/4], by Taylor series.
void sincospi_small(q t, q* s, q* c) {
  q x = kPi * t;
  q x2 = x * x;
  q term = x, ss = x;
  for (int k = 1; k < 40; ++k) {
    term *= -x2 / (q)((2 * k) * (2 * k + 1));
    ss += term;
    if (qabs(term) < 1e-40Q) break;
  }
  term = 1;
  q cc = 1;
  for (int k = 1; k < 40; ++k) {
    term *= -x2 / (q)((2 * k - 1) * (2 * k));
    cc += term;
    if (qabs(term) < 1e-40Q) break;
  }
  *s = ss;
  *c = cc;
}

// sin and cos of pi * num / den with exact integer octant reduction.
void sincospi(int64_t num, int64_t den, q* s, q* c) {
  int64_t r = num % (2 * den);
  if (r < 0) r += 2 * den;
  q sgs = 1, sgc = 1;
  if (r >= den) {  // pi + a
    r -= den;
    sgs = -1;
    sgc = -1;
  }
  if (2 * r > den) {  // pi - a
    r = den - r;
    sgc = -sgc;
  }
  q ss, cc;
  if (4 * r > den) {  // pi/2 - a, t = (den - 2r) / (2 den)
    sincospi_small((q)(den - 2 * r) / (q)(2 * den), &cc, &ss);
  } else {
    sincospi_small((q)r / (q)den, &ss, &cc);
  }
  *s = sgs * ss;
  *c = sgc * cc;
}

// Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int m, std::vector<q>* x, std::vector<q>* w) {
  x->resize(m);
  w->resize(m);
  for (int i = 0; i < m; ++i) {
    q z = (q)std::cos(M_PI * (i + 0.75) / (m + 0.5));
    q dp = 1;
    for (int it = 0; it < 100; ++it) {
      q p0 = 1, p1 = z;
      for (int k = 1; k < m; ++k) {
        q p2 = ((2 * k + 1) * z * p1 - k * p0) / (q)(k + 1);
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1);
      q dz = p1 / dp;
      z -= dz;
      if (qabs(dz) < 1e-36Q) break;
    }
    (*x)[i] = z;
    (*w)[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

// Element matrices on [-1, 1] for the Lagrange basis at -1 + 2k/n (Sect. 2),
// integrated exactly by (n+1)-point Gauss-Legendre.
void element_matrices_q(int n, std::vector<q>* A, std::vector<q>* C) {
  std::vector<q> xn(n + 1), xg, wg;
  for (int k = 0; k <= n; ++k) xn[k] = -1 + (q)(2 * k) / (q)n;
  gauss_legendre(n + 1, &xg, &wg);
  int m = n + 1;
  std::vector<q> val((n + 1) * m), der((n + 1) * m);
  for (int l = 0; l <= n; ++l) {
    for (int g = 0; g < m; ++g) {
      q x = xg[g];
      q v = 1;
      for (int j = 0; j <= n; ++j)
        if (j != l) v *= (x - xn[j]) / (xn[l] - xn[j]);
      q d = 0;
      for (int j = 0; j <= n; ++j) {
        if (j == l) continue;
        q t = 1 / (xn[l] - xn[j]);
        for (int p = 0; p <= n; ++p)
          if (p != l && p != j) t *= (x - xn[p]) / (xn[l] - xn[p]);
        d += t;
      }
      val[l * m + g] = v;
      der[l * m + g] = d;
    }
  }
  A->assign((n + 1) * (n + 1), 0);
  C->assign((n + 1) * (n + 1), 0);
  for (int i = 0; i <= n; ++i)
    for (int j = 0; j <= n; ++j) {
      q sa = 0, sc = 0;
      for (int g = 0; g < m; ++g) {
        sa += wg[g] * der[i * m + g] * der[j * m + g];
        sc += wg[g] * val[i * m + g] * val[j * m + g];
      }
      (*A)[i * (n + 1) + j] = sa;
      (*C)[i * (n + 1) + j] = sc;
    }
}

// One term of a channel vector: local index, weight, trig kind, phase.
struct Term {
  int i;
  int w;
  bool is_cos;
  int phase;  // -1, 0, +1 in units of psi
};

std::vector<std::vector<Term>> channel_terms(int n, bool k0) {
  std::vector<std::vector<Term>> b;
  if (!k0) b.push_back({{0, 1, false, -1}, {n, 1, false, +1}});
  for (int m = 1; m <= num_even(n); ++m) {
    if (2 * m == n)
      b.push_back({{m, 1, false, 0}});
    else
      b.push_back({{m, 1, false, 0}, {n - m, 1, false, 0}});
  }
  for (int m = 1; m <= num_odd(n); ++m) b.push_back({{m, 1, true, 0}, {n - m, -1, true, 0}});
  return b;
}

// Symmetric-definite pencil (Ma, Mc) of order r: eigenvalues ascending and
// Mc-orthonormal eigenvectors V (column j = vector j), by Cholesky of Mc and
// cyclic Jacobi on L^{-1} Ma L^{-T}.  Returns false on breakdown.
bool pencil_eigen(int r, std::vector<q> Ma, std::vector<q> Mc, std::vector<q>* lam,
                  std::vector<q>* V) {
  std::vector<q> L(r * r, 0);
  for (int j = 0; j < r; ++j) {
    q s = Mc[j * r + j];
    for (int k = 0; k < j; ++k) s -= L[j * r + k] * L[j * r + k];
    if (!(s > 0)) return false;
    L[j * r + j] = qsqrt(s);
    for (int i = j + 1; i < r; ++i) {
      q t = Mc[i * r + j];
      for (int k = 0; k < j; ++k) t -= L[i * r + k] * L[j * r + k];
      L[i * r + j] = t / L[j * r + j];
    }
  }
  // H = L^{-1} Ma L^{-T}: first T = L^{-1} Ma (forward substitution per column)
  std::vector<q> T(r * r), H(r * r);
  for (int c = 0; c < r; ++c)
    for (int i = 0; i < r; ++i) {
      q s = Ma[i * r + c];
      for (int k = 0; k < i; ++k) s -= L[i * r + k] * T[k * r + c];
      T[i * r + c] = s / L[i * r + i];
    }
  // H = T L^{-T}  <=>  H^T = L^{-1} T^T
  for (int c = 0; c < r; ++c)
    for (int i = 0; i < r; ++i) {
      q s = T[c * r + i];
      for (int k = 0; k < i; ++k) s -= L[i * r + k] * H[c * r + k];
      H[c * r + i] = s / L[i * r + i];
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < i; ++j) {
      q a = (H[i * r + j] + H[j * r + i]) / 2;
      H[i * r + j] = H[j * r + i] = a;
    }
  std::vector<q> W(r * r, 0);
  for (int i = 0; i < r; ++i) W[i * r + i] = 1;
  q norm = 0;
  for (int i = 0; i < r * r; ++i) norm += H[i] * H[i];
  for (int sweep = 0; sweep < 60; ++sweep) {
    q off = 0;
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j)
        if (i != j) off += H[i * r + j] * H[i * r + j];
    if (off <= 1e-66Q * norm) break;
    for (int p = 0; p < r - 1; ++p)
      for (int s = p + 1; s < r; ++s) {
        q apq = H[p * r + s];
        if (apq == 0) continue;
        q app = H[p * r + p], aqq = H[s * r + s];
        q theta = (aqq - app) / (2 * apq);
        q t = (theta >= 0 ? 1 : -1) / (qabs(theta) + qsqrt(theta * theta + 1));
        q c = 1 / qsqrt(t * t + 1), sn = t * c;
        for (int k = 0; k < r; ++k) {
          q hkp = H[k * r + p], hks = H[k * r + s];
          H[k * r + p] = c * hkp - sn * hks;
          H[k * r + s] = sn * hkp + c * hks;
        }
        for (int k = 0; k < r; ++k) {
          q hpk = H[p * r + k], hsk = H[s * r + k];
          H[p * r + k] = c * hpk - sn * hsk;
          H[s * r + k] = sn * hpk + c * hsk;
        }
        for (int k = 0; k < r; ++k) {
          q wkp = W[k * r + p], wks = W[k * r + s];
          W[k * r + p] = c * wkp - sn * wks;
          W[k * r + s] = sn * wkp + c * wks;
        }
      }
  }
  // V = L^{-T} W (back substitution per column)
  std::vector<q> Vt(r * r);
  for (int c = 0; c < r; ++c)
    for (int i = r - 1; i >= 0; --i) {
      q s = W[i * r + c];
      for (int k = i + 1; k < r; ++k) s -= L[k * r + i] * Vt[k * r + c];
      Vt[i * r + c] = s / L[i * r + i];
    }
  std::vector<int> order(r);
  for (int i = 0; i < r; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return H[a * r + a] < H[b * r + b]; });
  lam->resize(r);
  V->resize(r * r);
  for (int j = 0; j < r; ++j) {
    (*lam)[j] = H[order[j] * r + order[j]];
    for (int i = 0; i < r; ++i) (*V)[i * r + j] = Vt[i * r + order[j]];
  }
  return true;
}

struct AxisJob {
  int n;
  int64_t K;
  const std::vector<q>* A;
  const std::vector<q>* C;
  AxisTables* out;
  bool ok;
};

// Projected pencil at frequency k (1..K-1) and its eigenpairs.
bool frequency_block(int n, int64_t K, int64_t k, const std::vector<q>& A,
                     const std::vector<q>& C, AxisTables* t) {
  q sp, cp, s2p, c2p;
  sincospi(k, 2 * K, &sp, &cp);  // psi = pi k / (2K)
  sincospi(k, K, &s2p, &c2p);    // 2 psi
  auto terms = channel_terms(n, false);
  int r = n;
  auto kap = [&](const Term& a, const Term& b) -> q {
    int d = a.phase - b.phase;  // phase difference in units of psi
    q cosd = d == 0 ? (q)1 : (d == 2 || d == -2 ? c2p : cp);
    q sind = d == 0 ? (q)0 : (d == 2 ? s2p : d == -2 ? -s2p : d == 1 ? sp : -sp);
    if (a.is_cos == b.is_cos) return cosd;
    if (!a.is_cos) return sind;   // sum sin(x + a) cos(x + b) = (K/2) sin(a - b)
    return -sind;                 // sum cos(x + a) sin(x + b) = (K/2) sin(b - a)
  };
  std::vector<q> Ma(r * r), Mc(r * r);
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      q sa = 0, sc = 0;
      for (const Term& ta : terms[a])
        for (const Term& tb : terms[b]) {
          q f = (q)(ta.w * tb.w) * kap(ta, tb);
          sa += f * A[ta.i * (n + 1) + tb.i];
          sc += f * C[ta.i * (n + 1) + tb.i];
        }
      Ma[a * r + b] = sa * (q)K / 2;
      Mc[a * r + b] = sc * (q)K / 2;
    }
  std::vector<q> lam, V;
  if (!pencil_eigen(r, Ma, Mc, &lam, &V)) return false;
  for (int l = 0; l < r; ++l) {
    if (V[0 * r + l] < 0)
      for (int c = 0; c < r; ++c) V[c * r + l] = -V[c * r + l];
    t->lam[(n - 1) + (k - 1) * n + l] = (double)lam[l];
  }
  double* Qk = &t->Q[(size_t)k * n * n];
  for (int c = 0; c < r; ++c)
    for (int l = 0; l < r; ++l) Qk[c * n + l] = (double)V[c * r + l];
  return true;
}

// Bubble-only block (k = 0): channels even m (alternating pattern) and odd m
// (constant pattern); sum over the K elements gives the factor K.
bool zero_block(int n, int64_t K, const std::vector<q>& A, const std::vector<q>& C,
                AxisTables* t) {
  int r = n - 1;
  if (r == 0) return true;
  auto terms = channel_terms(n, true);
  int ne = num_even(n);
  std::vector<q> Ma(r * r, 0), Mc(r * r, 0);
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      if ((a < ne) != (b < ne)) continue;  // even/odd blocks decouple (bisymmetry)
      q sa = 0, sc = 0;
      for (const Term& ta : terms[a])
        for (const Term& tb : terms[b]) {
          sa += (q)(ta.w * tb.w) * A[ta.i * (n + 1) + tb.i];
          sc += (q)(ta.w * tb.w) * C[ta.i * (n + 1) + tb.i];
        }
      Ma[a * r + b] = sa * (q)K;
      Mc[a * r + b] = sc * (q)K;
    }
  std::vector<q> lam, V;
  if (!pencil_eigen(r, Ma, Mc, &lam, &V)) return false;
  for (int l = 0; l < r; ++l) {
    int big = 0;
    for (int c = 1; c < r; ++c)
      if (qabs(V[c * r + l]) > qabs(V[big * r + l]) * (1 + 1e-20Q)) big = c;
    if (V[big * r + l] < 0)
      for (int c = 0; c < r; ++c) V[c * r + l] = -V[c * r + l];
    t->lam[l] = (double)lam[l];
  }
  for (int c = 0; c < r; ++c)
    for (int l = 0; l < r; ++l) t->Q[c * n + l] = (double)V[c * r + l];
  return true;
}

// Tables of the condensed per-frequency solve.  At frequency k >= 1
// (psi = pi k / (2K)) the projected pencil is K/2 times
//   [ a0 + a1 cos 2psi     cos psi ve^T   sin psi vo^T ]
//   [ cos psi ve           E              0            ]
//   [ sin psi vo           0              O            ]
// (stiffness; the mass pencil likewise): the bubble blocks E (even
// channels) and O (odd) do not depend on k, and the nodal couplings only
// through cos psi and sin psi.  With We, Wo the mass-orthonormal
// eigenvectors of (E_A, E_C) and (O_A, O_C) (eigenvalues nu), the shifted
// system (coef A_k + bd C_k) x = y is an arrowhead system in the bubble
// eigenbasis.  Stored: We (ne x ne, [channel][mode]), Wo (no x no), nu,
// gA = W^T vA, gC = W^T vC (even modes then odd), and cc0, cc1 with
// cc0 + cc1 cos^2 psi the nodal Schur complement of the mass pencil.
bool condensed_tables(int n, const std::vector<q>& A, const std::vector<q>& C, AxisTables* t) {
  const int ne = num_even(n), no = num_odd(n), nb = n - 1;
  auto terms = channel_terms(n, true);
  auto blk = [&](const std::vector<q>& X, int a, int b) {
    q s = 0;
    for (const Term& ta : terms[a])
      for (const Term& tb : terms[b]) s += (q)(ta.w * tb.w) * X[ta.i * (n + 1) + tb.i];
    return s;
  };
  // nodal coupling of bubble channel a: even channels see the sum of the two
  // end rows (cos psi), odd channels their difference (sin psi)
  auto cpl = [&](const std::vector<q>& X, int a) {
    q s = 0;
    const bool odd = a >= ne;
    for (const Term& tb : terms[a])
      s += (q)tb.w * (odd ? X[n * (n + 1) + tb.i] - X[tb.i] : X[tb.i] + X[n * (n + 1) + tb.i]);
    return s;
  };
  std::vector<q> W(nb * nb, 0), nu(nb, 0), gA(nb, 0), gC(nb, 0);
  for (int part = 0; part < 2; ++part) {
    const int r = part == 0 ? ne : no, o = part == 0 ? 0 : ne;
    if (r == 0) continue;
    std::vector<q> Ma(r * r), Mc(r * r);
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < r; ++b) {
        Ma[a * r + b] = blk(A, o + a, o + b);
        Mc[a * r + b] = blk(C, o + a, o + b);
      }
    std::vector<q> lam, V;
    if (!pencil_eigen(r, Ma, Mc, &lam, &V)) return false;
    for (int m = 0; m < r; ++m) {
      nu[o + m] = lam[m];
      q sa = 0, sc = 0;
      for (int c = 0; c < r; ++c) {
        W[(o + c) * nb + o + m] = V[c * r + m];
        sa += V[c * r + m] * cpl(A, o + c);
        sc += V[c * r + m] * cpl(C, o + c);
      }
      gA[o + m] = sa;
      gC[o + m] = sc;
    }
  }
  q Ge = 0, Go = 0;
  for (int m = 0; m < nb; ++m) (m < ne ? Ge : Go) += gC[m] * gC[m];
  const q c0 = C[0] + C[n * (n + 1) + n], c1 = C[n] + C[n * (n + 1)];
  t->arrow.clear();
  for (int c = 0; c < ne; ++c)
    for (int m = 0; m < ne; ++m) t->arrow.push_back((double)W[c * nb + m]);
  for (int c = 0; c < no; ++c)
    for (int m = 0; m < no; ++m) t->arrow.push_back((double)W[(ne + c) * nb + ne + m]);
  for (int m = 0; m < nb; ++m) t->arrow.push_back((double)nu[m]);
  for (int m = 0; m < nb; ++m) t->arrow.push_back((double)gA[m]);
  for (int m = 0; m < nb; ++m) t->arrow.push_back((double)gC[m]);
  // cos 2psi = 2 cos^2 psi - 1, sin^2 psi = 1 - cos^2 psi
  t->arrow.push_back((double)(c0 - c1 - Go));
  t->arrow.push_back((double)(2 * c1 - Ge + Go));
  return true;
}

// Tables of the banded solve along an axis (Sect. 4, algorithm (b)): the
// element's bubble block of the shifted matrix coef A + sigma C is
// diagonalized once in the mass-orthonormal eigenbasis V of the pencil
// (A_BB, C_BB) (eigenvalues lam), so per line only the n - 1 reciprocals
// 1 / (coef lam + sigma) are needed to eliminate the bubbles element by
// element; the couplings of the modes to the element's end nodes give the
// nodal tridiagonal system.  Its entries are formed without cancellation:
// the condensed stiffness part (a0, -a0: rows summing to zero) comes from
// this 113-bit table, and only terms proportional to sigma are added per
// line (tL, tX: the sigma-independent parts of those terms).
bool band_tables(int n, const std::vector<q>& A, const std::vector<q>& C, AxisTables* t) {
  const int nb = n - 1, m = n + 1;
  const BandLayout bl(n);
  t->band.assign(bl.size, 0.0);
  q a0 = A[0];
  if (nb > 0) {
    std::vector<q> Ma(nb * nb), Mc(nb * nb);
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) {
        Ma[a * nb + b] = A[(1 + a) * m + 1 + b];
        Mc[a * nb + b] = C[(1 + a) * m + 1 + b];
      }
    std::vector<q> lam, V;
    if (!pencil_eigen(nb, Ma, Mc, &lam, &V)) return false;
    for (int a = 0; a < nb; ++a)
      for (int l = 0; l < nb; ++l) t->band[bl.V + a * nb + l] = (double)V[a * nb + l];
    for (int l = 0; l < nb; ++l) {
      if (!(lam[l] > 0)) return false;
      q aL = 0, cL = 0, aR = 0, cR = 0;
      for (int a = 0; a < nb; ++a) {
        aL += V[a * nb + l] * A[(1 + a) * m + 0];
        cL += V[a * nb + l] * C[(1 + a) * m + 0];
        aR += V[a * nb + l] * A[(1 + a) * m + n];
        cR += V[a * nb + l] * C[(1 + a) * m + n];
      }
      t->band[bl.lam + l] = (double)lam[l];
      t->band[bl.hAL + l] = (double)aL;
      t->band[bl.hCL + l] = (double)cL;
      t->band[bl.hAR + l] = (double)aR;
      t->band[bl.hCR + l] = (double)cR;
      t->band[bl.tL + l] = (double)(2 * aL * cL - aL * aL / lam[l]);
      t->band[bl.tX + l] = (double)(aL * cR + aR * cL - aL * aR / lam[l]);
      a0 -= aL * aL / lam[l];
    }
  }
  t->band[bl.nn + 0] = (double)C[0];
  t->band[bl.nn + 1] = (double)C[n];
  t->band[bl.nn + 2] = (double)a0;
  return true;
}

}  // namespace

void element_matrices(int n, std::vector<double>* A, std::vector<double>* C) {
  std::vector<q> Aq, Cq;
  element_matrices_q(n, &Aq, &Cq);
  A->resize(Aq.size());
  C->resize(Cq.size());
  for (size_t i = 0; i < Aq.size(); ++i) {
    (*A)[i] = (double)Aq[i];
    (*C)[i] = (double)Cq[i];
  }
}

void element_matrices_dd(int n, std::vector<double>* A, std::vector<double>* C) {
  std::vector<q> Aq, Cq;
  element_matrices_q(n, &Aq, &Cq);
  const size_t m = Aq.size();
  A->assign(2 * m, 0.0);
  C->assign(2 * m, 0.0);
  for (size_t i = 0; i < m; ++i) {
    double ah = (double)Aq[i], ch = (double)Cq[i];
    (*A)[i] = ah;
    (*A)[m + i] = (double)(Aq[i] - (q)ah);
    (*C)[i] = ch;
    (*C)[m + i] = (double)(Cq[i] - (q)ch);
  }
}

int build_axis_tables(int n, int64_t K, double diff, double X, AxisTables* t) {
  const int kEINVAL = -1, kESPECTRUM = -4;
  if (n < 1 || K < 2) return kEINVAL;
  std::vector<q> A, C;
  element_matrices_q(n, &A, &C);
  t->n = n;
  t->K = K;
  t->M = (int64_t)n * K - 1;
  t->coef = diff * 4.0 * ((double)K / X) * ((double)K / X);
  t->lam.assign(t->M, 0.0);
  t->Q.assign((size_t)K * n * n, 0.0);
  if (!zero_block(n, K, A, C, t)) return kESPECTRUM;
  if (!condensed_tables(n, A, C, t)) return kESPECTRUM;
  if (!band_tables(n, A, C, t)) return kESPECTRUM;
  unsigned hw = std::thread::hardware_concurrency();
  int nthreads = (int)std::max(1u, std::min(hw == 0 ? 1u : hw, 16u));
  if (K < 64) nthreads = 1;
  std::vector<int> ok(nthreads, 1);
  auto work = [&](int tid) {
    for (int64_t k = 1 + tid; k < K; k += nthreads)
      if (!frequency_block(n, K, k, A, C, t)) ok[tid] = 0;
  };
  if (nthreads == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int i = 0; i < nthreads; ++i) th.emplace_back(work, i);
    for (auto& x : th) x.join();
  }
  for (int v : ok)
    if (!v) return kESPECTRUM;
  for (double v : t->lam)
    if (!(v > 0) || !std::isfinite(v)) return kESPECTRUM;
  // mixed-radix stages for a line held in one LDS tile (K <= 1024); longer
  // lines that are not a power of two take Bluestein's tables
  t->radices = (K & (K - 1)) && K <= 1024 ? mixed_radices(K) : std::vector<int>();
  if ((K & (K - 1)) && t->radices.empty()) {
    // Bluestein tables for a length-K DFT: chirp c_j = exp(-i pi j^2 / K)
    // (argument reduced exactly: j^2 mod 2K), and the spectrum of the
    // conjugate chirp b (b_m = conj(c_m) at m and L - m, |m| < K, zero
    // elsewhere) over L >= 2K - 1 points, divided by L.
    int64_t L = 1;
    while (L < 2 * K - 1) L *= 2;
    t->L = L;
    t->chirp.resize(2 * K);
    std::vector<long double> br(L, 0.0L), bi(L, 0.0L);
    for (int64_t j = 0; j < K; ++j) {
      q sn, cs;
      sincospi((j * j) % (2 * K), K, &sn, &cs);
      t->chirp[2 * j] = (double)cs;
      t->chirp[2 * j + 1] = -(double)sn;
      br[j] = (long double)cs;
      bi[j] = (long double)sn;
      if (j > 0) {
        br[L - j] = (long double)cs;
        bi[L - j] = (long double)sn;
      }
    }
    // iterative radix-2 FFT (exp(-2 pi i/L)) in extended precision
    std::vector<long double> wr(L / 2), wi(L / 2);
    for (int64_t m = 0; m < L / 2; ++m) {
      q sn, cs;
      sincospi(2 * m, L, &sn, &cs);
      wr[m] = (long double)cs;
      wi[m] = -(long double)sn;
    }
    for (int64_t i = 1, j = 0; i < L; ++i) {
      int64_t bit = L >> 1;
      for (; j & bit; bit >>= 1) j ^= bit;
      j ^= bit;
      if (i < j) {
        std::swap(br[i], br[j]);
        std::swap(bi[i], bi[j]);
      }
    }
    for (int64_t len = 2; len <= L; len *= 2) {
      const int64_t step = L / len;
      for (int64_t i0 = 0; i0 < L; i0 += len)
        for (int64_t m = 0; m < len / 2; ++m) {
          long double xr = br[i0 + m + len / 2], xi = bi[i0 + m + len / 2];
          long double tr = xr * wr[m * step] - xi * wi[m * step];
          long double ti = xr * wi[m * step] + xi * wr[m * step];
          br[i0 + m + len / 2] = br[i0 + m] - tr;
          bi[i0 + m + len / 2] = bi[i0 + m] - ti;
          br[i0 + m] += tr;
          bi[i0 + m] += ti;
        }
    }
    t->bhat.resize(2 * L);
    t->twl.resize(2 * L);
    for (int64_t m = 0; m < L; ++m) {
      t->bhat[2 * m] = (double)(br[m] / (long double)L);
      t->bhat[2 * m + 1] = (double)(bi[m] / (long double)L);
      q sn, cs;
      sincospi(2 * m, L, &sn, &cs);
      t->twl[2 * m] = (double)cs;
      t->twl[2 * m + 1] = -(double)sn;
    }
  }
  t->twf.resize(2 * K);
  t->twm.resize(2 * K);
  t->twd.resize(2 * K);
  for (int64_t k = 0; k < K; ++k) {
    q s, c;
    sincospi(2 * k, K, &s, &c);
    t->twf[2 * k] = (double)c;
    t->twf[2 * k + 1] = -(double)s;
    sincospi(k, 2 * K, &s, &c);
    t->twm[2 * k] = (double)c;
    t->twm[2 * k + 1] = -(double)s;
    sincospi(k, K, &s, &c);
    t->twd[2 * k] = (double)c;
    t->twd[2 * k + 1] = -(double)s;
  }
  return 0;
}

}  // namespace fftfem
