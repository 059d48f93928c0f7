// Operator apply (double-double, for y = A u and the refinement residual), the
// refinement bookkeeping kernels and the tiled transpose (gfx950).
#include "device_common.h"
#include "launch.h"

namespace fftfem {

// Dynamic LDS of the kernels in this file.
extern __shared__ double2 fftfem_ops_lds[];

// ---------------------------------------------------------------------------
// Double-double arithmetic for the operator apply.  The stiffness part of A
// is a second-difference operator whose norm exceeds its smallest eigenvalue
// by about (nK)^2; a residual f - A u rounded at float64 (and float64-rounded
// element matrices, whose rows then no longer sum to zero) leaves an error of
// that size relative to the solution, far above what refinement must reach.
// Every product and sum of the apply is therefore carried as an unevaluated
// sum hi + lo of two doubles (error-free transformations), with the element
// matrices rounded from 113-bit values into hi + lo pairs.  Contraction of
// a * b + c into fma is disabled in these helpers: the error-free sums depend
// on each operation being rounded on its own.
struct dd {
  double h, l;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// s += x * v, x and v given as hi + lo pairs (vl = 0 for a float64 input)
template <bool LO>
__device__ __forceinline__ void dd_fma(dd& s, double xh, double xl, double vh, double vl) {
#pragma clang fp contract(off)
  double p = xh * vh;
  double e = __builtin_fma(xh, vh, -p);
  if constexpr (LO) e = __builtin_fma(xh, vl, e);
  e = __builtin_fma(xl, vh, e);
  double t, err;
  two_sum(s.h, p, t, err);
  s.h = t;
  s.l += err + e;
}

// s += c * x for a float64 scalar c
__device__ __forceinline__ void dd_axpy(dd& s, double c, dd x) {
#pragma clang fp contract(off)
  double p = c * x.h;
  double e = __builtin_fma(c, x.h, -p);
  e = __builtin_fma(c, x.l, e);
  double t, err;
  two_sum(s.h, p, t, err);
  s.h = t;
  s.l += err + e;
}

__device__ __forceinline__ dd dd_norm(dd s) {
#pragma clang fp contract(off)
  double h = s.h + s.l;
  return {h, s.l - (h - s.h)};
}

// The same row in plain float64 arithmetic (hi parts of the element
// matrices only; the operator of the incremental residual r - A c, where c
// is a small correction and its float64 rounding is far below the accuracy
// the refinement needs).
template <int NORD>
__device__ __forceinline__ double row_apply_f64(const double* v, int g, const double* X) {
  constexpr int n = NORD;
  const bool node = (g + 1) % n == 0;
  const int l = node ? n : g % n + 1;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t <= n; ++t) s = __builtin_fma(X[l * (n + 1) + t], v[g - l + t], s);
  if (node) {
#pragma unroll
    for (int t = 0; t <= n; ++t) s = __builtin_fma(X[t], v[g + t], s);
  }
  return s;
}

// One row of a 1D element-assembled matrix at position g of a line
// (Sect. 2: element-by-element assembly of A and C).  With v = 0 outside
// the line (Dirichlet):
//   node (g+1) % n == 0:  sum_t X[n][t] v[g-n+t] + sum_t X[0][t] v[g+t]
//   bubble l = g % n + 1: sum_t X[l][t] v[g-l+t]
// The first sum of a node has the form of a bubble row with l = n, so all
// lanes of a wave run it together and only the nodes' second sum diverges.
// X holds (n+1)^2 hi values followed by (n+1)^2 lo values.
template <int NORD, bool LO>
__device__ __forceinline__ dd row_apply(const double* vh, const double* vl, int g, const double* X) {
  constexpr int n = NORD;
  constexpr int XX = (NORD + 1) * (NORD + 1);
  const bool node = (g + 1) % n == 0;
  const int l = node ? n : g % n + 1;
  dd s{0.0, 0.0};
#pragma unroll
  for (int t = 0; t <= n; ++t) {
    int j = g - l + t;
    dd_fma<LO>(s, X[l * (n + 1) + t], X[XX + l * (n + 1) + t], vh[j], LO ? vl[j] : 0.0);
  }
  if (node) {
#pragma unroll
    for (int t = 0; t <= n; ++t)
      dd_fma<LO>(s, X[t], X[XX + t], vh[g + t], LO ? vl[g + t] : 0.0);
  }
  return s;
}

// Both products of a row, C v and A v, at position g of a float64 line
// (the fused 2D pass): four independent partial sums (the two matrices,
// even and odd t) instead of two serial chains of n + 1 error-free
// multiply-adds, joined at the end.
template <int NORD>
__device__ __forceinline__ void row_apply2(const double* v, int g, const double* Xc, const double* Xa, dd& C,
                                           dd& A) {
#pragma clang fp contract(off)
  constexpr int n = NORD;
  constexpr int XX = (NORD + 1) * (NORD + 1);
  const bool node = (g + 1) % n == 0;
  const int l = node ? n : g % n + 1;
  dd c0{0, 0}, c1{0, 0}, a0{0, 0}, a1{0, 0};
#pragma unroll
  for (int t = 0; t <= n; ++t) {
    const int o = l * (n + 1) + t;
    const double x = v[g - l + t];
    dd_fma<false>((t & 1) ? c1 : c0, Xc[o], Xc[XX + o], x, 0.0);
    dd_fma<false>((t & 1) ? a1 : a0, Xa[o], Xa[XX + o], x, 0.0);
  }
  if (node) {
#pragma unroll
    for (int t = 0; t <= n; ++t) {
      const double x = v[g + t];
      dd_fma<false>((t & 1) ? c1 : c0, Xc[t], Xc[XX + t], x, 0.0);
      dd_fma<false>((t & 1) ? a1 : a0, Xa[t], Xa[XX + t], x, 0.0);
    }
  }
  dd_axpy(c0, 1.0, c1);
  dd_axpy(a0, 1.0, a1);
  C = c0;
  A = a0;
}

// ---------------------------------------------------------------------------
// 1D operator pass along one axis.  With a and c the stiffness and mass rows
// above, for each position of each line:
//   o1 = c1[0] a(in1) + c1[1] c(in1) + c1[2] a(in2) + c1[3] c(in2)
//        (o1 = f - that, when f is given)
//   o2 = c2[0] a(in1) + c2[1] c(in1) + c2[2] a(in2) + c2[3] c(in2)
// Chained along the axes these give the sum-factorized tensor operator.
// Tiles: G lines x TL positions with an n-dof halo on each side, staged in
// LDS as separate hi and lo planes.  DD: double-double arithmetic (error-free
// products and sums); otherwise plain float64 (LO false, hi outputs only).
template <int NORD, bool LO, bool DD>
__device__ __forceinline__ void apply_body(const ApplyArgs& a, int bid, int nblk) {
#pragma clang fp contract(off)
  static_assert(DD || !LO, "double-double inputs need double-double arithmetic");
  if (a.flag && *a.flag) return;
  constexpr int n = NORD;
  constexpr int XX = (NORD + 1) * (NORD + 1);
  double* sm = reinterpret_cast<double*>(fftfem_ops_lds);
  __shared__ double Xa[2 * XX], Xc[2 * XX];
  const int tid = threadIdx.x;
  for (int i = tid; i < XX; i += kThreads) {
    Xa[i] = a.Ael[0][i];
    Xa[XX + i] = a.Ael[1][i];
    Xc[i] = a.Cel[0][i];
    Xc[XX + i] = a.Cel[1][i];
  }
  const int G = a.G, TL = a.TL, W = TL + 2 * n;
  const int64_t nseg = (a.M + TL - 1) / TL;
  const int64_t tile = xcd_remap(bid, nblk);
  const int64_t lg = tile / nseg, seg = tile - lg * nseg;
  const int64_t l0 = lg * G, s0 = seg * TL;
  const bool lines_fast = a.es > 1;
  const bool two = a.in2[0] != nullptr;
  const int plane = G * W;
  double* v1h = sm;
  double* v1l = sm + plane;
  double* v2h = sm + (LO ? 2 : 1) * plane;
  double* v2l = v2h + plane;
  for (int t = tid; t < plane; t += kThreads) {
    int g, i;
    if (lines_fast) {
      g = t % G;
      i = t / G;
    } else {
      i = t % W;
      g = t / W;
    }
    int64_t line = l0 + g;
    int64_t pos = s0 - n + i;
    double x1h = 0, x1l = 0, x2h = 0, x2l = 0;
    if (line < a.nlines && pos >= 0 && pos < a.M) {
      int64_t outer = line / a.es, inner = line - outer * a.es;
      int64_t idx = outer * a.M * a.es + inner + pos * a.es;
      x1h = a.in1[0][idx];
      if (LO) x1l = a.in1[1][idx];
      if (two) {
        x2h = a.in2[0][idx];
        if (LO) x2l = a.in2[1][idx];
      }
    }
    const int o = g * W + i;
    v1h[o] = x1h;
    if (LO) v1l[o] = x1l;
    if (two) {
      v2h[o] = x2h;
      if (LO) v2l[o] = x2l;
    }
  }
  __syncthreads();
  // which of the four row products any output needs (uniform over the grid)
  const bool needA1 = a.c1[0] != 0 || a.c2[0] != 0, needC1 = a.c1[1] != 0 || a.c2[1] != 0;
  const bool needA2 = two && (a.c1[2] != 0 || a.c2[2] != 0);
  const bool needC2 = two && (a.c1[3] != 0 || a.c2[3] != 0);
  for (int t = tid; t < G * TL; t += kThreads) {
    int g, i;
    if (lines_fast) {
      g = t % G;
      i = t / G;
    } else {
      i = t % TL;
      g = t / TL;
    }
    int64_t line = l0 + g;
    int64_t pos = s0 + i;
    if (line >= a.nlines || pos >= a.M) continue;
    // window pointers shifted so that index = position along the line
    const int sh = g * W + n - (int)s0;
    if constexpr (!DD) {
      double A1 = 0, C1 = 0, A2 = 0, C2v = 0;
      if (needA1) A1 = row_apply_f64<NORD>(v1h + sh, (int)pos, Xa);
      if (needC1) C1 = row_apply_f64<NORD>(v1h + sh, (int)pos, Xc);
      if (needA2) A2 = row_apply_f64<NORD>(v2h + sh, (int)pos, Xa);
      if (needC2) C2v = row_apply_f64<NORD>(v2h + sh, (int)pos, Xc);
      int64_t outer = line / a.es, inner = line - outer * a.es;
      int64_t idx = outer * a.M * a.es + inner + pos * a.es;
      double r = a.c1[0] * A1;
      r = __builtin_fma(a.c1[1], C1, r);
      r = __builtin_fma(a.c1[2], A2, r);
      r = __builtin_fma(a.c1[3], C2v, r);
      if (a.f) r = a.f[idx] - r;
      if (a.o1_kind == 0)
        ((float*)a.o1[0])[idx] = (float)r;
      else
        ((double*)a.o1[0])[idx] = r;
      if (a.o2[0]) {
        double q = a.c2[0] * A1;
        q = __builtin_fma(a.c2[1], C1, q);
        q = __builtin_fma(a.c2[2], A2, q);
        q = __builtin_fma(a.c2[3], C2v, q);
        a.o2[0][idx] = q;
      }
      continue;
    }
    dd A1{0, 0}, C1{0, 0}, A2{0, 0}, C2v{0, 0};
    if (needA1) A1 = row_apply<NORD, LO>(v1h + sh, v1l + sh, (int)pos, Xa);
    if (needC1) C1 = row_apply<NORD, LO>(v1h + sh, v1l + sh, (int)pos, Xc);
    if (needA2) A2 = row_apply<NORD, LO>(v2h + sh, v2l + sh, (int)pos, Xa);
    if (needC2) C2v = row_apply<NORD, LO>(v2h + sh, v2l + sh, (int)pos, Xc);
    int64_t outer = line / a.es, inner = line - outer * a.es;
    int64_t idx = outer * a.M * a.es + inner + pos * a.es;
    dd r{0, 0};
    dd_axpy(r, a.c1[0], A1);
    dd_axpy(r, a.c1[1], C1);
    dd_axpy(r, a.c1[2], A2);
    dd_axpy(r, a.c1[3], C2v);
    if (a.f) {
      double hh, e;
      two_sum(a.f[idx], -r.h, hh, e);
      r = {hh, e - r.l};
    }
    r = dd_norm(r);
    if (a.o1_kind == 0) {
      ((float*)a.o1[0])[idx] = (float)r.h;
    } else {
      ((double*)a.o1[0])[idx] = r.h;
      if (a.o1_kind == 2) ((double*)a.o1[1])[idx] = r.l;
    }
    if (a.o2[0]) {
      dd q{0, 0};
      dd_axpy(q, a.c2[0], A1);
      dd_axpy(q, a.c2[1], C1);
      dd_axpy(q, a.c2[2], A2);
      dd_axpy(q, a.c2[3], C2v);
      q = dd_norm(q);
      a.o2[0][idx] = q.h;
      a.o2[1][idx] = q.l;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused 2D operator pass (both axes of order n in one kernel), for the
// refinement residual and the operator apply:
//   A u = c0 (A_0 x C_1) u + c1 (C_0 x A_1) u + react (C_0 x C_1) u
//       = A_0 v + C_0 z,   v = c0 C_1 u,  z = c1 A_1 u + react C_1 u,
// v and z taken along axis 1 (rows), then A_0 and C_0 along axis 0 (the
// sum factorization of the two-pass apply, in one pass over the array).
//
// One wave owns 64 columns (lane l: column col0 + l) and a chunk of E
// elements along axis 0, which it walks one element at a time.  For element
// e (rows t = 0..n: global row n e + t - 1, t = 0 and t = n its end nodes)
// the wave stages rows t = 1..n (with n columns of halo on each side) in
// LDS, forms v_t and z_t in registers, and accumulates the element's local
// products y_q += A_0[q][t] v_t + C_0[q][t] z_t for all q = 0..n at once
// (n + 1 independent accumulators; row t = 0 is the previous element's
// row n, kept in registers).  Then the bubbles q = 1..n-1 are complete; the
// node between elements e-1 and e is the previous element's y_n plus this
// element's y_0.  A chunk also walks the element after it (without writing
// its bubbles) to complete its last node.  The next element's rows and this
// element's f (or r) values are loaded into registers one element ahead.
//
// DD: double-double arithmetic throughout, out = f - A u (or A u when f is
// null), u float64.  Otherwise plain float64: out -= A u in place (the
// incremental residual r - A c).
template <int NORD, bool DD>
__device__ __forceinline__ void resid2_body(const Resid2Args& a, int bid, int nblk) {
#pragma clang fp contract(off)
  if (a.flag && *a.flag) return;
  constexpr int n = NORD, XX = (n + 1) * (n + 1), W = 64 + 2 * n;
  __shared__ double Xa[2 * XX], Xc[2 * XX];
  __shared__ double stg[n * W];
  const int lane = threadIdx.x;
  for (int i = lane; i < 2 * XX; i += 64) {
    Xa[i] = a.Ael[i];
    Xc[i] = a.Cel[i];
  }
  const int64_t M0 = a.M0, M1 = a.M1;
  const int ncb = (int)((M1 + 63) / 64);
  const int tile = xcd_remap(bid, nblk);
  const int ch = tile / ncb, cb = tile - ch * ncb;
  const int e0 = ch * a.E;
  const int e1 = e0 + a.E < a.K0 ? e0 + a.E : a.K0;  // elements whose rows this chunk writes
  const int elast = e1 < a.K0 ? e1 : e1 - 1;         // plus the next one, for the last node
  const int64_t col0 = (int64_t)cb * 64, col = col0 + lane;
  const bool colok = col < M1;
  const double* src = DD ? a.f : a.out;  // subtracted from (null: out = A u)

  // values of global row r at columns col0 - n + lane and col0 - n + 64 + lane
  // (zero outside the array: the Dirichlet boundary)
  auto load_row = [&](int64_t r, double& x0, double& x1) {
    x0 = x1 = 0.0;
    if (r < 0 || r >= M0) return;
    const int64_t c0 = col0 - n + lane, c1 = c0 + 64;
    const double* row = a.u + r * M1;
    if (c0 >= 0 && c0 < M1) x0 = row[c0];
    if (lane < W - 64 && c1 < M1) x1 = row[c1];
  };
  auto stage = [&](int sr, double x0, double x1) {
    stg[sr * W + lane] = x0;
    if (lane < W - 64) stg[sr * W + 64 + lane] = x1;
  };
  // The element matrices are read from LDS at each use through an offset
  // the compiler cannot see (zero): otherwise it keeps all 4 (n + 1)^2 values
  // (they do not change from element to element) in registers and spills.
  auto opaque0 = []() {
    int z = 0;
    __asm__ volatile("" : "+v"(z));
    return z;
  };
  // v and z of staged row sr at this lane's column
  auto rowvz = [&](int sr, dd& v, dd& z) {
    const double* vrow = stg + sr * W + n - col0;  // index = global column
    const int o0 = opaque0();
    const double* Xa_ = Xa + o0;
    const double* Xc_ = Xc + o0;
    if constexpr (DD) {
      dd C, A;
      row_apply2<NORD>(vrow, (int)col, Xc_, Xa_, C, A);
      v = dd{0, 0};
      z = dd{0, 0};
      dd_axpy(v, a.c0, C);
      dd_axpy(z, a.c1, A);
      dd_axpy(z, a.react, C);
      v = dd_norm(v);
      z = dd_norm(z);
    } else {
      const double C = row_apply_f64<NORD>(vrow, (int)col, Xc_);
      const double A = row_apply_f64<NORD>(vrow, (int)col, Xa_);
      v = dd{a.c0 * C, 0};
      z = dd{__builtin_fma(a.c1, A, a.react * C), 0};
    }
  };
  // acc[q] += A_0[q][t] v + C_0[q][t] z for q = 0..n
  auto accumulate = [&](dd* acc, int t, const dd& v, const dd& z) {
    const int o0 = opaque0();
#pragma unroll
    for (int q = 0; q <= n; ++q) {
      const int o = q * (n + 1) + t + o0;
      if constexpr (DD) {
        dd_fma<true>(acc[q], Xa[o], Xa[XX + o], v.h, v.l);
        dd_fma<true>(acc[q], Xc[o], Xc[XX + o], z.h, z.l);
      } else {
        acc[q].h = __builtin_fma(Xa[o], v.h, acc[q].h);
        acc[q].h = __builtin_fma(Xc[o], z.h, acc[q].h);
      }
    }
  };
  auto put = [&](int64_t g, double fv, const dd& y) {
    if (!colok || g < 0 || g >= M0) return;
    const int64_t idx = g * M1 + col;
    if constexpr (DD) {
      dd r = y;
      if (src) {
        double hh, er;
        two_sum(fv, -y.h, hh, er);
        r = {hh, er - y.l};
      }
      r = dd_norm(r);
      a.out[idx] = r.h;
    } else {
      a.out[idx] = fv - y.h;
    }
  };
  auto load_f = [&](int64_t g) -> double { return (src && colok && g >= 0 && g < M0) ? src[g * M1 + col] : 0.0; };

  // prologue: row t = 0 of element e0 (its left node)
  dd v0, z0;
  {
    double x0, x1;
    load_row((int64_t)n * e0 - 1, x0, x1);
    stage(0, x0, x1);
    __syncthreads();
    rowvz(0, v0, z0);
    __syncthreads();
  }
  // float64 pass: the next element's rows are loaded one element ahead
  // (registers allow it; the double-double pass has no room for them)
  constexpr bool PF = !DD;
  double ux[PF ? n : 1][2];
  if constexpr (PF) {
#pragma unroll
    for (int t = 1; t <= n; ++t) load_row((int64_t)n * e0 + t - 1, ux[t - 1][0], ux[t - 1][1]);
  }
  dd carry{0, 0};  // the previous element's contribution to its right node
  for (int e = e0; e <= elast; ++e) {
    // rows t = 1..n of element e into the staging area
#pragma unroll
    for (int t = 1; t <= n; ++t) {
      if constexpr (PF) {
        stage(t - 1, ux[t - 1][0], ux[t - 1][1]);
      } else {
        double x0, x1;
        load_row((int64_t)n * e + t - 1, x0, x1);
        stage(t - 1, x0, x1);
      }
    }
    __syncthreads();
    if constexpr (PF) {
      if (e < elast) {
#pragma unroll
        for (int t = 1; t <= n; ++t) load_row((int64_t)n * (e + 1) + t - 1, ux[t - 1][0], ux[t - 1][1]);
      }
    }
    dd acc[n + 1];
#pragma unroll
    for (int q = 0; q <= n; ++q) acc[q] = dd{0, 0};
    accumulate(acc, 0, v0, z0);
    // one row at a time (not unrolled: unrolled, the scheduler starts the
    // LDS reads of all rows at once and spills)
#pragma unroll 1
    for (int t = 1; t <= n; ++t) {
      dd v, z;
      rowvz(t - 1, v, z);
      accumulate(acc, t, v, z);
      if (t == n) {
        v0 = v;
        z0 = z;
      }
    }
    // subtrahends of this element's outputs: row n e - 1 (its left node,
    // t = 0) and its bubbles (t = 1..n-1); loaded after the products, which
    // leaves the registers to the accumulators (other waves cover the wait)
    double fc[n];
#pragma unroll
    for (int t = 0; t < n; ++t) fc[t] = load_f((int64_t)n * e + t - 1);
    __syncthreads();  // the staging area is free for the next element
    // the node between elements e - 1 and e (a row of this chunk when e > e0)
    if (e > e0) {
      dd y = carry;
      dd_axpy(y, 1.0, acc[0]);
      put((int64_t)n * e - 1, fc[0], y);
    }
    if (e < e1) {
#pragma unroll
      for (int t = 1; t < n; ++t) put((int64_t)n * e + t - 1, fc[t], acc[t]);
    }
    carry = acc[n];
  }
}

// Waves per SIMD: 4 for the float64 pass (at most 128 VGPRs), 3 for the
// double-double one (at most 168; its n + 1 double-double accumulators,
// carried row and node partial spill at 128 for n >= 8).  The one-wave
// workgroups on a CU hide each other's row loads.
// Plane pass of the 3D operator (axes 1 and 2 of one order n), the first of
// the two passes of the 3D residual: per plane i_0, with the same walk as
// resid2_body (one wave per 64 columns of axis 2 and a chunk of E elements
// of axis 1), the two products
//   P = (C_1 x C_2) u,   Q = (c0 A_1 x C_2 + c1 C_1 x A_2 + react C_1 x C_2) u
// (c0, c1: the coefficients of axes 1 and 2), from the rows' C_2 u and
// A_2 u: P accumulates C_1 (C_2 u), Q accumulates A_1 (c0 C_2 u) and
// C_1 (c1 A_2 u + react C_2 u).  The axis-0 pass then forms
// f - (diff_0 4/h_0^2) A_0 P - C_0 Q.  DD: both in double-double (hi, lo
// planes); otherwise float64.
template <int NORD, bool DD>
__device__ __forceinline__ void resid3p_body(const Resid2Args& a, int bid, int nblk) {
#pragma clang fp contract(off)
  if (a.flag && *a.flag) return;
  constexpr int n = NORD, XX = (n + 1) * (n + 1), W = 64 + 2 * n;
  __shared__ double Xa[2 * XX], Xc[2 * XX];
  __shared__ double stg[n * W];
  const int lane = threadIdx.x;
  for (int i = lane; i < 2 * XX; i += 64) {
    Xa[i] = a.Ael[i];
    Xc[i] = a.Cel[i];
  }
  const int64_t M0 = a.M0, M1 = a.M1;
  const int ncb = (int)((M1 + 63) / 64);
  const int nch = (a.K0 + a.E - 1) / a.E;
  const int tile = xcd_remap(bid, nblk);
  const int per = ncb * nch;
  const int plane = tile / per, rest = tile - plane * per;
  const int ch = rest / ncb, cb = rest - ch * ncb;
  const int64_t pb = (int64_t)plane * M0 * M1;
  const double* u = a.u + pb;
  const int e0 = ch * a.E;
  const int e1 = e0 + a.E < a.K0 ? e0 + a.E : a.K0;
  const int elast = e1 < a.K0 ? e1 : e1 - 1;
  const int64_t col0 = (int64_t)cb * 64, col = col0 + lane;
  const bool colok = col < M1;

  auto load_row = [&](int64_t r, double& x0, double& x1) {
    x0 = x1 = 0.0;
    if (r < 0 || r >= M0) return;
    const int64_t c0 = col0 - n + lane, c1 = c0 + 64;
    const double* row = u + r * M1;
    if (c0 >= 0 && c0 < M1) x0 = row[c0];
    if (lane < W - 64 && c1 < M1) x1 = row[c1];
  };
  auto stage = [&](int sr, double x0, double x1) {
    stg[sr * W + lane] = x0;
    if (lane < W - 64) stg[sr * W + 64 + lane] = x1;
  };
  auto opaque0 = []() {
    int z = 0;
    __asm__ volatile("" : "+v"(z));
    return z;
  };
  // the row's inputs of the two accumulations: zp = C_2 u (for P), vq =
  // c0 C_2 u and zq = c1 A_2 u + react C_2 u (for Q)
  auto rowvz = [&](int sr, dd& zp, dd& vq, dd& zq) {
    const double* vrow = stg + sr * W + n - col0;
    const int o0 = opaque0();
    const double* Xa_ = Xa + o0;
    const double* Xc_ = Xc + o0;
    if constexpr (DD) {
      dd C, A;
      row_apply2<NORD>(vrow, (int)col, Xc_, Xa_, C, A);
      zp = dd_norm(C);
      vq = dd{0, 0};
      zq = dd{0, 0};
      dd_axpy(vq, a.c0, C);
      dd_axpy(zq, a.c1, A);
      dd_axpy(zq, a.react, C);
      vq = dd_norm(vq);
      zq = dd_norm(zq);
    } else {
      const double C = row_apply_f64<NORD>(vrow, (int)col, Xc_);
      const double A = row_apply_f64<NORD>(vrow, (int)col, Xa_);
      zp = dd{C, 0};
      vq = dd{a.c0 * C, 0};
      zq = dd{__builtin_fma(a.c1, A, a.react * C), 0};
    }
  };
  auto accumulate = [&](dd* ap, dd* aq, int t, const dd& zp, const dd& vq, const dd& zq) {
    const int o0 = opaque0();
#pragma unroll
    for (int q = 0; q <= n; ++q) {
      const int o = q * (n + 1) + t + o0;
      if constexpr (DD) {
        dd_fma<true>(ap[q], Xc[o], Xc[XX + o], zp.h, zp.l);
        dd_fma<true>(aq[q], Xa[o], Xa[XX + o], vq.h, vq.l);
        dd_fma<true>(aq[q], Xc[o], Xc[XX + o], zq.h, zq.l);
      } else {
        ap[q].h = __builtin_fma(Xc[o], zp.h, ap[q].h);
        aq[q].h = __builtin_fma(Xa[o], vq.h, aq[q].h);
        aq[q].h = __builtin_fma(Xc[o], zq.h, aq[q].h);
      }
    }
  };
  auto put = [&](int64_t g, const dd& P, const dd& Q) {
    if (!colok || g < 0 || g >= M0) return;
    const int64_t idx = pb + g * M1 + col;
    if constexpr (DD) {
      const dd p2 = dd_norm(P), q2 = dd_norm(Q);
      a.out[idx] = p2.h;
      a.out_l[idx] = p2.l;
      a.out2[idx] = q2.h;
      a.out2_l[idx] = q2.l;
    } else {
      a.out[idx] = P.h;
      a.out2[idx] = Q.h;
    }
  };

  dd zp0, vq0, zq0;
  {
    double x0, x1;
    load_row((int64_t)n * e0 - 1, x0, x1);
    stage(0, x0, x1);
    __syncthreads();
    rowvz(0, zp0, vq0, zq0);
    __syncthreads();
  }
  dd carp{0, 0}, carq{0, 0};
  for (int e = e0; e <= elast; ++e) {
#pragma unroll
    for (int t = 1; t <= n; ++t) {
      double x0, x1;
      load_row((int64_t)n * e + t - 1, x0, x1);
      stage(t - 1, x0, x1);
    }
    __syncthreads();
    dd ap[n + 1], aq[n + 1];
#pragma unroll
    for (int q = 0; q <= n; ++q) ap[q] = aq[q] = dd{0, 0};
    accumulate(ap, aq, 0, zp0, vq0, zq0);
#pragma unroll 1
    for (int t = 1; t <= n; ++t) {
      dd zp, vq, zq;
      rowvz(t - 1, zp, vq, zq);
      accumulate(ap, aq, t, zp, vq, zq);
      if (t == n) {
        zp0 = zp;
        vq0 = vq;
        zq0 = zq;
      }
    }
    __syncthreads();
    if (e > e0) {
      dd P = carp, Q = carq;
      dd_axpy(P, 1.0, ap[0]);
      dd_axpy(Q, 1.0, aq[0]);
      put((int64_t)n * e - 1, P, Q);
    }
    if (e < e1) {
#pragma unroll
      for (int t = 1; t < n; ++t) put((int64_t)n * e + t - 1, ap[t], aq[t]);
    }
    carp = ap[n];
    carq = aq[n];
  }
}

template <int NORD, bool DD>
__global__ __launch_bounds__(64, DD ? 2 : 4) void resid3p_kernel(Resid2Args a) {
  resid3p_body<NORD, DD>(a, blockIdx.x, gridDim.x);
}

template <int NORD, bool DD>
__global__ __launch_bounds__(64, DD ? 2 : 4) void resid3p_kernel_grouped(const Resid2Args* __restrict__ jobs,
                                                                         const int* __restrict__ job_of,
                                                                         const int* __restrict__ start) {
  const int j = __builtin_amdgcn_readfirstlane(job_of[blockIdx.x]);
  const int b0 = __builtin_amdgcn_readfirstlane(start[j]), b1 = __builtin_amdgcn_readfirstlane(start[j + 1]);
  resid3p_body<NORD, DD>(jobs[j], (int)blockIdx.x - b0, b1 - b0);
}

template <int NORD, bool DD>
__global__ __launch_bounds__(64, DD ? 3 : 4) void resid2_kernel(Resid2Args a) {
  resid2_body<NORD, DD>(a, blockIdx.x, gridDim.x);
}

// Grouped launch: block b runs tile b - start[j] of job j = job_of[b].
template <int NORD, bool DD>
__global__ __launch_bounds__(64, DD ? 3 : 4) void resid2_kernel_grouped(const Resid2Args* __restrict__ jobs,
                                                                   const int* __restrict__ job_of,
                                                                   const int* __restrict__ start) {
  const int j = __builtin_amdgcn_readfirstlane(job_of[blockIdx.x]);
  const int b0 = __builtin_amdgcn_readfirstlane(start[j]), b1 = __builtin_amdgcn_readfirstlane(start[j + 1]);
  resid2_body<NORD, DD>(jobs[j], (int)blockIdx.x - b0, b1 - b0);
}

template <int NORD, bool LO, bool DD>
__global__ __launch_bounds__(kThreads) void apply_kernel(ApplyArgs a) {
  apply_body<NORD, LO, DD>(a, blockIdx.x, gridDim.x);
}

// Grouped launch: block b runs tile b - start[j] of job j = job_of[b].
template <int NORD, bool LO, bool DD>
__global__ __launch_bounds__(kThreads) void apply_kernel_grouped(const ApplyArgs* __restrict__ jobs,
                                                                 const int* __restrict__ job_of,
                                                                 const int* __restrict__ start) {
  const int j = __builtin_amdgcn_readfirstlane(job_of[blockIdx.x]);
  const int b0 = __builtin_amdgcn_readfirstlane(start[j]), b1 = __builtin_amdgcn_readfirstlane(start[j + 1]);
  apply_body<NORD, LO, DD>(jobs[j], (int)blockIdx.x - b0, b1 - b0);
}

// ---------------------------------------------------------------------------
// Refinement bookkeeping.  stats layout (doubles): [0] iterations applied,
// [1] state: 0 running (or no refinement), 1 tolerance reached, -1 a
// non-finite correction or iterate, -2 a correction no smaller than the one
// before; [2 + i] relative correction of iteration i.  The flag stops every
// later launch of the solve when it is nonzero: 1 is set here, bit 2 by an
// output pass that wrote a NaN or Inf.
__device__ __forceinline__ void reset_body(int* flag, double* stats, int nstats) {
  int i = threadIdx.x;
  if (i == 0) *flag = 0;
  for (int j = i; j < nstats; j += blockDim.x) stats[j] = 0;
}

__global__ void reset_kernel(int* flag, double* stats, int nstats) { reset_body(flag, stats, nstats); }

// count consecutive flags and statistics blocks (right-hand sides) at once
__global__ void reset_many_kernel(int* flags, double* stats, int nstats, int count) {
  for (int r = blockIdx.x; r < count; r += gridDim.x) reset_body(flags + r, stats + (size_t)r * nstats, nstats);
}

__global__ void reset_kernel_grouped(const ResetJob* __restrict__ jobs) {
  const ResetJob& j = jobs[blockIdx.x];
  reset_body(j.flag, j.stats, j.nstats);
}

__device__ __forceinline__ void reduce_body(const double* partials, int nparts, int iter, double tol, int* flag,
                                            double* stats) {
  if (*flag) return;
  __shared__ double r0[kThreads], r1[kThreads];
  int tid = threadIdx.x;
  double a = 0, b = 0;
  for (int i = tid; i < nparts; i += kThreads) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  r0[tid] = a;
  r1[tid] = b;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      r0[tid] += r0[tid + s];
      r1[tid] += r1[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    // ||c||^2 and ||u||^2 of this step; a NaN or Inf in either (non-finite
    // data, a float32 overflow) makes rel NaN, a correction of a zero iterate
    // makes it +Inf, and neither counts as converged
    const double c2 = r0[0], u2 = r1[0];
    double rel;
    if (!(c2 - c2 == 0.0) || !(u2 - u2 == 0.0))
      rel = __builtin_nan("");
    else if (u2 > 0)
      rel = sqrt(c2 / u2);
    else
      rel = c2 > 0 ? __builtin_inf() : 0.0;
    stats[2 + iter] = rel;
    stats[0] = iter;
    if (!(rel - rel == 0.0)) {
      stats[1] = -1;
      *flag = 1;
    } else if (iter > 0 && rel <= tol) {
      stats[1] = 1;
      *flag = 1;
    } else if (iter >= 2 && !(rel < stats[1 + iter])) {
      // stationary refinement contracts every step; a correction that does
      // not shrink means round-off level or divergence: stop
      stats[1] = -2;
      *flag = 1;
    }
  }
}

__global__ void reduce_kernel(const double* partials, int nparts, int iter, double tol, int* flag,
                              double* stats) {
  reduce_body(partials, nparts, iter, tol, flag, stats);
}

__global__ void reduce_kernel_grouped(const ReduceJob* __restrict__ jobs) {
  const ReduceJob& j = jobs[blockIdx.x];
  reduce_body(j.partials, j.nparts, j.iter, j.tol, j.flag, j.stats);
}

// ---------------------------------------------------------------------------
// Out-of-place transpose of a batch of R x C matrices: out[b][c][r] = in[b][r][c].
// 64 x 64 tiles through LDS (one padding column against bank conflicts);
// every global access is a contiguous 256-thread segment.
template <typename T>
__device__ __forceinline__ void transpose_body(const T* __restrict__ in, T* __restrict__ out, int64_t R,
                                               int64_t C, int64_t ntr, int64_t ntc, int blk, int nblk) {
  constexpr int TS = 64;
  __shared__ T tile[TS][TS + 1];
  const int64_t bid = xcd_remap(blk, nblk);
  const int64_t per = ntr * ntc;
  const int64_t b = bid / per;
  const int64_t rem = bid - b * per;
  const int64_t tr = rem / ntc, tc = rem - tr * ntc;
  const int64_t r0 = tr * TS, c0 = tc * TS;
  const T* src = in + b * R * C;
  T* dst = out + b * R * C;
  const int tx = threadIdx.x & (TS - 1), ty = threadIdx.x >> 6;  // 64 x 4
#pragma unroll
  for (int i = 0; i < TS; i += 4) {
    int64_t r = r0 + ty + i, c = c0 + tx;
    if (r < R && c < C) tile[ty + i][tx] = src[r * C + c];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TS; i += 4) {
    int64_t c = c0 + ty + i, r = r0 + tx;
    if (r < R && c < C) dst[c * R + r] = tile[tx][ty + i];
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void transpose_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                             int64_t R, int64_t C, int64_t ntr, int64_t ntc) {
  transpose_body<T>(in, out, R, C, ntr, ntc, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void transpose_kernel_grouped(const TransposeJob* __restrict__ jobs,
                                                                     const int* __restrict__ job_of,
                                                                     const int* __restrict__ start) {
  const int j = __builtin_amdgcn_readfirstlane(job_of[blockIdx.x]);
  const int b0 = __builtin_amdgcn_readfirstlane(start[j]), b1 = __builtin_amdgcn_readfirstlane(start[j + 1]);
  const TransposeJob& t = jobs[j];
  transpose_body<T>((const T*)t.in, (T*)t.out, t.R, t.C, t.ntr, t.ntc, (int)blockIdx.x - b0, b1 - b0);
}

template <typename T>
hipError_t launch_transpose_grouped(const GroupedOps& g, hipStream_t s) {
  hipLaunchKernelGGL((transpose_kernel_grouped<T>), dim3(g.nblocks), dim3(kThreads), 0, s,
                     (const TransposeJob*)g.jobs, g.job_of, g.start);
  return hipGetLastError();
}
template hipError_t launch_transpose_grouped<float>(const GroupedOps&, hipStream_t);
template hipError_t launch_transpose_grouped<double>(const GroupedOps&, hipStream_t);

hipError_t launch_apply_grouped(int n, bool lo, bool dd, const GroupedOps& g, hipStream_t s) {
  const ApplyArgs* jobs = (const ApplyArgs*)g.jobs;
  switch (n) {
#define FFTFEM_CASE(N)                                                                                       \
  case N:                                                                                                    \
    if (!dd)                                                                                                 \
      hipLaunchKernelGGL((apply_kernel_grouped<N, false, false>), dim3(g.nblocks), dim3(kThreads), g.lds, s, \
                         jobs, g.job_of, g.start);                                                           \
    else if (lo)                                                                                             \
      hipLaunchKernelGGL((apply_kernel_grouped<N, true, true>), dim3(g.nblocks), dim3(kThreads), g.lds, s,   \
                         jobs, g.job_of, g.start);                                                           \
    else                                                                                                     \
      hipLaunchKernelGGL((apply_kernel_grouped<N, false, true>), dim3(g.nblocks), dim3(kThreads), g.lds, s,  \
                         jobs, g.job_of, g.start);                                                           \
    return hipGetLastError();
    FFTFEM_CASE(1)
    FFTFEM_CASE(2)
    FFTFEM_CASE(3)
    FFTFEM_CASE(4)
    FFTFEM_CASE(5)
    FFTFEM_CASE(6)
    FFTFEM_CASE(7)
    FFTFEM_CASE(8)
    FFTFEM_CASE(9)
#undef FFTFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_reset_grouped(const ResetJob* jobs, int njobs, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel_grouped, dim3(njobs), dim3(64), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_reduce_grouped(const ReduceJob* jobs, int njobs, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel_grouped, dim3(njobs), dim3(kThreads), 0, s, jobs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transpose(const T* in, T* out, int64_t batch, int64_t R, int64_t C, hipStream_t s) {
  int64_t ntr = (R + 63) / 64, ntc = (C + 63) / 64;
  int64_t nb = batch * ntr * ntc;
  hipLaunchKernelGGL((transpose_kernel<T>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, R, C, ntr, ntc);
  return hipGetLastError();
}
template hipError_t launch_transpose<float>(const float*, float*, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<double>(const double*, double*, int64_t, int64_t, int64_t, hipStream_t);

hipError_t launch_apply(int n, const ApplyArgs& a, int nblocks, size_t lds, hipStream_t s) {
  const bool lo = a.in1[1] != nullptr;
  if (!a.dd && lo) return hipErrorInvalidValue;
  switch (n) {
#define FFTFEM_CASE(N)                                                                                \
  case N:                                                                                             \
    if (!a.dd)                                                                                        \
      hipLaunchKernelGGL((apply_kernel<N, false, false>), dim3(nblocks), dim3(kThreads), lds, s, a);  \
    else if (lo)                                                                                      \
      hipLaunchKernelGGL((apply_kernel<N, true, true>), dim3(nblocks), dim3(kThreads), lds, s, a);    \
    else                                                                                              \
      hipLaunchKernelGGL((apply_kernel<N, false, true>), dim3(nblocks), dim3(kThreads), lds, s, a);   \
    return hipGetLastError();
    FFTFEM_CASE(1)
    FFTFEM_CASE(2)
    FFTFEM_CASE(3)
    FFTFEM_CASE(4)
    FFTFEM_CASE(5)
    FFTFEM_CASE(6)
    FFTFEM_CASE(7)
    FFTFEM_CASE(8)
    FFTFEM_CASE(9)
#undef FFTFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_reset(int* flag, double* stats, int nstats, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, flag, stats, nstats);
  return hipGetLastError();
}

hipError_t launch_reset_many(int* flags, double* stats, int nstats, int count, hipStream_t s) {
  if (count < 1) return hipSuccess;
  const int nb = count < 4096 ? count : 4096;
  hipLaunchKernelGGL(reset_many_kernel, dim3(nb), dim3(64), 0, s, flags, stats, nstats, count);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, int iter, double tol, int* flag,
                         double* stats, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, nparts, iter, tol,
                     flag, stats);
  return hipGetLastError();
}


hipError_t launch_resid2_grouped(int n, bool dd, const GroupedOps& g, hipStream_t s) {
  const Resid2Args* jobs = (const Resid2Args*)g.jobs;
  switch (n) {
#define FFTFEM_CASE(N)                                                                                      \
  case N:                                                                                                   \
    if (dd)                                                                                                 \
      hipLaunchKernelGGL((resid2_kernel_grouped<N, true>), dim3(g.nblocks), dim3(64), 0, s, jobs,      \
                         g.job_of, g.start);                                                                \
    else                                                                                                    \
      hipLaunchKernelGGL((resid2_kernel_grouped<N, false>), dim3(g.nblocks), dim3(64), 0, s, jobs,     \
                         g.job_of, g.start);                                                                \
    return hipGetLastError();
    FFTFEM_CASE(1)
    FFTFEM_CASE(2)
    FFTFEM_CASE(3)
    FFTFEM_CASE(4)
    FFTFEM_CASE(5)
    FFTFEM_CASE(6)
    FFTFEM_CASE(7)
    FFTFEM_CASE(8)
    FFTFEM_CASE(9)
#undef FFTFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

int64_t resid2_blocks(const Resid2Args& a) {
  return (a.planes > 0 ? a.planes : 1) * ((a.M1 + 63) / 64) * ((a.K0 + a.E - 1) / a.E);
}

hipError_t launch_resid3p(int n, bool dd, const Resid2Args& a, hipStream_t s) {
  if (a.K0 < 1 || a.E < 1 || a.M1 < 1 || a.planes < 1) return hipErrorInvalidValue;
  const int64_t nb = resid2_blocks(a);
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  switch (n) {
#define FFTFEM_CASE(N)                                                                              \
  case N:                                                                                           \
    if (dd)                                                                                         \
      hipLaunchKernelGGL((resid3p_kernel<N, true>), dim3((unsigned)nb), dim3(64), 0, s, a);        \
    else                                                                                            \
      hipLaunchKernelGGL((resid3p_kernel<N, false>), dim3((unsigned)nb), dim3(64), 0, s, a);       \
    return hipGetLastError();
    FFTFEM_CASE(1)
    FFTFEM_CASE(2)
    FFTFEM_CASE(3)
    FFTFEM_CASE(4)
    FFTFEM_CASE(5)
    FFTFEM_CASE(6)
    FFTFEM_CASE(7)
    FFTFEM_CASE(8)
    FFTFEM_CASE(9)
#undef FFTFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_resid3p_grouped(int n, bool dd, const GroupedOps& g, hipStream_t s) {
  const Resid2Args* jobs = (const Resid2Args*)g.jobs;
  switch (n) {
#define FFTFEM_CASE(N)                                                                                       \
  case N:                                                                                                    \
    if (dd)                                                                                                  \
      hipLaunchKernelGGL((resid3p_kernel_grouped<N, true>), dim3(g.nblocks), dim3(64), 0, s, jobs, g.job_of, \
                         g.start);                                                                           \
    else                                                                                                     \
      hipLaunchKernelGGL((resid3p_kernel_grouped<N, false>), dim3(g.nblocks), dim3(64), 0, s, jobs,          \
                         g.job_of, g.start);                                                                 \
    return hipGetLastError();
    FFTFEM_CASE(1)
    FFTFEM_CASE(2)
    FFTFEM_CASE(3)
    FFTFEM_CASE(4)
    FFTFEM_CASE(5)
    FFTFEM_CASE(6)
    FFTFEM_CASE(7)
    FFTFEM_CASE(8)
    FFTFEM_CASE(9)
#undef FFTFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_resid2(int n, bool dd, const Resid2Args& a, hipStream_t s) {
  if (a.K0 < 1 || a.E < 1 || a.M1 < 1) return hipErrorInvalidValue;
  const int64_t ncb = (a.M1 + 63) / 64, nch = (a.K0 + a.E - 1) / a.E;
  const int64_t nb = ncb * nch;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  switch (n) {
#define FFTFEM_CASE(N)                                                                              \
  case N:                                                                                           \
    if (dd)                                                                                         \
      hipLaunchKernelGGL((resid2_kernel<N, true>), dim3((unsigned)nb), dim3(64), 0, s, a);     \
    else                                                                                            \
      hipLaunchKernelGGL((resid2_kernel<N, false>), dim3((unsigned)nb), dim3(64), 0, s, a);    \
    return hipGetLastError();
    FFTFEM_CASE(1)
    FFTFEM_CASE(2)
    FFTFEM_CASE(3)
    FFTFEM_CASE(4)
    FFTFEM_CASE(5)
    FFTFEM_CASE(6)
    FFTFEM_CASE(7)
    FFTFEM_CASE(8)
    FFTFEM_CASE(9)
#undef FFTFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fftfem
