// The banded solve along an axis of algorithm (b) of Sect. 4 (gfx950).
//
// After the FC_n transforms along every other axis, each line along axis 0
// carries one shifted 1D system (coef A + sigma C) x = y of the assembled
// nth-order stiffness A and mass C (Sect. 2), sigma = react + the other axes'
// terms coef_d lambda_d.  Its matrix couples the n - 1 bubble unknowns of an
// element only to each other and to the element's two end nodes, so the
// bubbles are eliminated element by element (static condensation) and what
// remains is a tridiagonal system in the K - 1 mesh nodes.  The bubble block
// coef A_BB + sigma C_BB is the same in every element; in the
// mass-orthonormal eigenbasis V of the pencil (A_BB, C_BB) (eigenvalues
// lam) it is diagonal, coef lam_m + sigma, so the elimination needs n - 1
// reciprocals per line and two n - 1 by n - 1 products per element.
//
// With t = V^T y_B, z_m = t_m / (coef lam_m + sigma) and h_L, h_R the mode
// couplings to the left and right node, the condensed element matrix is
// [[a, b], [b, a]] (the element is mirror symmetric), and element e adds
// -h_L . z to the right-hand side of its left node and -h_R . z to its right
// node.  The node system has diagonal 2a and off-diagonal b = -s; written as
// s tridiag(-1, 2, -1) + d I with d = 2 (a + b), both s and d are formed
// without cancellation (s from the 113-bit condensed stiffness a0 minus a
// term proportional to sigma, d proportional to sigma), and the
// elimination carries e_j = den_j - s, which obeys
// e_j = d + s e_{j-1} / den_{j-1} (e_1 = s + d), a sum of non-negative terms.
// The small eigenvalues of the node system, 2 s (1 - cos(pi k / K)) + d,
// then keep their relative accuracy; forming 2a and b directly would lose
// about (K / pi)^2 eps of it.  A backward sweep substitutes the nodes and
// recovers the bubbles x_B = V (z - (h_L x_L + h_R x_R) / (coef lam + sigma)).
//
// Element i of line l is at i * nlines + l, so threads taking consecutive
// lines read and write consecutive values.  Three forms follow: one sweep
// per line (band_kernel), three element-parallel kernels for few long lines,
// and one LDS-tiled kernel for short lines.
#include "device_common.h"
#include "launch.h"

namespace fftfem {

// Per-line constants: r_m = 1 / (coef lam_m + sigma), the node couplings
// h_L, h_R of the bubble modes, and the node system's s and d.
struct BandLine {
  double r[kMaxLineOrder], hL[kMaxLineOrder], hR[kMaxLineOrder];
  double s, d;
};

// sigma of a line: react + the other axes' terms.
__device__ __forceinline__ double band_sigma(const BandArgs& a, int64_t line) {
  double sg = a.react;
  for (int e = 0; e < a.nother; ++e) sg += a.mu_o[e][(line / a.so[e]) % a.Mo[e]];
  return sg;
}

template <int NORD>
__device__ __forceinline__ void band_line(const BandArgs& a, int64_t line, BandLine& L) {
  constexpr int nb = NORD - 1;
  constexpr int oL = nb * nb, oAL = oL + nb, oCL = oAL + nb, oAR = oCL + nb, oCR = oAR + nb, otL = oCR + nb,
                otX = otL + nb, oN = otX + nb;
  const double* __restrict__ tb = a.tab;
  const double sg = band_sigma(a, line);
  const double cf = a.coef;
  // a = cf a0 + sg PL, b = -cf a0 + sg PX
  double PL = tb[oN + 0], PX = tb[oN + 1];
#pragma unroll
  for (int m = 0; m < nb; ++m) {
    const double r = 1.0 / (cf * tb[oL + m] + sg);
    const double cl = tb[oCL + m], cr = tb[oCR + m];
    L.r[m] = r;
    L.hL[m] = cf * tb[oAL + m] + sg * cl;
    L.hR[m] = cf * tb[oAR + m] + sg * cr;
    PL -= r * (cf * tb[otL + m] + sg * cl * cl);
    PX -= r * (cf * tb[otX + m] + sg * cl * cr);
  }
  L.s = cf * tb[oN + 2] - sg * PX;
  L.d = 2.0 * sg * (PL + PX);
}

// z = diag(r) V^T y_B of one element (bubble values at p[m S]).
template <int NORD>
__device__ __forceinline__ void band_z(const double* __restrict__ tb, const BandLine& L, const double* p,
                                       int64_t S, double* z) {
  constexpr int nb = NORD - 1, NB = nb > 0 ? nb : 1;
  double y[NB];
#pragma unroll
  for (int i = 0; i < nb; ++i) y[i] = p[(int64_t)i * S];
#pragma unroll
  for (int m = 0; m < nb; ++m) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < nb; ++i) t += tb[i * nb + m] * y[i];
    z[m] = L.r[m] * t;
  }
}

// One thread per line; the next element's values are loaded before the
// current one is processed.
template <int NORD>
__global__ __launch_bounds__(kBlock) void band_kernel(BandArgs a) {
  constexpr int nb = NORD - 1, NB = nb > 0 ? nb : 1;
  const int64_t line = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (line >= a.nlines) return;
  const double* __restrict__ tb = a.tab;
  BandLine L;
  band_line<NORD>(a, line, L);
  const double sn = L.s, dn = L.d;
  const int64_t S = a.nlines;
  const int K = a.K;
  const double* in = a.in + line;
  double* out = a.out + line;
  double* cp = a.cp + line;

  // forward: condensation and elimination of the node system
  double cur[NORD], nxt[NORD];
  cur[0] = 0.0;
#pragma unroll
  for (int m = 0; m < nb; ++m) cur[1 + m] = in[(int64_t)m * S];
  double carry = 0.0, ex = 0.0, rho = 0.0, gprev = 0.0;
  for (int e = 0; e < K; ++e) {
    if (e + 1 < K) {
      const int64_t b1 = (int64_t)(e + 1) * NORD;
      nxt[0] = in[(b1 - 1) * S];
#pragma unroll
      for (int m = 0; m < nb; ++m) nxt[1 + m] = in[(b1 + m) * S];
    }
    const int64_t b0 = (int64_t)e * NORD;
    double z[NB];
    double pL = 0.0, pR = 0.0;
#pragma unroll
    for (int m = 0; m < nb; ++m) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < nb; ++i) t += tb[i * nb + m] * cur[1 + i];
      z[m] = L.r[m] * t;
      pL += L.hL[m] * z[m];
      pR += L.hR[m] * z[m];
    }
#pragma unroll
    for (int m = 0; m < nb; ++m) out[(b0 + m) * S] = z[m];
    if (e > 0) {
      const double g = cur[0] + carry - pL;
      ex = e == 1 ? sn + dn : dn + rho * ex;
      const double inv = 1.0 / (sn + ex);
      rho = sn * inv;
      gprev = (g + sn * gprev) * inv;
      cp[(int64_t)(e - 1) * S] = rho;
      out[(b0 - 1) * S] = gprev;
    }
    carry = -pR;
#pragma unroll
    for (int m = 0; m < NORD; ++m) cur[m] = nxt[m];
  }

  // backward: node substitution x_j = g'_j + rho_j x_{j+1}, bubble recovery
  {
    const int64_t b0 = (int64_t)(K - 1) * NORD;
    cur[0] = K > 1 ? out[(b0 - 1) * S] : 0.0;
    nxt[0] = K > 1 ? cp[(int64_t)(K - 2) * S] : 0.0;
#pragma unroll
    for (int m = 0; m < nb; ++m) cur[1 + m] = out[(b0 + m) * S];
  }
  double xR = 0.0, pc = nxt[0];
  for (int e = K - 1; e >= 0; --e) {
    double pn = 0.0;
    if (e > 0) {
      const int64_t b1 = (int64_t)(e - 1) * NORD;
      nxt[0] = e > 1 ? out[(b1 - 1) * S] : 0.0;
      pn = e > 1 ? cp[(int64_t)(e - 2) * S] : 0.0;
#pragma unroll
      for (int m = 0; m < nb; ++m) nxt[1 + m] = out[(b1 + m) * S];
    }
    const int64_t b0 = (int64_t)e * NORD;
    double xL = 0.0;
    if (e > 0) {
      xL = cur[0] + pc * xR;
      out[(b0 - 1) * S] = xL;
    }
    double w[NB];
#pragma unroll
    for (int m = 0; m < nb; ++m) w[m] = cur[1 + m] - L.r[m] * (L.hL[m] * xL + L.hR[m] * xR);
#pragma unroll
    for (int i = 0; i < nb; ++i) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < nb; ++m) v += tb[i * nb + m] * w[m];
      out[(b0 + i) * S] = v;
    }
    xR = xL;
    pc = pn;
#pragma unroll
    for (int m = 0; m < NORD; ++m) cur[m] = nxt[m];
  }
}

// The same solve in three kernels, for grids with too few lines to fill the
// chip with one thread per line (2D: M_2 lines).  The condensation and the
// bubble recovery are independent per element and run one thread per
// (line, group of kBandEPTc or kBandEPTb elements); only the node elimination, K - 1
// values per line, stays sequential.
//   1. cond: y (in) -> the condensed node right-hand sides g in w's node
//      slots (a thread recomputes the last z of the element before its
//      group); w's bubble slots are not written;
//   2. nodes: the tridiagonal node system on w's node slots, forward
//      elimination (g' and the pivots as pairs into a compact array) and
//      back substitution: the node values x in w's node slots;
//   3. back: z again from y's bubble slots, x_B = V (z - (h_L x_L + h_R
//      x_R) / (.)) and the node values into out (out may be in: a thread
//      reads only the bubble slots of its own elements).
// Recomputing z (n - 1 squared multiply-adds per element) instead of
// storing it saves a write and a read of the bubble values: 8 (n - 1) / n
// bytes per value of the array each way.
// elements per thread of the condensation and of the bubble recovery
constexpr int kBandEPTc = 16, kBandEPTb = 4;

// The condensation and the bubble recovery keep of the per-line constants
// only r in registers.  The table (V and the coupling coefficients,
// (n - 1)(n + 4) values) is copied to LDS and read at each use through an
// offset the compiler cannot see (zero), one column of V at a time (a
// scheduling barrier after each): otherwise the scheduler loads the whole
// table into vector registers at once (three waves per SIMD instead of five).
// The couplings h_L, h_R are one multiply-add each where they are used.
template <int NORD>
__device__ __forceinline__ const double* band_table_lds(const BandArgs& a, double* stb) {
  constexpr int nb = NORD - 1, ntab = nb * (nb + 5);
  for (int i = threadIdx.x; i < ntab; i += blockDim.x) stb[i] = a.tab[i];
  __syncthreads();
  return stb;
}

__device__ __forceinline__ const double* band_opaque(const double* p) {
  int z0 = 0;
  asm volatile("" : "+v"(z0));
  return p + z0;
}

// h_L . z and h_R . z of one element, z = diag(r) V^T y (y: its bubble values).
template <int NORD>
__device__ __forceinline__ void band_couple(const double* stb, const double* r, double cf, double sg,
                                            const double* y, double& pL, double& pR) {
  constexpr int nb = NORD - 1;
  constexpr int oL = nb * nb, oAL = oL + nb, oCL = oAL + nb, oAR = oCL + nb, oCR = oAR + nb;
  const double* tb = band_opaque(stb);
  pL = pR = 0.0;
#pragma unroll
  for (int m = 0; m < nb; ++m) {
    double tm = 0.0;
#pragma unroll
    for (int i = 0; i < nb; ++i) tm += tb[i * nb + m] * y[i];
    const double z = r[m] * tm;
    pL += (cf * tb[oAL + m] + sg * tb[oCL + m]) * z;
    pR += (cf * tb[oAR + m] + sg * tb[oCR + m]) * z;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The bubble values of the element at p (stride S) and the node value before it.
template <int NORD>
__device__ __forceinline__ void band_load_elem(const double* p, int64_t S, bool node, double* y, double& yn) {
  constexpr int nb = NORD - 1;
#pragma unroll
  for (int i = 0; i < nb; ++i) y[i] = p[(int64_t)i * S];
  yn = node ? p[-S] : 0.0;
}

template <int NORD>
__global__ __launch_bounds__(kBlock) void band_cond_kernel(BandArgs a) {
  constexpr int nb = NORD - 1, NB = nb > 0 ? nb : 1;
  __shared__ double stb_[nb * (nb + 5) > 0 ? nb * (nb + 5) : 1];
  const double* stb = band_table_lds<NORD>(a, stb_);
  const int64_t ng = (a.K + kBandEPTc - 1) / kBandEPTc;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= a.nlines * ng) return;
  const int64_t line = t % a.nlines, grp = t / a.nlines;
  const int64_t S = a.nlines;
  const double sg = band_sigma(a, line), cf = a.coef;
  double r[NB];
#pragma unroll
  for (int m = 0; m < nb; ++m) r[m] = 1.0 / (cf * stb[nb * nb + m] + sg);
  const double* in = a.in + line;
  double* w = a.cp + line;
  const int e0 = (int)grp * kBandEPTc, e1 = min(a.K, e0 + kBandEPTc);
  double carry = 0.0;  // -h_R . z of the element before
  double y[NB], yn;
  if (e0 > 0 && nb > 0) {
    double pL, pR;
    band_load_elem<NORD>(in + (int64_t)(e0 - 1) * NORD * S, S, false, y, yn);
    band_couple<NORD>(stb, r, cf, sg, y, pL, pR);
    carry = -pR;
  }
  // the loads of element e + 1 are issued before the arithmetic of element e
  band_load_elem<NORD>(in + (int64_t)e0 * NORD * S, S, e0 > 0, y, yn);
  for (int e = e0; e < e1; ++e) {
    const int64_t b0 = (int64_t)e * NORD;
    double y1[NB] = {}, yn1 = 0.0;
    if (e + 1 < e1) band_load_elem<NORD>(in + (b0 + NORD) * S, S, true, y1, yn1);
    double pL = 0.0, pR = 0.0;
    if constexpr (nb > 0) band_couple<NORD>(stb, r, cf, sg, y, pL, pR);
    if (e > 0) w[(b0 - 1) * S] = yn + carry - pL;
    carry = -pR;
#pragma unroll
    for (int i = 0; i < nb; ++i) y[i] = y1[i];
    yn = yn1;
  }
}

// Node elimination by a twisted factorization, two lanes per line: lane
// t < 32 eliminates nodes 1 .. m - 1 downward and lane t + 32 nodes
// K - 1 .. m + 1 upward (m = K / 2), each with the recurrence of band_kernel
// (the node matrix reads the same from either end, so both halves have the
// same non-negative pivot terms).  The middle node then has the equation
//   (d + rho_{m-1} e_{m-1} + rho'_{m+1} e'_{m+1}) x_m = g_m + s g'_{m-1} + s g''_{m+1},
// again a sum of non-negative terms in the pivot; both lanes form it in the
// same order, and each substitutes back outward from x_m.  Each lane's chain
// of divisions is half a line long, and the grid has twice as many waves.
// The sweeps load kBandNF right-hand sides, then kBandNB pairs (g', pivot),
// one block ahead.  One-wave workgroups spread the few waves (2D: M_2 / 32)
// over as many CUs as possible: each wave's sweeps are bound by its own
// memory latency.
constexpr int kBandNF = 24, kBandNB = 24, kBandNodesBlock = 64, kBandNodesLines = 32;

template <int NORD>
__global__ __launch_bounds__(kBandNodesBlock) void band_nodes_kernel(BandArgs a) {
  const int half = threadIdx.x >> 5;  // 0: top half, 1: bottom half
  const int64_t line = (int64_t)blockIdx.x * kBandNodesLines + (threadIdx.x & 31);
  const bool live = line < a.nlines;  // every lane takes part in the exchange
  const int64_t S = a.nlines;
  BandLine L;
  band_line<NORD>(a, live ? line : 0, L);
  const double sn = L.s, dn = L.d;
  const int nn = a.K - 1;  // node j (1..K-1) at slot j NORD - 1 of w
  const int m = (nn + 1) >> 1;
  const int cnt = half ? nn - m : m - 1;  // nodes this lane eliminates
  const int jf = half ? nn : 1, dj = half ? -1 : 1;
  const int64_t st = (int64_t)NORD * S;
  double* wn = a.cp + (live ? line : 0) + (int64_t)(NORD - 1) * S;  // node 1
  // (g'_j, pivot_j) of node j at pair (j - 1) S + line: one 16-byte access per step
  double2* pr = reinterpret_cast<double2*>(a.pr) + (live ? line : 0);
  auto slot = [&](int i) { return (int64_t)(jf + dj * i - 1); };  // 0-based node of step i
  double ex = sn, rho = 1.0, gprev = 0.0;  // e_1 = d + 1 * s
  {
    double g[kBandNF], gn[kBandNF];
#pragma unroll
    for (int i = 0; i < kBandNF; ++i) g[i] = live && i < cnt ? wn[slot(i) * st] : 0.0;
    for (int i0 = 0; i0 < cnt; i0 += kBandNF) {
#pragma unroll
      for (int i = 0; i < kBandNF; ++i) {
        const int k = i0 + kBandNF + i;
        gn[i] = live && k < cnt ? wn[slot(k) * st] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < kBandNF; ++i)
        if (i0 + i < cnt) {
          ex = dn + rho * ex;
          const double inv = 1.0 / (sn + ex);
          rho = sn * inv;
          gprev = (g[i] + sn * gprev) * inv;
          if (live) pr[slot(i0 + i) * S] = make_double2(gprev, rho);
        }
#pragma unroll
      for (int i = 0; i < kBandNF; ++i) g[i] = gn[i];
    }
  }
  // the middle node: this half's terms and the other half's, summed top first
  const double gm = live ? wn[(int64_t)(m - 1) * st] : 0.0;
  const double cme = rho * ex, rme = sn * gprev;
  const double coth = __shfl_xor(cme, 32), roth = __shfl_xor(rme, 32);
  const double ctop = half ? coth : cme, cbot = half ? cme : coth;
  const double rtop = half ? roth : rme, rbot = half ? rme : roth;
  double x = (gm + rtop + rbot) / (dn + ctop + cbot);
  if (live && half == 0) wn[(int64_t)(m - 1) * st] = x;
  // back substitution outward: x_j = g'_j + pivot_j x_(j toward m), one block ahead
  double2 q[kBandNB], qn[kBandNB];
#pragma unroll
  for (int i = 0; i < kBandNB; ++i) {
    const int k = cnt - 1 - i;
    q[i] = live && k >= 0 ? pr[slot(k) * S] : make_double2(0.0, 0.0);
  }
  for (int k0 = cnt - 1; k0 >= 0; k0 -= kBandNB) {
#pragma unroll
    for (int i = 0; i < kBandNB; ++i) {
      const int k = k0 - kBandNB - i;
      qn[i] = live && k >= 0 ? pr[slot(k) * S] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < kBandNB; ++i)
      if (k0 - i >= 0) {
        x = q[i].x + q[i].y * x;
        if (live) wn[slot(k0 - i) * st] = x;
      }
#pragma unroll
    for (int i = 0; i < kBandNB; ++i) q[i] = qn[i];
  }
}

template <int NORD>
__global__ __launch_bounds__(kBlock) void band_back_kernel(BandArgs a) {
  constexpr int nb = NORD - 1, NB = nb > 0 ? nb : 1;
  constexpr int oL = nb * nb, oAL = oL + nb, oCL = oAL + nb, oAR = oCL + nb, oCR = oAR + nb;
  __shared__ double stb_[nb * (nb + 5) > 0 ? nb * (nb + 5) : 1];
  const double* stb = band_table_lds<NORD>(a, stb_);
  const int64_t ng = (a.K + kBandEPTb - 1) / kBandEPTb;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= a.nlines * ng) return;
  const int64_t line = t % a.nlines, grp = t / a.nlines;
  const int64_t S = a.nlines;
  const double sg = band_sigma(a, line), cf = a.coef;
  double r[NB];
#pragma unroll
  for (int m = 0; m < nb; ++m) r[m] = 1.0 / (cf * stb[oL + m] + sg);
  const double* w = a.cp + line;
  const double* in = a.in + line;
  double* out = a.out + line;
  const int e0 = (int)grp * kBandEPTb, e1 = min(a.K, e0 + kBandEPTb);
  double xL = e0 > 0 ? w[((int64_t)e0 * NORD - 1) * S] : 0.0;
  for (int e = e0; e < e1; ++e) {
    const int64_t b0 = (int64_t)e * NORD;
    const double xR = e + 1 < a.K ? w[(b0 + NORD - 1) * S] : 0.0;
    if (e > 0) out[(b0 - 1) * S] = xL;
    if constexpr (nb > 0) {
      const double* tb = band_opaque(stb);
      double y[NB], v[NB];
#pragma unroll
      for (int i = 0; i < nb; ++i) y[i] = in[(b0 + i) * S];
#pragma unroll
      for (int m = 0; m < nb; ++m) {
        double tm = 0.0;
#pragma unroll
        for (int i = 0; i < nb; ++i) tm += tb[i * nb + m] * y[i];
        const double hL = cf * tb[oAL + m] + sg * tb[oCL + m], hR = cf * tb[oAR + m] + sg * tb[oCR + m];
        v[m] = r[m] * tm - r[m] * (hL * xL + hR * xR);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int i = 0; i < nb; ++i) {
        double x = 0.0;
#pragma unroll
        for (int m = 0; m < nb; ++m) x += tb[i * nb + m] * v[m];
        out[(b0 + i) * S] = x;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    xL = xR;
  }
}

// The same solve in one kernel for short lines (K G <= 1024): a workgroup
// of 256 threads takes G adjacent lines; thread t works on line t mod G and
// on elements t / G + (256 / G) i.  The condensation keeps z in registers and leaves the
// node couplings h_L . z, h_R . z and the node loads in LDS; G threads then
// eliminate the node systems from LDS, and every thread recovers its
// elements' bubbles and nodes and stores them.  y is read once and x written
// once, with no work array.
constexpr int kBandTileBlock = 256;  // threads per workgroup of the tiled form
constexpr int kBandTileEPT = 4;      // elements per thread: K G <= kBandTileBlock kBandTileEPT

// 1 / x on the node elimination's dependency chain (x > 0 normal).
__device__ __forceinline__ double band_inv(double x) { return 1.0 / x; }

// Workgroups are dispatched to the 8 XCDs in turn (workgroup i to XCD i mod
// 8), and each XCD has its own L2.  A tile's rows are 128-byte segments that
// start anywhere in a cache line (the line count is usually odd), so
// neighbouring tiles share cache lines; mapping consecutive workgroups of one
// XCD to consecutive tiles keeps those shared lines in one L2.  A bijection
// of [0, nblk): XCD x takes tiles [x q + min(x, r), ...) with q = nblk / 8,
// r = nblk mod 8.
__device__ __forceinline__ unsigned band_tile_of(unsigned b, unsigned nblk) {
  const unsigned q = nblk / 8, r = nblk % 8, x = b % 8, slot = b / 8;
  return x * q + min(x, r) + slot;
}

template <int NORD, int G>
__global__ __launch_bounds__(kBandTileBlock, 3) void band_tile_kernel(BandArgs a) {
  constexpr int nb = NORD - 1, NB = nb > 0 ? nb : 1;
  constexpr int oL = nb * nb, oAL = oL + nb, oCL = oAL + nb, oAR = oCL + nb, oCR = oAR + nb;
  constexpr int STEP = kBandTileBlock / G;
  extern __shared__ double band_lds[];
  __shared__ double stb_[nb * (nb + 5) > 0 ? nb * (nb + 5) : 1];
  const double* stb = band_table_lds<NORD>(a, stb_);
  const int K = a.K;
  double* pl = band_lds;                    // [K][G]: h_L . z of element e
  double* pq = pl + (size_t)K * G;          // [K][G]: h_R . z
  double* yn = pq + (size_t)K * G;          // [K][G]: load of the left node of e; then g'; then x
  double* pv = yn + (size_t)K * G;          // [K][G]: pivots
  const int tid = threadIdx.x, l = tid % G, es = tid / G;
  const int64_t line = (int64_t)band_tile_of(blockIdx.x, gridDim.x) * G + l;
  const bool live = line < a.nlines;
  const int64_t S = a.nlines;
  const double sg = band_sigma(a, live ? line : 0), cf = a.coef;
  double r[NB];
#pragma unroll
  for (int m = 0; m < nb; ++m) r[m] = 1.0 / (cf * stb[oL + m] + sg);
  const double* in = a.in + (live ? line : 0);
  double* out = a.out + (live ? line : 0);
  // z of this thread's elements stay in registers across the node solve;
  // the table is read from LDS one column at a time (as in band_couple)
  double zr[kBandTileEPT][NB];
#pragma unroll
  for (int i = 0; i < kBandTileEPT; ++i) {
    const int e = es + STEP * i;
    if (e < K && live) {
      const int64_t b0 = (int64_t)e * NORD;
      double pL = 0.0, pR = 0.0;
      if constexpr (nb > 0) {
        const double* tb = band_opaque(stb);
        double y[NB];
#pragma unroll
        for (int j = 0; j < nb; ++j) y[j] = in[(b0 + j) * S];
#pragma unroll
        for (int m = 0; m < nb; ++m) {
          double tm = 0.0;
#pragma unroll
          for (int j = 0; j < nb; ++j) tm += tb[j * nb + m] * y[j];
          zr[i][m] = r[m] * tm;
          pL += (cf * tb[oAL + m] + sg * tb[oCL + m]) * zr[i][m];
          pR += (cf * tb[oAR + m] + sg * tb[oCR + m]) * zr[i][m];
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      pl[e * G + l] = pL;
      pq[e * G + l] = pR;
      yn[e * G + l] = e > 0 ? in[(b0 - 1) * S] : 0.0;
    }
  }
  __syncthreads();
  if (tid < G && live) {
    // s and d of the node system as in band_line, from the r already held
    constexpr int otL = oCR + nb, otX = otL + nb, oN = otX + nb;
    const double* __restrict__ tb = a.tab;
    double PL = tb[oN + 0], PX = tb[oN + 1];
#pragma unroll
    for (int m = 0; m < nb; ++m) {
      const double cl = tb[oCL + m], cr = tb[oCR + m];
      PL -= r[m] * (cf * tb[otL + m] + sg * cl * cl);
      PX -= r[m] * (cf * tb[otX + m] + sg * cl * cr);
    }
    const double sn = cf * tb[oN + 2] - sg * PX, dn = 2.0 * sg * (PL + PX);
    double ex = sn, rho = 1.0, gprev = 0.0;
    for (int j = 1; j < K; ++j) {
      const double g = yn[j * G + l] - pq[(j - 1) * G + l] - pl[j * G + l];
      ex = dn + rho * ex;
      const double inv = band_inv(sn + ex);
      rho = sn * inv;
      gprev = (g + sn * gprev) * inv;
      pv[j * G + l] = rho;
      yn[j * G + l] = gprev;
    }
    double x = 0.0;
    for (int j = K - 1; j >= 1; --j) {
      x = yn[j * G + l] + pv[j * G + l] * x;
      yn[j * G + l] = x;
    }
    yn[l] = 0.0;  // element 0 has no left node
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBandTileEPT; ++i) {
    const int e = es + STEP * i;
    if (e < K && live) {
      const int64_t b0 = (int64_t)e * NORD;
      const double xL = yn[e * G + l];
      const double xR = e + 1 < K ? yn[(e + 1) * G + l] : 0.0;
      if (e > 0) out[(b0 - 1) * S] = xL;
      if constexpr (nb > 0) {
        const double* tb = band_opaque(stb);
        double w[NB];
#pragma unroll
        for (int m = 0; m < nb; ++m) {
          const double hL = cf * tb[oAL + m] + sg * tb[oCL + m], hR = cf * tb[oAR + m] + sg * tb[oCR + m];
          w[m] = zr[i][m] - r[m] * (hL * xL + hR * xR);
        }
#pragma unroll
        for (int j = 0; j < nb; ++j) {
          double x = 0.0;
#pragma unroll
          for (int m = 0; m < nb; ++m) x += tb[j * nb + m] * w[m];
          out[(b0 + j) * S] = x;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }
}

// Lines per workgroup of the tiled form for K elements (0: not applicable).
int band_tile_lines(int K) {
  if (16 * K <= kBandTileBlock * kBandTileEPT) return 16;
  if (8 * K <= kBandTileBlock * kBandTileEPT) return 8;
  return 0;
}

hipError_t launch_band_tile(int n, const BandArgs& a, hipStream_t s) {
  const int G = band_tile_lines(a.K);
  if (a.nlines < 1 || a.K < 1 || G == 0) return hipErrorInvalidValue;
  const int64_t nblk = (a.nlines + G - 1) / G;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = (size_t)4 * a.K * G * sizeof(double);
  switch (n * 100 + G) {
#define FFTFEM_CASE(N)                                                                                    \
  case N * 100 + 16:                                                                                      \
    hipLaunchKernelGGL((band_tile_kernel<N, 16>), dim3((unsigned)nblk), dim3(kBandTileBlock), lds, s, a);         \
    return hipGetLastError();                                                                             \
  case N * 100 + 8:                                                                                       \
    hipLaunchKernelGGL((band_tile_kernel<N, 8>), dim3((unsigned)nblk), dim3(kBandTileBlock), lds, s, a);          \
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

hipError_t launch_band_split(int n, int step, const BandArgs& a, hipStream_t s) {
  if (a.nlines < 1 || a.K < 1 || a.in == a.cp || a.out == a.cp || !a.pr || step < 0 || step > 2)
    return hipErrorInvalidValue;
  const int64_t ept = step == 0 ? kBandEPTc : kBandEPTb;
  const int64_t nb_el = (a.nlines * ((a.K + ept - 1) / ept) + kBlock - 1) / kBlock;
  const int64_t nb_ln = (a.nlines + kBandNodesLines - 1) / kBandNodesLines;
  if (nb_el > 0x7fffffff || nb_ln > 0x7fffffff) return hipErrorInvalidValue;
  if (step == 1 && a.K < 2) return hipSuccess;  // no nodes
  switch (n) {
#define FFTFEM_CASE(N)                                                                          \
  case N:                                                                                       \
    if (step == 0)                                                                              \
      hipLaunchKernelGGL((band_cond_kernel<N>), dim3((unsigned)nb_el), dim3(kBlock), 0, s, a);  \
    else if (step == 1)                                                                         \
      hipLaunchKernelGGL((band_nodes_kernel<N>), dim3((unsigned)nb_ln), dim3(kBandNodesBlock), 0, s, a); \
    else                                                                                        \
      hipLaunchKernelGGL((band_back_kernel<N>), dim3((unsigned)nb_el), dim3(kBlock), 0, s, a);  \
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

hipError_t launch_band(int n, const BandArgs& a, hipStream_t s) {
  if (a.nlines < 1 || a.K < 1) return hipErrorInvalidValue;
  const int64_t nblocks = (a.nlines + kBlock - 1) / kBlock;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  switch (n) {
#define FFTFEM_CASE(N)                                                                      \
  case N:                                                                                   \
    hipLaunchKernelGGL((band_kernel<N>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, a);   \
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
