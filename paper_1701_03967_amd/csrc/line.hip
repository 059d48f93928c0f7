// Line passes of the fast direct solver (gfx950).
//
// A line pass applies, along one axis of an N-D array, the direct FC_n
// transform (FWD), the inverse F_n transform (INV), or both with the
// pointwise division in between (MID), to a tile of G lines held in LDS
// (Sect. 3, Theorem 2; Sect. 4, algorithm (a)).  For one line of
// M = nK - 1 dofs:
//
//   load       coalesced global -> LDS (raw line layout); for strided axes
//              the G lines of a tile are adjacent in memory, so a row of the
//              tile is one contiguous segment;
//   gather     per element j: nodal value and the even/odd bubble channels
//              of Sect. 2 (registers), then written into the packed FFT
//              buffers: nodes as the odd extension of length 2K packed into K
//              complex values, bubble channels two per complex buffer in the
//              even/odd reordering that makes a DCT-II a K-point DFT (even
//              channels sign-alternated: their DST-II comes out of the same
//              DCT-II);
//   FFT        in-place Stockham, radix 16/8/4/2;
//   contract   per FFT index pair {k, K-k}: untangle the packed spectra into
//              the DST-I (nodes), DST-II (even) and DCT-II (odd) values of
//              frequencies k and K-k and apply the n x n table Q_k
//              (Q_k^T forward, Q_k inverse); k = 0 is the bubble-only block;
//   inverse    DST-I again (as a forward DFT, computed as a conjugated inverse
//              DFT), DCT-III/DST-III via the Hermitian pre-twiddle and an
//              unnormalized inverse DFT;
//   scatter    channels -> bubble vectors and nodes -> LDS -> coalesced store.
//
// Data move between phases through registers across barriers, so the raw
// line, the FFT buffers and the spectral output share one LDS region per
// line.  K and G are powers of two; all index arithmetic is shifts and masks.
#include "device_common.h"
#include "fft.h"
#include "launch.h"
#include "spectral.h"

namespace fftfem {

// Dynamic LDS of the line kernels.
extern __shared__ double2 fftfem_lds[];

#ifndef FFTFEM_MINW64
#define FFTFEM_MINW64 4
#endif
#ifndef FFTFEM_MINW32
#define FFTFEM_MINW32 4
#endif

// Threads per line-kernel workgroup: 512 for both precisions.  A float64
// line of K = 1024 elements fills half the LDS of a CU, so two tiles share
// a CU; at <= 128 VGPRs their 16 waves (four per SIMD) hide more latency
// than eight 256-thread waves with room for 256 VGPRs.  Every tile has
// G * K <= 1024 element tasks and G * K / 2 contraction tasks.
#ifndef FFTFEM_NT64
#define FFTFEM_NT64 512
#endif

// Value pairs per thread and sweep of the flat float64 tile loads: 10 x 512
// covers the largest tile (9 x 1024 - 1 values) in one sweep, so its loads
// take one memory round trip.
constexpr int kFlatPairs = 10;

template <typename T>
struct LineCfg {
  static constexpr int NT = sizeof(T) == 8 ? FFTFEM_NT64 : 512;
  static constexpr int TPT = 1024 / NT;  // element tasks per thread
  static constexpr int CPT = 512 / NT;   // contraction tasks per thread
  // minimum waves per SIMD the register allocation must allow: two 512-thread
  // tiles per CU (<= 128 VGPRs)
  static constexpr int MINW = sizeof(T) == 8 ? FFTFEM_MINW64 : FFTFEM_MINW32;
};

// Flat float64 tile I/O with the non-temporal hint: each value is read or
// written once, and the streaming lines should not evict the tables that
// every tile rereads (Q_k, twiddles) from L2.
typedef double fftfem_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const fftfem_d2v t = __builtin_nontemporal_load(reinterpret_cast<const fftfem_d2v*>(p));
  return double2{t.x, t.y};
}
__device__ __forceinline__ void st_stream(double2* p, double x, double y) {
  const fftfem_d2v t = {x, y};
  __builtin_nontemporal_store(t, reinterpret_cast<fftfem_d2v*>(p));
}

template <typename T>
__device__ __forceinline__ int64_t line_base(const LineArgs<T>& a, int64_t line) {
  int64_t outer = line / a.es;
  int64_t inner = line - outer * a.es;
  return outer * a.M * a.es + inner;
}

template <typename T>
__device__ __forceinline__ T other_den(const LineArgs<T>& a, int64_t base) {
  T d = a.react;
  for (int e = 0; e < a.nother; ++e) {
    int64_t c = (base / a.so[e]) % a.Mo[e];
    d += a.mu_o[e][c];
  }
  return d;
}

// The fused MID pass needs, per frequency k, x = Q_k diag(1/(bd + mu_kl))
// Q_k^T y, i.e. the solution of the shifted n x n system
// (coef A_k + bd C_k) x = y of the projected pencil.  Its bubble blocks do
// not depend on k and couple to the nodal channel only through cos psi and
// sin psi (psi = pi k / (2K)), so in the bubble eigenbasis (We, Wo: fixed
// per axis) the system is an arrowhead one, solved by eliminating the
// bubble modes: O(n) work and one division per frequency instead of two
// n x n products with a table of n^2 values per frequency.  The nodal
// Schur complement comes from the product form
//   den = (cc0 + cc1 cos^2 psi) prod_l (mu_kl + bd) / prod_m (nu_m + bd),
// every factor a sum of positive terms, so it keeps full relative accuracy
// at the lowest frequencies, where the direct form
// alpha_k - sum_m s_m^2 g_m^2 / D_m cancels.
//
// Per line (bd = react + the other axes' terms): r_m = 1 / (nu_m + bd) and
// g_m = coef gA_m + bd gC_m for the n - 1 bubble modes (even, then odd).
template <typename T, int NORD>
__device__ __forceinline__ void cond_line(const T* __restrict__ ar, T bd, T* r, T* g) {
  constexpr int ne = NORD / 2, no = (NORD - 1) / 2, nb = NORD - 1;
  constexpr int onu = ne * ne + no * no, ogA = onu + nb, ogC = ogA + nb;
#pragma unroll
  for (int m = 0; m < nb; ++m) {
    r[m] = (T)1 / (ar[onu + m] + bd);
    g[m] = ar[ogA + m] + bd * ar[ogC + m];
  }
}

// Bubble channels into (BACK = false: W^T) or out of (BACK = true: W) the
// bubble eigenbasis; v and w hold the n - 1 bubble values, even then odd.
template <typename T, int NORD, bool BACK>
__device__ __forceinline__ void cond_basis(const T* __restrict__ ar, const T* v, T* w) {
  constexpr int ne = NORD / 2, no = (NORD - 1) / 2;
#pragma unroll
  for (int i = 0; i < ne; ++i) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < ne; ++j) acc += (BACK ? ar[i * ne + j] : ar[j * ne + i]) * v[j];
    w[i] = acc;
  }
#pragma unroll
  for (int i = 0; i < no; ++i) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < no; ++j)
      acc += (BACK ? ar[ne * ne + i * no + j] : ar[ne * ne + j * no + i]) * v[ne + j];
    w[ne + i] = acc;
  }
}

// Frequency k >= 1: ch (nodal, even, odd channel values) -> out; cs, sn =
// cos psi, sin psi; mu: the n values mu_kl; twoK = 2 / K (the projected
// pencil is K/2 times the element-level one).
template <typename T, int NORD>
__device__ __forceinline__ void cond_solve(const T* __restrict__ ar, const T* r, const T* g, T bd, T cs,
                                           T sn, const T* __restrict__ mu, T twoK, const T* ch, T* out) {
  constexpr int ne = NORD / 2, no = (NORD - 1) / 2, nb = NORD - 1;
  constexpr int occ = ne * ne + no * no + 3 * nb;
  constexpr int NC = nb > 0 ? nb : 1;
  T yh[NC], xh[NC];
  if constexpr (nb > 0) cond_basis<T, NORD, false>(ar, ch + 1, yh);
  T se = 0, so = 0;
#pragma unroll
  for (int m = 0; m < ne; ++m) se += g[m] * r[m] * yh[m];
#pragma unroll
  for (int m = ne; m < nb; ++m) so += g[m] * r[m] * yh[m];
  const T num = ch[0] - cs * se - sn * so;
  T den = (ar[occ] + ar[occ + 1] * cs * cs) * (mu[0] + bd);
#pragma unroll
  for (int l = 1; l < NORD; ++l) den *= (mu[l] + bd) * r[l - 1];
  const T x0 = twoK * num / den;
#pragma unroll
  for (int m = 0; m < nb; ++m) xh[m] = r[m] * (twoK * yh[m] - (m < ne ? cs : sn) * g[m] * x0);
  out[0] = x0;
  if constexpr (nb > 0) cond_basis<T, NORD, true>(ar, xh, out + 1);
}

// The bubble-only block (k = 0, projected pencil K times the element-level
// bubble blocks): ch and out hold the n - 1 bubble values.
template <typename T, int NORD>
__device__ __forceinline__ void cond_solve0(const T* __restrict__ ar, const T* r, T invK, const T* ch,
                                            T* out) {
  constexpr int nb = NORD - 1;
  constexpr int NC = nb > 0 ? nb : 1;
  if constexpr (nb > 0) {
    T yh[NC];
    cond_basis<T, NORD, false>(ar, ch, yh);
#pragma unroll
    for (int m = 0; m < nb; ++m) yh[m] *= r[m] * invK;
    cond_basis<T, NORD, true>(ar, yh, out);
  }
}

// This file is compiled six times: FFTFEM_LINE_KIND = 0 for element counts K
// that are powers of two (shift/mask index arithmetic, Stockham FFTs), 1 for
// other K with prime factors <= 7 (divisions, mixed-radix Stockham FFTs),
// 2 for the rest (divisions, Bluestein DFTs); each kernel object carries only
// its own DFT, which keeps the register allocation of the general-K kernels
// from paying for code they never run.  The kind is a template argument of
// the kernels, so the objects define different symbols.
#ifndef FFTFEM_LINE_KIND
#define FFTFEM_LINE_KIND 0
#endif
// and once per precision (FFTFEM_LINE_REAL: float or double)
#ifndef FFTFEM_LINE_REAL
#define FFTFEM_LINE_REAL double
#endif
constexpr int kLineKind = FFTFEM_LINE_KIND;

// Length-K DFTs of the nfft buffers of a tile: Stockham for K a power of
// two, mixed-radix Stockham for other K whose prime factors are at most 7,
// Bluestein otherwise.
template <typename T, bool INV, int NT, int KIND>
__device__ __forceinline__ void line_dft(const LineArgs<T>& a, C2<T>* buf, int nfft, int ls) {
  const int lrmax = a.lrmax ? a.lrmax : 4;
  if constexpr (KIND == 0) {
    fft_all<T, INV, NT>(buf, nfft, a.log2K, reinterpret_cast<const C2<T>*>(a.twf), ls, lrmax);
  } else if constexpr (KIND == 1) {
    fft_mixed<T, INV, NT>(buf, nfft, a.K, a.radpack, a.nrad, reinterpret_cast<const C2<T>*>(a.twf), ls);
  } else {
    bluestein<T, INV, NT>(buf, nfft, a.K, a.log2L, reinterpret_cast<const C2<T>*>(a.chirp),
                          reinterpret_cast<const C2<T>*>(a.bhat), reinterpret_cast<const C2<T>*>(a.twl), ls,
                          lrmax);
  }
}

// Body of a line pass for tile `bid` of `nblk` tiles (the launch, or one job
// of a grouped launch).
template <typename T, int NORD, int MODE, bool UPD, bool LF, int KIND>
__device__ __forceinline__ void line_body(const LineArgs<T>& a, int bid, int nblk) {
  constexpr int kNT = LineCfg<T>::NT, kMaxTPT = LineCfg<T>::TPT, kMaxCPT = LineCfg<T>::CPT;
  if (a.flag && *a.flag) return;
  constexpr int n = NORD, ne = NORD / 2, no = (NORD - 1) / 2, P = NORD / 2, NB = 1 + P;
  constexpr int NC = NORD > 1 ? NORD - 1 : 1;
  C2<T>* buf = reinterpret_cast<C2<T>*>(fftfem_lds);
  T* raw = reinterpret_cast<T*>(fftfem_lds);
  const int tid = threadIdx.x;
  const int K = a.K, lk = a.log2K, lg = a.log2G, G = 1 << lg;
  const int M = n * K - 1;
  const int ls = a.fl + (G > 1 ? 1 : 0);  // complex slots per FFT buffer (pad between lines)
  // raw line data (loaded input, spectral output, scattered result) is
  // packed at M slots per line: it never coexists with the FFT buffers
  // (NB ls complex slots per line), which it aliases across barriers
  const int RS = M;
  const int64_t l0 = (int64_t)xcd_remap(bid, nblk) << lg;
  const rsrc_t qtab = table_rsrc(a.Q, (uint32_t)(K * n * n));
  const C2<T>* twf = reinterpret_cast<const C2<T>*>(a.twf);
  const C2<T>* twm = reinterpret_cast<const C2<T>*>(a.twm);
  const C2<T>* twd = reinterpret_cast<const C2<T>*>(a.twd);

  // ---------------- coalesced bulk transfers between HBM and LDS ----------
  auto bulk_load = [&](const void* src, int f64) {
    if constexpr (LF) {
      const int g = tid & (G - 1);
      const int64_t line = l0 + g;
      const bool ok = line < a.nlines;
      const int64_t base = ok ? line_base(a, line) : 0;
      T* dst = raw + g * RS;
      const int step = kNT >> lg;
      for (int i0 = tid >> lg; i0 < M; i0 += 16 * step) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          int i = i0 + u * step;
          v[u] = (ok && i < M) ? load_in<T>(src, f64, base + (int64_t)i * a.es) : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          int i = i0 + u * step;
          if (i < M) dst[i] = v[u];
        }
      }
    } else {
      // ies != 0: element i of line l at l + i ies (a transposed layout)
      if (a.ies) {
        for (int g = 0; g < G; ++g) {
          const int64_t line = l0 + g;
          if (line >= a.nlines) break;
          T* dst = raw + g * RS;
          for (int i0 = tid; i0 < M; i0 += 4 * kNT) {
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              int i = i0 + u * kNT;
              v[u] = i < M ? load_in<T>(src, f64, line + (int64_t)i * a.ies) : (T)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              int i = i0 + u * kNT;
              if (i < M) dst[i] = v[u];
            }
          }
        }
        return;
      }
      // the lines of a contiguous tile are adjacent: one flat segment of
      // nl M values, loaded in one sweep into the packed raw layout (a loop
      // over the lines would wait for each line's loads before issuing the
      // next line's)
      const int nl = (int)(a.nlines - l0 < (int64_t)G ? a.nlines - l0 : (int64_t)G);
      const int nflat = nl * M;
      const int64_t base = l0 * (int64_t)M;
      if constexpr (sizeof(T) == 8) {
        // float64: 16-byte loads of value pairs (the first value alone when
        // the segment does not start 16-byte aligned, the last when one is
        // left over)
        const double* sp = reinterpret_cast<const double*>(src) + base;
        const int head = (reinterpret_cast<uintptr_t>(sp) & 15) ? 1 : 0;
        const int np = (nflat - head) >> 1;
        const double2* s2 = reinterpret_cast<const double2*>(sp + head);
        for (int i0 = tid; i0 < np; i0 += kFlatPairs * kNT) {
          double2 v[kFlatPairs];
#pragma unroll
          for (int u = 0; u < kFlatPairs; ++u) {
            int i = i0 + u * kNT;
            v[u] = i < np ? ld_stream(s2 + i) : double2{0.0, 0.0};
          }
#pragma unroll
          for (int u = 0; u < kFlatPairs; ++u) {
            int i = i0 + u * kNT;
            if (i < np) {
              raw[head + 2 * i] = v[u].x;
              raw[head + 2 * i + 1] = v[u].y;
            }
          }
        }
        if (tid == 0 && nflat > 0) {
          if (head) raw[0] = sp[0];
          if ((nflat - head) & 1) raw[nflat - 1] = sp[nflat - 1];
        }
        return;
      }
      for (int i0 = tid; i0 < nflat; i0 += 16 * kNT) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          int i = i0 + u * kNT;
          v[u] = i < nflat ? load_in<T>(src, f64, base + i) : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          int i = i0 + u * kNT;
          if (i < nflat) raw[i] = v[u];
        }
      }
    }
  };
  double acc_c = 0, acc_u = 0;
  // output pass: any NaN or Inf written (v - v is 0 exactly for finite v)
  const bool chk = !UPD && a.bad != nullptr;
  bool nonfinite = false;
  auto put = [&](int64_t idx, T v) {
    if constexpr (UPD) {
      double u = a.upd[idx] + (double)v;
      ((double*)a.out)[idx] = u;
      if (a.cor) a.cor[idx] = (double)v;
      acc_c += (double)v * (double)v;
      acc_u += u * u;
    } else {
      store_out<T>(a.out, a.out_kind, idx, v);
      if (chk) nonfinite |= !(v - v == (T)0);
    }
  };
  auto bulk_store = [&]() {
    if constexpr (LF) {
      const int g = tid & (G - 1);
      const int64_t line = l0 + g;
      if (line < a.nlines) {
        const int64_t base = line_base(a, line);
        const T* srcl = raw + g * RS;
        const int step = kNT >> lg;
        for (int i = tid >> lg; i < M; i += step) put(base + (int64_t)i * a.es, srcl[i]);
      }
    } else {
      // oes != 0: element i of line l to l + i oes (a transposed layout)
      if (a.oes) {
        for (int g = 0; g < G; ++g) {
          const int64_t line = l0 + g;
          if (line >= a.nlines) break;
          const T* srcl = raw + g * RS;
          for (int i = tid; i < M; i += kNT) put(line + (int64_t)i * a.oes, srcl[i]);
        }
        return;
      }
      const int nl = (int)(a.nlines - l0 < (int64_t)G ? a.nlines - l0 : (int64_t)G);
      const int nflat = nl * M;
      const int64_t base = l0 * (int64_t)M;
      if constexpr (sizeof(T) == 8 && !UPD) {
        if (a.out_kind != 2) {
          // float64 output: 16-byte stores of value pairs
          double* op = reinterpret_cast<double*>(a.out) + base;
          const int head = (reinterpret_cast<uintptr_t>(op) & 15) ? 1 : 0;
          const int np = (nflat - head) >> 1;
          double2* o2 = reinterpret_cast<double2*>(op + head);
          for (int i = tid; i < np; i += kNT) {
            const double v0 = raw[head + 2 * i], v1 = raw[head + 2 * i + 1];
            st_stream(o2 + i, v0, v1);
            if (chk) nonfinite |= !(v0 - v0 == 0.0) || !(v1 - v1 == 0.0);
          }
          if (tid == 0 && nflat > 0) {
            if (head) put(base, raw[0]);
            if ((nflat - head) & 1) put(base + nflat - 1, raw[nflat - 1]);
          }
          return;
        }
      }
      for (int i = tid; i < nflat; i += kNT) put(base + i, raw[i]);
    }
  };

  // element tasks (g, j'), j' < K, and contraction tasks (g, kappa),
  // kappa < ceil(K/2): kappa >= 1 pairs the frequencies kappa and K - kappa,
  // kappa = 0 is the bubble block (and frequency K/2 when K is even)
  constexpr bool pow2 = KIND == 0;
  const int kh = (K + 1) >> 1;
  const int lkh = lk - 1;
  const int ntask = G * K;
  const int nctask = G * kh;
  auto esplit = [&](int t, int& g, int& jp) {
    if constexpr (pow2) {
      g = t >> lk;
      jp = t & (K - 1);
    } else {
      g = t / K;
      jp = t - g * K;
    }
  };
  auto csplit = [&](int t, int& g, int& kap) {
    if constexpr (pow2) {
      g = t >> lkh;
      kap = t & ((1 << lkh) - 1);
    } else {
      g = t / kh;
      kap = t - g * kh;
    }
  };
  const bool keven = (K & 1) == 0;  // frequency K/2 exists

  if constexpr (MODE == FWD || MODE == MID) {
    bulk_load(a.in, a.in_f64);
    __syncthreads();
    // ---- gather: element j' -> nodal value (node j'+1) and channels ----
    T hv[kMaxTPT][NORD];
#pragma unroll
    for (int s = 0; s < kMaxTPT; ++s) {
      int t = tid + s * kNT;
      if (t < ntask) {
        int g, jp;
        esplit(t, g, jp);
        const T* r = raw + g * RS + jp * n;
        T y[NORD];
#pragma unroll
        for (int m = 0; m < n - 1; ++m) y[m] = r[m];
        y[n - 1] = (jp < K - 1) ? r[n - 1] : (T)0;
        T sg = (jp & 1) ? (T)-1 : (T)1;
        hv[s][0] = y[n - 1];
#pragma unroll
        for (int m = 1; m <= ne; ++m) hv[s][m] = sg * ((2 * m == n) ? y[m - 1] : y[m - 1] + y[n - m - 1]);
#pragma unroll
        for (int m = 1; m <= no; ++m) hv[s][ne + m] = y[m - 1] - y[n - m - 1];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kMaxTPT; ++s) {
      int t = tid + s * kNT;
      if (t < ntask) {
        int g, jp;
        esplit(t, g, jp);
        C2<T>* Z = buf + g * NB * ls;
        if (jp < K - 1) {
          int j = jp + 1;
          T x = hv[s][0];
          set_comp(Z, j >> 1, j & 1, x);
          int t2 = 2 * K - j;
          set_comp(Z, t2 >> 1, t2 & 1, -x);
        } else {
          write_nodal_zeros(Z, K);
        }
        int q = (jp & 1) ? K - 1 - (jp >> 1) : (jp >> 1);
#pragma unroll
        for (int b = 0; b < n - 1; ++b) set_comp(Z + (1 + b / 2) * ls, q, b & 1, hv[s][1 + b]);
        if ((n - 1) & 1) set_comp(Z + P * ls, q, 1, (T)0);
      }
    }
    __syncthreads();
    line_dft<T, false, kNT, KIND>(a, buf, G * NB, ls);
  } else {
    bulk_load(a.in, a.in_f64);
    __syncthreads();
  }

  // ---------------- contraction per frequency pair -------------------------
  if constexpr (MODE == MID) {
    // The nodal forward values of this thread's tasks are read first: the
    // nodal inverse inputs of a task land in slots that other tasks read.
    // After the barrier every task runs start to finish on its own (bubble
    // slots are pair-local), so no per-task state outlives its iteration and
    // the loop is not unrolled: the register footprint is that of one task.
    T nf[kMaxCPT][2];
#pragma unroll
    for (int s = 0; s < kMaxCPT; ++s) {
      int t = tid + s * kNT;
      nf[s][0] = nf[s][1] = (T)0;
      if (t < nctask) {
        int g, kap;
        csplit(t, g, kap);
        const C2<T>* B = buf + g * NB * ls;
        if (kap == 0) {
          if (keven) nf[s][1] = nodal_post<T>(B, K, K >> 1, twd, false);
        } else {
          nf[s][0] = nodal_post<T>(B, K, kap, twd, false);
          nf[s][1] = nodal_post<T>(B, K, K - kap, twd, false);
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < kMaxCPT; ++s) {
      int t = tid + s * kNT;
      if (t >= nctask) break;
      T nfa = nf[0][0], nfb = nf[0][1];
#pragma unroll
      for (int u = 1; u < kMaxCPT; ++u)
        if (s == u) {
          nfa = nf[u][0];
          nfb = nf[u][1];
        }
      int g, kap;
        csplit(t, g, kap);
      int kb = kap == 0 ? 0 : K - kap;
      C2<T>* B = buf + g * NB * ls;
      // per-line denominator base: react + the other axes' terms
      T bd = (T)1;
      {
        const int64_t line = l0 + g;
        if (line < a.nlines) bd = other_den(a, line_base(a, line));
      }
      T ca[NC], cb[NC];
      if constexpr (NORD > 1) {
        if (kap != 0) bubble_post<T, NORD>(B, ls, kap, kb, twm, ca, cb);
      }
      // frequencies of the task: ka = kap (0: the bubble block), kb = K - kap
      // (K/2 when kap = 0; for odd K, kap = 0 has no second frequency and
      // chain b runs on the bubble block again, its result unused)
      const int ka = kap, kbq = kap == 0 ? (keven ? (K >> 1) : 0) : K - kap;
      T cha[NORD], chb[NORD];
      if (kap == 0) {
        if constexpr (NORD > 1) {
          bubble_post<T, NORD>(B, ls, 0, 0, twm, ca, cb);
#pragma unroll
          for (int b = 0; b < NORD - 1; ++b) cha[b] = ca[b];
          bubble_post<T, NORD>(B, ls, kbq, kbq, twm, ca, cb);
        }
        cha[NORD - 1] = 0;
        channel_vec<T, NORD>(nfb, ca, ca, chb);
      } else {
        channel_vec<T, NORD>(nfa, ca, cb, cha);
        channel_vec<T, NORD>(nfb, cb, ca, chb);
      }
      T res[2][NORD];
      {
        T lr[NC], lgc[NC];
        if constexpr (NORD > 1) cond_line<T, NORD>(a.arrow, bd, lr, lgc);
        const T twoK = (T)2 / (T)K;
        if (ka == 0) {
          cond_solve0<T, NORD>(a.arrow, lr, (T)0.5 * twoK, cha, res[0]);
          res[0][NORD - 1] = 0;
        } else {
          const C2<T> w = twm[ka];
          cond_solve<T, NORD>(a.arrow, lr, lgc, bd, w.x, -w.y, a.mu_self + (n - 1 + (ka - 1) * n), twoK, cha,
                              res[0]);
        }
        if (kbq != 0) {
          const C2<T> w = twm[kbq];
          cond_solve<T, NORD>(a.arrow, lr, lgc, bd, w.x, -w.y, a.mu_self + (n - 1 + (kbq - 1) * n), twoK, chb,
                              res[1]);
        } else {
#pragma unroll
          for (int c = 0; c < NORD; ++c) res[1][c] = 0;
        }
      }
      // inverse inputs: bubble pre-twiddles (pair-local slots), nodal values
      if constexpr (NORD > 1) {
        T ya[NC], yb[NC];
        if (kap == 0) {
#pragma unroll
          for (int b = 0; b < NORD - 1; ++b) ya[b] = res[0][b];  // index 0 of every channel (k = 0 block)
#pragma unroll
          for (int m = 1; m <= ne; ++m) yb[m - 1] = res[1][m];
#pragma unroll
          for (int m = 1; m <= no; ++m) yb[ne + m - 1] = res[1][ne + m];
#pragma unroll
          for (int p = 1; p <= P; ++p) {
            int b0 = 2 * (p - 1), b1 = b0 + 1;
            bool has1 = b1 < NORD - 1;
            slot(B + p * ls, 0) = {ya[b0], has1 ? ya[b1] : (T)0};
            if (keven) {
              int h = K >> 1;
              C2<T> va = herm<T>(yb[b0], yb[b0], h, twm);
              C2<T> vb = has1 ? herm<T>(yb[b1], yb[b1], h, twm) : C2<T>{0, 0};
              slot(B + p * ls, h) = {va.x - vb.y, va.y + vb.x};
            }
          }
        } else {
          // channel spectra at FFT index kap (ya) and kb (yb): even channels
          // of frequency k sit at K - k, odd channels at k
#pragma unroll
          for (int m = 1; m <= ne; ++m) {
            ya[m - 1] = res[1][m];
            yb[m - 1] = res[0][m];
          }
#pragma unroll
          for (int m = 1; m <= no; ++m) {
            ya[ne + m - 1] = res[0][ne + m];
            yb[ne + m - 1] = res[1][ne + m];
          }
#pragma unroll
          for (int p = 1; p <= P; ++p) {
            int b0 = 2 * (p - 1), b1 = b0 + 1;
            bool has1 = b1 < NORD - 1;
            C2<T> va = herm<T>(ya[b0], yb[b0], kap, twm);
            C2<T> vb = has1 ? herm<T>(ya[b1], yb[b1], kap, twm) : C2<T>{0, 0};
            slot(B + p * ls, kap) = {va.x - vb.y, va.y + vb.x};
            va = herm<T>(yb[b0], ya[b0], kb, twm);
            vb = has1 ? herm<T>(yb[b1], ya[b1], kb, twm) : C2<T>{0, 0};
            slot(B + p * ls, kb) = {va.x - vb.y, va.y + vb.x};
          }
        }
      }
      if (kap == 0) {
        write_nodal_zeros(B, K);
        if (keven) write_nodal_inv(B, K, K >> 1, res[1][0]);
      } else {
        write_nodal_inv(B, K, kap, res[0][0]);
        write_nodal_inv(B, K, K - kap, res[1][0]);
      }
    }
    __syncthreads();
    line_dft<T, true, kNT, KIND>(a, buf, G * NB, ls);
  } else {
  // held across a barrier: spectral results (FWD) or channel spectra (INV)
  T hw[kMaxCPT][2][NORD];
#pragma unroll
  for (int s = 0; s < kMaxCPT; ++s) {
    int t = tid + s * kNT;
    if (t >= nctask) continue;
    int g, kap;
        csplit(t, g, kap);
    // frequencies of the task: ka = kap (0: the bubble block), kb = K - kap
    // (K/2 when kap = 0; for odd K, kap = 0 has no second frequency and
    // chain b runs on the bubble block again, its result unused)
    const bool hasb = kap != 0 || keven;
    const int ka = kap, kbq = kap == 0 ? (keven ? (K >> 1) : 0) : K - kap;
    const int ra = ka == 0 ? n - 1 : n;
    const int offa = ka == 0 ? 0 : n - 1 + (ka - 1) * n;
    const int offb = kbq == 0 ? 0 : n - 1 + (kbq - 1) * n;
    if constexpr (MODE == FWD) {
      const C2<T>* B = buf + g * NB * ls;
      T ca[NC], cb[NC], cha[NORD], chb[NORD];
      if (kap == 0) {
        if constexpr (NORD > 1) {
          bubble_post<T, NORD>(B, ls, 0, 0, twm, ca, cb);
#pragma unroll
          for (int b = 0; b < NORD - 1; ++b) cha[b] = ca[b];
          bubble_post<T, NORD>(B, ls, kbq, kbq, twm, ca, cb);
        }
        cha[NORD - 1] = 0;
        channel_vec<T, NORD>(hasb ? nodal_post<T>(B, K, kbq, twd, false) : (T)0, ca, ca, chb);
      } else {
        if constexpr (NORD > 1) bubble_post<T, NORD>(B, ls, kap, K - kap, twm, ca, cb);
        channel_vec<T, NORD>(nodal_post<T>(B, K, ka, twd, false), ca, cb, cha);
        channel_vec<T, NORD>(nodal_post<T>(B, K, kbq, twd, false), cb, ca, chb);
      }
      contract_fwd2<T, NORD>(qtab, K, ka, kbq, cha, chb, hw[s][0], hw[s][1], cha[0]);
#pragma unroll
      for (int l = 0; l < NORD; ++l)
        if (l >= ra) hw[s][0][l] = 0;
    } else {
      const T* rs = raw + g * RS;
      T wa[NORD], wb[NORD];
#pragma unroll
      for (int l = 0; l < NORD; ++l) {
        wa[l] = l < ra ? rs[offa + l] : (T)0;
        wb[l] = hasb ? rs[offb + l] : (T)0;
      }
      contract_inv2<T, NORD>(qtab, K, ka, kbq, wa, wb, hw[s][0], hw[s][1], wa[0] + wb[0]);
    }
  }
  __syncthreads();

  if constexpr (MODE == FWD) {
    // spectral results -> LDS (line layout) -> coalesced store
#pragma unroll
    for (int s = 0; s < kMaxCPT; ++s) {
      int t = tid + s * kNT;
      if (t >= nctask) continue;
      int g, kap;
        csplit(t, g, kap);
      T* rs = raw + g * RS;
#pragma unroll
      for (int fi = 0; fi < 2; ++fi) {
        int k = fi == 0 ? kap : (kap == 0 ? (K >> 1) : K - kap);
        if (fi == 1 && kap == 0 && !keven) continue;
        int r = k == 0 ? n - 1 : n;
        int off = k == 0 ? 0 : n - 1 + (k - 1) * n;
#pragma unroll
        for (int l = 0; l < NORD; ++l)
          if (l < r) rs[off + l] = hw[s][fi][l];
      }
    }
    __syncthreads();
    bulk_store();
    return;
  } else {
    // write the inverse-transform inputs: nodal (and, for INV, bubbles)
#pragma unroll
    for (int s = 0; s < kMaxCPT; ++s) {
      int t = tid + s * kNT;
      if (t >= nctask) continue;
      int g, kap;
        csplit(t, g, kap);
      int kb = kap == 0 ? 0 : K - kap;
      C2<T>* B = buf + g * NB * ls;
      if (kap == 0) {
        write_nodal_zeros(B, K);
        if (keven) write_nodal_inv(B, K, K >> 1, hw[s][1][0]);
      } else {
        write_nodal_inv(B, K, kap, hw[s][0][0]);
        write_nodal_inv(B, K, K - kap, hw[s][1][0]);
      }
      if constexpr (MODE == INV && NORD > 1) {
        T ya[NC], yb[NC];
        if (kap == 0) {
#pragma unroll
          for (int b = 0; b < NORD - 1; ++b) ya[b] = hw[s][0][b];
#pragma unroll
          for (int m = 1; m <= ne; ++m) yb[m - 1] = hw[s][1][m];
#pragma unroll
          for (int m = 1; m <= no; ++m) yb[ne + m - 1] = hw[s][1][ne + m];
#pragma unroll
          for (int p = 1; p <= P; ++p) {
            int b0 = 2 * (p - 1), b1 = b0 + 1;
            bool has1 = b1 < NORD - 1;
            slot(B + p * ls, 0) = {ya[b0], has1 ? ya[b1] : (T)0};
            if (keven) {
              int h = K >> 1;
              C2<T> va = herm<T>(yb[b0], yb[b0], h, twm);
              C2<T> vb = has1 ? herm<T>(yb[b1], yb[b1], h, twm) : C2<T>{0, 0};
              slot(B + p * ls, h) = {va.x - vb.y, va.y + vb.x};
            }
          }
        } else {
#pragma unroll
          for (int m = 1; m <= ne; ++m) {
            ya[m - 1] = hw[s][1][m];
            yb[m - 1] = hw[s][0][m];
          }
#pragma unroll
          for (int m = 1; m <= no; ++m) {
            ya[ne + m - 1] = hw[s][0][ne + m];
            yb[ne + m - 1] = hw[s][1][ne + m];
          }
#pragma unroll
          for (int p = 1; p <= P; ++p) {
            int b0 = 2 * (p - 1), b1 = b0 + 1;
            bool has1 = b1 < NORD - 1;
            C2<T> va = herm<T>(ya[b0], yb[b0], kap, twm);
            C2<T> vb = has1 ? herm<T>(ya[b1], yb[b1], kap, twm) : C2<T>{0, 0};
            slot(B + p * ls, kap) = {va.x - vb.y, va.y + vb.x};
            va = herm<T>(yb[b0], ya[b0], kb, twm);
            vb = has1 ? herm<T>(yb[b1], ya[b1], kb, twm) : C2<T>{0, 0};
            slot(B + p * ls, kb) = {va.x - vb.y, va.y + vb.x};
          }
        }
      }
    }
    __syncthreads();
    line_dft<T, true, kNT, KIND>(a, buf, G * NB, ls);
  }
  }

  // ---------------- scatter: channels -> bubble vectors and nodes ----------
  {
    T hv[kMaxTPT][NORD];
#pragma unroll
    for (int s = 0; s < kMaxTPT; ++s) {
      int t = tid + s * kNT;
      if (t < ntask) {
        int g, jp;
        esplit(t, g, jp);
        const C2<T>* Z = buf + g * NB * ls;
        hv[s][n - 1] = jp < K - 1 ? nodal_post<T>(Z, K, jp + 1, twd, true) : (T)0;
        int q = (jp & 1) ? K - 1 - (jp >> 1) : (jp >> 1);
        T sg = (jp & 1) ? (T)-1 : (T)1;
#pragma unroll
        for (int m = 1; m <= ne; ++m) {
          int be = m - 1;
          T E = sg * get_comp(Z + (1 + be / 2) * ls, q, be & 1);
          if (2 * m == n) {
            hv[s][m - 1] = E;
          } else {
            int bo = ne + m - 1;
            T O = get_comp(Z + (1 + bo / 2) * ls, q, bo & 1);
            hv[s][m - 1] = E + O;
            hv[s][n - m - 1] = E - O;
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kMaxTPT; ++s) {
      int t = tid + s * kNT;
      if (t < ntask) {
        int g, jp;
        esplit(t, g, jp);
        T* r = raw + g * RS + jp * n;
#pragma unroll
        for (int m = 0; m < n - 1; ++m) r[m] = hv[s][m];
        if (jp < K - 1) r[n - 1] = hv[s][n - 1];
      }
    }
    __syncthreads();
    bulk_store();
  }
  if (chk) {
    // one vector atomic per wave that saw a non-finite value
    if (__ballot(nonfinite) != 0 && (tid & 63) == 0) atomicOr(a.bad, 2);
  }
  if constexpr (UPD) {
    __shared__ double red[2][kNT];
    red[0][tid] = acc_c;
    red[1][tid] = acc_u;
    __syncthreads();
    for (int s = kNT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        red[0][tid] += red[0][tid + s];
        red[1][tid] += red[1][tid + s];
      }
      __syncthreads();
    }
    if (tid == 0) {
      a.partials[2 * bid] = red[0][0];
      a.partials[2 * bid + 1] = red[1][0];
    }
  }
}

template <typename T, int NORD, int MODE, bool UPD, bool LF, int KIND>
__global__ __launch_bounds__(LineCfg<T>::NT, LineCfg<T>::MINW) void line_kernel(LineArgs<T> a) {
  line_body<T, NORD, MODE, UPD, LF, KIND>(a, blockIdx.x, gridDim.x);
}

// Grouped launch: block b runs tile b - start[j] of job j = job_of[b].
template <typename T, int NORD, int MODE, bool UPD, bool LF, int KIND>
__global__ __launch_bounds__(LineCfg<T>::NT, LineCfg<T>::MINW) void line_kernel_grouped(
    const LineArgs<T>* __restrict__ jobs, const int* __restrict__ job_of, const int* __restrict__ start) {
  const int j = __builtin_amdgcn_readfirstlane(job_of[blockIdx.x]);
  const int b0 = __builtin_amdgcn_readfirstlane(start[j]), b1 = __builtin_amdgcn_readfirstlane(start[j + 1]);
  line_body<T, NORD, MODE, UPD, LF, KIND>(jobs[j], (int)blockIdx.x - b0, b1 - b0);
}

template <typename F>
static void allow_lds(F* fn, size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int NORD, int MODE, bool UPD>
static hipError_t go(bool lf, const LineArgs<T>& a, int nblocks, size_t lds, hipStream_t s) {
  if (lf) {
    allow_lds(line_kernel<T, NORD, MODE, UPD, true, kLineKind>, lds);
    hipLaunchKernelGGL((line_kernel<T, NORD, MODE, UPD, true, kLineKind>), dim3(nblocks), dim3(LineCfg<T>::NT),
                       lds, s, a);
  } else {
    allow_lds(line_kernel<T, NORD, MODE, UPD, false, kLineKind>, lds);
    hipLaunchKernelGGL((line_kernel<T, NORD, MODE, UPD, false, kLineKind>), dim3(nblocks), dim3(LineCfg<T>::NT),
                       lds, s, a);
  }
  return hipGetLastError();
}

template <typename T, int NORD>
static hipError_t launch_line_n(int mode, bool upd, const LineArgs<T>& a, int nblocks, size_t lds,
                                hipStream_t s) {
  bool lf = a.es > 1;
  if (mode == FWD) return go<T, NORD, FWD, false>(lf, a, nblocks, lds, s);
  if (mode == INV)
    return upd ? go<T, NORD, INV, true>(lf, a, nblocks, lds, s) : go<T, NORD, INV, false>(lf, a, nblocks, lds, s);
  return upd ? go<T, NORD, MID, true>(lf, a, nblocks, lds, s) : go<T, NORD, MID, false>(lf, a, nblocks, lds, s);
}

template <typename T, int NORD, int MODE, bool UPD>
static hipError_t go_grouped(bool lf, const GroupedLaunch<T>& g, hipStream_t s) {
  if (lf) {
    allow_lds(line_kernel_grouped<T, NORD, MODE, UPD, true, kLineKind>, g.lds);
    hipLaunchKernelGGL((line_kernel_grouped<T, NORD, MODE, UPD, true, kLineKind>), dim3(g.nblocks),
                       dim3(LineCfg<T>::NT), g.lds, s, g.jobs, g.job_of, g.start);
  } else {
    allow_lds(line_kernel_grouped<T, NORD, MODE, UPD, false, kLineKind>, g.lds);
    hipLaunchKernelGGL((line_kernel_grouped<T, NORD, MODE, UPD, false, kLineKind>), dim3(g.nblocks),
                       dim3(LineCfg<T>::NT), g.lds, s, g.jobs, g.job_of, g.start);
  }
  return hipGetLastError();
}

template <typename T, int NORD>
static hipError_t grouped_n(int mode, bool upd, bool lf, const GroupedLaunch<T>& g, hipStream_t s) {
  if (mode == FWD) return go_grouped<T, NORD, FWD, false>(lf, g, s);
  if (mode == INV) return upd ? go_grouped<T, NORD, INV, true>(lf, g, s) : go_grouped<T, NORD, INV, false>(lf, g, s);
  return upd ? go_grouped<T, NORD, MID, true>(lf, g, s) : go_grouped<T, NORD, MID, false>(lf, g, s);
}

#if FFTFEM_LINE_KIND == 0
#define FFTFEM_LAUNCH_LINE launch_line_p2
#define FFTFEM_LAUNCH_GROUPED launch_line_grouped_p2
#elif FFTFEM_LINE_KIND == 1
#define FFTFEM_LAUNCH_LINE launch_line_mr
#define FFTFEM_LAUNCH_GROUPED launch_line_grouped_mr
#else
#define FFTFEM_LAUNCH_LINE launch_line_bs
#define FFTFEM_LAUNCH_GROUPED launch_line_grouped_bs
#endif

template <typename T>
hipError_t FFTFEM_LAUNCH_GROUPED(int n, int mode, bool upd, bool lf, const GroupedLaunch<T>& g, hipStream_t s) {
  switch (n) {
#define FFTFEM_CASE(N) \
  case N:              \
    return grouped_n<T, N>(mode, upd, lf, g, s);
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
template hipError_t FFTFEM_LAUNCH_GROUPED<FFTFEM_LINE_REAL>(int, int, bool, bool,
                                                            const GroupedLaunch<FFTFEM_LINE_REAL>&, hipStream_t);

template <typename T>
hipError_t FFTFEM_LAUNCH_LINE(int n, int mode, bool upd, const LineArgs<T>& a, int nblocks, size_t lds,
                              hipStream_t s) {
  switch (n) {
#define FFTFEM_CASE(N) \
  case N:              \
    return launch_line_n<T, N>(mode, upd, a, nblocks, lds, s);
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

template hipError_t FFTFEM_LAUNCH_LINE<FFTFEM_LINE_REAL>(int, int, bool, const LineArgs<FFTFEM_LINE_REAL>&, int,
                                                         size_t, hipStream_t);

}  // namespace fftfem
