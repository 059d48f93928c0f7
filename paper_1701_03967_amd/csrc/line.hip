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

namespace fftfem {

// Dynamic LDS of the line kernels.
extern __shared__ double2 fftfem_lds[];

// Threads per line-kernel workgroup: 512 for float32; 256 for float64, whose
// register footprint allows no more than eight waves per CU anyway.  Every
// tile has G * K <= 1024 element tasks and G * K / 2 contraction tasks.
template <typename T>
struct LineCfg {
  static constexpr int NT = sizeof(T) == 8 ? 256 : 512;
  static constexpr int TPT = 1024 / NT;  // element tasks per thread
  static constexpr int CPT = 512 / NT;   // contraction tasks per thread
};

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

// DCT-II values of the packed bubble buffers at indices ia and ib (= K - ia
// mod K): out_a[b], out_b[b] for every bubble channel b.
template <typename T, int NORD>
__device__ __forceinline__ void bubble_post(const C2<T>* B, int ls, int ia, int ib,
                                            const C2<T>* twm, T* out_a, T* out_b) {
  constexpr int P = NORD / 2;
#pragma unroll
  for (int p = 1; p <= P; ++p) {
    C2<T> Va = B[p * ls + ia], Vb = B[p * ls + ib];
    C2<T> sm = {Va.x + Vb.x, Va.y - Vb.y};  // Va + conj(Vb)
    C2<T> df = {Va.x - Vb.x, Va.y + Vb.y};  // Va - conj(Vb)
    C2<T> wa = twm[ia], wb = twm[ib];
    C2<T> sa = cmul(wa, sm), da = cmul(wa, df);
    C2<T> smb = {sm.x, -sm.y}, dfb = {-df.x, df.y};  // Vb + conj(Va), Vb - conj(Va)
    C2<T> sb = cmul(wb, smb), db = cmul(wb, dfb);
    out_a[2 * (p - 1)] = sa.x * (T)0.5;
    out_b[2 * (p - 1)] = sb.x * (T)0.5;
    if (2 * (p - 1) + 1 < NORD - 1) {
      out_a[2 * (p - 1) + 1] = da.y * (T)0.5;
      out_b[2 * (p - 1) + 1] = db.y * (T)0.5;
    }
  }
}

// DST-I value at frequency k from the packed odd-extension spectrum Z.
template <typename T>
__device__ __forceinline__ T nodal_post(const C2<T>* Z, int K, int k, const C2<T>* twd,
                                        bool conj_in) {
  C2<T> zk = Z[k], zm = Z[K - k];
  if (conj_in) {
    zk.y = -zk.y;
    zm.y = -zm.y;
  }
  C2<T> F = {(zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5};
  C2<T> d = {zk.x - zm.x, zk.y + zm.y};
  C2<T> Gv = {d.y * (T)0.5, -d.x * (T)0.5};
  C2<T> Y = cmul(twd[k], Gv);
  return -(F.y + Y.y) * (T)0.5;
}

// exp(i pi idx/(2K)) (y~[idx] - i y~[K-idx]) / 2 with y~[0] = 2 y[0], y~[K] = 0.
template <typename T>
__device__ __forceinline__ C2<T> herm(T y_idx, T y_mirror, int idx, const C2<T>* twm) {
  if (idx == 0) return {y_idx, (T)0};
  C2<T> v = {y_idx * (T)0.5, -y_mirror * (T)0.5};
  return cmulc(v, twm[idx]);
}

// conj of the odd-extension packing: y_t -> component t%2 of Z[t/2], imaginary negated
template <typename T>
__device__ __forceinline__ void write_nodal_inv(C2<T>* Z, int K, int k, T val) {
  int t = k;
  set_comp(Z, t >> 1, t & 1, (t & 1) ? -val : val);
  t = 2 * K - k;
  set_comp(Z, t >> 1, t & 1, (t & 1) ? val : -val);
}

template <typename T>
__device__ __forceinline__ void write_nodal_zeros(C2<T>* Z, int K) {
  set_comp(Z, 0, 0, (T)0);
  set_comp(Z, K >> 1, K & 1, (T)0);
}

// Channel vector of frequency k from post-processed spectra at the index
// pair (ia, ib = K - ia): nodal, even channels (DST-II at k = DCT-II of the
// alternated input at K - k), odd channels (DCT-II at k).
template <typename T, int NORD>
__device__ __forceinline__ void channel_vec(T nodal, const T* at_k, const T* at_mk, T* ch) {
  constexpr int ne = NORD / 2, no = (NORD - 1) / 2;
  ch[0] = nodal;
#pragma unroll
  for (int m = 1; m <= ne; ++m) ch[m] = at_mk[m - 1];
#pragma unroll
  for (int m = 1; m <= no; ++m) ch[ne + m] = at_k[ne + m - 1];
}

// Q is stored structure-of-arrays: entry (c, l) of frequency k at
// Q[(c * n + l) * K + k], so the lanes of a wave (consecutive k) read
// consecutive addresses.  Block k = 0 is zero-padded to n x n.
template <typename T, int NORD>
__device__ __forceinline__ void contract_fwd(const T* __restrict__ Q, int K, int k, const T* ch, T* w) {
#pragma unroll
  for (int l = 0; l < NORD; ++l) w[l] = 0;
#pragma unroll
  for (int c = 0; c < NORD; ++c) {
    T q[NORD];
#pragma unroll
    for (int l = 0; l < NORD; ++l) q[l] = Q[(c * NORD + l) * K + k];
#pragma unroll
    for (int l = 0; l < NORD; ++l) w[l] += q[l] * ch[c];
  }
}

template <typename T, int NORD>
__device__ __forceinline__ void contract_inv(const T* __restrict__ Q, int K, int k, const T* w, T* ch) {
#pragma unroll
  for (int c = 0; c < NORD; ++c) {
    T q[NORD];
#pragma unroll
    for (int l = 0; l < NORD; ++l) q[l] = Q[(c * NORD + l) * K + k];
    T acc = 0;
#pragma unroll
    for (int l = 0; l < NORD; ++l) acc += q[l] * w[l];
    ch[c] = acc;
  }
}

template <typename T, int NORD, int MODE, bool UPD, bool LF>
__global__ __launch_bounds__(LineCfg<T>::NT) void line_kernel(LineArgs<T> a) {
  constexpr int kNT = LineCfg<T>::NT, kMaxTPT = LineCfg<T>::TPT, kMaxCPT = LineCfg<T>::CPT;
  if (a.flag && *a.flag) return;
  constexpr int n = NORD, ne = NORD / 2, no = (NORD - 1) / 2, P = NORD / 2, NB = 1 + P;
  constexpr int NC = NORD > 1 ? NORD - 1 : 1;
  C2<T>* buf = reinterpret_cast<C2<T>*>(fftfem_lds);
  T* raw = reinterpret_cast<T*>(fftfem_lds);
  const int tid = threadIdx.x;
  const int K = a.K, lk = a.log2K, lg = a.log2G, G = 1 << lg;
  const int M = n * K - 1;
  const int ls = K + (G > 1 ? 1 : 0);  // complex slots per FFT buffer (pad between lines)
  const int LS = NB * ls * 2;  // T slots per line
  const int64_t l0 = (int64_t)xcd_remap(blockIdx.x, gridDim.x) << lg;
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
      T* dst = raw + g * LS;
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
      for (int g = 0; g < G; ++g) {
        const int64_t line = l0 + g;
        if (line >= a.nlines) break;
        const int64_t base = line * (int64_t)M;
        T* dst = raw + g * LS;
        for (int i0 = tid; i0 < M; i0 += 16 * kNT) {
          T v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            int i = i0 + u * kNT;
            v[u] = i < M ? load_in<T>(src, f64, base + i) : (T)0;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            int i = i0 + u * kNT;
            if (i < M) dst[i] = v[u];
          }
        }
      }
    }
  };
  double acc_c = 0, acc_u = 0;
  auto put = [&](int64_t idx, T v) {
    if constexpr (UPD) {
      double u = a.upd[idx] + (double)v;
      ((double*)a.out)[idx] = u;
      acc_c += (double)v * (double)v;
      acc_u += u * u;
    } else {
      store_out<T>(a.out, a.out_kind, idx, v);
    }
  };
  auto bulk_store = [&]() {
    if constexpr (LF) {
      const int g = tid & (G - 1);
      const int64_t line = l0 + g;
      if (line < a.nlines) {
        const int64_t base = line_base(a, line);
        const T* srcl = raw + g * LS;
        const int step = kNT >> lg;
        for (int i = tid >> lg; i < M; i += step) put(base + (int64_t)i * a.es, srcl[i]);
      }
    } else {
      for (int g = 0; g < G; ++g) {
        const int64_t line = l0 + g;
        if (line >= a.nlines) break;
        const int64_t base = line * (int64_t)M;
        const T* srcl = raw + g * LS;
        for (int i = tid; i < M; i += kNT) put(base + i, srcl[i]);
      }
    }
  };

  // per-line denominator base react + sum of the other axes' terms (MID)
  __shared__ T bden[64];
  if constexpr (MODE == MID) {
    if (tid < G) {
      int64_t line = l0 + tid;
      bden[tid] = line < a.nlines ? other_den(a, line_base(a, line)) : (T)1;
    }
  }
  const int ntask = G << lk;         // element tasks (g, j')
  const int lkh = lk - 1;
  const int nctask = G << lkh;       // contraction tasks (g, kappa), kappa < K/2

  if constexpr (MODE == FWD || MODE == MID) {
    bulk_load(a.in, a.in_f64);
    __syncthreads();
    // ---- gather: element j' -> nodal value (node j'+1) and channels ----
    T hv[kMaxTPT][NORD];
#pragma unroll
    for (int s = 0; s < kMaxTPT; ++s) {
      int t = tid + s * kNT;
      if (t < ntask) {
        int g = t >> lk, jp = t & (K - 1);
        const T* r = raw + g * LS + jp * n;
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
        int g = t >> lk, jp = t & (K - 1);
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
    fft_all<T, false, kNT>(buf, G * NB, lk, twf, ls);
  } else {
    bulk_load(a.in, a.in_f64);
    __syncthreads();
  }

  // ---------------- contraction per frequency pair -------------------------
  // held across a barrier: spectral results (FWD), channel spectra (INV), or
  // the nodal inverse inputs (MID)
  T hw[kMaxCPT][2][NORD];
#pragma unroll
  for (int s = 0; s < kMaxCPT; ++s) {
    int t = tid + s * kNT;
    if (t >= nctask) continue;
    int g = t >> lkh, kap = t & ((1 << lkh) - 1);
    int kb = kap == 0 ? 0 : K - kap;
    C2<T>* B = buf + g * NB * ls;
    const T* rs = raw + g * LS;
    T bd = (T)1;
    if constexpr (MODE == MID) bd = bden[g];
    T ca[NC], cb[NC];
    if constexpr (MODE != INV) {
      if constexpr (NORD > 1) {
        if (kap != 0) bubble_post<T, NORD>(B, ls, kap, kb, twm, ca, cb);
      }
    }
#pragma unroll
    for (int fi = 0; fi < 2; ++fi) {
      // fi = 0: k = kap (0 -> bubble block); fi = 1: k = K - kap (K/2 when kap = 0)
      int k = fi == 0 ? kap : (kap == 0 ? (K >> 1) : K - kap);
      if (fi == 1 && kap == 0 && K == 1) continue;
      int r = k == 0 ? n - 1 : n;
      int off = k == 0 ? 0 : n - 1 + (k - 1) * n;
      T ch[NORD], w[NORD];
      if constexpr (MODE != INV) {
        if (kap == 0) {
          // k = 0 (spectra at index 0) or k = K/2 (spectra at index K/2)
          if constexpr (NORD > 1) bubble_post<T, NORD>(B, ls, k, k, twm, ca, cb);
        }
        if (k == 0) {
#pragma unroll
          for (int b = 0; b < NORD - 1; ++b) ch[b] = ca[b];
          ch[NORD - 1] = 0;
        } else if (kap == 0) {  // k = K/2
          channel_vec<T, NORD>(nodal_post<T>(B, K, k, twd, false), ca, ca, ch);
        } else if (fi == 0) {
          channel_vec<T, NORD>(nodal_post<T>(B, K, k, twd, false), ca, cb, ch);
        } else {
          channel_vec<T, NORD>(nodal_post<T>(B, K, k, twd, false), cb, ca, ch);
        }
        if constexpr (MODE == MID && sizeof(T) == 4) {
          // one load of Q_k for the forward contraction, the division and the inverse
          T q[NORD][NORD];
#pragma unroll
          for (int c = 0; c < NORD; ++c)
#pragma unroll
            for (int l = 0; l < NORD; ++l) q[c][l] = a.Q[(c * NORD + l) * K + k];
#pragma unroll
          for (int l = 0; l < NORD; ++l) {
            T acc = 0;
#pragma unroll
            for (int c = 0; c < NORD; ++c) acc += q[c][l] * ch[c];
            w[l] = l < r ? acc / (bd + a.mu_self[off + l]) : (T)0;
          }
#pragma unroll
          for (int c = 0; c < NORD; ++c) {
            T acc = 0;
#pragma unroll
            for (int l = 0; l < NORD; ++l) acc += q[c][l] * w[l];
            hw[s][fi][c] = acc;
          }
          continue;
        }
        contract_fwd<T, NORD>(a.Q, K, k, ch, w);
        if constexpr (MODE == MID) {
#pragma unroll
          for (int l = 0; l < NORD; ++l) w[l] = l < r ? w[l] / (bd + a.mu_self[off + l]) : (T)0;
        }
      } else {
#pragma unroll
        for (int l = 0; l < NORD; ++l) w[l] = l < r ? rs[off + l] : (T)0;
      }
      if constexpr (MODE == FWD) {
#pragma unroll
        for (int l = 0; l < NORD; ++l) hw[s][fi][l] = w[l];
        continue;
      }
      contract_inv<T, NORD>(a.Q, K, k, w, ch);
#pragma unroll
      for (int c = 0; c < NORD; ++c) hw[s][fi][c] = ch[c];
    }
    if constexpr (MODE == MID) {
      // bubble pre-twiddle now (pair-local); nodal after the barrier
      if constexpr (NORD > 1) {
        T ya[NC], yb[NC];
        if (kap == 0) {
#pragma unroll
          for (int b = 0; b < NORD - 1; ++b) {
            ya[b] = hw[s][0][b];  // index 0 of every channel (k = 0 block)
          }
#pragma unroll
          for (int m = 1; m <= ne; ++m) yb[m - 1] = hw[s][1][m];
#pragma unroll
          for (int m = 1; m <= no; ++m) yb[ne + m - 1] = hw[s][1][ne + m];
#pragma unroll
          for (int p = 1; p <= P; ++p) {
            int b0 = 2 * (p - 1), b1 = b0 + 1;
            bool has1 = b1 < NORD - 1;
            C2<T> v0 = {ya[b0], has1 ? ya[b1] : (T)0};
            B[p * ls] = v0;
            int h = K >> 1;
            C2<T> va = herm<T>(yb[b0], yb[b0], h, twm);
            C2<T> vb = has1 ? herm<T>(yb[b1], yb[b1], h, twm) : C2<T>{0, 0};
            B[p * ls + h] = {va.x - vb.y, va.y + vb.x};
          }
        } else {
          // channel spectra at FFT index kap (ya) and kb (yb): even channels
          // of frequency k sit at K - k, odd channels at k
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
            B[p * ls + kap] = {va.x - vb.y, va.y + vb.x};
            va = herm<T>(yb[b0], ya[b0], kb, twm);
            vb = has1 ? herm<T>(yb[b1], ya[b1], kb, twm) : C2<T>{0, 0};
            B[p * ls + kb] = {va.x - vb.y, va.y + vb.x};
          }
        }
      }
    }
  }
  __syncthreads();

  if constexpr (MODE == FWD) {
    // spectral results -> LDS (line layout) -> coalesced store
#pragma unroll
    for (int s = 0; s < kMaxCPT; ++s) {
      int t = tid + s * kNT;
      if (t >= nctask) continue;
      int g = t >> lkh, kap = t & ((1 << lkh) - 1);
      T* rs = raw + g * LS;
#pragma unroll
      for (int fi = 0; fi < 2; ++fi) {
        int k = fi == 0 ? kap : (kap == 0 ? (K >> 1) : K - kap);
        if (fi == 1 && kap == 0 && K == 1) continue;
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
      int g = t >> lkh, kap = t & ((1 << lkh) - 1);
      int kb = kap == 0 ? 0 : K - kap;
      C2<T>* B = buf + g * NB * ls;
      if (kap == 0) {
        write_nodal_zeros(B, K);
        write_nodal_inv(B, K, K >> 1, hw[s][1][0]);
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
            B[p * ls] = {ya[b0], has1 ? ya[b1] : (T)0};
            int h = K >> 1;
            C2<T> va = herm<T>(yb[b0], yb[b0], h, twm);
            C2<T> vb = has1 ? herm<T>(yb[b1], yb[b1], h, twm) : C2<T>{0, 0};
            B[p * ls + h] = {va.x - vb.y, va.y + vb.x};
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
            B[p * ls + kap] = {va.x - vb.y, va.y + vb.x};
            va = herm<T>(yb[b0], ya[b0], kb, twm);
            vb = has1 ? herm<T>(yb[b1], ya[b1], kb, twm) : C2<T>{0, 0};
            B[p * ls + kb] = {va.x - vb.y, va.y + vb.x};
          }
        }
      }
    }
    __syncthreads();
    fft_all<T, true, kNT>(buf, G * NB, lk, twf, ls);
  }

  // ---------------- scatter: channels -> bubble vectors and nodes ----------
  {
    T hv[kMaxTPT][NORD];
#pragma unroll
    for (int s = 0; s < kMaxTPT; ++s) {
      int t = tid + s * kNT;
      if (t < ntask) {
        int g = t >> lk, jp = t & (K - 1);
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
        int g = t >> lk, jp = t & (K - 1);
        T* r = raw + g * LS + jp * n;
#pragma unroll
        for (int m = 0; m < n - 1; ++m) r[m] = hv[s][m];
        if (jp < K - 1) r[n - 1] = hv[s][n - 1];
      }
    }
    __syncthreads();
    bulk_store();
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
      a.partials[2 * blockIdx.x] = red[0][0];
      a.partials[2 * blockIdx.x + 1] = red[1][0];
    }
  }
}

template <typename F>
static void allow_lds(F* fn, size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int NORD, int MODE, bool UPD>
static hipError_t go(bool lf, const LineArgs<T>& a, int nblocks, size_t lds, hipStream_t s) {
  if (lf) {
    allow_lds(line_kernel<T, NORD, MODE, UPD, true>, lds);
    hipLaunchKernelGGL((line_kernel<T, NORD, MODE, UPD, true>), dim3(nblocks), dim3(LineCfg<T>::NT), lds, s, a);
  } else {
    allow_lds(line_kernel<T, NORD, MODE, UPD, false>, lds);
    hipLaunchKernelGGL((line_kernel<T, NORD, MODE, UPD, false>), dim3(nblocks), dim3(LineCfg<T>::NT), lds, s, a);
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

template <typename T>
hipError_t launch_line(int n, int mode, bool upd, const LineArgs<T>& a, int nblocks, size_t lds,
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

template hipError_t launch_line<float>(int, int, bool, const LineArgs<float>&, int, size_t, hipStream_t);
template hipError_t launch_line<double>(int, int, bool, const LineArgs<double>&, int, size_t, hipStream_t);

}  // namespace fftfem
