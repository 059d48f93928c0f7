// HIP kernels (gfx950) of the fast direct FEM solver.
//
// A "line pass" applies, along one axis of an N-D array, the direct FC_n
// transform (FWD), the inverse F_n transform (INV) or both with the pointwise
// division in between (MID), to a tile of G lines held in LDS (Sect. 3,
// Theorem 2; Sect. 4, algorithm (a)).  Per line of M = nK - 1 dofs:
//
//   gather     nodal values -> odd extension of length 2K packed as K complex
//              values (y_{2q} + i y_{2q+1}); bubble vectors -> even/odd
//              channels (Sect. 2 split), two real channels per complex buffer,
//              in the even/odd reordering that turns a DCT-II into a K-point
//              complex DFT; even channels are sign-alternated so that their
//              DST-II comes out of the same DCT-II.
//   FFT        in-place Stockham radix-4/2 on all buffers of the tile.
//   contract   per frequency pair {k, K-k} one thread untangles the packed
//              spectra (DST-I of the nodes, DST-II of the even channels,
//              DCT-II of the odd channels) and applies the n x n table Q_k
//              (Q_k^T forward, Q_k inverse); k = 0 is the bubble-only block.
//   inverse    the transposes: DST-I again (as a forward DFT, done as a
//              conjugated inverse DFT), DCT-III/DST-III via the Hermitian
//              pre-twiddle and an unnormalized inverse DFT.
//   scatter    channels -> bubble vectors and nodes, written to HBM.
//
// Workgroups are 256 threads; blockIdx is remapped so that consecutive tiles
// run on the same XCD (the hardware deals workgroups round-robin over the
// eight XCDs), which keeps neighbouring column tiles of a strided axis in one
// L2.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fftfem_internal.h"
#include "launch.h"

namespace fftfem {

constexpr int kThreads = 256;
constexpr int kMaxTasks = 4;  // contraction tasks held per thread in a MID pass

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int X = 8;
  int q = nblocks / X, r = nblocks % X;
  int xcd = bid % X, idx = bid / X;
  return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Dynamic LDS of every kernel in this file (one declaration: 16-byte aligned).
extern __shared__ double2 fftfem_lds[];

template <typename T>
__device__ __forceinline__ T load_in(const void* p, int f64, int64_t i) {
  return f64 ? (T)((const double*)p)[i] : ((const T*)p)[i];
}
template <typename T>
__device__ __forceinline__ void store_out(void* p, int f64, int64_t i, T v) {
  if (f64)
    ((double*)p)[i] = (double)v;
  else
    ((T*)p)[i] = v;
}
template <typename T>
__device__ __forceinline__ void set_comp(C2<T>* b, int idx, int comp, T v) {
  reinterpret_cast<T*>(b + idx)[comp] = v;
}
template <typename T>
__device__ __forceinline__ T get_comp(const C2<T>* b, int idx, int comp) {
  return reinterpret_cast<const T*>(b + idx)[comp];
}

// ---------------------------------------------------------------------------
// Batched in-place Stockham FFT over `nfft` contiguous buffers of length K.
// Each stage: every thread reads up to 8/R butterflies into registers,
// barrier, twiddle + R-point DFT, write, barrier.  Chunks of the butterfly
// range always cover whole buffers (K <= 2048), so reads and writes of a
// chunk touch the same set of elements.
template <typename T, int R, bool INVDIR>
__device__ __forceinline__ void butterfly(C2<T>* v) {
  if constexpr (R == 2) {
    C2<T> a = v[0], b = v[1];
    v[0] = {a.x + b.x, a.y + b.y};
    v[1] = {a.x - b.x, a.y - b.y};
  } else {
    C2<T> s02 = {v[0].x + v[2].x, v[0].y + v[2].y};
    C2<T> d02 = {v[0].x - v[2].x, v[0].y - v[2].y};
    C2<T> s13 = {v[1].x + v[3].x, v[1].y + v[3].y};
    C2<T> d13 = {v[1].x - v[3].x, v[1].y - v[3].y};
    // forward: multiply d13 by -i; inverse: by +i
    C2<T> rot = INVDIR ? C2<T>{-d13.y, d13.x} : C2<T>{d13.y, -d13.x};
    v[0] = {s02.x + s13.x, s02.y + s13.y};
    v[2] = {s02.x - s13.x, s02.y - s13.y};
    v[1] = {d02.x + rot.x, d02.y + rot.y};
    v[3] = {d02.x - rot.x, d02.y - rot.y};
  }
}

template <typename T, int R, bool INVDIR>
__device__ void fft_stage(C2<T>* buf, int nfft, int K, int Ns, const C2<T>* __restrict__ tw) {
  constexpr int MAXB = 8 / R;
  const int KR = K / R;
  const int total = nfft * KR;
  const int tid = threadIdx.x;
  const int tstride = K / (Ns * R);
  for (int base = 0; base < total; base += kThreads * MAXB) {
    C2<T> v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
      int b = base + t * kThreads + tid;
      dst[t] = -1;
      if (b < total) {
        int f = b / KR, j = b - f * KR;
        C2<T>* x = buf + (int64_t)f * K;
        int k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][r] = x[j + r * KR];
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C2<T> w = tw[r * k * tstride];
          v[t][r] = INVDIR ? cmulc(v[t][r], w) : cmul(v[t][r], w);
        }
        butterfly<T, R, INVDIR>(v[t]);
        dst[t] = f * K + (j - k) * R + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXB; ++t)
      if (dst[t] >= 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[dst[t] + r * Ns] = v[t][r];
      }
    __syncthreads();
  }
}

template <typename T, bool INVDIR>
__device__ void fft_all(C2<T>* buf, int nfft, int K, int log2K, const C2<T>* tw) {
  int Ns = 1, rem = log2K;
  if (rem & 1) {
    fft_stage<T, 2, INVDIR>(buf, nfft, K, Ns, tw);
    Ns *= 2;
    rem -= 1;
  }
  while (rem >= 2) {
    fft_stage<T, 4, INVDIR>(buf, nfft, K, Ns, tw);
    Ns *= 4;
    rem -= 2;
  }
}

// ---------------------------------------------------------------------------
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

// Untangle the packed forward spectra at FFT index pair {kap, kb} and form
// the channel vectors of the frequencies they carry.
template <typename T, int NORD>
struct PairSpectra {
  static constexpr int n = NORD, ne = NORD / 2, no = (NORD - 1) / 2, P = NORD / 2;
  T ca[NORD > 1 ? NORD - 1 : 1];  // DCT-II value of bubble channel b at index kap
  T cb[NORD > 1 ? NORD - 1 : 1];  // ... at index kb
};

template <typename T, int NORD>
__device__ __forceinline__ void bubble_post(const C2<T>* B, int K, int kap, int kb,
                                            const C2<T>* twm, PairSpectra<T, NORD>& s) {
  constexpr int P = NORD / 2;
#pragma unroll
  for (int p = 1; p <= P; ++p) {
    C2<T> Va = B[p * K + kap], Vb = B[p * K + kb];
    // index kap: Pv = Va, Qv = conj(Vb)
    {
      C2<T> w = twm[kap];
      C2<T> sm = {Va.x + Vb.x, Va.y - Vb.y};
      C2<T> df = {Va.x - Vb.x, Va.y + Vb.y};
      C2<T> ws = cmul(w, sm), wd = cmul(w, df);
      s.ca[2 * (p - 1)] = ws.x * (T)0.5;
      if (2 * (p - 1) + 1 < NORD - 1) s.ca[2 * (p - 1) + 1] = wd.y * (T)0.5;
    }
    {
      C2<T> w = twm[kb];
      C2<T> sm = {Vb.x + Va.x, Vb.y - Va.y};
      C2<T> df = {Vb.x - Va.x, Vb.y + Va.y};
      C2<T> ws = cmul(w, sm), wd = cmul(w, df);
      s.cb[2 * (p - 1)] = ws.x * (T)0.5;
      if (2 * (p - 1) + 1 < NORD - 1) s.cb[2 * (p - 1) + 1] = wd.y * (T)0.5;
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
  // F = (zk + conj zm)/2, G = (zk - conj zm)/(2i), Y = F + twd[k] G, value = -Im(Y)/2
  C2<T> F = {(zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5};
  C2<T> d = {zk.x - zm.x, zk.y + zm.y};
  C2<T> Gv = {d.y * (T)0.5, -d.x * (T)0.5};
  C2<T> Y = cmul(twd[k], Gv);
  return -(F.y + Y.y) * (T)0.5;
}

// Hermitian pre-twiddle of a DCT-III input at index idx:
// V = exp(i pi idx/(2K)) (y~[idx] - i y~[K-idx]) / 2, with y~[0] = 2 y[0], y~[K] = 0.
template <typename T>
__device__ __forceinline__ C2<T> herm(T y_idx, T y_mirror, int idx, const C2<T>* twm) {
  if (idx == 0) return {y_idx, (T)0};
  C2<T> w = twm[idx];
  C2<T> v = {y_idx * (T)0.5, -y_mirror * (T)0.5};
  return cmulc(v, w);
}

template <typename T>
__device__ __forceinline__ void write_nodal_inv(C2<T>* Z, int K, int k, T val) {
  // conj of the odd-extension packing: y_t -> component t%2 of Z[t/2], imaginary negated
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

template <typename T, int NORD, int MODE, bool UPD>
__global__ __launch_bounds__(kThreads) void line_kernel(LineArgs<T> a) {
  if (a.flag && *a.flag) return;
  constexpr int n = NORD, ne = NORD / 2, no = (NORD - 1) / 2, P = NORD / 2, NB = 1 + P;
  C2<T>* buf = reinterpret_cast<C2<T>*>(fftfem_lds);
  const int tid = threadIdx.x;
  const int K = a.K;
  const int G = a.G;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t l0 = (int64_t)tile * G;
  const bool lines_fast = a.es > 1;
  const C2<T>* twf = reinterpret_cast<const C2<T>*>(a.twf);
  const C2<T>* twm = reinterpret_cast<const C2<T>*>(a.twm);
  const C2<T>* twd = reinterpret_cast<const C2<T>*>(a.twd);
  const int halfK = (K + 1) / 2;  // contraction tasks per line

  if constexpr (MODE == FWD || MODE == MID) {
    // ---- gather: nodes -> odd extension (packed) ----
    for (int t = tid; t < G * K; t += kThreads) {
      int g, j;
      if (lines_fast) {
        g = t % G;
        j = t / G;
      } else {
        j = t % K;
        g = t / K;
      }
      C2<T>* Z = buf + (int64_t)g * NB * K;
      int64_t line = l0 + g;
      if (j == 0) {
        write_nodal_zeros(Z, K);
        continue;
      }
      T x = 0;
      if (line < a.nlines) x = load_in<T>(a.in, a.in_f64, line_base(a, line) + (int64_t)(j * n - 1) * a.es);
      set_comp(Z, j >> 1, j & 1, x);
      int tt = 2 * K - j;
      set_comp(Z, tt >> 1, tt & 1, -x);
    }
    // ---- gather: bubbles -> even/odd channels, reordered for the DCT ----
    if constexpr (ne > 0) {
      for (int t = tid; t < G * K * ne; t += kThreads) {
        int g, rest, jp, m;
        if (lines_fast) {
          g = t % G;
          rest = t / G;
        } else {
          g = t / (K * ne);
          rest = t - g * (K * ne);
        }
        m = rest % ne + 1;
        jp = rest / ne;
        C2<T>* B = buf + (int64_t)g * NB * K;
        int64_t line = l0 + g;
        int qi = (jp & 1) ? K - 1 - (jp >> 1) : (jp >> 1);
        T sg = (jp & 1) ? (T)-1 : (T)1;
        T va = 0, vb = 0;
        bool mid = (2 * m == n);
        if (line < a.nlines) {
          int64_t base = line_base(a, line);
          va = load_in<T>(a.in, a.in_f64, base + (int64_t)(jp * n + m - 1) * a.es);
          if (!mid) vb = load_in<T>(a.in, a.in_f64, base + (int64_t)(jp * n + n - m - 1) * a.es);
        }
        int be = m - 1;
        set_comp(B + (1 + be / 2) * K, qi, be & 1, sg * (mid ? va : va + vb));
        if (!mid) {
          int bo = ne + m - 1;
          set_comp(B + (1 + bo / 2) * K, qi, bo & 1, va - vb);
        }
        if (((n - 1) & 1) && m == 1) set_comp(B + P * K, qi, 1, (T)0);
      }
    }
    __syncthreads();
    fft_all<T, false>(buf, G * NB, K, a.log2K, twf);
  }

  // ---- contraction (and division) per frequency pair ----
  T hold[kMaxTasks][2];
  int hold_g[kMaxTasks], hold_kap[kMaxTasks];
  int nheld = 0;
  for (int t = tid; t < G * halfK; t += kThreads) {
    int g, kap;
    if (lines_fast) {
      g = t % G;
      kap = t / G;
    } else {
      kap = t % halfK;
      g = t / halfK;
    }
    int64_t line = l0 + g;
    bool valid = line < a.nlines;
    int64_t base = valid ? line_base(a, line) : 0;
    C2<T>* B = buf + (int64_t)g * NB * K;
    int kb = (K - kap) % K;
    // frequencies handled: kap==0 -> {0 (bubble block), K/2 if K even}; else {kap, K-kap}
    int kf[2];
    int nf = 0;
    if (kap == 0) {
      kf[nf++] = 0;
      if (!(K & 1)) kf[nf++] = K / 2;
    } else {
      kf[nf++] = kap;
      kf[nf++] = K - kap;
    }
    PairSpectra<T, NORD> s;
    if constexpr (MODE != INV) {
      if constexpr (NORD > 1) bubble_post<T, NORD>(B, K, kap, kb, twm, s);
    }
    // DCT-III inputs per channel at indices kap (ya) and kb (yb), filled below
    T ya[NORD > 1 ? NORD - 1 : 1], yb[NORD > 1 ? NORD - 1 : 1];
    T nodal_out[2] = {0, 0};
    T ymid[NORD > 1 ? NORD - 1 : 1];  // DCT-III input at K/2 (kap == 0, K even)
    for (int fi = 0; fi < nf; ++fi) {
      int k = kf[fi];
      T ch[NORD];
      const T* Qk = a.Q + (int64_t)k * n * n;
      T w[NORD];
      int off;
      int r;  // rank of the block
      if (k == 0) {
        r = n - 1;
        off = 0;
      } else {
        r = n;
        off = n - 1 + (k - 1) * n;
      }
      if constexpr (MODE != INV) {
        if (k == 0) {
#pragma unroll
          for (int b = 0; b < NORD - 1; ++b) ch[b] = s.ca[b];  // index 0 for every bubble channel
        } else {
          // which stored index holds k: kap or kb
          bool at_kap = (k == kap);
          ch[0] = nodal_post<T>(B, K, k, twd, false);
          if (k == K / 2 && kap == 0) {
            // K even, middle frequency: spectra at index K/2 for all channels
            PairSpectra<T, NORD> s2;
            if constexpr (NORD > 1) bubble_post<T, NORD>(B, K, K / 2, K / 2, twm, s2);
#pragma unroll
            for (int m = 1; m <= ne; ++m) ch[m] = s2.ca[m - 1];
#pragma unroll
            for (int m = 1; m <= no; ++m) ch[ne + m] = s2.ca[ne + m - 1];
          } else {
            // even channels: DST-II at k = DCT-II at K-k; odd: DCT-II at k
#pragma unroll
            for (int m = 1; m <= ne; ++m) ch[m] = at_kap ? s.cb[m - 1] : s.ca[m - 1];
#pragma unroll
            for (int m = 1; m <= no; ++m) ch[ne + m] = at_kap ? s.ca[ne + m - 1] : s.cb[ne + m - 1];
          }
        }
#pragma unroll
        for (int l = 0; l < NORD; ++l) {
          T acc = 0;
#pragma unroll
          for (int c = 0; c < NORD; ++c)
            if (c < r && l < r) acc += Qk[c * n + l] * ch[c];
          w[l] = acc;
        }
      }
      if constexpr (MODE == FWD) {
        if (valid)
          for (int l = 0; l < r; ++l)
            store_out<T>(a.out, a.out_f64, base + (int64_t)(off + l) * a.es, w[l]);
        continue;
      }
      if constexpr (MODE == INV) {
#pragma unroll
        for (int l = 0; l < NORD; ++l)
          w[l] = (valid && l < r) ? load_in<T>(a.in, a.in_f64, base + (int64_t)(off + l) * a.es) : (T)0;
      }
      if constexpr (MODE == MID) {
        T bd = valid ? other_den(a, base) : (T)1;
#pragma unroll
        for (int l = 0; l < NORD; ++l)
          if (l < r) w[l] = w[l] / (bd + a.mu_self[off + l]);
      }
      // inverse contraction: channel spectra
#pragma unroll
      for (int c = 0; c < NORD; ++c) {
        T acc = 0;
#pragma unroll
        for (int l = 0; l < NORD; ++l)
          if (c < r && l < r) acc += Qk[c * n + l] * w[l];
        ch[c] = acc;
      }
      // route channel spectra to DCT-III inputs
      if (k == 0) {
#pragma unroll
        for (int b = 0; b < NORD - 1; ++b) ya[b] = ch[b];  // index 0 (kap = kb = 0)
      } else if (kap == 0) {
        // k = K/2: every channel's DCT-III input sits at index K/2
        nodal_out[1] = ch[0];
#pragma unroll
        for (int m = 1; m <= ne; ++m) ymid[m - 1] = ch[m];
#pragma unroll
        for (int m = 1; m <= no; ++m) ymid[ne + m - 1] = ch[ne + m];
      } else {
        bool at_kap = (k == kap);
        nodal_out[at_kap ? 0 : 1] = ch[0];
        // odd: DCT-III index k; even: reversed, index K-k
#pragma unroll
        for (int m = 1; m <= ne; ++m) {
          if (at_kap)
            yb[m - 1] = ch[m];
          else
            ya[m - 1] = ch[m];
        }
#pragma unroll
        for (int m = 1; m <= no; ++m) {
          if (at_kap)
            ya[ne + m - 1] = ch[ne + m];
          else
            yb[ne + m - 1] = ch[ne + m];
        }
      }
    }
    if constexpr (MODE == FWD) continue;
    // ---- pre-twiddle for the inverse transforms (pair-local for bubbles) ----
    if constexpr (NORD > 1) {
#pragma unroll
      for (int p = 1; p <= P; ++p) {
        int b0 = 2 * (p - 1), b1 = b0 + 1;
        bool has1 = b1 < NORD - 1;
        if (kap == 0) {
          C2<T> v0a = herm<T>(ya[b0], (T)0, 0, twm);
          C2<T> v0b = has1 ? herm<T>(ya[b1], (T)0, 0, twm) : C2<T>{0, 0};
          B[p * K + 0] = {v0a.x - v0b.y, v0a.y + v0b.x};
          if (!(K & 1)) {
            int h = K / 2;
            C2<T> va = herm<T>(ymid[b0], ymid[b0], h, twm);
            C2<T> vb = has1 ? herm<T>(ymid[b1], ymid[b1], h, twm) : C2<T>{0, 0};
            B[p * K + h] = {va.x - vb.y, va.y + vb.x};
          }
        } else {
          C2<T> va = herm<T>(ya[b0], yb[b0], kap, twm);
          C2<T> vb = has1 ? herm<T>(ya[b1], yb[b1], kap, twm) : C2<T>{0, 0};
          B[p * K + kap] = {va.x - vb.y, va.y + vb.x};
          va = herm<T>(yb[b0], ya[b0], kb, twm);
          vb = has1 ? herm<T>(yb[b1], ya[b1], kb, twm) : C2<T>{0, 0};
          B[p * K + kb] = {va.x - vb.y, va.y + vb.x};
        }
      }
    }
    if constexpr (MODE == INV) {
      // nothing read the nodal buffer: write now
      if (kap == 0) {
        write_nodal_zeros(B, K);
        if (!(K & 1)) write_nodal_inv(B, K, K / 2, nodal_out[1]);
      } else {
        write_nodal_inv(B, K, kap, nodal_out[0]);
        write_nodal_inv(B, K, K - kap, nodal_out[1]);
      }
    } else {
      hold[nheld][0] = nodal_out[0];
      hold[nheld][1] = nodal_out[1];
      hold_g[nheld] = g;
      hold_kap[nheld] = kap;
      ++nheld;
    }
  }
  if constexpr (MODE == FWD) return;
  if constexpr (MODE == MID) {
    __syncthreads();  // every thread has read the forward nodal spectra
    for (int i = 0; i < nheld; ++i) {
      C2<T>* B = buf + (int64_t)hold_g[i] * NB * K;
      int kap = hold_kap[i];
      if (kap == 0) {
        write_nodal_zeros(B, K);
        if (!(K & 1)) write_nodal_inv(B, K, K / 2, hold[i][1]);
      } else {
        write_nodal_inv(B, K, kap, hold[i][0]);
        write_nodal_inv(B, K, K - kap, hold[i][1]);
      }
    }
  }
  __syncthreads();
  fft_all<T, true>(buf, G * NB, K, a.log2K, twf);

  // ---- scatter ----
  double acc_c = 0, acc_u = 0;
  for (int t = tid; t < G * K; t += kThreads) {
    int g, j;
    if (lines_fast) {
      g = t % G;
      j = t / G;
    } else {
      j = t % K;
      g = t / K;
    }
    int64_t line = l0 + g;
    if (j == 0 || line >= a.nlines) continue;
    const C2<T>* Z = buf + (int64_t)g * NB * K;
    T x = nodal_post<T>(Z, K, j, twd, true);
    int64_t idx = line_base(a, line) + (int64_t)(j * n - 1) * a.es;
    if constexpr (UPD) {
      double u = a.upd[idx] + (double)x;
      ((double*)a.out)[idx] = u;
      acc_c += (double)x * (double)x;
      acc_u += u * u;
    } else {
      store_out<T>(a.out, a.out_f64, idx, x);
    }
  }
  if constexpr (ne > 0) {
    for (int t = tid; t < G * K * ne; t += kThreads) {
      int g, rest;
      if (lines_fast) {
        g = t % G;
        rest = t / G;
      } else {
        g = t / (K * ne);
        rest = t - g * (K * ne);
      }
      int m = rest % ne + 1;
      int jp = rest / ne;
      int64_t line = l0 + g;
      if (line >= a.nlines) continue;
      const C2<T>* B = buf + (int64_t)g * NB * K;
      int qi = (jp & 1) ? K - 1 - (jp >> 1) : (jp >> 1);
      T sg = (jp & 1) ? (T)-1 : (T)1;
      int be = m - 1;
      T E = sg * get_comp(B + (1 + be / 2) * K, qi, be & 1);
      int64_t base = line_base(a, line);
      T v1, v2 = 0;
      bool mid = (2 * m == n);
      if (mid) {
        v1 = E;
      } else {
        int bo = ne + m - 1;
        T O = get_comp(B + (1 + bo / 2) * K, qi, bo & 1);
        v1 = E + O;
        v2 = E - O;
      }
      int64_t i1 = base + (int64_t)(jp * n + m - 1) * a.es;
      int64_t i2 = base + (int64_t)(jp * n + n - m - 1) * a.es;
      if constexpr (UPD) {
        double u1 = a.upd[i1] + (double)v1;
        ((double*)a.out)[i1] = u1;
        acc_c += (double)v1 * (double)v1;
        acc_u += u1 * u1;
        if (!mid) {
          double u2 = a.upd[i2] + (double)v2;
          ((double*)a.out)[i2] = u2;
          acc_c += (double)v2 * (double)v2;
          acc_u += u2 * u2;
        }
      } else {
        store_out<T>(a.out, a.out_f64, i1, v1);
        if (!mid) store_out<T>(a.out, a.out_f64, i2, v2);
      }
    }
  }
  if constexpr (UPD) {
    // block reduction of the two sums (fixed order: deterministic)
    __shared__ double red[2][kThreads];
    red[0][tid] = acc_c;
    red[1][tid] = acc_u;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
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

// ---------------------------------------------------------------------------
// 1D operator application along one axis (float64), for y = A u and the
// refinement residual.  For output position g of a line (Sect. 2, the
// element-by-element assembly of A and C):
//   node (g+1) % n == 0:  sum_t X[n][t] v[g-n+t] + sum_t X[0][t] v[g+t]
//   bubble l = g % n + 1: sum_t X[l][t] v[g-l+t]
// with v = 0 outside the line (Dirichlet).  Two inputs and two outputs with
// coefficient rows let one pass produce the sum-factorized partial products:
//   o1 = c1[0] A in1 + c1[1] C in1 + c1[2] A in2 + c1[3] C in2   (o1 = f - that, if sub_f)
//   o2 = c2[0] A in1 + c2[1] C in1 + c2[2] A in2 + c2[3] C in2
template <int NORD>
__device__ __forceinline__ void stencil(const double* __restrict__ v, int i, const double* X,
                                        double& out) {
  constexpr int n = NORD;
  double s = 0;
  if ((i + 1) % n == 0) {
#pragma unroll
    for (int t = 0; t <= n; ++t) s += X[n * (n + 1) + t] * v[i - n + t] + X[t] * v[i + t];
  } else {
    int l = i % n + 1;
#pragma unroll
    for (int t = 0; t <= n; ++t) s += X[l * (n + 1) + t] * v[i - l + t];
  }
  out = s;
}

template <int NORD>
__global__ __launch_bounds__(kThreads) void apply_kernel(ApplyArgs a) {
  if (a.flag && *a.flag) return;
  constexpr int n = NORD;
  double* sm = reinterpret_cast<double*>(fftfem_lds);
  __shared__ double Xa[(NORD + 1) * (NORD + 1)], Xc[(NORD + 1) * (NORD + 1)];
  const int tid = threadIdx.x;
  for (int i = tid; i < (n + 1) * (n + 1); i += kThreads) {
    Xa[i] = a.Ael[i];
    Xc[i] = a.Cel[i];
  }
  const int G = a.G, TL = a.TL, W = TL + 2 * n;
  const int64_t nseg = (a.M + TL - 1) / TL;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t lg = tile / nseg, seg = tile - lg * nseg;
  const int64_t l0 = lg * G, s0 = seg * TL;
  const bool lines_fast = a.es > 1;
  const bool two = a.in2 != nullptr;
  double* v1 = sm;
  double* v2 = sm + G * W;
  for (int t = tid; t < G * W; t += kThreads) {
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
    double x1 = 0, x2 = 0;
    if (line < a.nlines && pos >= 0 && pos < a.M) {
      int64_t outer = line / a.es, inner = line - outer * a.es;
      int64_t idx = outer * a.M * a.es + inner + pos * a.es;
      x1 = a.in1[idx];
      if (two) x2 = a.in2[idx];
    }
    v1[g * W + i] = x1;
    if (two) v2[g * W + i] = x2;
  }
  __syncthreads();
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
    // local index within the window: pos - (s0 - n); the stencil uses the
    // position along the line for the node/bubble pattern
    const double* w1 = v1 + g * W + n - s0;  // w1[pos] = window value at pos
    double A1, C1, A2 = 0, C2v = 0;
    stencil<NORD>(w1, (int)pos, Xa, A1);
    stencil<NORD>(w1, (int)pos, Xc, C1);
    if (two) {
      const double* w2 = v2 + g * W + n - s0;
      stencil<NORD>(w2, (int)pos, Xa, A2);
      stencil<NORD>(w2, (int)pos, Xc, C2v);
    }
    int64_t outer = line / a.es, inner = line - outer * a.es;
    int64_t idx = outer * a.M * a.es + inner + pos * a.es;
    double r1 = a.c1[0] * A1 + a.c1[1] * C1 + a.c1[2] * A2 + a.c1[3] * C2v;
    if (a.sub_f) r1 = a.f[idx] - r1;
    if (a.o1_f64)
      ((double*)a.o1)[idx] = r1;
    else
      ((float*)a.o1)[idx] = (float)r1;
    if (a.o2) a.o2[idx] = a.c2[0] * A1 + a.c2[1] * C1 + a.c2[2] * A2 + a.c2[3] * C2v;
  }
}

// ---------------------------------------------------------------------------
// Refinement bookkeeping.  stats layout (doubles): [0] iterations applied,
// [1] converged flag, [2 + i] relative correction of iteration i.
__global__ void reset_kernel(int* flag, double* stats, int nstats) {
  int i = threadIdx.x;
  if (i == 0) *flag = 0;
  for (int j = i; j < nstats; j += blockDim.x) stats[j] = 0;
}

__global__ void reduce_kernel(const double* partials, int nparts, int iter, double tol,
                              int* flag, double* stats) {
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
    double rel = r1[0] > 0 ? sqrt(r0[0] / r1[0]) : 0.0;
    stats[2 + iter] = rel;
    stats[0] = iter;
    if (iter > 0 && rel <= tol) {
      stats[1] = 1;
      *flag = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
template <typename F>
static void allow_lds(F* fn, size_t lds) {
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int NORD>
static hipError_t launch_line_n(int mode, bool upd, const LineArgs<T>& a, int nblocks,
                                size_t lds, hipStream_t s) {
  allow_lds(line_kernel<T, NORD, FWD, false>, lds);
  allow_lds(line_kernel<T, NORD, INV, false>, lds);
  allow_lds(line_kernel<T, NORD, INV, true>, lds);
  allow_lds(line_kernel<T, NORD, MID, false>, lds);
  allow_lds(line_kernel<T, NORD, MID, true>, lds);
  if (mode == FWD) {
    hipLaunchKernelGGL((line_kernel<T, NORD, FWD, false>), dim3(nblocks), dim3(kThreads), lds, s, a);
  } else if (mode == INV) {
    if (upd)
      hipLaunchKernelGGL((line_kernel<T, NORD, INV, true>), dim3(nblocks), dim3(kThreads), lds, s, a);
    else
      hipLaunchKernelGGL((line_kernel<T, NORD, INV, false>), dim3(nblocks), dim3(kThreads), lds, s, a);
  } else {
    if (upd)
      hipLaunchKernelGGL((line_kernel<T, NORD, MID, true>), dim3(nblocks), dim3(kThreads), lds, s, a);
    else
      hipLaunchKernelGGL((line_kernel<T, NORD, MID, false>), dim3(nblocks), dim3(kThreads), lds, s, a);
  }
  return hipGetLastError();
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

hipError_t launch_apply(int n, const ApplyArgs& a, int nblocks, size_t lds, hipStream_t s) {
  switch (n) {
#define FFTFEM_CASE(N)                                                                       \
  case N:                                                                                    \
    hipLaunchKernelGGL((apply_kernel<N>), dim3(nblocks), dim3(kThreads), lds, s, a);         \
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

hipError_t launch_reduce(const double* partials, int nparts, int iter, double tol, int* flag,
                         double* stats, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, nparts, iter, tol,
                     flag, stats);
  return hipGetLastError();
}

}  // namespace fftfem
