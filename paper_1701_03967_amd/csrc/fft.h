// Batched in-place Stockham FFT in LDS, radix 16/8/4/2, for power-of-two K.
//
// Chunks of the butterfly range (NT * 16/R butterflies) always cover whole
// buffers when K <= NT * 16.
//
// Buffer slots are addressed through slot() (an XOR swizzle that spreads
// the strided writes of the early stages over the LDS banks).
//
// Stage with radix R after Ns points have been combined: butterfly j
// (0 <= j < K/R) reads x[j + r K/R], r < R, multiplies input r by
// exp(-+2 pi i r (j mod Ns) / (Ns R)), takes an R-point DFT and writes output
// s to (j - j mod Ns) R + (j mod Ns) + s Ns.  Every thread first reads up to
// 16/R butterflies into registers, the workgroup synchronizes, and then all
// write: reads and writes of one pass always cover whole buffers, so the
// stage can run in place.  Twiddles come from a table exp(-2 pi i q / K).
#pragma once

#include "device_common.h"

namespace fftfem {

// cos/sin of pi/8 and pi/4
template <typename T>
struct Rt {
  static constexpr T c8 = (T)0.92387953251128675612818318939678829;
  static constexpr T s8 = (T)0.38268343236508977172845998403039887;
  static constexpr T h = (T)0.70710678118654752440084436210484904;
};

// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ C2<T> mul_mi(C2<T> a) {
  return INV ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(C2<T>& a, C2<T>& b) {
  C2<T> s = cadd(a, b), d = csub(a, b);
  a = s;
  b = d;
}

// 4-point DFT of (a, b, c, d) in place: outputs in natural order
template <typename T, bool INV>
__device__ __forceinline__ void dft4(C2<T>& a, C2<T>& b, C2<T>& c, C2<T>& d) {
  C2<T> s02 = cadd(a, c), d02 = csub(a, c), s13 = cadd(b, d), d13 = mul_mi<T, INV>(csub(b, d));
  a = cadd(s02, s13);
  c = csub(s02, s13);
  b = cadd(d02, d13);
  d = csub(d02, d13);
}

// constant twiddle w_N^e for N in {8, 16}, forward sign; conjugated for INV
template <typename T, bool INV>
__device__ __forceinline__ C2<T> tw_mul16(C2<T> v, int e) {
  // e in 0..15, w16^e = exp(-2 pi i e / 16)
  const T c8 = Rt<T>::c8, s8 = Rt<T>::s8, h = Rt<T>::h;
  C2<T> w;
  switch (e & 15) {
    case 0: return v;
    case 1: w = {c8, -s8}; break;
    case 2: w = {h, -h}; break;
    case 3: w = {s8, -c8}; break;
    case 4: return mul_mi<T, INV>(v);
    case 5: w = {-s8, -c8}; break;
    case 6: w = {-h, -h}; break;
    case 7: w = {-c8, -s8}; break;
    case 8: return C2<T>{-v.x, -v.y};
    case 9: w = {-c8, s8}; break;
    case 10: w = {-h, h}; break;
    case 11: w = {-s8, c8}; break;
    case 12: return mul_mi<T, !INV>(v);
    case 13: w = {s8, c8}; break;
    case 14: w = {h, h}; break;
    default: w = {c8, s8}; break;
  }
  return INV ? cmulc(v, w) : cmul(v, w);
}

// In-register R-point DFT, natural order in and out.
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(C2<T>* v) {
  if constexpr (R == 2) {
    dft2<T, INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<T, INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // r = r1 + 4 r2 (r1 < 4, r2 < 2); s = s2 + 2 s1
    C2<T> y[4][2];
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1) {
      y[r1][0] = cadd(v[r1], v[r1 + 4]);
      y[r1][1] = csub(v[r1], v[r1 + 4]);
      y[r1][1] = tw_mul16<T, INV>(y[r1][1], 2 * r1);  // w8^(r1 * 1)
    }
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      C2<T> a = y[0][s2], b = y[1][s2], c = y[2][s2], d = y[3][s2];
      dft4<T, INV>(a, b, c, d);
      v[s2] = a;
      v[s2 + 2] = b;
      v[s2 + 4] = c;
      v[s2 + 6] = d;
    }
  } else {
    static_assert(R == 16, "radix");
    // r = r1 + 4 r2, s = s2 + 4 s1
    C2<T> y[4][4];
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1) {
      C2<T> a = v[r1], b = v[r1 + 4], c = v[r1 + 8], d = v[r1 + 12];
      dft4<T, INV>(a, b, c, d);
      y[r1][0] = a;
      y[r1][1] = tw_mul16<T, INV>(b, r1);
      y[r1][2] = tw_mul16<T, INV>(c, 2 * r1);
      y[r1][3] = tw_mul16<T, INV>(d, 3 * r1);
    }
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      C2<T> a = y[0][s2], b = y[1][s2], c = y[2][s2], d = y[3][s2];
      dft4<T, INV>(a, b, c, d);
      v[s2] = a;
      v[s2 + 4] = b;
      v[s2 + 8] = c;
      v[s2 + 12] = d;
    }
  }
}

template <typename T, int R, bool INV, int NT>
__device__ __forceinline__ void fft_stage(C2<T>* buf, int nfft, int lk, int Ns, int lns,
                                          const C2<T>* __restrict__ tw, int ls) {
  constexpr int MAXB = 16 / R;
  constexpr int LR = R == 2 ? 1 : (R == 4 ? 2 : (R == 8 ? 3 : 4));
  const int K = 1 << lk;
  const int lkr = lk - LR;  // log2(K/R)
  const int KR = 1 << lkr;
  const int total = nfft << lkr;
  const int tid = threadIdx.x;
  const int lts = lk - lns - LR;  // log2 of the twiddle stride K/(Ns R)
  for (int base = 0; base < total; base += NT * MAXB) {
    C2<T> v[MAXB][R];
    int dst[MAXB], fb[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
      int b = base + t * NT + tid;
      dst[t] = -1;
      if (b < total) {
        int f = b >> lkr, j = b & (KR - 1);
        const C2<T>* x = buf + f * ls;
        int k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][r] = slot(x, j + r * KR);
        if (Ns > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            C2<T> w = tw[(r * k) << lts];
            v[t][r] = INV ? cmulc(v[t][r], w) : cmul(v[t][r], w);
          }
        }
        dft_small<T, R, INV>(v[t]);
        fb[t] = f * ls;
        dst[t] = ((j - k) << LR) + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXB; ++t)
      if (dst[t] >= 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) slot(buf + fb[t], dst[t] + r * Ns) = v[t][r];
      }
    __syncthreads();
  }
}

// All stages: the largest radix up to 2^lrmax (16, 8 or 4) while possible,
// then one stage of a smaller radix.  Buffer f starts at buf + f * ls
// (ls >= K complex values).
template <typename T, bool INV, int NT>
__device__ void fft_all(C2<T>* buf, int nfft, int lk, const C2<T>* tw, int ls, int lrmax = 4) {
  int lns = 0, rem = lk;
  if (lrmax >= 4)
    while (rem >= 4) {
      fft_stage<T, 16, INV, NT>(buf, nfft, lk, 1 << lns, lns, tw, ls);
      lns += 4;
      rem -= 4;
    }
  if (lrmax >= 3)
    while (rem >= 3) {
      fft_stage<T, 8, INV, NT>(buf, nfft, lk, 1 << lns, lns, tw, ls);
      lns += 3;
      rem -= 3;
    }
  while (rem >= 2) {
    fft_stage<T, 4, INV, NT>(buf, nfft, lk, 1 << lns, lns, tw, ls);
    lns += 2;
    rem -= 2;
  }
  if (rem == 1) fft_stage<T, 2, INV, NT>(buf, nfft, lk, 1 << lns, lns, tw, ls);
}

// cos(2 pi j / R) and sin(2 pi j / R), j < R, for the odd radices.
template <typename T, int R>
struct OddRoots;
template <typename T>
struct OddRoots<T, 3> {
  static constexpr T c[3] = {(T)1, (T)-0.5, (T)-0.5};
  static constexpr T s[3] = {(T)0, (T)0.866025403784438646763723170752936183,
                             (T)-0.866025403784438646763723170752936183};
};
template <typename T>
struct OddRoots<T, 5> {
  static constexpr T c[5] = {(T)1, (T)0.309016994374947424102293417182819059,
                             (T)-0.809016994374947424102293417182819059,
                             (T)-0.809016994374947424102293417182819059,
                             (T)0.309016994374947424102293417182819059};
  static constexpr T s[5] = {(T)0, (T)0.951056516295153572116439333379382143,
                             (T)0.587785252292473129168705954639072769,
                             (T)-0.587785252292473129168705954639072769,
                             (T)-0.951056516295153572116439333379382143};
};
template <typename T>
struct OddRoots<T, 7> {
  static constexpr T c[7] = {(T)1,
                             (T)0.623489801858733530525004884004239811,
                             (T)-0.222520933956314404288902564496794759,
                             (T)-0.900968867902419126236102319507445051,
                             (T)-0.900968867902419126236102319507445051,
                             (T)-0.222520933956314404288902564496794759,
                             (T)0.623489801858733530525004884004239811};
  static constexpr T s[7] = {(T)0,
                             (T)0.78183148246802980870844452667405775,
                             (T)0.974927912181823607018131682993931217,
                             (T)0.433883739117558120475768332848358755,
                             (T)-0.433883739117558120475768332848358755,
                             (T)-0.974927912181823607018131682993931217,
                             (T)-0.78183148246802980870844452667405775};
};

// In-register R-point DFT for odd R, natural order in and out: with
// p_m = v_m + v_{R-m}, d_m = v_m - v_{R-m} (m = 1 .. (R-1)/2),
//   X_s, X_{R-s} = v_0 + sum_m p_m cos(2 pi m s / R) -/+ i sum_m d_m sin(2 pi m s / R)
// (forward, exp(-2 pi i j s / R); the inverse swaps the signs).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_odd(C2<T>* v) {
  constexpr int H = (R - 1) / 2;
  using RT = OddRoots<T, R>;
  C2<T> p[H + 1], d[H + 1];
  C2<T> sum = v[0];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    p[m] = cadd(v[m], v[R - m]);
    d[m] = csub(v[m], v[R - m]);
    sum = cadd(sum, p[m]);
  }
  C2<T> out[R];
  out[0] = sum;
#pragma unroll
  for (int s = 1; s <= H; ++s) {
    C2<T> a = v[0], b = {(T)0, (T)0};
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      const T cs = RT::c[(m * s) % R], sn = RT::s[(m * s) % R];
      a.x += p[m].x * cs;
      a.y += p[m].y * cs;
      b.x += d[m].x * sn;
      b.y += d[m].y * sn;
    }
    // -i b = (b.y, -b.x); +i b = (-b.y, b.x)
    const C2<T> mib = {b.y, -b.x}, pib = {-b.y, b.x};
    out[s] = cadd(a, INV ? pib : mib);
    out[R - s] = cadd(a, INV ? mib : pib);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = out[r];
}

// Stockham stage of radix R (2, 3, 4, 5, 7, 8 or 16) for any K divisible
// by Ns R, after Ns points have been combined: the index arithmetic of
// fft_stage with divisions, and twiddles exp(-+2 pi i r (j mod Ns) / (Ns R))
// read from the length-K table at r (j mod Ns) K / (Ns R).  The butterflies
// of whole buffers are read into registers (chunks of at most NT max(1, 8/R)
// butterflies: K <= 1024 and NT >= 512 keep every buffer in one chunk), the
// workgroup synchronizes, and then all write, so the stage runs in place.
template <typename T, int R, bool INV, int NT>
__device__ void fft_stage_mr(C2<T>* buf, int nfft, int K, int Ns, const C2<T>* __restrict__ tw, int ls) {
  static_assert(NT >= 512, "a buffer's butterflies must fit in one chunk");
  constexpr int MAXB = R >= 8 ? 1 : 8 / R;  // at most 8 values in registers (16 for radix 16)
  const int KR = K / R;
  const int stride = K / (Ns * R);
  const int tid = threadIdx.x;
  int fpc = (NT * MAXB) / KR;
  if (fpc < 1) fpc = 1;
  for (int f0 = 0; f0 < nfft; f0 += fpc) {
    const int nf = nfft - f0 < fpc ? nfft - f0 : fpc;
    const int nb = nf * KR;
    C2<T> v[MAXB][R];
    int dst[MAXB], fb[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
      const int b = t * NT + tid;
      dst[t] = -1;
      if (b < nb) {
        const int fl = b / KR, j = b - fl * KR;
        const int f = f0 + fl;
        const int k = j % Ns;
        const C2<T>* x = buf + f * ls;
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][r] = slot(x, j + r * KR);
        if (Ns > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const C2<T> w = tw[r * k * stride];
            v[t][r] = INV ? cmulc(v[t][r], w) : cmul(v[t][r], w);
          }
        }
        if constexpr (R == 3 || R == 5 || R == 7)
          dft_odd<T, R, INV>(v[t]);
        else
          dft_small<T, R, INV>(v[t]);
        fb[t] = f * ls;
        dst[t] = (j - k) * R + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXB; ++t)
      if (dst[t] >= 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) slot(buf + fb[t], dst[t] + r * Ns) = v[t][r];
      }
    __syncthreads();
  }
}

// Length-K DFTs by mixed-radix Stockham stages, for K whose prime factors
// are at most 7: nrad stages, stage i's radix coded in bits 3i..3i+2 of
// radpack (0..6: radix 2, 3, 4, 5, 7, 8, 16; product K).  Output in natural
// order in slots 0..K-1.  Ends with a barrier.
template <typename T, bool INV, int NT>
__device__ void fft_mixed(C2<T>* buf, int nfft, int K, uint64_t radpack, int nrad, const C2<T>* tw, int ls) {
  int Ns = 1;
  for (int i = 0; i < nrad; ++i) {
    const int code = (int)((radpack >> (3 * i)) & 7);
    switch (code) {
      case 0: fft_stage_mr<T, 2, INV, NT>(buf, nfft, K, Ns, tw, ls); Ns *= 2; break;
      case 1: fft_stage_mr<T, 3, INV, NT>(buf, nfft, K, Ns, tw, ls); Ns *= 3; break;
      case 2: fft_stage_mr<T, 4, INV, NT>(buf, nfft, K, Ns, tw, ls); Ns *= 4; break;
      case 3: fft_stage_mr<T, 5, INV, NT>(buf, nfft, K, Ns, tw, ls); Ns *= 5; break;
      case 4: fft_stage_mr<T, 7, INV, NT>(buf, nfft, K, Ns, tw, ls); Ns *= 7; break;
      case 5: fft_stage_mr<T, 8, INV, NT>(buf, nfft, K, Ns, tw, ls); Ns *= 8; break;
      default: fft_stage_mr<T, 16, INV, NT>(buf, nfft, K, Ns, tw, ls); Ns *= 16; break;
    }
  }
}

// Length-K DFT for K not a power of two (Bluestein's chirp-z): with
// c_j = exp(-i pi j^2 / K), jk = (j^2 + k^2 - (k - j)^2) / 2 gives
//   X_k = c_k sum_j (x_j c_j) conj(c_{k-j}),
// a convolution computed as a cyclic one of length L >= 2K - 1 (a power of
// two) with two Stockham FFTs and the precomputed spectrum of conj(c)
// (bhat, already divided by L).  INV (exp(+2 pi i jk/K)): conjugated chirp
// and spectrum.  Data in slots 0..K-1 of each buffer; slots up to L - 1 are
// scratch.  Ends with a barrier.
template <typename T, bool INV, int NT>
__device__ void bluestein(C2<T>* buf, int nfft, int K, int lL, const C2<T>* __restrict__ chirp,
                          const C2<T>* __restrict__ bhat, const C2<T>* tw, int ls, int lrmax) {
  const int L = 1 << lL;
  const int tid = threadIdx.x;
  for (int i = tid; i < (nfft << lL); i += NT) {
    const int f = i >> lL, j = i & (L - 1);
    C2<T>& v = slot(buf + f * ls, j);
    if (j < K) {
      const C2<T> c = chirp[j];
      v = INV ? cmulc(v, c) : cmul(v, c);
    } else {
      v = C2<T>{0, 0};
    }
  }
  __syncthreads();
  fft_all<T, false, NT>(buf, nfft, lL, tw, ls, lrmax);
  for (int i = tid; i < (nfft << lL); i += NT) {
    const int f = i >> lL, j = i & (L - 1);
    C2<T>& v = slot(buf + f * ls, j);
    const C2<T> b = bhat[j];
    v = INV ? cmulc(v, b) : cmul(v, b);
  }
  __syncthreads();
  fft_all<T, true, NT>(buf, nfft, lL, tw, ls, lrmax);
  for (int i = tid; i < nfft * K; i += NT) {
    const int f = i / K, j = i - f * K;
    C2<T>& v = slot(buf + f * ls, j);
    const C2<T> c = chirp[j];
    v = INV ? cmulc(v, c) : cmul(v, c);
  }
  __syncthreads();
}

}  // namespace fftfem
