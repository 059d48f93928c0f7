// Per-frequency pieces of the FC_n transform and its inverse shared by the
// line passes held in LDS (line.hip) and the multi-pass transforms of long
// lines (long.hip): untangling the packed spectra of the node and bubble
// channels, the inverse pre-twiddles, and the n x n contractions with the
// table Q of Theorem 1's eigenvectors (Sect. 3).  Buffers are addressed
// through the LDS swizzle in the line passes and plainly in global work
// arrays (the SW template argument).
#pragma once

#include "device_common.h"

namespace fftfem {

// Slot access of a complex buffer: through the LDS swizzle (SW, the line
// passes) or plain (the global work arrays of the long-line transforms).
template <bool SW, typename T>
__device__ __forceinline__ const C2<T>& sl(const C2<T>* b, int i) {
  if constexpr (SW) return slot(b, i);
  else return b[i];
}
template <bool SW, typename T>
__device__ __forceinline__ void setc(C2<T>* b, int i, int comp, T v) {
  if constexpr (SW) set_comp(b, i, comp, v);
  else reinterpret_cast<T*>(b + i)[comp] = v;
}

// DCT-II values of the packed bubble buffers at indices ia and ib (= K - ia
// mod K): out_a[b], out_b[b] for every bubble channel b.
template <typename T, int NORD, bool SW = true>
__device__ __forceinline__ void bubble_post(const C2<T>* B, int ls, int ia, int ib,
                                            const C2<T>* twm, T* out_a, T* out_b) {
  constexpr int P = NORD / 2;
#pragma unroll
  for (int p = 1; p <= P; ++p) {
    C2<T> Va = sl<SW>(B + p * ls, ia), Vb = sl<SW>(B + p * ls, ib);
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
template <typename T, bool SW = true>
__device__ __forceinline__ T nodal_post(const C2<T>* Z, int K, int k, const C2<T>* twd,
                                        bool conj_in) {
  C2<T> zk = sl<SW>(Z, k), zm = sl<SW>(Z, K - k);
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
template <typename T, bool SW = true>
__device__ __forceinline__ void write_nodal_inv(C2<T>* Z, int K, int k, T val) {
  int t = k;
  setc<SW>(Z, t >> 1, t & 1, (t & 1) ? -val : val);
  t = 2 * K - k;
  setc<SW>(Z, t >> 1, t & 1, (t & 1) ? val : -val);
}

template <typename T, bool SW = true>
__device__ __forceinline__ void write_nodal_zeros(C2<T>* Z, int K) {
  setc<SW>(Z, 0, 0, (T)0);
  setc<SW>(Z, K >> 1, K & 1, (T)0);
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
// Q[(c n + l) K + k], so the lanes of a wave (consecutive k) read one
// contiguous segment per entry.  The table is read through a buffer
// resource: the row offset 8 (c n + l) K is a scalar operand and the lane
// offset 8 k the only vector one (plain pointer arithmetic here gets
// re-associated into per-load 64-bit vector addresses, issued one at a
// time).  Reads past the table return 0 instead of faulting.  Block k = 0 is
// zero-padded to n x n.
using rsrc_t = __amdgpu_buffer_rsrc_t;

template <typename T>
__device__ __forceinline__ rsrc_t table_rsrc(const T* p, uint32_t count) {
  // third descriptor word for the gfx9 family: raw 32-bit element format
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, count * (uint32_t)sizeof(T),
                                           0x00020000);
}

template <typename T>
__device__ __forceinline__ T ldq(rsrc_t r, uint32_t lane_off, uint32_t row_off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, row_off, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, row_off, 0));
}

template <typename T, int NORD>
__device__ __forceinline__ uint32_t qrow(int c, int l, int K) {
  return (uint32_t)((c * NORD + l) * K) * (uint32_t)sizeof(T);
}

template <typename T, int NORD>
__device__ __forceinline__ void contract_fwd(rsrc_t Q, int K, int k, const T* ch, T* w) {
  const uint32_t ko = (uint32_t)k * (uint32_t)sizeof(T);
#pragma unroll
  for (int l = 0; l < NORD; ++l) w[l] = 0;
#pragma unroll
  for (int c = 0; c < NORD; ++c)
#pragma unroll
    for (int l = 0; l < NORD; ++l) w[l] += ldq<T>(Q, ko, qrow<T, NORD>(c, l, K)) * ch[c];
}

template <typename T, int NORD>
__device__ __forceinline__ void contract_inv(rsrc_t Q, int K, int k, const T* w, T* ch) {
  const uint32_t ko = (uint32_t)k * (uint32_t)sizeof(T);
#pragma unroll
  for (int c = 0; c < NORD; ++c) {
    T acc = 0;
#pragma unroll
    for (int l = 0; l < NORD; ++l) acc += ldq<T>(Q, ko, qrow<T, NORD>(c, l, K)) * w[l];
    ch[c] = acc;
  }
}

// Contractions of the fused MID pass: the forward contraction, division and
// inverse contraction of the two frequencies k and K - k of a task run as
// two interleaved chains.  Left alone, the scheduler would issue the n^2
// table loads of all four contractions up front (several hundred live
// registers: one wave per SIMD, or spills).  Here the lane offset used by
// row c + D goes through empty asm statements that also consume that
// chain's accumulators after row c, so each chain has D rows in flight, and
// a contraction's first rows wait for `dep` (the previous stage's result).
template <typename V>
__device__ __forceinline__ uint32_t after(uint32_t o, V v) {
  __asm__ volatile("" : "+v"(o) : "v"(v));
  return o;
}

// The same, tied to all n accumulators (the scheduler would otherwise finish
// only the one the asm consumes and keep the other columns' inputs live).
template <typename T, int NORD>
__device__ __forceinline__ uint32_t after_all(uint32_t o, const T* v) {
#pragma unroll
  for (int l = 0; l < NORD; ++l) __asm__ volatile("" : "+v"(o) : "v"(v[l]));
  return o;
}

#ifndef FFTFEM_MID_ROWS
#define FFTFEM_MID_ROWS 2
#endif

template <typename T, int NORD>
__device__ __forceinline__ void contract_fwd2(rsrc_t Q, int K, int ka, int kb, const T* cha,
                                              const T* chb, T* wa, T* wb, T dep) {
  constexpr int D = FFTFEM_MID_ROWS < NORD ? FFTFEM_MID_ROWS : NORD;
  const uint32_t oa = (uint32_t)ka * (uint32_t)sizeof(T), ob = (uint32_t)kb * (uint32_t)sizeof(T);
  T qa[NORD][NORD], qb[NORD][NORD];
  {
    const uint32_t pa = after(oa, dep), pb = after(ob, dep);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int l = 0; l < NORD; ++l) {
        qa[c][l] = ldq<T>(Q, pa, qrow<T, NORD>(c, l, K));
        qb[c][l] = ldq<T>(Q, pb, qrow<T, NORD>(c, l, K));
      }
  }
#pragma unroll
  for (int l = 0; l < NORD; ++l) wa[l] = wb[l] = 0;
#pragma unroll
  for (int c = 0; c < NORD; ++c) {
#pragma unroll
    for (int l = 0; l < NORD; ++l) {
      wa[l] += qa[c][l] * cha[c];
      wb[l] += qb[c][l] * chb[c];
    }
    if (c + D < NORD) {
      const uint32_t pa = after_all<T, NORD>(oa, wa), pb = after_all<T, NORD>(ob, wb);
#pragma unroll
      for (int l = 0; l < NORD; ++l) {
        qa[c + D][l] = ldq<T>(Q, pa, qrow<T, NORD>(c + D, l, K));
        qb[c + D][l] = ldq<T>(Q, pb, qrow<T, NORD>(c + D, l, K));
      }
    }
  }
}

template <typename T, int NORD>
__device__ __forceinline__ void contract_inv2(rsrc_t Q, int K, int ka, int kb, const T* wa,
                                              const T* wb, T* cha, T* chb, T dep) {
  constexpr int D = FFTFEM_MID_ROWS < NORD ? FFTFEM_MID_ROWS : NORD;
  const uint32_t oa = (uint32_t)ka * (uint32_t)sizeof(T), ob = (uint32_t)kb * (uint32_t)sizeof(T);
  T qa[NORD][NORD], qb[NORD][NORD];
  {
    const uint32_t pa = after(oa, dep), pb = after(ob, dep);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int l = 0; l < NORD; ++l) {
        qa[c][l] = ldq<T>(Q, pa, qrow<T, NORD>(c, l, K));
        qb[c][l] = ldq<T>(Q, pb, qrow<T, NORD>(c, l, K));
      }
  }
#pragma unroll
  for (int c = 0; c < NORD; ++c) {
    T acca = 0, accb = 0;
#pragma unroll
    for (int l = 0; l < NORD; ++l) {
      acca += qa[c][l] * wa[l];
      accb += qb[c][l] * wb[l];
    }
    cha[c] = acca;
    chb[c] = accb;
    if (c + D < NORD) {
      const uint32_t pa = after(oa, acca), pb = after(ob, accb);
#pragma unroll
      for (int l = 0; l < NORD; ++l) {
        qa[c + D][l] = ldq<T>(Q, pa, qrow<T, NORD>(c + D, l, K));
        qb[c + D][l] = ldq<T>(Q, pb, qrow<T, NORD>(c + D, l, K));
      }
    }
  }
}

}  // namespace fftfem
