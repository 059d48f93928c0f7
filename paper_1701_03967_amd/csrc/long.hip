// Transforms of long lines (gfx950): the direct FC_n transform and its
// inverse (Sect. 3, Theorem 2) for one-dimensional plans whose element count
// K (1024 < K <= 2^20) exceeds what one LDS tile holds.  The steps of a line
// pass run as separate passes over global work arrays of NB = 1 + floor(n/2)
// complex buffers per line (ls slots each), packed as in the line passes (the
// node channel's odd extension of length 2K, then the bubble channel pairs in
// the reordering that makes their DCT-II a K-point DFT):
//
//   forward:  gather -> K-point DFT -> contraction
//   inverse:  contraction -> inverse K-point DFT -> scatter
//
// The K-point DFT of every buffer is a four-step DFT of a power-of-two
// length D = K1 K2 (K1, K2 <= 2048), as two passes, "columns" and "rows":
// the buffer viewed as K1 x K2 (index i1 K2 + i2), length-K1 DFTs down the
// columns with the twiddles exp(-+2 pi i i2 k1 / D), then length-K2 DFTs
// along the rows, stored transposed so that frequency k1 + K1 k2 lands at
// index k1 + K1 k2 (natural order).  K a power of two: D = K, two passes.
// Otherwise Bluestein's chirp-z with D = L >= 2K - 1 (as in the line passes):
// with c_j = exp(-i pi j^2 / K), X_k = c_k sum_j (x_j c_j) conj(c_{k-j}), a
// cyclic convolution of length L done as a forward and an inverse D-point
// DFT, four passes: the chirp multiplication and the zero padding fused into
// the loads of the first column pass, the product with the spectrum of
// conj(c) (divided by L) into the loads of the second column pass, the final
// chirp and the truncation to K into the stores of the last row pass
// (conjugated chirp and spectrum for the inverse DFT).
//
// The sub-DFTs run in LDS with the Stockham stages of fft.h; forward and
// inverse DFTs differ only in the sign of the twiddles.  A tile holds Gc
// columns (Gr rows) of about 4096 points: the global reads and writes of one
// tile row are runs of Gc (Gr) complex values, and consecutive tiles share
// one XCD so that the halves of a 128-byte line read or written by
// neighbouring tiles meet in one L2.  The twiddle exp(-2 pi i m / D) is the
// product of two cached tables (high bits and low ten bits of m).  The
// per-frequency untangling and the contractions with Q_k are those of the
// line passes (spectral.h); a contraction thread takes one frequency pair of
// several lines, so the Q rows it reads are fetched from HBM once for all of
// them.
#include "device_common.h"
#include "fft.h"
#include "launch.h"
#include "spectral.h"

namespace fftfem {

extern __shared__ double2 fftfem_long_lds[];

constexpr int kLongThreads = 256;
constexpr int kLongLgTilePts = 12;  // 4096 points per four-step tile (one chunk of the Stockham stages)
constexpr int kLongTwBits = 10;     // low bits of the twiddle index (table of 1024)
static_assert((1 << kLongLgTilePts) == kLongThreads * 16, "a tile is one chunk of the Stockham stages");
constexpr int kLongPT = 16;  // tile points per thread at most

using CD = C2<double>;

__device__ __forceinline__ CD* long_buf(double* w, int64_t line, int b, int NB, int ls) {
  return reinterpret_cast<CD*>(w) + ((size_t)line * NB + b) * (size_t)ls;
}

// Element jp of line l: node jp + 1 and the bubble channels into the work
// buffers of wa (as the gather of the line passes).
template <int NORD>
__global__ __launch_bounds__(kLongThreads) void long_gather_kernel(LongArgs a) {
  constexpr int n = NORD, ne = NORD / 2, no = (NORD - 1) / 2, P = NORD / 2, NB = 1 + P;
  const int K = a.K, ls = a.ls;
  const int64_t t = (int64_t)blockIdx.x * kLongThreads + threadIdx.x;
  if (t >= a.nlines * K) return;
  const int64_t l = t / K;
  const int jp = (int)(t - l * K);
  const double* r = a.in + l * a.M + (int64_t)jp * n;
  double y[NORD], hv[NORD];
#pragma unroll
  for (int m = 0; m < n - 1; ++m) y[m] = r[m];
  y[n - 1] = jp < K - 1 ? r[n - 1] : 0.0;
  const double sg = (jp & 1) ? -1.0 : 1.0;
  hv[0] = y[n - 1];
#pragma unroll
  for (int m = 1; m <= ne; ++m) hv[m] = sg * ((2 * m == n) ? y[m - 1] : y[m - 1] + y[n - m - 1]);
#pragma unroll
  for (int m = 1; m <= no; ++m) hv[ne + m] = y[m - 1] - y[n - m - 1];
  CD* Z = long_buf(a.wa, l, 0, NB, ls);
  if (jp < K - 1) {
    const int j = jp + 1, t2 = 2 * K - j;
    setc<false>(Z, j >> 1, j & 1, hv[0]);
    setc<false>(Z, t2 >> 1, t2 & 1, -hv[0]);
  } else {
    write_nodal_zeros<double, false>(Z, K);
  }
  const int q = (jp & 1) ? K - 1 - (jp >> 1) : (jp >> 1);
#pragma unroll
  for (int b = 0; b < n - 1; ++b) setc<false>(Z + (1 + b / 2) * (size_t)ls, q, b & 1, hv[1 + b]);
  if ((n - 1) & 1) setc<false>(Z + P * (size_t)ls, q, 1, 0.0);
}

// Four-step DFT, first half: 2^lgc adjacent columns (i2) of one buffer,
// length-K1 DFTs over i1, then the twiddles exp(-+2 pi i i2 k1 / D); in
// place.  pre = 1 (2): the input is x_i c_i (x_i conj(c_i)) for i < K and 0
// beyond (the start of Bluestein's convolution); pre = 3 (4): x_i bhat_i
// (x_i conj(bhat_i)), the product with the spectrum of its kernel.
template <bool INV>
__global__ __launch_bounds__(kLongThreads) void long_cols_kernel(LongArgs a, double* w) {
  const int K1 = a.K1, K2 = a.K2, lg = a.lgc, G = 1 << lg, K = a.K, pre = a.pre;
  const int ncb = K2 >> lg;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t buf = tile / ncb;
  const int c0 = (int)(tile - buf * ncb) << lg;
  CD* X = reinterpret_cast<CD*>(w) + buf * (size_t)a.ls;
  CD* L = reinterpret_cast<CD*>(fftfem_long_lds);
  const int ls = K1 + 1;
  const int tid = threadIdx.x;
  const int total = G * K1;
  // all of a thread's loads in flight before the first LDS store
  CD v[kLongPT];
  if (pre == 0) {
#pragma unroll
    for (int j = 0; j < kLongPT; ++j) {
      const int i = tid + j * kLongThreads;
      if (i < total) v[j] = X[(i >> lg) * K2 + c0 + (i & (G - 1))];
    }
  } else {
    // x_i and the factor f_i for i < lim, 0 and 1 beyond
    const CD* fac = reinterpret_cast<const CD*>(pre <= 2 ? a.chirp : a.bhat);
    const int lim = pre <= 2 ? K : K1 * K2;
    CD c[kLongPT];
#pragma unroll
    for (int j = 0; j < kLongPT; ++j) {
      const int i = tid + j * kLongThreads;
      const int idx = (i >> lg) * K2 + c0 + (i & (G - 1));
      const bool in = i < total && idx < lim;
      v[j] = in ? X[idx] : CD{0.0, 0.0};
      c[j] = in ? fac[idx] : CD{1.0, 0.0};
    }
    const bool conj = (pre & 1) == 0;
#pragma unroll
    for (int j = 0; j < kLongPT; ++j) v[j] = conj ? cmulc(v[j], c[j]) : cmul(v[j], c[j]);
  }
#pragma unroll
  for (int j = 0; j < kLongPT; ++j) {
    const int i = tid + j * kLongThreads;
    if (i < total) slot(L + (i & (G - 1)) * ls, i >> lg) = v[j];
  }
  __syncthreads();
  fft_all<double, INV, kLongThreads>(L, G, a.lk1, reinterpret_cast<const CD*>(a.tw1), ls, 4);
  const CD* twlo = reinterpret_cast<const CD*>(a.twlo);
  const CD* twhi = reinterpret_cast<const CD*>(a.twhi);
#pragma unroll
  for (int j = 0; j < kLongPT; ++j) {
    const int i = tid + j * kLongThreads;
    if (i < total) {
      const int k1 = i >> lg, g = i & (G - 1);
      const CD u = slot(L + g * ls, k1);
      const int m = (c0 + g) * k1;  // < D <= 2^21
      const CD tw = cmul(twhi[m >> kLongTwBits], twlo[m & ((1 << kLongTwBits) - 1)]);
      X[(size_t)k1 * K2 + c0 + g] = INV ? cmulc(u, tw) : cmul(u, tw);
    }
  }
}

// Four-step DFT, second half: 2^lgr adjacent rows (k1) of one buffer of w,
// length-K2 DFTs over i2, stored into the same buffer of out at
// k = k1 + K1 k2.  post = 1 (2): times c_k (conj(c_k)) and only k < K stored
// (the end of Bluestein's convolution).
template <bool INV>
__global__ __launch_bounds__(kLongThreads) void long_rows_kernel(LongArgs a, const double* w, double* out) {
  const int K1 = a.K1, K2 = a.K2, lg = a.lgr, G = 1 << lg, K = a.K, post = a.post;
  const int nrb = K1 >> lg;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t buf = tile / nrb;
  const int r0 = (int)(tile - buf * nrb) << lg;
  const CD* X = reinterpret_cast<const CD*>(w) + buf * (size_t)a.ls;
  CD* Y = reinterpret_cast<CD*>(out) + buf * (size_t)a.ls;
  CD* L = reinterpret_cast<CD*>(fftfem_long_lds);
  const CD* chirp = reinterpret_cast<const CD*>(a.chirp);
  const int ls = K2 + 1;
  const int tid = threadIdx.x;
  const int total = G * K2;
  // the tile's rows are one contiguous segment of the buffer; all of a
  // thread's loads in flight before the first LDS store
  const CD* Xs = X + (size_t)r0 * K2;
  CD v[kLongPT];
#pragma unroll
  for (int j = 0; j < kLongPT; ++j) {
    const int i = tid + j * kLongThreads;
    v[j] = i < total ? Xs[i] : CD{0.0, 0.0};
  }
#pragma unroll
  for (int j = 0; j < kLongPT; ++j) {
    const int i = tid + j * kLongThreads;
    if (i < total) slot(L + (i >> a.lk2) * ls, i & (K2 - 1)) = v[j];
  }
  __syncthreads();
  fft_all<double, INV, kLongThreads>(L, G, a.lk2, reinterpret_cast<const CD*>(a.tw2), ls, 4);
  for (int i = tid; i < total; i += kLongThreads) {
    {
      const int k2 = i >> lg, g = i & (G - 1);
      const int k = r0 + g + K1 * k2;
      CD u = slot(L + g * ls, k2);
      if (post == 0 || k < K) {
        if (post != 0) u = post == 1 ? cmul(u, chirp[k]) : cmulc(u, chirp[k]);
        Y[k] = u;
      }
    }
  }
}

// Frequency pair tasks of a line: kap = 0 .. ceil(K/2) - 1 takes the
// frequencies kap and K - kap; kap = 0 the bubble-only block and, for even
// K, frequency K/2.
__host__ __device__ inline int long_pair_tasks(int K) { return (K + 1) >> 1; }

// Frequencies of task kap of line l: untangled spectra of the buffers of wb
// -> coefficients (y, s~) in the spectral order of the line (k = 0 block of
// n - 1, then n per k).
template <int NORD>
__device__ __forceinline__ void long_contract_fwd_line(const LongArgs& a, int64_t l, int kap, double* wa,
                                                       double* wb) {
  constexpr int n = NORD, NC = NORD > 1 ? NORD - 1 : 1;
  const int K = a.K, ls = a.ls;
  const bool keven = (K & 1) == 0;
  const bool hasb = kap != 0 || keven;
  const int ka = kap, kb = kap == 0 ? (K >> 1) : K - kap;
  const CD* B = long_buf(a.wb, l, 0, 1 + NORD / 2, ls);
  const CD* twm = reinterpret_cast<const CD*>(a.twm);
  const CD* twd = reinterpret_cast<const CD*>(a.twd);
  double ca[NC], cb[NC], cha[NORD], chb[NORD];
  if (kap == 0) {
    if constexpr (NORD > 1) {
      bubble_post<double, NORD, false>(B, ls, 0, 0, twm, ca, cb);
#pragma unroll
      for (int b = 0; b < NORD - 1; ++b) cha[b] = ca[b];
      if (keven) bubble_post<double, NORD, false>(B, ls, kb, kb, twm, ca, cb);
    }
    cha[NORD - 1] = 0;
    if (keven) channel_vec<double, NORD>(nodal_post<double, false>(B, K, kb, twd, false), ca, ca, chb);
  } else {
    if constexpr (NORD > 1) bubble_post<double, NORD, false>(B, ls, ka, kb, twm, ca, cb);
    channel_vec<double, NORD>(nodal_post<double, false>(B, K, ka, twd, false), ca, cb, cha);
    channel_vec<double, NORD>(nodal_post<double, false>(B, K, kb, twd, false), cb, ca, chb);
  }
  const rsrc_t qtab = table_rsrc(a.Q, (uint32_t)((size_t)K * n * n));
  if (!hasb) {
#pragma unroll
    for (int c = 0; c < NORD; ++c) chb[c] = 0.0;
  }
  // both frequencies as two chains with a few table rows in flight (without
  // a second frequency the chain repeats the first one's block, unused)
  contract_fwd2<double, NORD>(qtab, K, ka, hasb ? kb : ka, cha, chb, wa, wb, cha[0]);
  if (!hasb) {
#pragma unroll
    for (int c = 0; c < NORD; ++c) wb[c] = 0.0;
  }
}

// The spectral coefficients of the tasks of one block: workgroup b takes the
// tasks kap0 .. kap0 + 255 of a group of lpt lines.  Without kap = 0 their
// coefficients form two contiguous runs of a line, the frequencies kap
// (ascending) and K - kap (descending): staged in LDS, they are read and
// written by consecutive threads in 8-byte steps instead of n-strided ones.
struct LongRuns {
  int64_t grp;     // line group
  int kap;         // this thread's task
  int lo, cnt;     // tasks lo .. lo + cnt - 1 (lo >= 1) form the runs
  int64_t baseA;   // offset of frequency lo's coefficients
  int64_t baseB;   // offset of frequency K - (lo + cnt - 1)'s coefficients
};

__device__ __forceinline__ LongRuns long_runs(const LongArgs& a, int n) {
  LongRuns r;
  const int nt = long_pair_tasks(a.K);
  const int nkb = (nt + kLongThreads - 1) / kLongThreads;
  r.grp = blockIdx.x / nkb;
  const int k0 = (int)(blockIdx.x - r.grp * nkb) * kLongThreads;
  r.kap = k0 + (int)threadIdx.x;
  r.lo = k0 > 0 ? k0 : 1;
  const int hi = k0 + kLongThreads < nt ? k0 + kLongThreads : nt;
  r.cnt = hi > r.lo ? hi - r.lo : 0;
  r.baseA = n - 1 + (int64_t)(r.lo - 1) * n;
  r.baseB = n - 1 + (int64_t)(a.K - (hi - 1) - 1) * n;
  return r;
}

template <int NORD>
__global__ __launch_bounds__(kLongThreads) void long_contract_fwd_kernel(LongArgs a) {
  constexpr int n = NORD;
  __shared__ double SA[kLongThreads * NORD], SB[kLongThreads * NORD];
  const LongRuns r = long_runs(a, n);
  const bool act = r.kap < long_pair_tasks(a.K);
  const int pa = r.kap - r.lo, pb = r.lo + r.cnt - 1 - r.kap;
  const int64_t lend = (r.grp + 1) * a.lpt < a.nlines ? (r.grp + 1) * a.lpt : a.nlines;
  for (int64_t l = r.grp * a.lpt; l < lend; ++l) {
    double wa[NORD], wb[NORD];
    double* rs = a.out + l * a.M;
    if (act) {
      long_contract_fwd_line<NORD>(a, l, r.kap, wa, wb);
      if (r.kap == 0) {
        // the k = 0 block, and frequency K/2 for even K
#pragma unroll
        for (int c = 0; c < NORD - 1; ++c) rs[c] = wa[c];
        if ((a.K & 1) == 0) {
#pragma unroll
          for (int c = 0; c < NORD; ++c) rs[n - 1 + (int64_t)((a.K >> 1) - 1) * n + c] = wb[c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < NORD; ++c) {
          SA[pa * n + c] = wa[c];
          SB[pb * n + c] = wb[c];
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r.cnt * n; i += kLongThreads) {
      rs[r.baseA + i] = SA[i];
      rs[r.baseB + i] = SB[i];
    }
    __syncthreads();
  }
}

// The inverse: coefficients of the frequencies of task kap -> channel
// spectra with the Hermitian pre-twiddles -> slots of the buffers of wa.
template <int NORD>
__device__ __forceinline__ void long_contract_inv_line(const LongArgs& a, int64_t l, int kap, const double* wa,
                                                       const double* wb) {
  constexpr int n = NORD, ne = NORD / 2, no = (NORD - 1) / 2, P = NORD / 2, NC = NORD > 1 ? NORD - 1 : 1;
  const int K = a.K, ls = a.ls;
  const bool keven = (K & 1) == 0;
  const bool hasb = kap != 0 || keven;
  const int kh = K >> 1;
  const int ka = kap, kb = kap == 0 ? kh : K - kap;
  double h0[NORD], h1[NORD];
  const rsrc_t qtab = table_rsrc(a.Q, (uint32_t)((size_t)K * n * n));
  contract_inv2<double, NORD>(qtab, K, ka, hasb ? kb : ka, wa, wb, h0, h1, wa[0] + wb[0]);
  if (!hasb) {
#pragma unroll
    for (int c = 0; c < NORD; ++c) h1[c] = 0.0;
  }
  CD* B = long_buf(a.wa, l, 0, 1 + P, ls);
  const CD* twm = reinterpret_cast<const CD*>(a.twm);
  if (kap == 0) {
    write_nodal_zeros<double, false>(B, K);
    if (keven) write_nodal_inv<double, false>(B, K, kh, h1[0]);
  } else {
    write_nodal_inv<double, false>(B, K, kap, h0[0]);
    write_nodal_inv<double, false>(B, K, K - kap, h1[0]);
  }
  if constexpr (NORD > 1) {
    double ya[NC], yb[NC];
    if (kap == 0) {
#pragma unroll
      for (int b = 0; b < NORD - 1; ++b) ya[b] = h0[b];
#pragma unroll
      for (int m = 1; m <= ne; ++m) yb[m - 1] = h1[m];
#pragma unroll
      for (int m = 1; m <= no; ++m) yb[ne + m - 1] = h1[ne + m];
#pragma unroll
      for (int p = 1; p <= P; ++p) {
        const int b0 = 2 * (p - 1), b1 = b0 + 1;
        const bool has1 = b1 < NORD - 1;
        B[p * (size_t)ls + 0] = CD{ya[b0], has1 ? ya[b1] : 0.0};
        if (keven) {
          const CD va = herm<double>(yb[b0], yb[b0], kh, twm);
          const CD vb = has1 ? herm<double>(yb[b1], yb[b1], kh, twm) : CD{0, 0};
          B[p * (size_t)ls + kh] = CD{va.x - vb.y, va.y + vb.x};
        }
      }
    } else {
#pragma unroll
      for (int m = 1; m <= ne; ++m) {
        ya[m - 1] = h1[m];
        yb[m - 1] = h0[m];
      }
#pragma unroll
      for (int m = 1; m <= no; ++m) {
        ya[ne + m - 1] = h0[ne + m];
        yb[ne + m - 1] = h1[ne + m];
      }
#pragma unroll
      for (int p = 1; p <= P; ++p) {
        const int b0 = 2 * (p - 1), b1 = b0 + 1;
        const bool has1 = b1 < NORD - 1;
        CD va = herm<double>(ya[b0], yb[b0], kap, twm);
        CD vb = has1 ? herm<double>(ya[b1], yb[b1], kap, twm) : CD{0, 0};
        B[p * (size_t)ls + kap] = CD{va.x - vb.y, va.y + vb.x};
        va = herm<double>(yb[b0], ya[b0], K - kap, twm);
        vb = has1 ? herm<double>(yb[b1], ya[b1], K - kap, twm) : CD{0, 0};
        B[p * (size_t)ls + (K - kap)] = CD{va.x - vb.y, va.y + vb.x};
      }
    }
  }
}

template <int NORD>
__global__ __launch_bounds__(kLongThreads) void long_contract_inv_kernel(LongArgs a) {
  // n-strided loads of the coefficients: staging them through LDS (as the
  // forward contraction does for its stores) measured slower here
  constexpr int n = NORD;
  const LongRuns r = long_runs(a, n);
  if (r.kap >= long_pair_tasks(a.K)) return;
  const bool keven = (a.K & 1) == 0;
  const bool hasb = r.kap != 0 || keven;
  const int64_t offa = r.kap == 0 ? 0 : n - 1 + (int64_t)(r.kap - 1) * n;
  const int64_t offb = n - 1 + (int64_t)((r.kap == 0 ? a.K >> 1 : a.K - r.kap) - 1) * n;
  const int ra = r.kap == 0 ? n - 1 : n;
  const int64_t lend = (r.grp + 1) * a.lpt < a.nlines ? (r.grp + 1) * a.lpt : a.nlines;
  for (int64_t l = r.grp * a.lpt; l < lend; ++l) {
    const double* rs = a.in + l * a.M;
    double wa[NORD], wb[NORD];
#pragma unroll
    for (int c = 0; c < NORD; ++c) {
      wa[c] = c < ra ? rs[offa + c] : 0.0;
      wb[c] = hasb ? rs[offb + c] : 0.0;
    }
    long_contract_inv_line<NORD>(a, l, r.kap, wa, wb);
  }
}

// Element jp of line l from the inverse-transformed buffers of wb: node
// jp + 1 and the element's bubbles (as the scatter of the line passes).
template <int NORD>
__global__ __launch_bounds__(kLongThreads) void long_scatter_kernel(LongArgs a) {
  constexpr int n = NORD, ne = NORD / 2, P = NORD / 2, NB = 1 + P;
  const int K = a.K, ls = a.ls;
  const int64_t t = (int64_t)blockIdx.x * kLongThreads + threadIdx.x;
  if (t >= a.nlines * K) return;
  const int64_t l = t / K;
  const int jp = (int)(t - l * K);
  const CD* Z = long_buf(a.wb, l, 0, NB, ls);
  const CD* twd = reinterpret_cast<const CD*>(a.twd);
  double hv[NORD];
  hv[n - 1] = jp < K - 1 ? nodal_post<double, false>(Z, K, jp + 1, twd, true) : 0.0;
  const int q = (jp & 1) ? K - 1 - (jp >> 1) : (jp >> 1);
  const double sg = (jp & 1) ? -1.0 : 1.0;
#pragma unroll
  for (int m = 1; m <= ne; ++m) {
    const int be = m - 1;
    const double E = sg * reinterpret_cast<const double*>(Z + (1 + be / 2) * (size_t)ls + q)[be & 1];
    if (2 * m == n) {
      hv[m - 1] = E;
    } else {
      const int bo = ne + m - 1;
      const double O = reinterpret_cast<const double*>(Z + (1 + bo / 2) * (size_t)ls + q)[bo & 1];
      hv[m - 1] = E + O;
      hv[n - m - 1] = E - O;
    }
  }
  double* r = a.out + l * a.M + (int64_t)jp * n;
#pragma unroll
  for (int m = 0; m < n - 1; ++m) r[m] = hv[m];
  if (jp < K - 1) r[n - 1] = hv[n - 1];
  if (a.bad) {
    bool nonfinite = false;
#pragma unroll
    for (int m = 0; m < n; ++m) nonfinite |= !(hv[m] - hv[m] == 0.0);
    if (nonfinite) atomicOr(a.bad + l / a.lpf, 2);
  }
}

// Spectral coefficients of every line divided by react + mu (the axis'
// denominators) + mu_line[l] (the other axis' denominator of line l, when
// the lines are those of a transposed two-axis array): the middle step of a
// solve.
__global__ __launch_bounds__(kLongThreads) void long_divide_kernel(LongArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kLongThreads + threadIdx.x;
  if (t >= a.nlines * a.M) return;
  const int64_t l = t / a.M, i = t - l * a.M;
  a.out[t] = a.in[t] / (a.react + a.mu[i] + (a.mu_line ? a.mu_line[l] : 0.0));
}

static hipError_t grid_launch_check(int64_t threads, unsigned* nb) {
  const int64_t b = (threads + kLongThreads - 1) / kLongThreads;
  if (b < 1 || b > 0x7fffffff) return hipErrorInvalidValue;
  *nb = (unsigned)b;
  return hipSuccess;
}

template <int NORD>
static hipError_t long_step_n(int step, const LongArgs& a, hipStream_t s) {
  unsigned nb = 0;
  hipError_t e;
  const int64_t ngrp = (a.nlines + a.lpt - 1) / a.lpt;
  const int64_t nkb = (long_pair_tasks(a.K) + kLongThreads - 1) / kLongThreads;  // contraction blocks per group
  switch (step) {
    case LONG_GATHER:
      if ((e = grid_launch_check(a.nlines * a.K, &nb))) return e;
      hipLaunchKernelGGL((long_gather_kernel<NORD>), dim3(nb), dim3(kLongThreads), 0, s, a);
      break;
    case LONG_CONTRACT_FWD:
      if ((e = grid_launch_check(ngrp * nkb * kLongThreads, &nb))) return e;
      hipLaunchKernelGGL((long_contract_fwd_kernel<NORD>), dim3(nb), dim3(kLongThreads), 0, s, a);
      break;
    case LONG_CONTRACT_INV:
      if ((e = grid_launch_check(ngrp * nkb * kLongThreads, &nb))) return e;
      hipLaunchKernelGGL((long_contract_inv_kernel<NORD>), dim3(nb), dim3(kLongThreads), 0, s, a);
      break;
    case LONG_SCATTER:
      if ((e = grid_launch_check(a.nlines * a.K, &nb))) return e;
      hipLaunchKernelGGL((long_scatter_kernel<NORD>), dim3(nb), dim3(kLongThreads), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

void long_tiles(int lk1, int lk2, int* lgc, int* lgr) {
  // log2 of the columns (rows) per tile: 4096 points per tile (at least 4
  // columns of up to 1024 points, 2 of 2048), at most the other dimension
  auto pick = [](int lk, int lother) {
    const int lg = kLongLgTilePts - lk;
    return lg < lother ? lg : lother;
  };
  *lgc = pick(lk1, lk2);
  *lgr = pick(lk2, lk1);
}

static size_t tile_lds_bytes(int K, int lg) { return (size_t)((K + 1) << lg) * sizeof(CD); }

hipError_t launch_long(int n, int step, bool inv, const LongArgs& a, double* w, double* out, hipStream_t s) {
  const int D = a.K1 * a.K2;
  const bool pow2 = (a.K & (a.K - 1)) == 0;
  if (a.K < 2 || a.K > (1 << 20) || a.K1 != 1 << a.lk1 || a.K2 != 1 << a.lk2 || a.lk1 < 1 || a.lk2 < 1 ||
      a.lk1 > 11 || a.lk2 > 11 || (pow2 ? D != a.K : D < 2 * a.K - 1) || a.ls != D ||
      D > (1 << (2 * kLongTwBits + 1)) || a.nlines < 1 || a.lpt < 1 || (a.bad && a.lpf < 1))
    return hipErrorInvalidValue;
  // the Bluestein factors: only for K not a power of two, with their tables
  if (a.pre < 0 || a.pre > 4 || a.post < 0 || a.post > 2 || (pow2 && (a.pre || a.post)) ||
      (((a.pre && a.pre <= 2) || a.post) && !a.chirp) || (a.pre >= 3 && !a.bhat))
    return hipErrorInvalidValue;
  // a tile is one chunk of the Stockham stages (whole buffers, in place)
  if (a.lgc < 0 || a.lgc > a.lk2 || a.lgr < 0 || a.lgr > a.lk1 || a.lk1 + a.lgc > kLongLgTilePts ||
      a.lk2 + a.lgr > kLongLgTilePts)
    return hipErrorInvalidValue;
  const int NB = 1 + n / 2;
  if (step == LONG_COLS || step == LONG_ROWS) {
    const int64_t tiles = a.nlines * NB * (int64_t)(step == LONG_COLS ? a.K2 >> a.lgc : a.K1 >> a.lgr);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = step == LONG_COLS ? tile_lds_bytes(a.K1, a.lgc) : tile_lds_bytes(a.K2, a.lgr);
    if (step == LONG_COLS) {
      auto fn = inv ? long_cols_kernel<true> : long_cols_kernel<false>;
      (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(kLongThreads), lds, s, a, w);
    } else {
      auto fn = inv ? long_rows_kernel<true> : long_rows_kernel<false>;
      (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(kLongThreads), lds, s, a, (const double*)w, out);
    }
    return hipGetLastError();
  }
  if (step == LONG_DIVIDE) {
    unsigned nb = 0;
    hipError_t e = grid_launch_check(a.nlines * a.M, &nb);
    if (e) return e;
    hipLaunchKernelGGL(long_divide_kernel, dim3(nb), dim3(kLongThreads), 0, s, a);
    return hipGetLastError();
  }
  switch (n) {
#define FFTFEM_CASE(N) \
  case N:              \
    return long_step_n<N>(step, a, s);
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
