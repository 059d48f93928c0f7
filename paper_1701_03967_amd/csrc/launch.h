// Kernel argument blocks and launchers shared by the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fftfem {

enum { FWD = 0, INV = 1, MID = 2 };

template <typename T>
struct LineArgs {
  const void* in;
  void* out;
  const double* upd;      // INV with update: out = upd + result (float64)
  double* cor;            // INV with update, optional: the result (the correction) as float64
  int in_f64;
  int out_kind;           // 0: T, 1: double, 2: float
  int K, log2K;
  int64_t M, es, nlines;
  int64_t ies, oes;       // contiguous tiles only: nonzero = element stride of a
                          // transposed input / output (element i of line l at l + i ies)
  int G, log2G;           // lines per tile (a power of two)
  int lrmax;              // log2 of the largest FFT radix (4, 3 or 2; 0: 4)
  const T* Q;             // K blocks of n*n
  const T* twf;           // K complex exp(-2 pi i q/K)
  const T* twm;           // K complex exp(-i pi k/(2K))
  const T* twd;           // K complex exp(-i pi k/K)
  int L, log2L;           // K not a power of two without a mixed-radix plan: Bluestein length (else 0)
  int fl;                 // complex slots per FFT buffer: K, the padded K of a mixed-radix plan, or L
  int nrad;               // mixed-radix stages (K not a power of two, prime factors <= 7; else 0)
  uint64_t radpack;       // their radices, 3 bits per stage (stage i at bit 3 i): codes 0..6 for
                          // radix 2, 3, 4, 5, 7, 8, 16; product K
  const T* chirp;         // K complex exp(-i pi j^2/K)
  const T* bhat;          // L complex, spectrum of the conjugate chirp / L
  const T* twl;           // L complex exp(-2 pi i q/L)
  const T* arrow;         // condensed per-frequency solve (MID): bubble eigenbases
                          // We, Wo, then coef nu, coef gA, gC (n - 1 each), cc0, cc1
  const T* mu_self;       // M: diff_d 4/h_d^2 lambda along this axis
  const T* mu_o[2];       // other axes
  int64_t so[2], Mo[2];   // their strides and lengths
  int nother;
  T react;
  double* partials;       // per-block (sum c^2, sum u^2) in update mode
  const int* flag;        // nonzero: skip (refinement converged)
  int* bad;               // non-null (output pass without update): or 2 into it when
                          // a written value is NaN or Inf
};

// One operator pass along an axis (see apply_kernel).  Inputs and the
// outputs o2 and o1 (o1_kind 2) are double-double: [0] hi, [1] lo planes.
struct ApplyArgs {
  const double* in1[2];   // lo may be null: a float64 input
  const double* in2[2];   // hi null: one input; lo null iff in1 lo is null
  const double* f;        // non-null: o1 = f - result
  void* o1[2];
  double* o2[2];          // null: no second output
  int o1_kind;            // 0 float, 1 double, 2 double-double
  double c1[4], c2[4];
  int64_t M, es, nlines;
  int G, TL;
  const double* Ael[2];   // element matrices, hi and lo parts
  const double* Cel[2];
  const int* flag;
  int dd;                 // 1: double-double arithmetic; 0: plain float64 (no lo planes)
};


// The fused 2D operator pass (both axes of order n): out = f - A u (double-
// double, u and f float64; f null: out = A u) or out -= A u (plain float64,
// in place).  Tiles of 64 columns x E elements along axis 0.
struct Resid2Args {
  const double* u;
  const double* f;
  double* out;
  int64_t M0, M1;
  int K0, E;
  double c0, c1, react;   // diff_d 4 / h_d^2 of axes 0 and 1, reaction
  const double* Ael;      // element stiffness: (n+1)^2 hi values, then (n+1)^2 lo values
  const double* Cel;      // element mass, the same layout
  const int* flag;
  // plane pass of a 3D array (axes 1 and 2 of one order; M0, M1, K0 and c0,
  // c1 then refer to axes 1 and 2): planes = M_0, and the two products
  // (C_1 x C_2) u into out (hi) / out_l (lo, double-double) and
  // (c0 A_1 x C_2 + c1 C_1 x A_2 + react C_1 x C_2) u into out2 / out2_l
  int64_t planes;
  double* out_l;
  double* out2;
  double* out2_l;
};

// The banded solve along axis 0 (algorithm (b)): per line, the shifted 1D
// system (coef A + sigma C) x = y with sigma = react + the other axes'
// spectral terms.  Element i of line l sits at i * nlines + l (axis 0 of a
// row-major array).
struct BandArgs {
  const double* in;       // y (may equal out)
  double* out;            // x
  double* cp;             // one sweep: (K - 1) x nlines work (the elimination's pivots);
                          // three kernels: a work array of the size of y
  double* pr;             // three kernels: 2 (K - 1) x nlines work (node pairs), 16-byte aligned
  const double* tab;      // the axis' band tables (unscaled)
  double coef;            // diff 4 / h^2 of the axis
  double react;
  int K;
  int64_t nlines;
  const double* mu_o[2];  // other axes' spectral terms, strides and lengths
  int64_t so[2], Mo[2];
  int nother;
};

// Multi-pass transforms of long lines (1D plans, K = K1 K2 > 1024): work
// arrays wa and wb of nlines x (1 + n/2) buffers of K complex values.
enum { LONG_GATHER = 0, LONG_COLS, LONG_ROWS, LONG_CONTRACT_FWD, LONG_CONTRACT_INV, LONG_SCATTER, LONG_DIVIDE };
struct LongArgs {
  const double* in;       // lines (gather, inverse contraction, divide)
  double* out;            // lines (forward contraction, scatter, divide)
  double* wa;             // gather / inverse-contraction output, column-pass buffers
  double* wb;             // buffers read by the forward contraction and the scatter
  int K;                  // elements per line
  int ls;                 // slots per work buffer: the DFT length D = K1 K2
  int K1, K2, lk1, lk2;   // D = K1 K2 = 2^(lk1 + lk2): K, or Bluestein's L >= 2K - 1
  int64_t M, nlines;
  const double* Q;        // (c n + l) K + k, float64
  const double* twm;      // K complex exp(-i pi k / (2K))
  const double* twd;      // K complex exp(-i pi k / K)
  const double* tw1;      // K1 complex exp(-2 pi i q / K1)
  const double* tw2;      // K2 complex exp(-2 pi i q / K2)
  const double* twlo;     // 1024 complex exp(-2 pi i q / D)
  const double* twhi;     // D / 1024 complex exp(-2 pi i 1024 q / D)
  const double* chirp;    // K not a power of two: K complex exp(-i pi j^2 / K)
  const double* bhat;     // and L complex: the spectrum of conj(chirp) (zero-padded, cyclic) / L
  const double* mu;       // M: the axis' spectral denominators (divide)
  double react;
  int* bad;               // scatter: when set, bit 2 of bad[l / lpf] marks NaN / Inf in line l
  int64_t lpf;            // lines per flag (1: one flag per line)
  const double* mu_line;  // divide: when set, mu_line[l] is added to line l's denominators
  int lgc, lgr;           // log2 of the columns per column tile and of the rows per row tile (long_tiles)
  int lpt;                // lines per contraction thread
  int pre, post;          // Bluestein factors of the column loads and the row stores (long.hip)
};
// step LONG_COLS / LONG_ROWS work on buffer array w (rows: into out), the
// others on the arrays of a
hipError_t launch_long(int n, int step, bool inv, const LongArgs& a, double* w, double* out, hipStream_t s);
void long_tiles(int lk1, int lk2, int* lgc, int* lgr);

// One axis pass of the Dirichlet lifting (extended axis of E = nK + 1 points
// -> its M = nK - 1 interior rows): out[o, i, ii] = sum_q X_ext[i + 1, q] in[o, q, ii].
struct LiftArgs {
  const double* in;       // shape outer x E x inner
  double* out;            // shape outer x M x inner
  const double* f;        // combine: out = (f ? f : out) - scale * result
  const double* X;        // (n + 1) x (n + 1) element matrix
  int n, K;
  int64_t outer, inner;
  int mask;               // the input is the extended b: its interior reads as zero
  int N;
  int64_t ext[3];         // extended shape of b (mask only)
  int combine;
  double scale;
};

// Jobs of the grouped operator, transpose and bookkeeping launches.
struct TransposeJob {
  const void* in;
  void* out;
  int64_t R, C, ntr, ntc;
};
struct ResetJob {
  int* flag;
  double* stats;
  int nstats;
};
struct ReduceJob {
  const double* partials;
  int nparts, iter;
  double tol;
  int* flag;
  double* stats;
};
// jobs: ApplyArgs or TransposeJob array (see launch_line's GroupedLaunch)
struct GroupedOps {
  const void* jobs;
  const int* job_of;
  const int* start;
  int nblocks;
  size_t lds;
};
hipError_t launch_apply_grouped(int n, bool lo, bool dd, const GroupedOps& g, hipStream_t s);
template <typename T>
hipError_t launch_transpose_grouped(const GroupedOps& g, hipStream_t s);
hipError_t launch_reset_grouped(const ResetJob* jobs, int njobs, hipStream_t s);
hipError_t launch_reduce_grouped(const ReduceJob* jobs, int njobs, hipStream_t s);

// A grouped launch: nblocks blocks over a device array of jobs; block b runs
// tile b - start[j] of job j = job_of[b] (start has one entry per job plus
// the total).  lds: the largest per-job tile.
template <typename T>
struct GroupedLaunch {
  const LineArgs<T>* jobs;
  const int* job_of;
  const int* start;
  int nblocks;
  size_t lds;
};

// Line-pass launchers, one per object built from line.hip: element counts
// that are powers of two (p2), other K with prime factors <= 7 (mr, mixed
// radix), and all others (bs, Bluestein).  line_kind() names the object a
// line of the arguments needs.
template <typename T>
hipError_t launch_line_grouped_p2(int n, int mode, bool upd, bool lf, const GroupedLaunch<T>& g, hipStream_t s);
template <typename T>
hipError_t launch_line_grouped_mr(int n, int mode, bool upd, bool lf, const GroupedLaunch<T>& g, hipStream_t s);
template <typename T>
hipError_t launch_line_grouped_bs(int n, int mode, bool upd, bool lf, const GroupedLaunch<T>& g, hipStream_t s);
template <typename T>
hipError_t launch_line_p2(int n, int mode, bool upd, const LineArgs<T>& a, int nblocks, size_t lds,
                          hipStream_t s);
template <typename T>
hipError_t launch_line_mr(int n, int mode, bool upd, const LineArgs<T>& a, int nblocks, size_t lds,
                          hipStream_t s);
template <typename T>
hipError_t launch_line_bs(int n, int mode, bool upd, const LineArgs<T>& a, int nblocks, size_t lds,
                          hipStream_t s);
template <typename T>
inline int line_kind(const LineArgs<T>& a) {
  return (a.K & (a.K - 1)) == 0 ? 0 : (a.nrad > 0 ? 1 : 2);
}
template <typename T>
inline hipError_t launch_line(int n, int mode, bool upd, const LineArgs<T>& a, int nblocks, size_t lds,
                              hipStream_t s) {
  switch (line_kind(a)) {
    case 0: return launch_line_p2<T>(n, mode, upd, a, nblocks, lds, s);
    case 1: return launch_line_mr<T>(n, mode, upd, a, nblocks, lds, s);
    default: return launch_line_bs<T>(n, mode, upd, a, nblocks, lds, s);
  }
}
template <typename T>
inline hipError_t launch_line_grouped(int kind, int n, int mode, bool upd, bool lf, const GroupedLaunch<T>& g,
                                      hipStream_t s) {
  switch (kind) {
    case 0: return launch_line_grouped_p2<T>(n, mode, upd, lf, g, s);
    case 1: return launch_line_grouped_mr<T>(n, mode, upd, lf, g, s);
    default: return launch_line_grouped_bs<T>(n, mode, upd, lf, g, s);
  }
}
hipError_t launch_apply(int n, const ApplyArgs& a, int nblocks, size_t lds, hipStream_t s);
hipError_t launch_resid2(int n, bool dd, const Resid2Args& a, hipStream_t s);
hipError_t launch_resid2_grouped(int n, bool dd, const GroupedOps& g, hipStream_t s);
int64_t resid2_blocks(const Resid2Args& a);  // workgroups of one launch (both forms)
hipError_t launch_resid3p(int n, bool dd, const Resid2Args& a, hipStream_t s);
hipError_t launch_resid3p_grouped(int n, bool dd, const GroupedOps& g, hipStream_t s);
hipError_t launch_band(int n, const BandArgs& a, hipStream_t s);
hipError_t launch_band_split(int n, int step, const BandArgs& a, hipStream_t s);  // step 0, 1, 2
hipError_t launch_band_tile(int n, const BandArgs& a, hipStream_t s);
hipError_t launch_lift(const LiftArgs& a, hipStream_t s);
// The Dirichlet lifting's static work area (doubles per device) and its
// device address on the current device.
constexpr size_t kLiftScratchDoubles = size_t(1) << 21;
hipError_t lift_scratch(double** ptr);
int band_tile_lines(int K);  // lines per workgroup of launch_band_tile for K elements, 0: K too large
template <typename T>
hipError_t launch_transpose(const T* in, T* out, int64_t batch, int64_t R, int64_t C, hipStream_t s);
hipError_t launch_reset(int* flag, double* stats, int nstats, hipStream_t s);
hipError_t launch_reset_many(int* flags, double* stats, int nstats, int count, hipStream_t s);
hipError_t launch_reduce(const double* partials, int nparts, int iter, double tol, int* flag,
                         double* stats, hipStream_t s);

constexpr int kBlock = 256;        // threads per workgroup of every kernel
constexpr int kLineTasks = 1024;   // G * K limit of one line-kernel tile
constexpr int64_t kLongMaxK = int64_t(1) << 20;  // largest K of the long-line transforms (1D)
constexpr size_t kLongWorkBytes = size_t(8) << 30;  // per work array of the long-line transforms (chunks of lines beyond)
constexpr int kMaxLineOrder = 9;   // element orders compiled into the line kernels

}  // namespace fftfem
