// C ABI of the solver: plan construction, solve schedule, operator apply,
// refinement loop and statistics.  Host code only; every arithmetic step of
// a solve runs in the HIP kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdio>

#include <algorithm>
#include <cmath>
#include <limits>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fftfem.h"
#include "fftfem_internal.h"
#include "launch.h"
#include "record.h"

using namespace fftfem;

namespace {

// Per-axis device tables: Q, twf, twm, twd, mu, for K not a power of two
// the Bluestein chirp, bhat and twl (null otherwise), the condensed
// per-frequency solve's constants and the banded solve's (algorithm (b)).
constexpr int kNumTables = 10;
struct DevTables {
  double* d[kNumTables] = {};
  float* f[kNumTables] = {};
};

}  // namespace

struct fftfem_plan_s {
  fftfem_desc desc{};
  int N = 0, n = 0, nrhs = 1;
  int64_t K[3] = {0, 0, 0}, M[3] = {0, 0, 0}, stride[3] = {0, 0, 0};
  int64_t size = 0;  // per right-hand side
  double coef[3] = {0, 0, 0};
  std::vector<AxisTables> host;
  DevTables dev[3];
  int nd[3] = {0, 0, 0};     // element order per axis
  double* Ael[3] = {};       // per-axis element matrices, hi then lo parts
  double* Cel[3] = {};
  float* W32 = nullptr;      // float32 workspace (float32 modes)
  float* W32b = nullptr;     // second float32 workspace (transposed 2D schedule)
  double* W64b = nullptr;    // float64 workspace (transposed 2D schedule, float64 mode)
  double* W64r = nullptr;    // float64 residual (float32 + refinement)
  bool algb = false;         // algorithm (b): banded solve along axis 0
  int band_form = 0;         // ... 0: one sweep per line, 1: three kernels (few lines),
                             // 2: one LDS-tiled kernel (short lines)
  double* Wband = nullptr;   // its work: (K_0 - 1) x (size / M_0) pivots, or (split) size values
  bool longK = false;        // an axis with K > 1024 (1D, or one or both of 2D): multi-pass transforms
  double* Wl[2] = {nullptr, nullptr};  // their work arrays: lines x (1 + n/2) x D complex each (the
                                       // largest over the axes) for long_chunk lines at a time
  int64_t long_chunk = 0;              // lines per pass (of nrhs in 1D, M of the other axis in 2D)
  // per axis: the four-step split of the DFT length D (K, or Bluestein's L),
  // the tile shapes, and the twiddles: sub-DFTs (K1, K2), low and high parts
  // of exp(-2 pi i m / D) (1024, D / 1024)
  struct LongAxis {
    int lk1 = 0, lk2 = 0, lgc = 0, lgr = 0;
    int64_t D = 0;
    double* tw[4] = {nullptr, nullptr, nullptr, nullptr};
  } lax[FFTFEM_MAX_DIMS];
                             // then 2 (K_0 - 1) x (size / M_0) node pairs
  bool tr2d = false;         // 2D: run the axis-0 pass on a transposed copy
  bool trfused = false;      // ... made by the axis-1 passes' own stores and loads (no transposes)
  double* tmp[8] = {};       // operator-apply partial products (double-double planes)
  double* cor = nullptr;     // while set: the update pass also stores its correction here
  int* bad = nullptr;        // while set: output passes without update report non-finite values here
  int ntmp = 0;
  double* partials = nullptr;
  int npartials = 0;
  int nparts_last = 0;       // partial sums written by the last update pass
  int* flags = nullptr;      // one per rhs
  double* stats = nullptr;   // (2 + FFTFEM_MAX_ITERS + 1) per rhs
  size_t bytes = 0;
  int lds_max = 65536;
  hipStream_t last = nullptr;
  // batched execution: launches are recorded (with their schedule position)
  // instead of issued while rec is set
  Recorder* rec = nullptr;
  int phase = 0;
  // timing runs of the tuner: forced lines per tile and FFT radix (0: none)
  int Gforce = 0, lrforce = 0;
  std::vector<void*> allocs;
  // per-kernel timing (measurement only)
  bool timing = false;
  struct Mark {
    int name;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<std::string> names;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
};

namespace {

constexpr int kStatsLen = 2 + FFTFEM_MAX_ITERS + 1;

int from_hip(hipError_t e) {
  if (e == hipSuccess) return FFTFEM_OK;
  if (e == hipErrorOutOfMemory) return FFTFEM_ENOMEM;
  return FFTFEM_EHIP;
}

hipEvent_t take_event(fftfem_plan_t p) {
  if (p->pool_used == p->pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->pool.push_back(e);
  }
  return p->pool[p->pool_used++];
}

// Brackets one launch with events when timing is on.
struct Timed {
  fftfem_plan_t p;
  hipStream_t s;
  hipEvent_t a = nullptr;
  int name = -1;
  Timed(fftfem_plan_t p_, hipStream_t s_, const std::string& nm) : p(p_), s(s_) {
    if (!p->timing) return;
    for (size_t i = 0; i < p->names.size(); ++i)
      if (p->names[i] == nm) name = (int)i;
    if (name < 0) {
      p->names.push_back(nm);
      name = (int)p->names.size() - 1;
    }
    a = take_event(p);
    if (a) (void)hipEventRecord(a, s);
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(p);
    if (!b) return;
    (void)hipEventRecord(b, s);
    p->marks.push_back({name, a, b});
  }
};

const char* mode_name(int mode, bool upd) {
  if (mode == FWD) return "fwd";
  if (mode == INV) return upd ? "inv_upd" : "inv";
  return upd ? "mid_upd" : "mid";
}

int dev_alloc(fftfem_plan_t p, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) return FFTFEM_OK;
  const char* fail = std::getenv("FFTFEM_TEST_FAIL_ALLOC");
  if (fail && fail[0] == '1') return FFTFEM_ENOMEM;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? FFTFEM_ENOMEM : FFTFEM_EHIP;
  }
  p->allocs.push_back(*ptr);
  p->bytes += bytes;
  return FFTFEM_OK;
}

template <typename T>
int upload(fftfem_plan_t p, T** dst, const std::vector<double>& src) {
  std::vector<T> tmp(src.begin(), src.end());
  int rc = dev_alloc(p, (void**)dst, tmp.size() * sizeof(T));
  if (rc) return rc;
  return from_hip(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int64_t x) {
  int r = 0;
  while ((int64_t(1) << r) < x) ++r;
  return r;
}

int validate(const fftfem_desc* d) {
  if (!d) return FFTFEM_EINVAL;
  if (d->N < 1 || d->N > FFTFEM_MAX_DIMS) return FFTFEM_EINVAL;
  if (d->n < 1 || d->n > FFTFEM_MAX_ORDER) return FFTFEM_EINVAL;
  for (int i = 0; i < d->N; ++i)
    if (d->n_axis[i] < 0 || d->n_axis[i] > FFTFEM_MAX_ORDER) return FFTFEM_EINVAL;
  if (d->flags & ~FFTFEM_ALGORITHM_B) return FFTFEM_EINVAL;
  if (d->precision < FFTFEM_FP64 || d->precision > FFTFEM_FP32_REFINE) return FFTFEM_EINVAL;
  if (d->max_iter < 0 || d->max_iter > FFTFEM_MAX_ITERS) return FFTFEM_EINVAL;
  if (d->nrhs < 0 || !(d->tol >= 0) || !std::isfinite(d->react)) return FFTFEM_EINVAL;
  for (int i = 0; i < d->N; ++i) {
    if (d->K[i] < 2) return FFTFEM_EINVAL;
    if (!(d->diff[i] > 0) || !std::isfinite(d->diff[i])) return FFTFEM_EINVAL;
    if (d->X[i] < 0 || !std::isfinite(d->X[i])) return FFTFEM_EINVAL;
  }
  return FFTFEM_OK;
}

// FFT buffer length of an axis: K (a power of two), K rounded up to a
// multiple of 32 (mixed radix: the LDS slot swizzle permutes within aligned
// blocks of up to 32 slots, so every permuted slot of the first K stays in
// the buffer), or the Bluestein length L.
int64_t fft_len(int64_t K) {
  if ((K & (K - 1)) == 0) return K;
  if (!mixed_radices(K).empty()) return (K + 31) & ~int64_t(31);
  int64_t L = 1;
  while (L < 2 * K - 1) L *= 2;
  return L;
}

// Tuned parameters are shared by element counts with the same FFT buffer
// length and kind of transform (power of two, mixed radix, Bluestein).
int64_t tune_class_of(int64_t K) {
  const int kind = (K & (K - 1)) == 0 ? 0 : (mixed_radices(K).empty() ? 1 : 2);
  return 4 * fft_len(K) + kind;
}


size_t line_lds(int n, int64_t K, size_t elt, bool pad = true) {
  return (size_t)(1 + n / 2) * (fft_len(K) + (pad ? 1 : 0)) * 2 * elt;  // pad slot per FFT buffer
}

// Lines per workgroup for a line pass: a power of two with G * K <= 1024
// (per-thread task registers), G lines of LDS within the budget (64 KB, or
// one line when a line alone is larger), at most 64 and at most nlines.
int choose_G(int n, int64_t K, size_t elt, int64_t nlines) {
  size_t per = line_lds(n, K, elt);
  size_t budget = std::max<size_t>(line_lds(n, K, elt, false), 65536);
  int G = 1;
  while (G < 64 && (size_t)(2 * G) * per <= budget && 2 * G * K <= kLineTasks && 2 * G <= nlines)
    G *= 2;
  return G;
}

}  // namespace

// ---- tuned line-pass parameters (process-wide) ----------------------------
bool TuneKey::operator<(const TuneKey& o) const {
  if (elt != o.elt) return elt < o.elt;
  if (n != o.n) return n < o.n;
  if (mode != o.mode) return mode < o.mode;
  if (lf != o.lf) return lf < o.lf;
  return K < o.K;
}

namespace {
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
}  // namespace

namespace fftfem {

void tune_set(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> l(g_tune_mu);
  g_tune[k] = v;
}

bool tune_get(const TuneKey& k, TuneVal* v) {
  std::lock_guard<std::mutex> l(g_tune_mu);
  if (g_tune.empty()) return false;
  auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}

void plan_set_recorder(fftfem_plan_t p, Recorder* r) { p->rec = r; }
void plan_set_stream(fftfem_plan_t p, hipStream_t s) { p->last = s; }
size_t plan_array_bytes(fftfem_plan_t p) { return (size_t)p->size * (size_t)p->nrhs * sizeof(double); }
int64_t tune_class(int64_t K) { return tune_class_of(K); }

}  // namespace fftfem

namespace {

template <typename A>
void record(fftfem_plan_t p, int kind, std::initializer_list<int> key, const A& args, int64_t nblocks,
            size_t lds) {
  Rec r;
  r.phase = p->phase;
  r.kind = kind;
  int i = 0;
  for (int k : key) r.key[i++] = k;
  for (; i < 5; ++i) r.key[i] = 0;
  r.args.resize(sizeof(A));
  std::memcpy(r.args.data(), &args, sizeof(A));
  r.nblocks = (int)nblocks;
  r.lds = lds;
  p->rec->recs.push_back(std::move(r));
}

int ilog2i(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

// Geometry of one line pass: which axis' tables, the line length, the
// element stride, the number of lines, and where the other axes' spectral
// indices are found (for the division in a MID pass).
struct Geom {
  int axis = 0;
  int64_t M = 0, es = 1, nlines = 0;
  int64_t ies = 0, oes = 0;  // transposed input / output layouts (contiguous tiles)
  int nother = 0;
  int oaxis[2] = {0, 0};
  int64_t so[2] = {1, 1}, Mo[2] = {1, 1};
};

Geom natural_geom(const fftfem_plan_s* p, int axis, bool others) {
  Geom g;
  g.axis = axis;
  g.M = p->M[axis];
  g.es = p->stride[axis];
  g.nlines = p->size / g.M;
  if (others)
    for (int e = 0; e < p->N; ++e)
      if (e != axis) {
        g.oaxis[g.nother] = e;
        g.so[g.nother] = p->stride[e];
        g.Mo[g.nother] = p->M[e];
        ++g.nother;
      }
  return g;
}

template <typename T>
const T* tab(const fftfem_plan_s* p, int axis, int which);
template <>
const double* tab<double>(const fftfem_plan_s* p, int axis, int which) {
  return p->dev[axis].d[which];
}
template <>
const float* tab<float>(const fftfem_plan_s* p, int axis, int which) {
  return p->dev[axis].f[which];
}

// One line pass.
template <typename T>
int line_pass(fftfem_plan_t p, const Geom& gm, int mode, const void* in, int in_f64, void* out,
              int out_kind, const double* upd, const int* flag, hipStream_t s, bool want_partials) {
  LineArgs<T> a{};
  const AxisTables& t = p->host[gm.axis];
  a.in = in;
  a.out = out;
  a.upd = upd;
  a.cor = upd ? p->cor : nullptr;
  a.in_f64 = in_f64;
  a.out_kind = out_kind;
  a.K = (int)t.K;
  a.log2K = ilog2(t.K);
  a.M = gm.M;
  a.es = gm.es;
  a.nlines = gm.nlines;
  a.ies = gm.ies;
  a.oes = gm.oes;
  const int n = p->nd[gm.axis];
  a.G = choose_G(n, t.K, sizeof(T), a.nlines);
  a.lrmax = 4;
  {
    TuneVal tv;
    const bool lf = gm.es > 1;
    if (p->Gforce) {
      a.G = p->Gforce;
      a.lrmax = p->lrforce;
    } else if (tune_get(TuneKey{(int)sizeof(T), n, mode, lf ? 1 : 0, tune_class(t.K)}, &tv)) {
      a.G = tv.G;
      a.lrmax = tv.lrmax;
    }
    // tuned or loaded values still respect this plan's lines, tasks and LDS
    while (a.G > 1 && (a.G > a.nlines || (int64_t)a.G * t.K > kLineTasks ||
                       (size_t)a.G * line_lds(n, t.K, sizeof(T)) > (size_t)p->lds_max))
      a.G /= 2;
  }
  a.log2G = ilog2i(a.G);
  a.Q = tab<T>(p, gm.axis, 0);
  a.twf = tab<T>(p, gm.axis, 1);
  a.twm = tab<T>(p, gm.axis, 2);
  a.twd = tab<T>(p, gm.axis, 3);
  a.mu_self = tab<T>(p, gm.axis, 4);
  a.L = (int)t.L;
  a.log2L = t.L ? ilog2(t.L) : 0;
  a.fl = (int)fft_len(t.K);
  a.nrad = (int)t.radices.size();
  if (a.nrad > 21) return FFTFEM_ENOTIMPL;
  a.radpack = 0;
  for (int i = 0; i < a.nrad; ++i) {
    const int R = t.radices[i];
    const uint64_t code = R == 2 ? 0 : R == 3 ? 1 : R == 4 ? 2 : R == 5 ? 3 : R == 7 ? 4 : R == 8 ? 5 : 6;
    a.radpack |= code << (3 * i);
  }
  a.chirp = tab<T>(p, gm.axis, 5);
  a.bhat = tab<T>(p, gm.axis, 6);
  a.twl = tab<T>(p, gm.axis, 7);
  a.arrow = tab<T>(p, gm.axis, 8);
  a.react = (T)p->desc.react;
  a.nother = gm.nother;
  for (int e = 0; e < gm.nother; ++e) {
    a.mu_o[e] = tab<T>(p, gm.oaxis[e], 4);
    a.so[e] = gm.so[e];
    a.Mo[e] = gm.Mo[e];
  }
  a.partials = want_partials ? p->partials : nullptr;
  a.flag = flag;
  a.bad = out_kind == 1 && upd == nullptr ? p->bad : nullptr;
  size_t lds = (size_t)a.G * line_lds(n, t.K, sizeof(T), a.G > 1);
  if (lds > (size_t)p->lds_max) return FFTFEM_ENOTIMPL;
  int64_t nblocks = (a.nlines + a.G - 1) / a.G;
  if (want_partials && nblocks > p->npartials) return FFTFEM_ENOTIMPL;
  if (want_partials) p->nparts_last = (int)nblocks;
  if (p->rec) {
    record(p, sizeof(T) == 4 ? REC_LINE32 : REC_LINE64,
           {n, mode, upd != nullptr ? 1 : 0, gm.es > 1 ? 1 : 0, line_kind(a)}, a, nblocks, lds);
    return FFTFEM_OK;
  }
  Timed tm(p, s, std::string(mode_name(mode, upd != nullptr)) + (sizeof(T) == 4 ? "32" : "64") +
                    "_ax" + std::to_string(gm.axis) + (gm.es == 1 && gm.axis != p->N - 1 ? "t" : ""));
  return from_hip(launch_line<T>(n, mode, upd != nullptr, a, (int)nblocks, lds, s));
}

template <typename T>
int transpose(fftfem_plan_t p, const T* in, T* out, int64_t R, int64_t C, hipStream_t s) {
  if (p->rec) {
    TransposeJob j{in, out, R, C, (R + 63) / 64, (C + 63) / 64};
    const int64_t batch = p->size / (R * C);
    if (batch != 1) return FFTFEM_ENOTIMPL;
    record(p, sizeof(T) == 4 ? REC_TR32 : REC_TR64, {}, j, j.ntr * j.ntc, 0);
    return FFTFEM_OK;
  }
  Timed tm(p, s, std::string("transpose") + (sizeof(T) == 4 ? "32" : "64"));
  return from_hip(launch_transpose<T>(in, out, p->size / (R * C), R, C, s));
}

// A double-double array: hi plane and lo plane (lo null: a float64 array).
struct DDp {
  const double* h;
  const double* l;
};

// One operator pass along `axis` (see ApplyArgs in launch.h).  out1 kind:
// 0 float, 1 double, 2 double-double (o1h, o1l).
int apply_pass(fftfem_plan_t p, int axis, DDp in1, DDp in2, const double* f, void* o1h, double* o1l,
               int o1_kind, double* o2h, double* o2l, const double c1[4], const double c2[4],
               const int* flag, hipStream_t s, bool dd = true) {
  ApplyArgs a{};
  a.dd = dd ? 1 : 0;
  a.in1[0] = in1.h;
  a.in1[1] = in1.l;
  a.in2[0] = in2.h;
  a.in2[1] = in2.l;
  a.f = f;
  a.o1[0] = o1h;
  a.o1[1] = o1l;
  a.o1_kind = o1_kind;
  a.o2[0] = o2h;
  a.o2[1] = o2l;
  for (int i = 0; i < 4; ++i) {
    a.c1[i] = c1[i];
    a.c2[i] = c2 ? c2[i] : 0.0;
  }
  a.M = p->M[axis];
  a.es = p->stride[axis];
  a.nlines = p->size / a.M;
  const int planes = (in1.l ? 2 : 1) * (in2.h ? 2 : 1);
  if (a.es > 1) {
    a.G = 32;
    a.TL = planes > 2 ? 32 : 64;
  } else {
    a.G = 4;
    a.TL = 512;
  }
  const int n = p->nd[axis];
  const int XX = (n + 1) * (n + 1);
  a.Ael[0] = p->Ael[axis];
  a.Ael[1] = p->Ael[axis] + XX;
  a.Cel[0] = p->Cel[axis];
  a.Cel[1] = p->Cel[axis] + XX;
  a.flag = flag;
  int64_t W = a.TL + 2 * n;
  size_t lds = (size_t)planes * a.G * W * sizeof(double);
  int64_t nblocks = ((a.nlines + a.G - 1) / a.G) * ((a.M + a.TL - 1) / a.TL);
  if (p->rec) {
    record(p, REC_APPLY, {n, in1.l ? 1 : 0, dd ? 1 : 0}, a, nblocks, lds);
    return FFTFEM_OK;
  }
  Timed tm(p, s, std::string(dd ? "apply_ax" : "apply64_ax") + std::to_string(axis));
  return from_hip(launch_apply(n, a, (int)nblocks, lds, s));
}

// y = A u (out_kind 1) or r = f - A u (f non-null; out_kind 0 stores it as
// float), for one right-hand side.  Sum factorization over the axes, last
// axis first, with double-double partial products:
//   1D: c0 a u + react c u
//   2D: pass axis 1: t = c u, s = a u;  pass axis 0: c0 a t + react c t + c1 c s
//   3D: pass axis 2: t = c u, s = a u;
//       pass axis 1: t2 = c t, s2 = c1 a t + react c t + c2 c s;
//       pass axis 0: c0 a t2 + c s2
// The fused 2D operator pass (resid2_kernel) applies to 2D plans whose two
// axes have the same element order (in batches too: the grouped launch
// runs the same body per job).  FFTFEM_RESID2=0 selects the two-pass form
// everywhere (tests compare the two).
static bool fused2d(fftfem_plan_t p) {
  if (p->N != 2 || p->nd[0] != p->nd[1]) return false;
  const char* e = std::getenv("FFTFEM_RESID2");
  return !(e && e[0] == '0');
}

// Elements per one-wave workgroup along axis 0 of the fused pass: 16 (each
// chunk also walks one element past its end), fewer when the grid would
// not give every CU a few dozen waves.
static int fused2d_chunk(fftfem_plan_t p) {
  const int64_t ncb = (p->M[1] + 63) / 64;
  int E = 16;
  while (E > 1 && ncb * ((p->K[0] + E - 1) / E) < 8192) E /= 2;
  return E;
}

static int resid2(fftfem_plan_t p, const double* u, const double* f, double* out, bool dd, const int* flag,
                  hipStream_t s) {
  Resid2Args a{};
  a.u = u;
  a.f = f;
  a.out = out;
  a.M0 = p->M[0];
  a.M1 = p->M[1];
  a.K0 = (int)p->K[0];
  a.E = fused2d_chunk(p);
  a.c0 = p->coef[0];
  a.c1 = p->coef[1];
  a.react = p->desc.react;
  a.Ael = p->Ael[0];
  a.Cel = p->Cel[0];
  a.flag = flag;
  if (p->rec) {
    record(p, REC_RESID2, {p->nd[0], dd ? 1 : 0, 0, 0, 0}, a, (int)resid2_blocks(a), 0);
    return FFTFEM_OK;
  }
  Timed tm(p, s, dd ? "resid2dd" : "resid2f64");
  return from_hip(launch_resid2(p->nd[0], dd, a, s));
}

// The last pass of the 3D operator: out = f - (c_0 A_0 P + C_0 Q) (or
// without f: the product), P and Q from the first two passes or the plane
// pass in tmp[4..7]; double-double or plain float64 (out = r in place).
static int operator_apply_axis0(fftfem_plan_t p, const double* f, void* out, int out_kind, const int* flag,
                                hipStream_t s, int ph, bool dd) {
  double** T = p->tmp;
  p->phase = ph + 2;
  const double c1[4] = {p->coef[0], 0, 0, 1};
  if (dd)
    return apply_pass(p, 0, {T[4], T[5]}, {T[6], T[7]}, f, out, nullptr, out_kind, nullptr, nullptr, c1, nullptr,
                      flag, s);
  return apply_pass(p, 0, {T[4], nullptr}, {T[6], nullptr}, f, out, nullptr, out_kind, nullptr, nullptr, c1,
                    nullptr, flag, s, false);
}

// The 3D plane pass (resid3p_kernel): axes 1 and 2 of one order, in batches
// too; FFTFEM_RESID2=0 selects the three-pass form.
static bool fused3d(fftfem_plan_t p) {
  if (p->N != 3 || p->nd[1] != p->nd[2]) return false;
  const char* e = std::getenv("FFTFEM_RESID2");
  return !(e && e[0] == '0');
}

// Passes 1 and 2 of the 3D operator in one: P = (C_1 x C_2) u into tmp[4]
// (and tmp[5], double-double lo), Q = (c_1 A_1 x C_2 + c_2 C_1 x A_2 +
// react C_1 x C_2) u into tmp[6] (tmp[7]).
static int resid3p(fftfem_plan_t p, const double* u, bool dd, const int* flag, hipStream_t s) {
  double** T = p->tmp;
  Resid2Args a{};
  a.u = u;
  a.out = T[4];
  a.out_l = dd ? T[5] : nullptr;
  a.out2 = T[6];
  a.out2_l = dd ? T[7] : nullptr;
  a.planes = p->M[0];
  a.M0 = p->M[1];
  a.M1 = p->M[2];
  a.K0 = (int)p->K[1];
  a.c0 = p->coef[1];
  a.c1 = p->coef[2];
  a.react = p->desc.react;
  a.Ael = p->Ael[1];
  a.Cel = p->Cel[1];
  a.flag = flag;
  const int64_t per_plane = (a.M1 + 63) / 64;
  int E = 16;
  while (E > 1 && a.planes * per_plane * ((a.K0 + E - 1) / E) < 8192) E /= 2;
  a.E = E;
  if (p->rec) {
    record(p, REC_RESID3P, {p->nd[1], dd ? 1 : 0, 0, 0, 0}, a, (int)resid2_blocks(a), 0);
    return FFTFEM_OK;
  }
  Timed tm(p, s, dd ? "resid3pdd" : "resid3pf64");
  return from_hip(launch_resid3p(p->nd[1], dd, a, s));
}

int operator_apply(fftfem_plan_t p, const double* u, const double* f, void* out, int out_kind,
                   const int* flag, hipStream_t s, int ph = 0) {
  const double* c = p->coef;
  double react = p->desc.react;
  double** T = p->tmp;
  const DDp none{nullptr, nullptr};
  int rc;
  p->phase = ph;
  if (out_kind == 1 && fused2d(p)) return resid2(p, u, f, (double*)out, true, flag, s);
  if (p->N == 2 && !T[3]) return FFTFEM_ENOTIMPL;  // long-line plan: no planes for the two-pass form
  if (fused3d(p)) {
    rc = resid3p(p, u, true, flag, s);
    if (rc) return rc;
    return operator_apply_axis0(p, f, out, out_kind, flag, s, ph, true);
  }
  if (p->N == 1) {
    double c1[4] = {c[0], react, 0, 0};
    return apply_pass(p, 0, {u, nullptr}, none, f, out, nullptr, out_kind, nullptr, nullptr, c1, nullptr,
                      flag, s);
  }
  const double cC[4] = {0, 1, 0, 0}, cA[4] = {1, 0, 0, 0};
  rc = apply_pass(p, p->N - 1, {u, nullptr}, none, nullptr, T[0], T[1], 2, T[2], T[3], cC, cA, flag, s);
  if (rc) return rc;
  p->phase = ph + 1;
  if (p->N == 2) {
    double c1[4] = {c[0], react, 0, c[1]};
    return apply_pass(p, 0, {T[0], T[1]}, {T[2], T[3]}, f, out, nullptr, out_kind, nullptr, nullptr, c1,
                      nullptr, flag, s);
  }
  double c4[4] = {c[1], react, 0, c[2]};
  rc = apply_pass(p, 1, {T[0], T[1]}, {T[2], T[3]}, nullptr, T[4], T[5], 2, T[6], T[7], cC, c4, flag, s);
  if (rc) return rc;
  return operator_apply_axis0(p, f, out, out_kind, flag, s, ph, true);
}

// out = F + scale C u with C = C_1 x ... x C_N (F may be null), in plain
// float64 (one right-hand side; no cancellation: the mass is positive
// definite and well conditioned, so float64 rounding of C u is at the level
// of the representation of F).
int mass_apply(fftfem_plan_t p, const double* u, const double* F, double* out, double scale, hipStream_t s) {
  double** T = p->tmp;
  const DDp none{nullptr, nullptr};
  const double cC[4] = {0, 1, 0, 0};
  // F - (-scale) C u, or scale C u without F
  const double last[4] = {0, F ? -scale : scale, 0, 0};
  int rc;
  p->phase = 0;
  if (p->N == 1)
    return apply_pass(p, 0, {u, nullptr}, none, F, out, nullptr, 1, nullptr, nullptr, last, nullptr, nullptr, s,
                      false);
  rc = apply_pass(p, p->N - 1, {u, nullptr}, none, nullptr, T[0], nullptr, 1, nullptr, nullptr, cC, nullptr,
                  nullptr, s, false);
  if (rc) return rc;
  if (p->N == 3) {
    rc = apply_pass(p, 1, {T[0], nullptr}, none, nullptr, T[4], nullptr, 1, nullptr, nullptr, cC, nullptr, nullptr,
                    s, false);
    if (rc) return rc;
    return apply_pass(p, 0, {T[4], nullptr}, none, F, out, nullptr, 1, nullptr, nullptr, last, nullptr, nullptr, s,
                      false);
  }
  return apply_pass(p, 0, {T[0], nullptr}, none, F, out, nullptr, 1, nullptr, nullptr, last, nullptr, nullptr, s,
                    false);
}

// r <- r - A c in plain float64 (N >= 2): the residual of u + c from the
// residual r of u, for a correction c that is small next to u (rounding of
// A c is then far below the refinement's target).  c is read from tmp[1];
// the passes write hi planes only (tmp[0], tmp[2]; in 3D also tmp[4], tmp[6]).
int operator_apply_incr(fftfem_plan_t p, double* r, const int* flag, hipStream_t s, int ph) {
  const double* c = p->coef;
  const double react = p->desc.react;
  double** T = p->tmp;
  const DDp none{nullptr, nullptr};
  const double cC[4] = {0, 1, 0, 0}, cA[4] = {1, 0, 0, 0};
  int rc;
  p->phase = ph;
  if (fused2d(p)) return resid2(p, T[1], nullptr, r, false, flag, s);
  if (fused3d(p)) {
    rc = resid3p(p, T[1], false, flag, s);
    if (rc) return rc;
    return operator_apply_axis0(p, r, r, 1, flag, s, ph, false);
  }
  rc = apply_pass(p, p->N - 1, {T[1], nullptr}, none, nullptr, T[0], nullptr, 1, T[2], nullptr, cC, cA, flag, s,
                  false);
  if (rc) return rc;
  p->phase = ph + 1;
  if (p->N == 2) {
    double c1[4] = {c[0], react, 0, c[1]};
    return apply_pass(p, 0, {T[0], nullptr}, {T[2], nullptr}, r, r, nullptr, 1, nullptr, nullptr, c1, nullptr,
                      flag, s, false);
  }
  double c4[4] = {c[1], react, 0, c[2]};
  rc = apply_pass(p, 1, {T[0], nullptr}, {T[2], nullptr}, nullptr, T[4], nullptr, 1, T[6], nullptr, cC, c4, flag,
                  s, false);
  if (rc) return rc;
  p->phase = ph + 2;
  double c1[4] = {c[0], 0, 0, 1};
  return apply_pass(p, 0, {T[4], nullptr}, {T[6], nullptr}, r, r, nullptr, 1, nullptr, nullptr, c1, nullptr, flag,
                    s, false);
}

// Forward on axes N-1..1, MID on axis 0, inverse on axes 1..N-1.
// work: T array used in place between passes (may equal out when T is double);
// work2: second T array for the transposed 2D schedule.
// mid64 (N = 1, T = float): run the single pass in float64.  Refinement
// residuals are dominated by the high-frequency rounding noise of the float32
// iterate (amplified by the stiffness); float32 transforms of them leak a
// fraction ~1e-7 of that noise into the lowest modes, which the division
// amplifies by up to cond(A).  In 1D the one float64 pass removes the leak.
// In 2D and 3D every forward pass before the division would have to run in
// float64 to the same end, at about the cost of a float64 solve, so those
// keep float32 and pay one more refinement step instead.
// Schedule positions (phase = ph + slot) of a chain's passes: 0 forward
// along axis N-1, N-1-d forward along axis d (0 < d < N-1), N-1 and N+1 the
// transposes around the middle pass N, N+1+d inverse along axis d.
constexpr int chain_slots(int N) { return 2 * N + 2; }

template <typename T>
int transform_chain(fftfem_plan_t p, const void* in, int in_f64, T* work, T* work2, double* out,
                    const double* upd, const int* flag, hipStream_t s, bool partials, bool mid64 = false,
                    int ph = 0) {
  int N = p->N, rc;
  p->phase = ph;
  if (N == 1) {
    if (mid64 && sizeof(T) == 4)
      return line_pass<double>(p, natural_geom(p, 0, true), MID, in, in_f64, out, 1, upd, flag, s, partials);
    return line_pass<T>(p, natural_geom(p, 0, true), MID, in, in_f64, out, 1, upd, flag, s, partials);
  }
  if (N == 2 && p->tr2d && p->trfused) {
    // No transposes: the forward pass along axis 1 stores the transposed
    // layout (M1 x M0) into work2, the middle pass reads it as contiguous
    // lines and stores back into the natural layout of `work`, and the
    // inverse pass runs on that in place (work == out when T is double).
    // Same schedule positions as the transposed schedule.
    Geom g1 = natural_geom(p, 1, true);
    g1.oes = p->M[0];
    rc = line_pass<T>(p, g1, FWD, in, in_f64, work2, 0, nullptr, flag, s, false);
    if (rc) return rc;
    Geom g;
    g.axis = 0;
    g.M = p->M[0];
    g.es = 1;
    g.nlines = p->M[1];
    g.nother = 1;
    g.oaxis[0] = 1;
    g.so[0] = p->M[0];
    g.Mo[0] = p->M[1];
    g.oes = p->M[1];
    p->phase = ph + N;
    rc = line_pass<T>(p, g, MID, work2, 0, work, 0, nullptr, flag, s, false);
    if (rc) return rc;
    p->phase = ph + 2 * N;
    return line_pass<T>(p, natural_geom(p, 1, true), INV, work, 0, out, 1, upd, flag, s, partials);
  }
  rc = line_pass<T>(p, natural_geom(p, N - 1, true), FWD, in, in_f64, work, 0, nullptr, flag, s, false);
  if (rc) return rc;
  for (int d = N - 2; d >= 1; --d) {
    p->phase = ph + N - 1 - d;
    rc = line_pass<T>(p, natural_geom(p, d, true), FWD, work, 0, work, 0, nullptr, flag, s, false);
    if (rc) return rc;
  }
  if (N == 2 && p->tr2d) {
    // axis 0 as contiguous lines of a transposed copy: (M0 x M1) -> (M1 x M0)
    p->phase = ph + N - 1;
    rc = transpose<T>(p, work, work2, p->M[0], p->M[1], s);
    if (rc) return rc;
    Geom g;
    g.axis = 0;
    g.M = p->M[0];
    g.es = 1;
    g.nlines = p->M[1];
    g.nother = 1;
    g.oaxis[0] = 1;
    g.so[0] = p->M[0];
    g.Mo[0] = p->M[1];
    p->phase = ph + N;
    rc = line_pass<T>(p, g, MID, work2, 0, work2, 0, nullptr, flag, s, false);
    if (rc) return rc;
    p->phase = ph + N + 1;
    rc = transpose<T>(p, work2, work, p->M[1], p->M[0], s);
    if (rc) return rc;
  } else {
    p->phase = ph + N;
    rc = line_pass<T>(p, natural_geom(p, 0, true), MID, work, 0, work, 0, nullptr, flag, s, false);
    if (rc) return rc;
  }
  for (int d = 1; d <= N - 2; ++d) {
    p->phase = ph + N + 1 + d;
    rc = line_pass<T>(p, natural_geom(p, d, true), INV, work, 0, work, 0, nullptr, flag, s, false);
    if (rc) return rc;
  }
  p->phase = ph + 2 * N;
  return line_pass<T>(p, natural_geom(p, N - 1, true), INV, work, 0, out, 1, upd, flag, s, partials);
}

// Mode of pass `pass` of the chain (0 .. 2N - 2): forward passes along axes
// N - 1 down to 1, the middle pass along axis 0, inverse passes along axes 1
// up to N - 1.
int chain_mode(const fftfem_plan_s* p, int pass) {
  return pass < p->N - 1 ? FWD : (pass == p->N - 1 ? MID : INV);
}

// Geometry of the tuner's passes, as the solve runs them.  2D: 0 forward
// along axis 1, 1 the middle pass along axis 0 (on the transposed copy when
// the solve uses one), 2 inverse along axis 1.
Geom tune_geom(fftfem_plan_t p, int pass) {
  if (p->N != 2) {
    const int N = p->N;
    const int axis = pass < N - 1 ? N - 1 - pass : (pass == N - 1 ? 0 : pass - N + 1);
    return natural_geom(p, axis, true);
  }
  if (pass != 1) {
    Geom g = natural_geom(p, p->N - 1, true);
    if (pass == 0 && p->trfused) g.oes = p->M[0];
    return g;
  }
  if (!p->tr2d) return natural_geom(p, 0, true);
  Geom g;
  g.axis = 0;
  g.M = p->M[0];
  g.es = 1;
  g.nlines = p->M[1];
  g.nother = 1;
  g.oaxis[0] = 1;
  g.so[0] = p->M[0];
  g.Mo[0] = p->M[1];
  if (p->trfused) g.oes = p->M[1];
  return g;
}

int64_t max_blocks_last_pass(const fftfem_plan_s* p, size_t elt) {
  int axis = p->N - 1;
  int64_t nlines = p->size / p->M[axis];
  int G = choose_G(p->nd[axis], p->K[axis], elt, nlines);
  return (nlines + G - 1) / G;
}

}  // namespace

extern "C" {

const char* fftfem_status_string(int st) {
  switch (st) {
    case FFTFEM_OK: return "ok";
    case FFTFEM_EINVAL: return "invalid argument";
    case FFTFEM_ENOMEM: return "out of memory";
    case FFTFEM_EHIP: return "HIP runtime error";
    case FFTFEM_ESPECTRUM: return "plan eigen-solve failed";
    case FFTFEM_EINDEF: return "operator not positive definite";
    case FFTFEM_ENOCONV: return "refinement did not converge";
    case FFTFEM_ENOTIMPL: return "configuration not supported";
    default: return "unknown status";
  }
}

void fftfem_destroy(fftfem_plan_t p) {
  if (!p) return;
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  for (void* a : p->allocs) (void)hipFree(a);
  delete p;
}

int fftfem_plan_ex(fftfem_plan_t* out, const fftfem_desc* din) { return plan_create(out, din, nullptr); }

}  // extern "C"

int fftfem::plan_create(fftfem_plan_t* out, const fftfem_desc* din, TableCache* cache) {
  if (!out) return FFTFEM_EINVAL;
  *out = nullptr;
  int rc = validate(din);
  if (rc) return rc;
  fftfem_desc d = *din;
  if (d.max_iter == 0) d.max_iter = 3;
  if (d.tol == 0) d.tol = 1e-12;
  if (d.nrhs == 0) d.nrhs = 1;
  for (int i = 0; i < d.N; ++i)
    if (d.X[i] == 0) d.X[i] = 1.0;
  for (int i = 0; i < d.N; ++i)
    if (d.n_axis[i] == 0) d.n_axis[i] = d.n;
  for (int i = 0; i < d.N; ++i)
    if (d.n_axis[i] > kMaxLineOrder) return FFTFEM_ENOTIMPL;
  const bool algb = (d.flags & FFTFEM_ALGORITHM_B) != 0;
  // a line-kernel tile holds at most kLineTasks element tasks; longer lines
  // take the multi-pass transforms: one axis, or two axes of which one or
  // both are longer than a tile (the other by the line passes), K up to
  // kLongMaxK, float64, algorithm (a), not in batches
  bool longK = false;
  {
    int nlong = 0;
    for (int i = 0; i < d.N; ++i) nlong += d.K[i] > kLineTasks ? 1 : 0;
    if (nlong > 0) {
      bool ok = d.N <= 2 && d.precision == FFTFEM_FP64 && !algb && !cache;
      for (int i = 0; i < d.N; ++i) ok = ok && d.K[i] <= kLongMaxK;
      if (!ok) return FFTFEM_ENOTIMPL;
      longK = true;
    }
  }
  if (algb && (d.precision != FFTFEM_FP64 || cache)) return FFTFEM_ENOTIMPL;
  fftfem_plan_s* p = new (std::nothrow) fftfem_plan_s();
  if (!p) return FFTFEM_ENOMEM;
  p->desc = d;
  p->algb = algb;
  p->longK = longK;
  p->N = d.N;
  p->n = d.n;
  p->nrhs = d.nrhs;
  p->size = 1;
  for (int i = 0; i < d.N; ++i) {
    p->nd[i] = d.n_axis[i];
    p->K[i] = d.K[i];
    p->M[i] = (int64_t)p->nd[i] * d.K[i] - 1;
    p->size *= p->M[i];
  }
  for (int i = 0; i < d.N; ++i) {
    p->stride[i] = 1;
    for (int e = i + 1; e < d.N; ++e) p->stride[i] *= p->M[e];
  }
  // tables (identical axes are computed once)
  p->host.resize(d.N);
  std::map<std::pair<int, int64_t>, int> seen;
  for (int i = 0; i < d.N; ++i) {
    const std::pair<int, int64_t> key{p->nd[i], d.K[i]};
    auto it = seen.find(key);
    if (it != seen.end()) {
      p->host[i] = p->host[it->second];
    } else if (cache && cache->get(p->nd[i], d.K[i], &p->host[i])) {
      seen[key] = i;
    } else {
      rc = build_axis_tables(p->nd[i], d.K[i], 1.0, 1.0, &p->host[i]);
      if (rc) {
        delete p;
        return rc;
      }
      if (cache) cache->put(p->nd[i], d.K[i], p->host[i]);
      seen[key] = i;
    }
    p->coef[i] = d.diff[i] * 4.0 * ((double)d.K[i] / d.X[i]) * ((double)d.K[i] / d.X[i]);
    p->host[i].coef = p->coef[i];
  }
  double dmin = d.react;
  for (int i = 0; i < d.N; ++i) {
    double m = p->host[i].lam[0];
    for (double v : p->host[i].lam) m = std::min(m, v);
    dmin += p->coef[i] * m;
  }
  if (!(dmin > 0)) {
    delete p;
    return FFTFEM_EINDEF;
  }
  int dev = 0;
  if ((rc = from_hip(hipGetDevice(&dev)))) {
    delete p;
    return rc;
  }
  int lmax = 0;
  if (hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
      lmax > 0)
    p->lds_max = lmax;
  // device tables
  for (int i = 0; i < d.N && !rc; ++i) {
    const AxisTables& t = p->host[i];
    std::vector<double> mu(t.lam.size());
    for (size_t c = 0; c < mu.size(); ++c) mu[c] = p->coef[i] * t.lam[c];
    // Q in structure-of-arrays order for the kernels: (c, l, k) -> (c n + l) K + k
    const int n = p->nd[i];
    std::vector<double> qs(t.Q.size());
    for (int64_t k = 0; k < t.K; ++k)
      for (int c = 0; c < n; ++c)
        for (int l = 0; l < n; ++l)
          qs[(size_t)(c * n + l) * t.K + k] = t.Q[(size_t)k * n * n + c * n + l];
    // condensed-solve constants with the stiffness parts scaled like mu
    std::vector<double> arrow = t.arrow;
    const ArrowLayout al(n);
    for (int m = 0; m < al.nb; ++m) {
      arrow[al.nu + m] *= p->coef[i];
      arrow[al.gA + m] *= p->coef[i];
    }
    const std::vector<double>* src[kNumTables] = {&qs,     &t.twf,  &t.twm, &t.twd, &mu,
                                                  &t.chirp, &t.bhat, &t.twl, &arrow, &t.band};
    for (int w = 0; w < kNumTables && !rc; ++w) {
      if (src[w]->empty()) continue;
      rc = upload<double>(p, &p->dev[i].d[w], *src[w]);
      if (!rc) rc = upload<float>(p, &p->dev[i].f[w], *src[w]);
    }
  }
  for (int i = 0; i < d.N && !rc; ++i) {
    std::vector<double> A, C;
    element_matrices_dd(p->nd[i], &A, &C);
    rc = upload<double>(p, &p->Ael[i], A);
    if (!rc) rc = upload<double>(p, &p->Cel[i], C);
  }
  // workspace
  size_t elt = d.precision == FFTFEM_FP64 ? sizeof(double) : sizeof(float);
  if (d.N == 2) {
    int G0 = choose_G(p->nd[0], p->K[0], elt, p->size / p->M[0]);
    p->tr2d = (size_t)G0 * elt < 64 && !p->longK;  // long-line plans take no line passes
    // float64: the axis-1 passes store and load the transposed layout
    // themselves (measured at n = 9, K = 1024: 3.38 ms against 3.54 ms with
    // the two transposes); float32: the transposes are cheaper (4-byte values)
    p->trfused = p->tr2d && d.precision == FFTFEM_FP64;
  }
  if (!rc && d.precision != FFTFEM_FP64)
    rc = dev_alloc(p, (void**)&p->W32, (size_t)p->size * sizeof(float));
  if (!rc && p->tr2d && d.precision != FFTFEM_FP64)
    rc = dev_alloc(p, (void**)&p->W32b, (size_t)p->size * sizeof(float));
  if (!rc && d.precision == FFTFEM_FP32_REFINE)
    rc = dev_alloc(p, (void**)&p->W64r, (size_t)p->size * sizeof(double));
  if (!rc && p->algb) {
    // short lines: the LDS-tiled kernel (y read once, x written once);
    // otherwise one thread per line, which fills the chip from about 64K
    // lines (256 CUs, 4 waves each), below that the element-parallel
    // three-kernel form.  FFTFEM_BAND_FORM (0, 1, 2) overrides the choice
    // where the form applies.
    const int64_t nl = p->size / p->M[0];
    const bool tile_ok = band_tile_lines((int)p->K[0]) > 0;
    p->band_form = tile_ok ? 2 : (nl < 65536 ? 1 : 0);
    if (const char* e = std::getenv("FFTFEM_BAND_FORM")) {
      const int f = std::atoi(e);
      if (f == 0 || f == 1 || (f == 2 && tile_ok)) p->band_form = f;
    }
    const size_t nodes = (size_t)std::max<int64_t>(1, p->K[0] - 1) * (size_t)nl;
    if (p->band_form == 0) rc = dev_alloc(p, (void**)&p->Wband, nodes * sizeof(double));
    if (p->band_form == 1)
      rc = dev_alloc(p, (void**)&p->Wband, ((size_t)((p->size + 1) & ~int64_t(1)) + 2 * nodes) * sizeof(double));
  }
  if (!rc && p->tr2d && d.precision == FFTFEM_FP64)
    rc = dev_alloc(p, (void**)&p->W64b, (size_t)p->size * sizeof(double));
  if (!rc && p->longK) {
    // per axis: the DFT length D (K, or Bluestein's L) and the twiddles of
    // the four-step passes (every (D/K_i)-th entry of the length-D table for
    // the sub-DFTs, its first 1024 entries and every 1024th for the
    // products); work arrays of D slots per buffer for long_chunk lines:
    // all the lines an axis transforms at once when that takes at most
    // kLongWorkBytes per array, else chunks of lines (FFTFEM_LONG_CHUNK sets
    // a smaller chunk)
    size_t per = 0;
    int64_t lines_max = 1;
    for (int ax = 0; ax < p->N && !rc; ++ax) {
      if (p->K[ax] <= kLineTasks) continue;  // a short axis of a two-axis plan: line passes
      const AxisTables& t = p->host[ax];
      auto& la = p->lax[ax];
      const bool pow2 = is_pow2(p->K[ax]);
      const int64_t D = pow2 ? p->K[ax] : t.L;
      const std::vector<double>& twD = pow2 ? t.twf : t.twl;
      const int lk = ilog2(D);
      la.lk1 = lk / 2;
      la.lk2 = lk - la.lk1;
      la.D = D;
      long_tiles(la.lk1, la.lk2, &la.lgc, &la.lgr);
      const int64_t lines = p->N == 1 ? p->nrhs : p->M[1 - ax];
      lines_max = std::max(lines_max, lines);
      per = std::max(per, (size_t)(1 + p->nd[ax] / 2) * 2 * (size_t)D);
      const int64_t len[4] = {int64_t(1) << la.lk1, int64_t(1) << la.lk2, 1024, D / 1024};
      const int64_t st[4] = {D / len[0], D / len[1], 1, 1024};
      for (int i = 0; i < 4 && !rc; ++i) {
        std::vector<double> tw((size_t)2 * len[i]);
        for (int64_t q = 0; q < len[i]; ++q) {
          tw[2 * q] = twD[2 * q * st[i]];
          tw[2 * q + 1] = twD[2 * q * st[i] + 1];
        }
        rc = upload<double>(p, &la.tw[i], tw);
      }
    }
    int64_t chunk = std::max<int64_t>(1, (int64_t)(kLongWorkBytes / (per * sizeof(double))));
    if (const char* e = std::getenv("FFTFEM_LONG_CHUNK")) {
      const long long v = std::atoll(e);
      if (v > 0) chunk = std::min<int64_t>(chunk, v);
    }
    p->long_chunk = std::min(chunk, lines_max);
    for (int i = 0; i < 2 && !rc; ++i)
      rc = dev_alloc(p, (void**)&p->Wl[i], (size_t)p->long_chunk * per * sizeof(double));
  }
  // full-size scratch: the operator passes' planes (2D: four, 3D: eight);
  // a two-axis long-line plan with one order uses only the first (the
  // transposed copy; its operator apply is the fused pass)
  p->ntmp = d.N == 1 ? 0 : (d.N == 2 ? (p->longK && p->nd[0] == p->nd[1] ? 1 : 4) : 8);
  for (int i = 0; i < p->ntmp && !rc; ++i)
    rc = dev_alloc(p, (void**)&p->tmp[i], (size_t)p->size * sizeof(double));
  if (!rc) {
    // one tile per line at most (tuned or forced lines per tile may be 1)
    p->npartials = (int)(p->size / p->M[d.N - 1]);
    rc = dev_alloc(p, (void**)&p->partials, (size_t)p->npartials * 2 * sizeof(double));
  }
  if (!rc) rc = dev_alloc(p, (void**)&p->flags, (size_t)p->nrhs * sizeof(int));
  if (!rc) rc = dev_alloc(p, (void**)&p->stats, (size_t)p->nrhs * kStatsLen * sizeof(double));
  if (!rc) {
    rc = from_hip(launch_reset_many(p->flags, p->stats, kStatsLen, p->nrhs, nullptr));
    if (!rc) rc = from_hip(hipDeviceSynchronize());
  }
  if (rc) {
    fftfem_destroy(p);
    return rc;
  }
  *out = p;
  return FFTFEM_OK;
}

extern "C" {

int fftfem_plan(fftfem_plan_t* out, int N, const int64_t* K, int n, const double* diff,
                double react) {
  if (!out) return FFTFEM_EINVAL;
  *out = nullptr;
  if (!K || !diff || N < 1 || N > FFTFEM_MAX_DIMS) return FFTFEM_EINVAL;
  fftfem_desc d{};
  d.N = N;
  d.n = n;
  d.react = react;
  for (int i = 0; i < N; ++i) {
    d.K[i] = K[i];
    d.diff[i] = diff[i];
  }
  d.precision = FFTFEM_FP64;
  return fftfem_plan_ex(out, &d);
}

static bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

// [a, a + na) and [b, b + nb) intersect
static bool overlap2(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

// Algorithm (b) of Sect. 4: FC_n transforms along axes N - 1 .. 1 (natural
// layout, f into u), the banded solve along axis 0 in place, the inverse
// transforms along axes 1 .. N - 1.
static int band_chain(fftfem_plan_t p, const double* f, double* u, hipStream_t s) {
  const int N = p->N;
  int rc = FFTFEM_OK;
  const double* src = f;
  for (int d = N - 1; d >= 1 && !rc; --d) {
    rc = line_pass<double>(p, natural_geom(p, d, false), FWD, src, 1, u, 1, nullptr, nullptr, s, false);
    src = u;
  }
  if (rc) return rc;
  const Geom g = natural_geom(p, 0, true);
  BandArgs a{};
  a.in = src;
  a.out = u;
  a.cp = p->Wband;
  a.pr = p->band_form == 1 ? p->Wband + ((p->size + 1) & ~int64_t(1)) : nullptr;  // 16-byte aligned pairs
  a.tab = p->dev[0].d[9];
  a.coef = p->coef[0];
  a.react = p->desc.react;
  a.K = (int)p->K[0];
  a.nlines = g.nlines;
  a.nother = g.nother;
  for (int e = 0; e < g.nother; ++e) {
    a.mu_o[e] = tab<double>(p, g.oaxis[e], 4);
    a.so[e] = g.so[e];
    a.Mo[e] = g.Mo[e];
  }
  if (p->band_form == 1) {
    static const char* names[3] = {"bandcond64_ax0", "bandnodes64_ax0", "bandback64_ax0"};
    for (int step = 0; step < 3 && !rc; ++step) {
      Timed tm(p, s, names[step]);
      rc = from_hip(launch_band_split(p->nd[0], step, a, s));
    }
  } else if (p->band_form == 2) {
    Timed tm(p, s, "bandtile64_ax0");
    rc = from_hip(launch_band_tile(p->nd[0], a, s));
  } else {
    Timed tm(p, s, "band64_ax0");
    rc = from_hip(launch_band(p->nd[0], a, s));
  }
  for (int d = 1; d < N && !rc; ++d)
    rc = line_pass<double>(p, natural_geom(p, d, false), INV, u, 1, u, 1, nullptr, nullptr, s, false);
  return rc;
}

// The FC_n transform (FWD: lines -> spectral coefficients), its inverse
// (INV) or both with the division by react + the axis' denominators (+
// mu_line[l] per line) in between (MID) of nlines consecutive lines along
// `axis` of a long-line plan, by the multi-pass kernels of long.hip.  The
// K-point DFTs of the channel buffers: K a power of two, a column and a row
// pass (wa -> wb); otherwise Bluestein's four passes (wa -> wb -> wa) with
// the chirp factors of the direction (conjugated for the inverse DFT).
// NaN / Inf written by the scatter sets bit 2 of bad[l / lpf].
static int long_transform(fftfem_plan_t p, int axis, int mode, const double* in, double* out, int64_t nlines,
                          hipStream_t s, int* bad = nullptr, int64_t lpf = 1, const double* mu_line = nullptr) {
  const auto& la = p->lax[axis];
  LongArgs a{};
  a.lpf = lpf;
  a.K = (int)p->K[axis];
  a.ls = (int)la.D;
  a.lk1 = la.lk1;
  a.lk2 = la.lk2;
  a.K1 = 1 << la.lk1;
  a.K2 = 1 << la.lk2;
  a.M = p->M[axis];
  a.Q = tab<double>(p, axis, 0);
  a.twm = tab<double>(p, axis, 2);
  a.twd = tab<double>(p, axis, 3);
  a.mu = tab<double>(p, axis, 4);
  a.chirp = tab<double>(p, axis, 5);
  a.bhat = tab<double>(p, axis, 6);
  a.tw1 = la.tw[0];
  a.tw2 = la.tw[1];
  a.twlo = la.tw[2];
  a.twhi = la.tw[3];
  a.lgc = la.lgc;
  a.lgr = la.lgr;
  a.react = p->desc.react;
  double* const W0 = p->Wl[0];
  double* const W1 = p->Wl[1];
  const bool pow2 = is_pow2(p->K[axis]);
  const int n = p->nd[axis];
  const std::string ax = "_ax" + std::to_string(axis);
  int rc = FFTFEM_OK;
  auto step = [&](int st, bool inv, double* w, double* o, const char* name) {
    if (rc) return;
    Timed tm(p, s, p->N == 1 ? std::string(name) : name + ax);
    rc = from_hip(launch_long(n, st, inv, a, w, o, s));
  };
  // DFTs of the buffers of W0 (forward or inverse); returns the array that
  // holds the spectra
  auto dft = [&](bool inv) -> double* {
    if (pow2) {
      step(LONG_COLS, inv, W0, nullptr, inv ? "lcols64i" : "lcols64");
      step(LONG_ROWS, inv, W0, W1, inv ? "lrows64i" : "lrows64");
      return W1;
    }
    a.pre = inv ? 2 : 1;
    step(LONG_COLS, false, W0, nullptr, inv ? "lbcols64i" : "lbcols64");
    a.pre = 0;
    step(LONG_ROWS, false, W0, W1, inv ? "lbrows64i" : "lbrows64");
    a.pre = inv ? 4 : 3;
    step(LONG_COLS, true, W1, nullptr, inv ? "lbcols64ic" : "lbcols64c");
    a.pre = 0;
    a.post = inv ? 2 : 1;
    step(LONG_ROWS, true, W1, W0, inv ? "lbrows64ic" : "lbrows64c");
    a.post = 0;
    return W0;
  };
  // the lines in chunks of at most long_chunk (the work arrays' size); the
  // non-finite flag of line l is bad[l / lpf], so a chunk boundary must not
  // split the lines of one flag unless all lines share one
  const int64_t chunk = p->long_chunk;
  if (bad && lpf > 1 && lpf < nlines && chunk % lpf) return FFTFEM_EINVAL;
  for (int64_t c0 = 0; c0 < nlines && !rc; c0 += chunk) {
    const int64_t nl = std::min(chunk, nlines - c0);
    const double* cin = in + c0 * a.M;
    double* cout = out + c0 * a.M;
    a.nlines = nl;
    a.bad = bad ? bad + (lpf >= nlines ? 0 : c0 / lpf) : nullptr;
    a.mu_line = mu_line ? mu_line + c0 : nullptr;
    // lines per contraction thread: enough threads to fill the chip (about
    // 2^18), the rest of the lines in a loop that reuses the cached Q rows
    a.lpt = (int)std::max<int64_t>(1, std::min<int64_t>(nl, nl * ((a.K + 1) / 2) >> 18));
    if (mode == FWD || mode == MID) {
      a.in = cin;
      a.out = cout;
      a.wa = W0;
      step(LONG_GATHER, false, nullptr, nullptr, "lgather64");
      a.wb = dft(false);
      step(LONG_CONTRACT_FWD, false, nullptr, nullptr, "lcfwd64");
    }
    if (mode == MID) {
      a.in = cout;
      a.out = cout;
      step(LONG_DIVIDE, false, nullptr, nullptr, "ldiv64");
    }
    if (mode == INV || mode == MID) {
      a.in = mode == INV ? cin : cout;
      a.out = cout;
      a.wa = W0;
      step(LONG_CONTRACT_INV, false, nullptr, nullptr, "lcinv64");
      a.wb = dft(true);
      step(LONG_SCATTER, false, nullptr, nullptr, "lscatter64");
    }
  }
  return rc;
}

// The rows (axis 1) of one right-hand side of a two-axis long-line plan:
// the multi-pass transforms when axis 1 is long, else one line pass.  NaN /
// Inf written by the pass sets bit 2 of *bad (when given).
static int rows_2d(fftfem_plan_t p, int mode, const double* in, double* out, hipStream_t s, int* bad = nullptr) {
  if (p->K[1] > kLineTasks) return long_transform(p, 1, mode, in, out, p->M[0], s, bad, p->M[0]);
  int* keep = p->bad;
  p->bad = bad;
  const int rc = line_pass<double>(p, natural_geom(p, 1, false), mode, in, 1, out, 1, nullptr, nullptr, s, false);
  p->bad = keep;
  return rc;
}

// The last axis of a long-line plan for every right-hand side: one call for
// one axis (the lines are the right-hand sides), one per right-hand side for
// two (the work arrays hold one right-hand side's M0 rows).
static int long_last_axis(fftfem_plan_t p, int mode, const double* in, double* out, hipStream_t s) {
  if (p->N == 1) return long_transform(p, 0, mode, in, out, p->nrhs, s);
  int rc = FFTFEM_OK;
  for (int r = 0; r < p->nrhs && !rc; ++r)
    rc = rows_2d(p, mode, in + (size_t)r * p->size, out + (size_t)r * p->size, s);
  return rc;
}

// Axis 0 of a two-axis long-line plan, one right-hand side: in (M0 x M1) is
// transposed into the plan's scratch, its M1 contiguous lines transformed
// there (mode as long_transform; the multi-pass transforms when axis 0 is
// long, else one line pass, whose MID step takes the axis-1 denominator of
// line l from axis 1's table, as mu_line does), and transposed back into out
// (which may be in).
static int long_axis0_2d(fftfem_plan_t p, int mode, const double* in, double* out, hipStream_t s,
                         const double* mu_line = nullptr) {
  double* T = p->tmp[0];
  const int64_t M0 = p->M[0], M1 = p->M[1];
  int rc = from_hip(launch_transpose<double>(in, T, 1, M0, M1, s));
  if (!rc) {
    if (p->K[0] > kLineTasks) {
      rc = long_transform(p, 0, mode, T, T, M1, s, nullptr, 1, mu_line);
    } else {
      Geom g;
      g.axis = 0;
      g.M = M0;
      g.es = 1;
      g.nlines = M1;
      if (mu_line) {
        g.nother = 1;
        g.oaxis[0] = 1;
        g.so[0] = M0;  // line l starts at l M0: other-axis index (l M0 / M0) mod M1 = l
        g.Mo[0] = M1;
      }
      rc = line_pass<double>(p, g, mode, T, 1, T, 1, nullptr, nullptr, s, false);
    }
  }
  if (!rc) rc = from_hip(launch_transpose<double>(T, out, 1, M1, M0, s));
  return rc;
}

int fftfem_solve(fftfem_plan_t p, const double* f, double* u, hipStream_t s) {
  if (!p || !f || !u) return FFTFEM_EINVAL;
  size_t bytes = (size_t)p->size * p->nrhs * sizeof(double);
  if (overlap(f, u, bytes)) return FFTFEM_EINVAL;
  p->last = s;
  int rc = FFTFEM_OK;
  if (p->longK) {
    // float64, no refinement: reset the statistics; one axis: every
    // right-hand side at once; two axes: per right-hand side, forward along
    // axis 1 (rows), the middle step along axis 0 on the transposed array
    // with the axis-1 denominators per line, the inverse along axis 1
    rc = from_hip(launch_reset_many(p->flags, p->stats, kStatsLen, p->nrhs, s));
    if (p->N == 1) {
      if (!rc) rc = long_transform(p, 0, MID, f, u, p->nrhs, s, p->flags);
      return rc;
    }
    for (int r = 0; r < p->nrhs && !rc; ++r) {
      const double* fr = f + (size_t)r * p->size;
      double* ur = u + (size_t)r * p->size;
      rc = rows_2d(p, FWD, fr, ur, s);
      if (!rc) rc = long_axis0_2d(p, MID, ur, ur, s, tab<double>(p, 1, 4));
      if (!rc) rc = rows_2d(p, INV, ur, ur, s, p->flags + r);
    }
    return rc;
  }
  for (int r = 0; r < p->nrhs && !rc; ++r) {
    const double* fr = f + (size_t)r * p->size;
    double* ur = u + (size_t)r * p->size;
    int* flag = p->flags + r;
    double* st = p->stats + (size_t)r * kStatsLen;
    // schedule positions: reset, the chain, then per refinement step the
    // operator passes, the chain and the convergence test (right-hand sides
    // in sequence: they share the workspace)
    const int N = p->N, SC = chain_slots(N), per_it = N + SC + 1;
    const int base = r * (1 + SC + p->desc.max_iter * per_it);
    p->phase = base;
    if (p->rec) {
      ResetJob j{flag, st, kStatsLen};
      record(p, REC_RESET, {}, j, 1, 0);
    } else {
      rc = from_hip(launch_reset(flag, st, kStatsLen, s));
    }
    if (rc) break;
    // the chains' output passes report NaN / Inf in u through the flag
    p->bad = flag;
    if (p->algb) {
      rc = band_chain(p, fr, ur, s);
      p->bad = nullptr;
      continue;
    }
    if (p->desc.precision == FFTFEM_FP64) {
      rc = transform_chain<double>(p, fr, 1, ur, p->W64b, ur, nullptr, nullptr, s, false, false, base + 1);
      p->bad = nullptr;
      continue;
    }
    rc = transform_chain<float>(p, fr, 1, p->W32, p->W32b, ur, nullptr, nullptr, s, false, false, base + 1);
    p->bad = nullptr;
    if (rc || p->desc.precision == FFTFEM_FP32) continue;
    for (int it = 1; it <= p->desc.max_iter && !rc; ++it) {
      const int pit = base + 1 + SC + (it - 1) * per_it;
      const bool one = N == 1;
      if (one) {
        // 1D: double-double residual every step, float64 chain
        rc = operator_apply(p, ur, fr, p->W64r, 1, flag, s, pit);
        if (!rc)
          rc = transform_chain<float>(p, p->W64r, 1, p->W32, p->W32b, ur, ur, flag, s, true, true, pit + N);
      } else {
        // first step: the double-double residual f - A u (float64); later
        // steps: r - A c in float64 with the stored correction c
        rc = it == 1 ? operator_apply(p, ur, fr, p->W64r, 1, flag, s, pit)
                     : operator_apply_incr(p, p->W64r, flag, s, pit);
        p->cor = p->tmp[1];
        if (!rc)
          rc = transform_chain<float>(p, p->W64r, 1, p->W32, p->W32b, ur, ur, flag, s, true, false, pit + N);
        p->cor = nullptr;
      }
      if (rc) break;
      p->phase = pit + N + SC;
      if (p->rec) {
        ReduceJob j{p->partials, p->nparts_last, it, p->desc.tol, flag, st};
        record(p, REC_REDUCE, {}, j, 1, 0);
      } else {
        rc = from_hip(launch_reduce(p->partials, p->nparts_last, it, p->desc.tol, flag, st, s));
      }
    }
  }
  return rc;
}

int fftfem_implicit_euler(fftfem_plan_t p, const double* F, double* u, double* work, int nsteps, hipStream_t s) {
  if (!p || !u || !work || nsteps < 0) return FFTFEM_EINVAL;
  if (!(p->desc.react > 0) || p->rec) return FFTFEM_EINVAL;
  const size_t bytes = (size_t)p->size * p->nrhs * sizeof(double);
  if (overlap(u, work, bytes) || (F && (overlap(F, work, bytes) || overlap(F, u, bytes)))) return FFTFEM_EINVAL;
  const double react = p->desc.react;
  int rc = FFTFEM_OK;
  for (int m = 0; m < nsteps && !rc; ++m) {
    for (int r = 0; r < p->nrhs && !rc; ++r) {
      const size_t o = (size_t)r * p->size;
      rc = mass_apply(p, u + o, F ? F + o : nullptr, work + o, react, s);
    }
    if (!rc) rc = fftfem_solve(p, work, u, s);
  }
  return rc;
}

int fftfem_apply_A(fftfem_plan_t p, const double* u, double* y, hipStream_t s) {
  if (!p || !u || !y) return FFTFEM_EINVAL;
  size_t bytes = (size_t)p->size * p->nrhs * sizeof(double);
  if (overlap(u, y, bytes)) return FFTFEM_EINVAL;
  p->last = s;
  int rc = FFTFEM_OK;
  for (int r = 0; r < p->nrhs && !rc; ++r)
    rc = operator_apply(p, u + (size_t)r * p->size, nullptr, y + (size_t)r * p->size, 1, nullptr, s);
  return rc;
}

int fftfem_get_stats(fftfem_plan_t p, fftfem_stats* out) {
  if (!p || !out) return FFTFEM_EINVAL;
  int rc = from_hip(hipStreamSynchronize(p->last));
  if (rc) return rc;
  std::vector<double> h((size_t)p->nrhs * kStatsLen);
  rc = from_hip(hipMemcpy(h.data(), p->stats, h.size() * sizeof(double), hipMemcpyDeviceToHost));
  if (rc) return rc;
  std::vector<int> fl((size_t)p->nrhs);
  rc = from_hip(hipMemcpy(fl.data(), p->flags, fl.size() * sizeof(int), hipMemcpyDeviceToHost));
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  // stop reasons ranked from best to worst; the worst right-hand side counts
  auto rank = [](int stop) {
    switch (stop) {
      case FFTFEM_STOP_NONE: return 0;
      case FFTFEM_STOP_TOL: return 1;
      case FFTFEM_STOP_MAX_ITER: return 2;
      case FFTFEM_STOP_STALLED: return 3;
      default: return 4;
    }
  };
  const bool refine = p->desc.precision == FFTFEM_FP32_REFINE && !p->algb;
  for (int r = 0; r < p->nrhs; ++r) {
    const double* st = &h[(size_t)r * kStatsLen];
    out->iterations = std::max(out->iterations, (int)st[0]);
    int stop = FFTFEM_STOP_NONE;
    if (fl[r] & 2)
      stop = FFTFEM_STOP_NONFINITE;  // an output pass wrote NaN or Inf
    else if (refine)
      stop = st[1] == 1    ? FFTFEM_STOP_TOL
             : st[1] == -1 ? FFTFEM_STOP_NONFINITE
             : st[1] == -2 ? FFTFEM_STOP_STALLED
                           : FFTFEM_STOP_MAX_ITER;
    if (rank(stop) > rank(out->stop)) out->stop = stop;
    for (int i = 0; i <= FFTFEM_MAX_ITERS; ++i) {
      const double v = st[2 + i];
      double& o = out->rel_correction[i];
      if (std::isnan(v) || std::isnan(o))
        o = std::numeric_limits<double>::quiet_NaN();
      else
        o = std::max(o, v);
    }
  }
  out->converged = out->stop == FFTFEM_STOP_NONE || out->stop == FFTFEM_STOP_TOL;
  return out->converged ? FFTFEM_OK : FFTFEM_ENOCONV;
}

size_t fftfem_workspace_bytes(const fftfem_plan_t p) { return p ? p->bytes : 0; }

int fftfem_set_timing(fftfem_plan_t p, int enable) {
  if (!p) return FFTFEM_EINVAL;
  p->timing = enable != 0;
  return FFTFEM_OK;
}

int fftfem_get_timing(fftfem_plan_t p, int max, char* names, double* avg_ms, int* count) {
  if (!p || max < 0 || (max > 0 && (!names || !avg_ms || !count))) return FFTFEM_EINVAL;
  int rc = from_hip(hipDeviceSynchronize());
  if (rc) return rc;
  std::vector<double> sum(p->names.size(), 0.0);
  std::vector<int> cnt(p->names.size(), 0);
  for (const auto& m : p->marks) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess) return FFTFEM_EHIP;
    sum[m.name] += ms;
    cnt[m.name] += 1;
  }
  int nk = (int)p->names.size();
  for (int i = 0; i < nk && i < max; ++i) {
    std::memset(names + 32 * i, 0, 32);
    std::strncpy(names + 32 * i, p->names[i].c_str(), 31);
    avg_ms[i] = cnt[i] ? sum[i] / cnt[i] : 0.0;
    count[i] = cnt[i];
  }
  p->marks.clear();
  p->names.clear();
  p->pool_used = 0;
  return nk;
}

int fftfem_plan_tables(const fftfem_plan_t p, int axis, double* lam, double* Q) {
  if (!p || axis < 0 || axis >= p->N || !lam) return FFTFEM_EINVAL;
  const AxisTables& t = p->host[axis];
  std::memcpy(lam, t.lam.data(), t.lam.size() * sizeof(double));
  if (Q) std::memcpy(Q, t.Q.data(), t.Q.size() * sizeof(double));
  return FFTFEM_OK;
}

int fftfem_axis_tables_host(int n, int64_t K, double* lam, double* Q) {
  if (!lam || n < 1 || n > FFTFEM_MAX_ORDER || K < 2) return FFTFEM_EINVAL;
  AxisTables t;
  int rc = build_axis_tables(n, K, 1.0, 1.0, &t);
  if (rc) return rc;
  std::memcpy(lam, t.lam.data(), t.lam.size() * sizeof(double));
  if (Q) std::memcpy(Q, t.Q.data(), t.Q.size() * sizeof(double));
  return FFTFEM_OK;
}

int fftfem_element_matrices_host(int n, double* A, double* C) {
  if (!A || !C || n < 1 || n > FFTFEM_MAX_ORDER) return FFTFEM_EINVAL;
  std::vector<double> a, c;
  element_matrices(n, &a, &c);
  std::memcpy(A, a.data(), a.size() * sizeof(double));
  std::memcpy(C, c.data(), c.size() * sizeof(double));
  return FFTFEM_OK;
}

int fftfem_coefficients(fftfem_plan_t p, const double* in, double* out, int kind, hipStream_t s) {
  if (!p || !in || !out || (kind != 0 && kind != 1) || p->rec) return FFTFEM_EINVAL;
  const size_t bytes = (size_t)p->size * p->nrhs * sizeof(double);
  if (in != out && overlap(in, out, bytes)) return FFTFEM_EINVAL;
  if (kind == 0 && in == out) return FFTFEM_EINVAL;
  p->last = s;
  int rc = FFTFEM_OK;
  if (p->longK) {
    // long lines: the rows of every right-hand side along the last axis,
    // then (two axes) axis 0 per right-hand side
    for (int r = 0; r < p->nrhs && !rc && kind == 0; ++r)
      rc = mass_apply(p, in + (size_t)r * p->size, nullptr, out + (size_t)r * p->size, 1.0, s);
    if (!rc) rc = long_last_axis(p, FWD, kind == 0 ? out : in, out, s);
    for (int r = 0; r < p->nrhs && !rc && p->N == 2; ++r)
      rc = long_axis0_2d(p, FWD, out + (size_t)r * p->size, out + (size_t)r * p->size, s);
    return rc;
  }
  for (int r = 0; r < p->nrhs && !rc; ++r) {
    const size_t o = (size_t)r * p->size;
    const double* src = in + o;
    if (kind == 0) {
      // values: the loads C w first (Theorem 2, item 3)
      rc = mass_apply(p, in + o, nullptr, out + o, 1.0, s);
      src = out + o;
    }
    for (int d = p->N - 1; d >= 0 && !rc; --d) {
      rc = line_pass<double>(p, natural_geom(p, d, false), FWD, src, 1, out + o, 1, nullptr, nullptr, s, false);
      src = out + o;
    }
  }
  return rc;
}

// Extended size (prod_d (M_d + 2)) of one right-hand side of the Dirichlet data.
static int64_t dirichlet_extended_size(fftfem_plan_t p) {
  int64_t esize = 1;
  for (int d = 0; d < p->N; ++d) esize *= p->M[d] + 2;
  return esize;
}

static int dirichlet_load_impl(fftfem_plan_t p, const double* b, const double* f, double* out, double* work,
                               hipStream_t s);

int fftfem_dirichlet_load(fftfem_plan_t p, const double* b, const double* f, double* out, double* work,
                          hipStream_t s) {
  if (!p || !b || !f || !out || !work || p->rec) return FFTFEM_EINVAL;
  const int64_t esize = dirichlet_extended_size(p);
  const size_t ib = (size_t)p->size * p->nrhs * sizeof(double), eb = (size_t)esize * p->nrhs * sizeof(double);
  const size_t wb = 2 * (size_t)esize * sizeof(double);
  if (overlap2(work, wb, out, ib) || overlap2(work, wb, b, eb) || overlap2(work, wb, f, ib))
    return FFTFEM_EINVAL;
  return dirichlet_load_impl(p, b, f, out, work, s);
}

int fftfem_dirichlet_load_noalloc(fftfem_plan_t p, const double* b, const double* f, double* out,
                                  hipStream_t s) {
  if (!p || !b || !f || !out || p->rec) return FFTFEM_EINVAL;
  if (2 * (size_t)dirichlet_extended_size(p) > kLiftScratchDoubles) return FFTFEM_EINVAL;
  double* work = nullptr;
  int rc = from_hip(lift_scratch(&work));
  if (rc) return rc;
  return dirichlet_load_impl(p, b, f, out, work, s);
}

static int dirichlet_load_impl(fftfem_plan_t p, const double* b, const double* f, double* out, double* work,
                               hipStream_t s) {
  const int N = p->N;
  int64_t E[3] = {1, 1, 1};
  for (int d = 0; d < N; ++d) E[d] = p->M[d] + 2;
  const int64_t esize = dirichlet_extended_size(p);
  const size_t ib = (size_t)p->size * p->nrhs * sizeof(double), eb = (size_t)esize * p->nrhs * sizeof(double);
  if (f != out && overlap(f, out, ib)) return FFTFEM_EINVAL;
  if (overlap2(b, eb, out, ib)) return FFTFEM_EINVAL;
  p->last = s;
  int rc = FFTFEM_OK;
  for (int r = 0; r < p->nrhs && !rc; ++r) {
    const double* br = b + (size_t)r * esize;
    const double* fr = f + (size_t)r * p->size;
    double* orr = out + (size_t)r * p->size;
    double* w[2] = {work, work + esize};
    // terms: coef_t C x .. x A_t x .. x C for t < N, react C x .. x C
    for (int t = 0; t <= N && !rc; ++t) {
      const double scale = t < N ? p->coef[t] : p->desc.react;
      if (t == N && scale == 0.0) break;
      int64_t L[3] = {E[0], E[1], E[2]};
      const double* src = br;
      for (int d = 0; d < N && !rc; ++d) {
        LiftArgs a{};
        a.in = src;
        a.n = p->nd[d];
        a.K = (int)p->K[d];
        a.X = d == t ? p->Ael[d] : p->Cel[d];  // float64 (hi) part
        a.outer = 1;
        for (int e = 0; e < d; ++e) a.outer *= L[e];
        a.inner = 1;
        for (int e = d + 1; e < N; ++e) a.inner *= L[e];
        a.mask = d == 0;
        a.N = N;
        for (int e = 0; e < 3; ++e) a.ext[e] = E[e];
        const bool last = d == N - 1;
        a.out = last ? orr : w[d % 2];
        a.combine = last;
        a.scale = scale;
        a.f = last && t == 0 ? fr : nullptr;
        Timed tm(p, s, "lift64_ax" + std::to_string(d));
        rc = from_hip(launch_lift(a, s));
        src = a.out;
        L[d] = p->M[d];
      }
    }
  }
  return rc;
}

int fftfem_synthesize(fftfem_plan_t p, const double* in, double* out, hipStream_t s) {
  if (!p || !in || !out || p->rec) return FFTFEM_EINVAL;
  const size_t bytes = (size_t)p->size * p->nrhs * sizeof(double);
  if (in != out && overlap(in, out, bytes)) return FFTFEM_EINVAL;
  p->last = s;
  if (p->longK) {
    // (two axes) axis 0 per right-hand side first, then the rows of every
    // right-hand side along the last axis
    int rc = FFTFEM_OK;
    const double* src = in;
    for (int r = 0; r < p->nrhs && !rc && p->N == 2; ++r)
      rc = long_axis0_2d(p, INV, in + (size_t)r * p->size, out + (size_t)r * p->size, s);
    if (p->N == 2) src = out;
    return rc ? rc : long_last_axis(p, INV, src, out, s);
  }
  int rc = FFTFEM_OK;
  for (int r = 0; r < p->nrhs && !rc; ++r) {
    const size_t o = (size_t)r * p->size;
    const double* src = in + o;
    for (int d = 0; d < p->N && !rc; ++d) {
      rc = line_pass<double>(p, natural_geom(p, d, false), INV, src, 1, out + o, 1, nullptr, nullptr, s, false);
      src = out + o;
    }
  }
  return rc;
}

int fftfem_tune_save(const char* path) {
  if (!path) return FFTFEM_EINVAL;
  std::lock_guard<std::mutex> l(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return FFTFEM_EINVAL;
  std::fprintf(f, "# fftfem line-pass parameters: elt n mode strided kclass G lrmax\n");
  for (const auto& kv : g_tune)
    std::fprintf(f, "%d %d %d %d %lld %d %d\n", kv.first.elt, kv.first.n, kv.first.mode, kv.first.lf,
                 (long long)kv.first.K, kv.second.G, kv.second.lrmax);
  const bool ok = std::fclose(f) == 0;
  return ok ? (int)g_tune.size() : FFTFEM_EINVAL;
}

int fftfem_tune_load(const char* path) {
  if (!path) return FFTFEM_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return FFTFEM_EINVAL;
  std::vector<std::pair<TuneKey, TuneVal>> rows;
  char line[256];
  bool bad = false;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int elt, n, mode, lf, G, lr;
    long long kc;
    if (std::sscanf(line, "%d %d %d %d %lld %d %d", &elt, &n, &mode, &lf, &kc, &G, &lr) != 7 ||
        (elt != 4 && elt != 8) || n < 1 || n > kMaxLineOrder || (mode != FWD && mode != MID && mode != INV) ||
        (lf != 0 && lf != 1) || kc < 1 || G < 1 || G > 64 || (G & (G - 1)) || lr < 2 || lr > 4) {
      bad = true;
      break;
    }
    rows.push_back({TuneKey{elt, n, mode, lf, (int64_t)kc}, TuneVal{G, lr}});
  }
  std::fclose(f);
  if (bad) return FFTFEM_EINVAL;
  for (const auto& r : rows) tune_set(r.first, r.second);
  return (int)rows.size();
}

int fftfem_debug_transform(fftfem_plan_t p, int axis, int dir, const double* in, double* out,
                           int dtype, hipStream_t s) {
  if (!p || !in || !out || axis < 0 || axis >= p->N || dir < -1 || dir > 1) return FFTFEM_EINVAL;
  if (dtype != 0 && dtype != 1) return FFTFEM_EINVAL;
  int mode = dir > 0 ? FWD : (dir < 0 ? INV : MID);
  p->last = s;
  if (p->longK) {
    // long lines: float64 only, every right-hand side; the last axis' rows
    // directly, axis 0 of a two-axis plan through the transposed array
    if (dtype != 0) return FFTFEM_ENOTIMPL;
    if (in != out && overlap(in, out, (size_t)p->size * p->nrhs * sizeof(double))) return FFTFEM_EINVAL;
    if (axis == p->N - 1) return long_last_axis(p, mode, in, out, s);
    int rc = FFTFEM_OK;
    for (int r = 0; r < p->nrhs && !rc; ++r)
      rc = long_axis0_2d(p, mode, in + (size_t)r * p->size, out + (size_t)r * p->size, s);
    return rc;
  }
  Geom g = natural_geom(p, axis, false);
  if (dtype == 0) return line_pass<double>(p, g, mode, in, 1, out, 1, nullptr, nullptr, s, false);
  return line_pass<float>(p, g, mode, in, 1, out, 1, nullptr, nullptr, s, false);
}

}  // extern "C"

namespace fftfem {

int plan_num_passes(fftfem_plan_t p) { return p ? 2 * p->N - 1 : 0; }

int plan_pass_info(fftfem_plan_t p, int pass, PassInfo* info) {
  if (!p || !info || pass < 0 || pass >= 2 * p->N - 1) return FFTFEM_EINVAL;
  if (p->N < 2 || p->longK) return FFTFEM_ENOTIMPL;
  const Geom g = tune_geom(p, pass);
  const int64_t K = p->K[g.axis];
  info->elt = p->desc.precision == FFTFEM_FP64 ? (int)sizeof(double) : (int)sizeof(float);
  info->n = p->nd[g.axis];
  info->mode = chain_mode(p, pass);
  info->lf = g.es > 1 ? 1 : 0;
  info->K = K;
  int G = 1;
  while (G < 64 && 2 * G * K <= kLineTasks && 2 * G <= g.nlines &&
         (size_t)(2 * G) * line_lds(info->n, K, info->elt) <= (size_t)p->lds_max)
    G *= 2;
  info->Gmax = G;
  return FFTFEM_OK;
}

int plan_time_pass(fftfem_plan_t p, int pass, int G, int lrmax, int reps, hipStream_t s, float* ms) {
  PassInfo info;
  int rc = plan_pass_info(p, pass, &info);
  if (rc) return rc;
  if (G < 1 || G > info.Gmax || (G & (G - 1)) || lrmax < 2 || lrmax > 4 || reps < 1) return FFTFEM_EINVAL;
  const Geom g = tune_geom(p, pass);
  // data for the timing runs: the plan's own scratch (float32 workspace; the
  // first two double-double planes for float64 plans), contents irrelevant
  const bool f64 = info.elt == (int)sizeof(double);
  float* buf = (p->N == 2 && pass == 1 && p->tr2d) ? p->W32b : p->W32;
  double* din = p->tmp[0];
  double* dout = p->tmp[1];
  auto run = [&]() {
    return f64 ? line_pass<double>(p, g, info.mode, din, 1, dout, 0, nullptr, nullptr, s, false)
               : line_pass<float>(p, g, info.mode, buf, 0, buf, 0, nullptr, nullptr, s, false);
  };
  hipEvent_t a = nullptr, b = nullptr;
  if ((rc = from_hip(hipEventCreate(&a)))) return rc;
  if ((rc = from_hip(hipEventCreate(&b)))) {
    (void)hipEventDestroy(a);
    return rc;
  }
  p->Gforce = G;
  p->lrforce = lrmax;
  Recorder* saved = p->rec;
  p->rec = nullptr;
  rc = run();  // warm-up
  if (!rc) rc = from_hip(hipEventRecord(a, s));
  for (int i = 0; i < reps && !rc; ++i) rc = run();
  if (!rc) rc = from_hip(hipEventRecord(b, s));
  if (!rc) rc = from_hip(hipEventSynchronize(b));
  if (!rc) rc = from_hip(hipEventElapsedTime(ms, a, b));
  if (!rc) *ms /= reps;
  p->rec = saved;
  p->Gforce = p->lrforce = 0;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // namespace fftfem
