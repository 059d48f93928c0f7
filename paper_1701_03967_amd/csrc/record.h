// Recording of a plan's launches (for the batched executor) and the table of
// tuned line-pass parameters.  Internal.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "fftfem.h"
#include "fftfem_internal.h"
#include "launch.h"

namespace fftfem {

// One launch a plan would issue, with its fully resolved arguments.
enum RecKind { REC_LINE32 = 0, REC_LINE64, REC_APPLY, REC_TR32, REC_TR64, REC_RESET, REC_REDUCE, REC_RESID2, REC_RESID3P };

struct Rec {
  int phase;                        // position in the plan's schedule (see fftfem_solve)
  int kind;                         // RecKind
  int key[5];                       // line: n, mode, upd, lf, pow2;  apply: n, lo, dd;  resid2, resid3p: n, dd
  std::vector<unsigned char> args;  // LineArgs<T>, ApplyArgs, Resid2Args, TransposeJob, ResetJob or ReduceJob
  int nblocks;
  size_t lds;
};

struct Recorder {
  std::vector<Rec> recs;
};

// Host axis tables shared by the plans of a batch, keyed by (n, K).
struct TableCache {
  std::mutex mu;
  std::map<std::pair<int, int64_t>, AxisTables> tabs;
  bool get(int n, int64_t K, AxisTables* t) {
    std::lock_guard<std::mutex> l(mu);
    auto it = tabs.find({n, K});
    if (it == tabs.end()) return false;
    *t = it->second;
    return true;
  }
  void put(int n, int64_t K, const AxisTables& t) {
    std::lock_guard<std::mutex> l(mu);
    tabs.emplace(std::make_pair(n, K), t);
  }
};

// fftfem_plan_ex with an optional table cache.
int plan_create(fftfem_plan_t* out, const fftfem_desc* d, TableCache* cache);

// While a recorder is attached, the plan's solve records its launches
// instead of issuing them.
void plan_set_recorder(fftfem_plan_t p, Recorder* r);
// The stream the plan's stats are synchronized with.
void plan_set_stream(fftfem_plan_t p, hipStream_t s);
size_t plan_array_bytes(fftfem_plan_t p);  // bytes of one f (all right-hand sides)

// Line-pass parameters chosen by measurement, for (precision, n, mode, lines
// strided, element count).  Consulted by every line pass; empty by default.
struct TuneKey {
  int elt, n, mode, lf;
  int64_t K;
  bool operator<(const TuneKey& o) const;
};
struct TuneVal {
  int G;      // lines per tile
  int lrmax;  // log2 of the largest FFT radix
};
// TuneKey::K: the class of an element count (its FFT length and whether it
// is a power of two)
int64_t tune_class(int64_t K);
void tune_set(const TuneKey& k, const TuneVal& v);
bool tune_get(const TuneKey& k, TuneVal* v);

// Candidate line-pass parameters for the tuner and a timing run of one pass
// of plan p (on its own scratch; plans with N >= 2).  pass 0 .. 2N - 2 in
// the order of the solve's chain: forward along axes N - 1 .. 1, the middle
// pass along axis 0 (in the layout the solve uses), inverse along 1 .. N - 1.
struct PassInfo {
  int elt;  // bytes per value of the pass (4 or 8)
  int n, mode, lf;
  int64_t K;
  int Gmax;  // largest admissible lines per tile
};
int plan_num_passes(fftfem_plan_t p);
int plan_pass_info(fftfem_plan_t p, int pass, PassInfo* info);
int plan_time_pass(fftfem_plan_t p, int pass, int G, int lrmax, int reps, hipStream_t s, float* ms);

}  // namespace fftfem
