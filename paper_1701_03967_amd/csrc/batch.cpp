// Batches of independent problems: one plan per problem, every problem's
// schedule recorded once, the passes of all problems that sit at the same
// position of the schedule and use the same kernel grouped into one launch
// over a device table of jobs, and the launches captured into one graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "fftfem.h"
#include "fftfem_internal.h"
#include "launch.h"
#include "record.h"

using namespace fftfem;

struct fftfem_batch_s {
  std::vector<fftfem_plan_t> plans;
  int flags = 0;
  bool tuned = false;
  // the graph and the pointers it was recorded for
  std::vector<const double*> f;
  std::vector<double*> u;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;  // capture stream
  void* jobs = nullptr;       // device job tables of the graph's launches
  size_t job_bytes = 0;
  hipStream_t last = nullptr;
};

namespace {

int hip_rc(hipError_t e) {
  if (e == hipSuccess) return FFTFEM_OK;
  if (e == hipErrorOutOfMemory) return FFTFEM_ENOMEM;
  return FFTFEM_EHIP;
}

void release_graph(fftfem_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->jobs) (void)hipFree(b->jobs);
  b->exec = nullptr;
  b->graph = nullptr;
  b->jobs = nullptr;
  b->job_bytes = 0;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// One grouped launch: all records of one kind and kernel at one phase.
struct Group {
  int phase, kind;
  int key[5];
  std::vector<const Rec*> recs;
  size_t off_jobs = 0, off_start = 0, off_jobof = 0;  // offsets in the job buffer
  int nblocks = 0;
  size_t lds = 0;
};

// Measures, for every line-pass kind of the plans (precision, n, mode,
// strided or not, element-count class) that the table does not hold yet,
// the candidate lines per tile and largest FFT radixes on the plan of that
// kind with the most data, and keeps the fastest (process-wide).
int tune_plans(const std::vector<fftfem_plan_t>& plans, hipStream_t s) {
  struct Cand {
    fftfem_plan_t p;
    int pass;
    int64_t lines;
  };
  std::map<std::tuple<int, int, int, int, int64_t>, Cand> kinds;
  for (fftfem_plan_t p : plans) {
    for (int pass = 0; pass < plan_num_passes(p); ++pass) {
      PassInfo info;
      if (plan_pass_info(p, pass, &info) != FFTFEM_OK) continue;
      const auto key = std::make_tuple(info.elt, info.n, info.mode, info.lf, tune_class(info.K));
      TuneVal known;
      if (tune_get(TuneKey{info.elt, info.n, info.mode, info.lf, tune_class(info.K)}, &known)) continue;
      const int64_t lines = (int64_t)fftfem_workspace_bytes(p);  // proxy for the problem size
      auto it = kinds.find(key);
      if (it == kinds.end() || it->second.lines < lines) kinds[key] = Cand{p, pass, lines};
    }
  }
  for (const auto& kv : kinds) {
    const Cand& c = kv.second;
    PassInfo info;
    int rc = plan_pass_info(c.p, c.pass, &info);
    if (rc) return rc;
    float best = 0;
    TuneVal bv{0, 4};
    for (int G = 1; G <= info.Gmax; G *= 2)
      for (int lr = 4; lr >= 2; --lr) {
        float ms = 0;
        rc = plan_time_pass(c.p, c.pass, G, lr, 3, s, &ms);
        if (rc) return rc;
        if (bv.G == 0 || ms < best) {
          best = ms;
          bv = TuneVal{G, lr};
        }
      }
    tune_set(TuneKey{info.elt, info.n, info.mode, info.lf, tune_class(info.K)}, bv);
  }
  return FFTFEM_OK;
}

int build_graph(fftfem_batch_s* b, const double* const* f, double* const* u, hipStream_t s) {
  release_graph(b);
  int rc;
  if (b->flags & FFTFEM_BATCH_TUNE && !b->tuned) {
    if ((rc = tune_plans(b->plans, s))) return rc;
    b->tuned = true;
  }
  // record every problem's schedule
  const int count = (int)b->plans.size();
  std::vector<Recorder> recs(count);
  for (int i = 0; i < count; ++i) {
    plan_set_recorder(b->plans[i], &recs[i]);
    rc = fftfem_solve(b->plans[i], f[i], u[i], s);
    plan_set_recorder(b->plans[i], nullptr);
    if (rc) return rc;
  }
  // group by (phase, kind, kernel)
  std::map<std::tuple<int, int, int, int, int, int, int>, Group> groups;
  for (int i = 0; i < count; ++i)
    for (const Rec& r : recs[i].recs) {
      auto key = std::make_tuple(r.phase, r.kind, r.key[0], r.key[1], r.key[2], r.key[3], r.key[4]);
      Group& g = groups[key];
      if (g.recs.empty()) {
        g.phase = r.phase;
        g.kind = r.kind;
        std::memcpy(g.key, r.key, sizeof(g.key));
      }
      g.recs.push_back(&r);
    }
  // job tables: per group the job structs, the block starts and the block -> job map
  size_t total = 0;
  for (auto& kv : groups) {
    Group& g = kv.second;
    const size_t jb = g.recs.front()->args.size();
    g.off_jobs = total;
    total = align256(total + jb * g.recs.size());
    int64_t nb = 0;
    for (const Rec* r : g.recs) {
      nb += r->nblocks;
      g.lds = std::max(g.lds, r->lds);
    }
    if (nb > 0x7fffffff) return FFTFEM_ENOTIMPL;
    g.nblocks = (int)nb;
    g.off_start = total;
    total = align256(total + sizeof(int) * (g.recs.size() + 1));
    g.off_jobof = total;
    total = align256(total + sizeof(int) * (size_t)std::max(nb, (int64_t)1));
  }
  std::vector<unsigned char> host(total, 0);
  for (auto& kv : groups) {
    Group& g = kv.second;
    const size_t jb = g.recs.front()->args.size();
    int* start = (int*)(host.data() + g.off_start);
    int* jobof = (int*)(host.data() + g.off_jobof);
    int acc = 0;
    for (size_t j = 0; j < g.recs.size(); ++j) {
      std::memcpy(host.data() + g.off_jobs + j * jb, g.recs[j]->args.data(), jb);
      start[j] = acc;
      for (int k = 0; k < g.recs[j]->nblocks; ++k) jobof[acc + k] = (int)j;
      acc += g.recs[j]->nblocks;
    }
    start[g.recs.size()] = acc;
  }
  if ((rc = hip_rc(hipMalloc(&b->jobs, std::max<size_t>(total, 256))))) {
    b->jobs = nullptr;
    return rc;
  }
  b->job_bytes = total;
  if ((rc = hip_rc(hipMemcpy(b->jobs, host.data(), total, hipMemcpyHostToDevice)))) return rc;
  // capture the launches in schedule order
  if (!b->cap && (rc = hip_rc(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)))) return rc;
  if ((rc = hip_rc(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)))) return rc;
  hipError_t e = hipSuccess;
  unsigned char* base = (unsigned char*)b->jobs;
  for (auto& kv : groups) {
    const Group& g = kv.second;
    const int* start = (const int*)(base + g.off_start);
    const int* jobof = (const int*)(base + g.off_jobof);
    const void* jobs = base + g.off_jobs;
    const int njobs = (int)g.recs.size();
    switch (g.kind) {
      case REC_LINE32: {
        GroupedLaunch<float> gl{(const LineArgs<float>*)jobs, jobof, start, g.nblocks, g.lds};
        e = launch_line_grouped<float>(g.key[4], g.key[0], g.key[1], g.key[2], g.key[3], gl, b->cap);
        break;
      }
      case REC_LINE64: {
        GroupedLaunch<double> gl{(const LineArgs<double>*)jobs, jobof, start, g.nblocks, g.lds};
        e = launch_line_grouped<double>(g.key[4], g.key[0], g.key[1], g.key[2], g.key[3], gl, b->cap);
        break;
      }
      case REC_APPLY:
        e = launch_apply_grouped(g.key[0], g.key[1] != 0, g.key[2] != 0, GroupedOps{jobs, jobof, start, g.nblocks, g.lds},
                                 b->cap);
        break;
      case REC_RESID3P:
        e = launch_resid3p_grouped(g.key[0], g.key[1] != 0, GroupedOps{jobs, jobof, start, g.nblocks, 0}, b->cap);
        break;
      case REC_RESID2:
        e = launch_resid2_grouped(g.key[0], g.key[1] != 0, GroupedOps{jobs, jobof, start, g.nblocks, 0}, b->cap);
        break;
      case REC_TR32:
        e = launch_transpose_grouped<float>(GroupedOps{jobs, jobof, start, g.nblocks, 0}, b->cap);
        break;
      case REC_TR64:
        e = launch_transpose_grouped<double>(GroupedOps{jobs, jobof, start, g.nblocks, 0}, b->cap);
        break;
      case REC_RESET:
        e = launch_reset_grouped((const ResetJob*)jobs, njobs, b->cap);
        break;
      case REC_REDUCE:
        e = launch_reduce_grouped((const ReduceJob*)jobs, njobs, b->cap);
        break;
      default:
        e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) break;
  }
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(b->cap, &graph);
  if (e == hipSuccess) e = ee;
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return hip_rc(e);
  }
  b->graph = graph;
  if ((rc = hip_rc(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)))) {
    b->exec = nullptr;
    return rc;
  }
  b->f.assign(f, f + count);
  b->u.assign(u, u + count);
  return FFTFEM_OK;
}

}  // namespace

extern "C" {

int fftfem_plan_batch(fftfem_batch_t* out, int count, const fftfem_desc* descs, int flags) {
  if (!out) return FFTFEM_EINVAL;
  *out = nullptr;
  if (count < 1 || !descs || (flags & ~FFTFEM_BATCH_TUNE)) return FFTFEM_EINVAL;
  fftfem_batch_s* b = new (std::nothrow) fftfem_batch_s();
  if (!b) return FFTFEM_ENOMEM;
  b->flags = flags;
  b->plans.assign(count, nullptr);
  // tables are computed on host threads; device uploads happen inside
  // plan_create (one problem per thread)
  TableCache cache;
  std::vector<int> rcs(count, FFTFEM_OK);
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int nth = std::max(1, std::min<int>(count, 8));
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
      (void)hipSetDevice(dev);
      for (int i = t; i < count; i += nth) rcs[i] = plan_create(&b->plans[i], &descs[i], &cache);
    });
  for (auto& x : th) x.join();
  for (int i = 0; i < count; ++i)
    if (rcs[i]) {
      int rc = rcs[i];
      fftfem_destroy_batch(b);
      return rc;
    }
  *out = b;
  return FFTFEM_OK;
}

int fftfem_solve_batch(fftfem_batch_t b, const double* const* f, double* const* u, hipStream_t s) {
  if (!b || !f || !u) return FFTFEM_EINVAL;
  const int count = (int)b->plans.size();
  for (int i = 0; i < count; ++i) {
    if (!f[i] || !u[i]) return FFTFEM_EINVAL;
    // as in fftfem_solve: u must not overlap f (the refinement rereads f)
    const size_t bytes = plan_array_bytes(b->plans[i]);
    const char *x = (const char*)f[i], *y = (const char*)u[i];
    if (x < y + bytes && y < x + bytes) return FFTFEM_EINVAL;
  }
  bool same = b->exec && (int)b->f.size() == count;
  for (int i = 0; same && i < count; ++i) same = b->f[i] == f[i] && b->u[i] == u[i];
  int rc;
  if (!same && (rc = build_graph(b, f, u, s))) return rc;
  b->last = s;
  for (fftfem_plan_t p : b->plans) plan_set_stream(p, s);
  return hip_rc(hipGraphLaunch(b->exec, s));
}

int fftfem_tune(fftfem_plan_t p, hipStream_t s) {
  if (!p) return FFTFEM_EINVAL;
  PassInfo info;
  int rc = plan_pass_info(p, 0, &info);
  if (rc) return rc;
  return tune_plans(std::vector<fftfem_plan_t>{p}, s);
}

int fftfem_batch_get_stats(fftfem_batch_t b, int i, fftfem_stats* out) {
  if (!b || !out || i < 0 || i >= (int)b->plans.size()) return FFTFEM_EINVAL;
  return fftfem_get_stats(b->plans[i], out);
}

size_t fftfem_batch_workspace_bytes(const fftfem_batch_t b) {
  if (!b) return 0;
  size_t t = b->job_bytes;
  for (fftfem_plan_t p : b->plans) t += fftfem_workspace_bytes(p);
  return t;
}

void fftfem_destroy_batch(fftfem_batch_t b) {
  if (!b) return;
  if (b->last) (void)hipStreamSynchronize(b->last);
  release_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (fftfem_plan_t p : b->plans) fftfem_destroy(p);
  delete b;
}

}  // extern "C"
