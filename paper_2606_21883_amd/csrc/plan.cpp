// Graph-captured solves (mpwos_plan_*) and the launch autotuner
// (mpwos_autotune).
//
// A plan owns the device buffers of one solve shape (queries, per-walk
// scores, estimates, counters, the seed word) and a HIP graph of its device
// work: counter reset, walk kernel(s), per-query reduction -- kernels only, so
// replays need no memset node.  The seed is read by the walk kernels from the
// plan's device word, so one instantiated graph serves every seed; execute
// copies the queries in, writes the seed with a one-thread kernel, launches
// the graph and copies the estimates out, all on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_internal.h"
#include "kernel_args.h"
#include "mpwos.h"

struct mpwos_plan {
  const mpwos_manifold* man = nullptr;
  mpwos::WalkArgs a;
  mpwos_options o;
  int64_t nq = 0, nw = 0;
  int n = 0;
  char* dev = nullptr;
  double* d_q = nullptr;
  double* d_S = nullptr;
  int32_t* d_K = nullptr;
  double* d_u = nullptr;
  double* d_se = nullptr;
  unsigned long long* d_stats = nullptr;  // ksum, kmax, ntrunc, (unused), queue, seed
  unsigned long long* d_hist = nullptr;   // K histogram, filled by mpwos_plan_stats
  double* d_table = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace mpwos {
namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void plan_free(mpwos_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->dev) (void)hipFree(p->dev);
  if (p->man) manifold_ref(p->man, -1);
  delete p;
}

}  // namespace
}  // namespace mpwos

using namespace mpwos;

extern "C" mpwos_status mpwos_plan_create(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g,
                                          double c, int64_t n_queries, int64_t n_walks, double eps,
                                          const mpwos_options* opt, mpwos_plan** out) {
  if (!out) return fail(MPWOS_EINVAL, "out is NULL");
  mpwos_options o;
  if (opt) o = *opt;
  else mpwos_options_default(&o);
  o.stream = nullptr;
  o.device_io = 1;
  o.walk_S = nullptr;
  o.walk_K = nullptr;
  if (n_queries > 0 && n_walks > ((int64_t)1 << 30) / n_queries)
    return fail(MPWOS_EINVAL, "a plan holds at most 2^30 walks");
  auto* p = new (std::nothrow) mpwos_plan;
  if (!p) return fail(MPWOS_ENOMEM, "host allocation");
  mpwos_status st = prepare_solve(manifold, f, g, c, n_queries, n_walks, eps, 0, o, p->a);
  if (st) {
    delete p;
    return st;
  }
  p->man = manifold;
  manifold_ref(manifold, +1);
  p->o = o;
  p->nq = n_queries;
  p->nw = n_walks;
  p->n = manifold_desc(manifold).n;
  const int64_t total = n_queries * n_walks;
  const bool table = fn_has_values(f->kind);
  size_t bytes = align256((size_t)n_queries * p->n * sizeof(double)) + align256((size_t)total * sizeof(double)) +
                 align256((size_t)total * sizeof(int32_t)) + 2 * align256((size_t)n_queries * sizeof(double)) +
                 align256(8 * sizeof(unsigned long long)) + align256(kKHistBins * sizeof(unsigned long long)) +
                 (table ? align256((size_t)f->n_values * sizeof(double)) : 0);
  hipError_t e = hipMalloc((void**)&p->dev, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->dev = nullptr;
    plan_free(p);
    return fail(MPWOS_ENOMEM, "plan: device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  char* q = p->dev;
  auto take = [&](size_t b) { char* r = q; q += align256(b); return r; };
  p->d_q = (double*)take((size_t)n_queries * p->n * sizeof(double));
  p->d_S = (double*)take((size_t)total * sizeof(double));
  p->d_K = (int32_t*)take((size_t)total * sizeof(int32_t));
  p->d_u = (double*)take((size_t)n_queries * sizeof(double));
  p->d_se = (double*)take((size_t)n_queries * sizeof(double));
  p->d_stats = (unsigned long long*)take(8 * sizeof(unsigned long long));
  p->d_hist = (unsigned long long*)take(kKHistBins * sizeof(unsigned long long));
  if (table) p->d_table = (double*)take((size_t)f->n_values * sizeof(double));
  e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess && table)
    e = hipMemcpy(p->d_table, f->values, (size_t)f->n_values * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    plan_free(p);
    return hip_fail(e, "plan: set-up");
  }
  WalkArgs& a = p->a;
  a.queries = p->d_q;
  a.nq = n_queries;
  a.nw = n_walks;
  a.q_offset = 0;
  a.idx_base = 0;
  a.count = total;
  a.walk_S = p->d_S;
  a.walk_K = p->d_K;
  a.seed_dev = (const uint64_t*)(p->d_stats + 5);
  if (table) a.f.values = p->d_table;
  // capture: counters, walks, reduction (kernels only)
  e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) e = launch_zero_u64(p->d_stats, 5, p->cap);
  if (e == hipSuccess) st = launch_walks(a, o, p->cap, p->d_stats + 4);
  if (e == hipSuccess && !st)
    e = launch_reduce(p->d_S, p->d_K, n_queries, n_walks, o.max_steps, p->d_u, p->d_se, p->d_stats + 0,
                      (int32_t*)(p->d_stats + 1), p->d_stats + 2, p->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(p->cap, &graph);
  p->graph = graph;
  if (st) {
    plan_free(p);
    return st;
  }
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    plan_free(p);
    return hip_fail(e, "plan: graph capture");
  }
  *out = p;
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_plan_execute(mpwos_plan* p, const double* queries, double* u_out, double* stderr_out,
                                           uint64_t seed, void* stream) {
  if (!p || !queries || !u_out) return fail(MPWOS_EINVAL, "NULL argument");
  hipStream_t s = stream ? (hipStream_t)stream : p->cap;
  const size_t qb = (size_t)p->nq * p->n * sizeof(double), ub = (size_t)p->nq * sizeof(double);
  hipError_t e = hipMemcpyAsync(p->d_q, queries, qb, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_set_u64(p->d_stats + 5, (unsigned long long)seed, s);
  if (e == hipSuccess) e = hipGraphLaunch(p->exec, s);
  if (e == hipSuccess) e = hipMemcpyAsync(u_out, p->d_u, ub, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && stderr_out) e = hipMemcpyAsync(stderr_out, p->d_se, ub, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "plan: execute");
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_plan_stats(mpwos_plan* p, void* stream, mpwos_stats* stats) {
  if (!p || !stats) return fail(MPWOS_EINVAL, "NULL argument");
  hipStream_t s = stream ? (hipStream_t)stream : p->cap;
  unsigned long long hs[8] = {};
  hipError_t e = hipMemcpyAsync(hs, p->d_stats, sizeof(hs), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "plan: stats");
  memset(stats, 0, sizeof(*stats));
  stats->walk_steps = (int64_t)hs[0];
  stats->k_max = (int32_t)(uint32_t)hs[1];
  stats->truncated = (int64_t)hs[2];
  stats->k_mean = (double)hs[0] / ((double)p->nq * (double)p->nw);
  // K quantiles of the last execution, from the per-walk K it left
  std::vector<unsigned long long> hh(kKHistBins);
  e = launch_zero_u64(p->d_hist, kKHistBins, s);
  if (e == hipSuccess) e = launch_khist(p->d_K, p->nq * p->nw, p->d_hist, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hh.data(), p->d_hist, hh.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "plan: K histogram");
  khist_quantiles(hh.data(), stats->k_p50, stats->k_p99);
  return hs[2] ? MPWOS_WTRUNC : MPWOS_OK;
}

extern "C" mpwos_status mpwos_plan_destroy(mpwos_plan* p) {
  if (!p) return fail(MPWOS_EINVAL, "plan is NULL");
  if (p->cap) (void)hipStreamSynchronize(p->cap);
  plan_free(p);
  return MPWOS_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
extern "C" mpwos_status mpwos_autotune(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g,
                                       double c, const double* queries, int64_t n_queries, int64_t n_walks,
                                       double eps, const mpwos_options* opt, mpwos_options* best,
                                       double* best_ms) {
  if (!manifold || !queries || !best) return fail(MPWOS_EINVAL, "NULL argument");
  mpwos_options base;
  if (opt) base = *opt;
  else mpwos_options_default(&base);
  base.device_io = 0;
  base.walk_S = nullptr;
  base.walk_K = nullptr;
  const mpwos_manifold_desc& d = manifold_desc(manifold);
  const int n = d.n;
  // a sample that fills the device: whole queries, walks per query capped
  WalkArgs probe;
  mpwos_status st = prepare_solve(manifold, f, g, c, n_queries, n_walks, eps, 0, base, probe);
  if (st) return st;
  const double k_est = probe.const_r ? std::ceil(std::log(base.tau_w) / std::log(probe.c0)) : 32.0;
  const double cost = philox_blocks_per_step(n, base.n_v);
  // Up to 2^24 walks (the whole solve at the headline sizes): the launch
  // forms differ in how they absorb uneven walk lengths and in how they fill
  // the device, which a small sample hides.  With a constant radius every
  // walk has the same length, so the trials keep the walks and cut their
  // length instead (max_steps) when the work would exceed the trial budget.
  const int64_t budget = (int64_t)1e10;  // Philox blocks of work per trial
  const int64_t want_walks = (int64_t)1 << 24;
  const int64_t caller_max_steps = base.max_steps;
  int64_t sample = std::min<int64_t>(want_walks, n_queries * n_walks);
  if (probe.const_r) {
    const double steps = std::floor((double)budget / ((double)sample * cost));
    if (steps < k_est) base.max_steps = (int64_t)std::max(16.0, steps);
  } else {
    sample = std::min<int64_t>(sample, std::max<int64_t>(64, (int64_t)(budget / (k_est * cost))));
  }
  const int64_t sw = std::min<int64_t>(n_walks, sample);
  const int64_t sq = std::max<int64_t>(1, std::min<int64_t>(n_queries, sample / sw));
  std::vector<mpwos_options> cand;
  auto add = [&](int block, int lanes, int persistent) {
    mpwos_options o = base;
    o.block_size = block;
    o.lanes_per_walk = lanes;
    o.persistent = persistent;
    cand.push_back(o);
  };
  if (n <= 3) {
    const std::vector<int> blocks = d.kind == MPWOS_POINT_CLOUD ? std::vector<int>{64, 128}
                                                                : std::vector<int>{64, 128, 192, 256};
    for (int b : blocks)
      for (int pz : {0, 1}) add(b, 1, pz);
  } else {
    for (int L : {4, 8, 16, 32, 64}) {
      int Lg, mb, nblk, rblk, rword;
      group_shape(n, L, Lg, mb, nblk, rblk, rword);
      if (mb > 8 && !(Lg == 64 && mb == 16)) continue;
      for (int b : {64, 128, 256})
        for (int pz : {0, 1}) add(b, L, pz);
    }
  }
  std::vector<double> u((size_t)sq), se((size_t)sq);
  double best_t = 1e300;
  int best_i = -1;
  for (size_t i = 0; i < cand.size(); ++i) {
    mpwos_stats s1, s2;
    st = mpwos_solve(manifold, f, g, c, queries, sq, sw, eps, 1, &cand[i], u.data(), se.data(), &s1);
    if (st < 0) continue;
    st = mpwos_solve(manifold, f, g, c, queries, sq, sw, eps, 2, &cand[i], u.data(), se.data(), &s2);
    if (st < 0) continue;
    if (s2.kernel_ms < best_t) {
      best_t = s2.kernel_ms;
      best_i = (int)i;
    }
  }
  if (best_i < 0) return fail(MPWOS_EINVAL, "autotune: no launch shape ran");
  *best = cand[(size_t)best_i];
  best->max_steps = caller_max_steps;
  if (opt) {
    best->stream = opt->stream;
    best->device_io = opt->device_io;
    best->walk_S = opt->walk_S;
    best->walk_K = opt->walk_K;
  }
  if (best_ms) *best_ms = best_t;
  return MPWOS_OK;
}
