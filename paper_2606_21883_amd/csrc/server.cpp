// Continuous-batching server (include/mpwos.h, "serving").
//
// Requests are validated and costed at submit time and queued.  A worker
// thread admits queued requests in arrival order while their device
// footprint fits the HBM budget and keeps a fixed number of walk slices in
// flight: two per stream on a few streams of default priority.  Whenever a
// slice completes (its event, polled by the host) the stream's slot takes the
// next slice, chosen round-robin over the admitted requests, so slices of
// different requests overlap on the device and a request that arrives while
// others run gets slots as soon as slices drain, without waiting for the
// others.  A request whose walks have all completed is reduced per query on a
// separate completion stream, copied out, released and signalled.
//
// A walk's score depends only on (request, query, walk) through the Philox
// counter, and the per-query reduction runs in a fixed order, so a served
// result is bit-identical to the same solve run alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_internal.h"
#include "kernel_args.h"
#include "mpwos.h"

namespace mpwos {

namespace {

constexpr int kStreams = 4;
constexpr int kDepth = 2;                  // slices in flight per stream
constexpr int kSlots = kStreams * kDepth;

struct SrvReq {
  uint64_t ticket = 0;
  mpwos_request r;
  std::vector<double> table;   // TABLE_S1 values (host copy)
  WalkArgs args;
  mpwos_options opt;
  int64_t total = 0;           // n_queries * n_walks
  int64_t next = 0;            // next walk to launch
  double k_est = 32.0;         // walk-steps per walk (exact when the radius is constant; a guess otherwise)
  double step_cost = 1.0;      // Philox blocks per walk-step
  int64_t min_walks = 1;       // walks that fill the device
  size_t bytes = 0;
  char* dev = nullptr;
  double* d_queries = nullptr;
  double* d_S = nullptr;
  int32_t* d_K = nullptr;
  double* d_u = nullptr;
  double* d_se = nullptr;
  unsigned long long* d_stats = nullptr;  // ksum, kmax, ntrunc, queue
  double* d_table = nullptr;
  int32_t status = MPWOS_OK;
  bool finished = false;
  bool async_alloc = false;    // device memory from the stream-ordered allocator
  int inflight = 0;            // slices launched and not yet completed
  bool queue_busy[kDepth] = {};  // per-slice work counters of the persistent kernels
  int64_t walk_steps = 0;
};

// One slot of in-flight work: a slice of walks of a request on a stream.
struct Slot {
  SrvReq* R = nullptr;
  hipEvent_t ev = nullptr;
  int queue = 0;
};

}  // namespace
}  // namespace mpwos

struct mpwos_server {
  size_t budget = 0;
  int64_t slice = 0;           // Philox blocks of work per slice (all admitted requests share it)
  int device = 0;
  int n_cu = 256;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  std::deque<mpwos::SrvReq*> pending;
  std::vector<mpwos::SrvReq*> active;
  std::unordered_map<uint64_t, mpwos::SrvReq*> reqs;
  uint64_t next_ticket = 1;
  size_t in_flight = 0;
  hipStream_t streams[mpwos::kStreams] = {};
  hipStream_t done_stream = nullptr;   // per-query reductions and copies out
  mpwos_server_stats st = {};
  std::chrono::steady_clock::time_point t0;
};

namespace mpwos {

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t request_bytes(const mpwos_request& r, int n) {
  size_t b = 0;
  b += align256((size_t)r.n_queries * n * sizeof(double));
  b += align256((size_t)r.n_queries * r.n_walks * sizeof(double));
  b += align256((size_t)r.n_queries * r.n_walks * sizeof(int32_t));
  b += 2 * align256((size_t)r.n_queries * sizeof(double));
  b += align256(8 * sizeof(unsigned long long));
  if (r.f.kind == MPWOS_FN_TABLE_S1) b += align256((size_t)r.f.n_values * sizeof(double));
  return b;
}

static mpwos_status admit(mpwos_server* s, SrvReq* R) {
  hipStream_t st = s->done_stream;
  // the stream-ordered allocator: freeing a request does not wait for the
  // device (a plain hipFree would synchronise with the slices of others)
  hipError_t e = hipMallocAsync((void**)&R->dev, R->bytes, st);
  R->async_alloc = e == hipSuccess;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = hipMalloc((void**)&R->dev, R->bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    R->dev = nullptr;
    return fail(MPWOS_ENOMEM, "server: device allocation failed");
  }
  const int n = R->args.n;
  char* p = R->dev;
  auto take = [&](size_t b) { char* q = p; p += align256(b); return q; };
  R->d_queries = (double*)take((size_t)R->r.n_queries * n * sizeof(double));
  R->d_S = (double*)take((size_t)R->total * sizeof(double));
  R->d_K = (int32_t*)take((size_t)R->total * sizeof(int32_t));
  R->d_u = (double*)take((size_t)R->r.n_queries * sizeof(double));
  R->d_se = (double*)take((size_t)R->r.n_queries * sizeof(double));
  R->d_stats = (unsigned long long*)take(8 * sizeof(unsigned long long));
  if (!R->table.empty()) R->d_table = (double*)take(R->table.size() * sizeof(double));
  e = hipMemcpyAsync(R->d_queries, R->r.queries, (size_t)R->r.n_queries * n * sizeof(double),
                     hipMemcpyHostToDevice, st);
  if (e == hipSuccess && R->d_table)
    e = hipMemcpyAsync(R->d_table, R->table.data(), R->table.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_zero_u64(R->d_stats, 8, st);
  // slices run on other streams: the uploads complete before the first launch
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "server: admission copies");
  WalkArgs& a = R->args;
  a.queries = R->d_queries;
  a.nq = R->r.n_queries;
  a.nw = R->r.n_walks;
  a.q_offset = 0;
  a.walk_S = R->d_S;
  a.walk_K = R->d_K;
  if (R->d_table) a.f.values = R->d_table;
  return MPWOS_OK;
}

// Every slice of R has completed (its events were observed): the reduction
// runs on the completion stream, which carries nothing else.
static mpwos_status finish(mpwos_server* s, SrvReq* R) {
  hipStream_t st = s->done_stream;
  hipError_t e = launch_reduce(R->d_S, R->d_K, R->r.n_queries, R->r.n_walks, R->opt.max_steps, R->d_u, R->d_se,
                               R->d_stats + 0, (int32_t*)(R->d_stats + 1), R->d_stats + 2, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(R->r.u_out, R->d_u, (size_t)R->r.n_queries * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && R->r.stderr_out)
    e = hipMemcpyAsync(R->r.stderr_out, R->d_se, (size_t)R->r.n_queries * sizeof(double), hipMemcpyDeviceToHost, st);
  unsigned long long hs[8] = {};
  if (e == hipSuccess) e = hipMemcpyAsync(hs, R->d_stats, sizeof(hs), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "server: completion");
  R->walk_steps = (int64_t)hs[0];
  return hs[2] ? MPWOS_WTRUNC : MPWOS_OK;
}

static void release(mpwos_server* s, SrvReq* R) {
  if (R->dev) {
    if (R->async_alloc) (void)hipFreeAsync(R->dev, s->done_stream);
    else (void)hipFree(R->dev);
  }
  R->dev = nullptr;
  manifold_ref(R->r.manifold, -1);
}

// Walks of R in one slice: a share of the slice budget by the request's cost
// per walk, at least what keeps the device busy together with the other
// slots, at most what is left.
static int64_t slice_walks(const mpwos_server* s, const SrvReq* R, int nact) {
  const double share = (double)s->slice / std::max(1, nact) / std::max(1.0, R->k_est * R->step_cost);
  int64_t walks = std::max<int64_t>((int64_t)share, R->min_walks / kSlots);
  walks = std::max<int64_t>(walks, 1);
  return std::min<int64_t>(walks, R->total - R->next);
}

static void worker_main(mpwos_server* s) {
  (void)hipSetDevice(s->device);
  Slot slots[kSlots];
  for (auto& sl : slots) (void)hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
  size_t rr = 0;
  auto last = std::chrono::steady_clock::now();
  for (;;) {
    std::vector<SrvReq*> fresh;
    std::vector<SrvReq*> active;
    bool busy_slot = false;
    for (auto& sl : slots) busy_slot = busy_slot || sl.R != nullptr;
    {
      const auto now = std::chrono::steady_clock::now();
      if (busy_slot) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.busy_seconds += std::chrono::duration<double>(now - last).count();
      }
      last = now;
    }
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (!busy_slot)
        s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
      if (s->stop && s->pending.empty() && s->active.empty() && !busy_slot) break;
      while (!s->pending.empty()) {
        SrvReq* R = s->pending.front();
        if (!s->active.empty() && s->in_flight + R->bytes > s->budget) break;
        s->pending.pop_front();
        s->in_flight += R->bytes;
        s->active.push_back(R);
        fresh.push_back(R);
        s->st.admitted += 1;
      }
      active = s->active;
      s->st.in_flight_bytes = (int64_t)s->in_flight;
    }
    for (SrvReq* R : fresh) {
      mpwos_status st = admit(s, R);
      if (st) {
        R->status = st;
        R->next = R->total;
      }
    }
    bool progress = !fresh.empty();
    // completed slices free their slots
    for (auto& sl : slots) {
      if (!sl.R) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess && sl.R->status >= 0) sl.R->status = hip_fail(q, "server: slice");
      sl.R->inflight -= 1;
      sl.R->queue_busy[sl.queue] = false;
      sl.R = nullptr;
      progress = true;
    }
    // requests whose walks have all completed: reduce, copy out, release
    std::vector<SrvReq*> done;
    for (SrvReq* R : active) {
      if (R->next < R->total || R->inflight > 0) continue;
      if (R->status >= 0) R->status = finish(s, R);
      release(s, R);
      done.push_back(R);
    }
    // fill free slots round-robin over the requests with walks left
    std::vector<SrvReq*> open;
    for (SrvReq* R : active)
      if (R->status >= 0 && R->next < R->total) open.push_back(R);
    const int nact = (int)open.size();
    for (int k = 0; k < kSlots && !open.empty(); ++k) {
      Slot& sl = slots[k];
      if (sl.R) continue;
      SrvReq* R = nullptr;
      int q = -1;
      for (size_t t = 0; t < open.size() && !R; ++t) {
        SrvReq* c = open[(rr + t) % open.size()];
        if (c->next >= c->total) continue;
        for (int j = 0; j < kDepth; ++j)
          if (!c->queue_busy[j]) { q = j; break; }
        if (q >= 0) { R = c; rr = (rr + t + 1) % open.size(); }
      }
      if (!R) break;
      WalkArgs a = R->args;
      a.idx_base = R->next;
      a.count = slice_walks(s, R, nact);
      hipStream_t st = s->streams[k % kStreams];
      mpwos_status ls = launch_walks(a, R->opt, st, R->d_stats + 3 + q);
      hipError_t e = ls ? hipErrorUnknown : hipEventRecord(sl.ev, st);
      if (ls || e != hipSuccess) {
        R->status = ls ? ls : hip_fail(e, "server: slice event");
        R->next = R->total;
        continue;
      }
      R->next += a.count;
      R->inflight += 1;
      R->queue_busy[q] = true;
      sl.R = R;
      sl.queue = q;
      progress = true;
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.rounds += 1;
    }
    if (!done.empty()) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (SrvReq* R : done) {
          R->finished = true;
          s->in_flight -= R->bytes;
          s->st.completed += 1;
          s->st.walk_steps += R->walk_steps;
          s->active.erase(std::find(s->active.begin(), s->active.end(), R));
        }
        s->st.in_flight_bytes = (int64_t)s->in_flight;
      }
      s->cv_done.notify_all();
    }
    if (!progress) {
      // slices still running: look again shortly, or sooner when work arrives
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(100));
    }
  }
  for (auto& sl : slots) (void)hipEventDestroy(sl.ev);
}

}  // namespace mpwos

using namespace mpwos;

extern "C" {

mpwos_status mpwos_server_create(size_t hbm_budget_bytes, int64_t slice_walk_steps, mpwos_server** out) {
  if (!out) return fail(MPWOS_EINVAL, "out is NULL");
  if (hbm_budget_bytes < ((size_t)1 << 20)) return fail(MPWOS_EINVAL, "HBM budget below 1 MiB");
  if (slice_walk_steps < 0) return fail(MPWOS_EINVAL, "slice_walk_steps must be >= 0");
  auto* s = new (std::nothrow) mpwos_server;
  if (!s) return fail(MPWOS_ENOMEM, "host allocation");
  s->budget = hbm_budget_bytes;
  s->slice = slice_walk_steps ? slice_walk_steps * 3 : ((int64_t)1 << 28);
  hipError_t e = hipGetDevice(&s->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, s->device);
  for (int i = 0; e == hipSuccess && i < kStreams; ++i) e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->done_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "server: stream creation");
  }
  s->n_cu = prop.multiProcessorCount;
  s->t0 = std::chrono::steady_clock::now();
  s->worker = std::thread(worker_main, s);
  *out = s;
  return MPWOS_OK;
}

mpwos_status mpwos_submit(mpwos_server* s, const mpwos_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return fail(MPWOS_EINVAL, "NULL argument");
  if (!req->queries || !req->u_out) return fail(MPWOS_EINVAL, "queries and u_out must not be NULL");
  if (!req->manifold) return fail(MPWOS_EINVAL, "manifold is NULL");
  auto* R = new (std::nothrow) SrvReq;
  if (!R) return fail(MPWOS_ENOMEM, "host allocation");
  R->r = *req;
  R->opt = req->opt;
  R->opt.stream = nullptr;
  R->opt.device_io = 0;
  R->opt.walk_S = nullptr;
  R->opt.walk_K = nullptr;
  const mpwos_fn* g = req->has_g ? &R->r.g : nullptr;
  if (req->f.kind == MPWOS_FN_TABLE_S1 && req->f.values && req->f.n_values > 0)
    R->table.assign(req->f.values, req->f.values + req->f.n_values);
  mpwos_status st = prepare_solve(req->manifold, &R->r.f, g, req->c, req->n_queries, req->n_walks, req->eps,
                                  req->seed, R->opt, R->args);
  if (!st) st = check_queries_host(req->manifold, R->args, req->queries, req->n_queries);
  if (st) {
    delete R;
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected += 1;
    return st;
  }
  const int n = R->args.n;
  R->total = req->n_queries * req->n_walks;
  R->bytes = request_bytes(*req, n);
  if (R->bytes > s->budget) {
    delete R;
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected += 1;
    return fail(MPWOS_ENOMEM, "request needs " + std::to_string(R->bytes) + " bytes, above the HBM budget");
  }
  if (R->args.const_r) R->k_est = std::ceil(std::log(R->opt.tau_w) / std::log(R->args.c0));
  R->step_cost = 1.0 + (double)((n + 3) / 4) * (1 + R->opt.n_v);
  const int lanes = (n <= 3) ? 1 : 64;
  R->min_walks = (int64_t)s->n_cu * 16 * 64 / lanes;   // walks that fill the device alone
  manifold_ref(req->manifold, +1);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      manifold_ref(req->manifold, -1);
      delete R;
      return fail(MPWOS_EBUSY, "server is shutting down");
    }
    R->ticket = s->next_ticket++;
    s->reqs[R->ticket] = R;
    s->pending.push_back(R);
    *ticket = R->ticket;
  }
  s->cv_work.notify_one();
  return MPWOS_OK;
}

mpwos_status mpwos_poll(mpwos_server* s, uint64_t ticket, int32_t* done, int32_t* result) {
  if (!s || !done) return fail(MPWOS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MPWOS_EINVAL, "unknown ticket");
  *done = it->second->finished ? 1 : 0;
  if (result) *result = it->second->finished ? it->second->status : MPWOS_OK;
  return MPWOS_OK;
}

mpwos_status mpwos_wait(mpwos_server* s, uint64_t ticket, int64_t timeout_ms, int32_t* result) {
  if (!s) return fail(MPWOS_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MPWOS_EINVAL, "unknown ticket");
  SrvReq* R = it->second;
  auto pred = [&] { return R->finished; };
  if (timeout_ms < 0) s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
    return fail(MPWOS_EBUSY, "timed out");
  if (result) *result = R->status;
  return MPWOS_OK;
}

mpwos_status mpwos_server_stats_get(mpwos_server* s, mpwos_server_stats* out) {
  if (!s || !out) return fail(MPWOS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return MPWOS_OK;
}

mpwos_status mpwos_server_destroy(mpwos_server* s) {
  if (!s) return fail(MPWOS_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->reqs) delete kv.second;
  for (auto& st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->done_stream) {
    (void)hipStreamSynchronize(s->done_stream);
    (void)hipStreamDestroy(s->done_stream);
  }
  delete s;
  return MPWOS_OK;
}

}  // extern "C"
