// Continuous-batching server (include/mpwos.h, "serving").
//
// Requests are validated and costed at submit time and queued.  A worker
// thread admits queued requests in arrival order while their device
// footprint fits the HBM budget and keeps a fixed number of batched launches
// in flight: two per stream on a few streams of default priority.  Classes
// whose launches run long (walks whose every step is costly: point clouds,
// the dumbbell's profile projection) are served on half of the streams, and
// no launch is queued behind a long one, so short requests never wait for a
// long launch to drain its stream.  Admitted
// requests that run the same kernel with the same problem data (manifold, f,
// g, sigma, eps, options) form a class; one launch carries slices of every
// request of a class, each request with its own queries, seed and outputs
// (a table of entries read by the kernel).  Whenever a launch completes (its
// event, polled by the host) its slot takes the next class round-robin, so
// small requests share the device instead of queueing behind each other and
// a request that arrives while others run joins the next launch of its class.
// A request whose walks have all completed is reduced per query on a separate
// completion stream, copied out, released and signalled.
//
// A walk's score depends only on (request, query, walk) through the Philox
// counter, and the per-query reduction runs in a fixed order, so a served
// result is bit-identical to the same solve run alone.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_internal.h"
#include "kernel_args.h"
#include "mpwos.h"

namespace mpwos {

namespace {

constexpr int kMaxStreams = 8;            // walk streams at most
constexpr int kMinStreams = 6;            // walk streams at least (CU-masked when the queues are fewer)
constexpr int kDepth = 2;                  // launches in flight per stream
constexpr int kSlots = kMaxStreams * kDepth;
constexpr int kMaxBatch = 512;             // requests per launch
constexpr double kLongMs = 20.0;           // launches of a long class take longer (device time, moving average)

struct SrvReq {
  uint64_t ticket = 0;
  mpwos_request r;
  std::vector<double> table;   // TABLE_S1 / DUMBBELL_POLY values (host copy)
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
  unsigned long long* d_stats = nullptr;  // ksum, kmax, ntrunc
  double* d_table = nullptr;
  char* h_io = nullptr;        // pinned staging: queries and table in, estimates and counters out
  size_t h_io_bytes = 0;
  bool h_io_own = false;       // staging of its own (too large for the shared block)
  hipEvent_t ready_ev = nullptr;  // uploads done (on the completion stream)
  hipEvent_t done_ev = nullptr;   // reduction and copies out done
  bool ready = false;          // ready_ev observed complete
  bool completing = false;     // reduction enqueued, done_ev pending
  int32_t status = MPWOS_OK;
  bool finished = false;
  bool async_alloc = false;    // device memory from the stream-ordered allocator
  int inflight = 0;            // launches holding walks of this request, not yet completed
  int64_t walk_steps = 0;
  std::string cls;             // batch class: the launch arguments less the per-request fields
  int64_t unit = 64;           // batch unit (walks) of the class's kernel
  char* d_state = nullptr;     // state records of time-sliced walks (or null)
  int64_t rec_bytes = 0;
  std::deque<std::pair<int64_t, int64_t>> resume;   // (first walk, count) of unfinished sliced walks
  double times[5] = {-1, -1, -1, -1, -1};           // submitted, admitted, first launch, walks done, delivered
};

// Pinned host memory for the asynchronous copies of admission and completion:
// one block allocated at creation and carved first-fit, so that no request
// calls the allocator (whose frees may wait for the device).
struct HostArena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  static size_t round(size_t b) { return (b + 63) & ~(size_t)63; }
  char* alloc(size_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      return base + off;
    }
    return nullptr;
  }
  void release(char* p, size_t bytes) {
    bytes = round(bytes);
    auto it = free_.emplace((size_t)(p - base), bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

constexpr size_t kArenaBytes = (size_t)64 << 20;
constexpr double kSliceBlocks = 1e6;       // Philox blocks per time-sliced walk and launch
constexpr int32_t kCloudSliceSteps = 256;  // steps per time-sliced point-cloud walk and launch
constexpr double kCloudWholeSteps = 4096;  // point-cloud walks known to be shorter run whole

// One slot of in-flight work: a batched launch on a stream, with its entry
// table (pinned host staging and device copy) and work counter.
struct ClassInfo {
  int inflight = 0;
  double last = -1.0;
  double ms = -1.0;            // device time of its launches, moving average (-1: none completed yet)
};

struct Slot {
  std::vector<SrvReq*> members;
  std::string cls;             // class of the launch in flight
  double issued = 0.0;         // when it was enqueued
  bool is_long = false;        // launch of a long class
  hipEvent_t t0 = nullptr;     // before the kernel (timing)
  hipEvent_t ev = nullptr;     // after the kernel and the table copy back (timing)
  BatchEntry* h_tab = nullptr;
  BatchEntry* d_tab = nullptr;
  unsigned long long* d_queue = nullptr;
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
  int n_streams = 2;           // walk streams in use; slot j runs on stream j % n_streams
  int n_long = 1;              // streams [0, n_long) take the long classes
  hipStream_t streams[mpwos::kMaxStreams] = {};
  hipStream_t done_stream = nullptr;   // per-query reductions and copies out
  mpwos::Slot slots[mpwos::kSlots];
  mpwos::HostArena arena;
  std::vector<hipEvent_t> events;      // idle events for requests
  mpwos_server_stats st = {};
  std::chrono::steady_clock::time_point t0;
};

namespace mpwos {

static double since(const mpwos_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device bytes of a request; a point-cloud request also holds its query
// check (distance to the reconstruction and local spacing per query).
static size_t request_bytes(const mpwos_request& r, int n, bool cloud) {
  size_t b = 0;
  if (cloud) b += align256((size_t)r.n_queries * 2 * sizeof(double));
  b += align256((size_t)r.n_queries * n * sizeof(double));
  b += align256((size_t)r.n_queries * r.n_walks * sizeof(double));
  b += align256((size_t)r.n_queries * r.n_walks * sizeof(int32_t));
  b += 2 * align256((size_t)r.n_queries * sizeof(double));
  b += align256(8 * sizeof(unsigned long long));
  if (fn_has_values(r.f.kind)) b += align256((size_t)r.f.n_values * sizeof(double));
  return b;
}

static hipEvent_t take_event(mpwos_server* s) {
  if (!s->events.empty()) {
    hipEvent_t e = s->events.back();
    s->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

static bool is_cloud(const SrvReq* R) { return R->args.kind == kCloud; }

// Staging bytes of R: queries and table in; u, stderr and 8 counters out;
// for a point cloud, the query check out.
static size_t staging_bytes(const SrvReq* R) {
  return HostArena::round((size_t)R->r.n_queries * R->args.n * sizeof(double)) +
         HostArena::round(R->table.size() * sizeof(double)) +
         HostArena::round((size_t)R->r.n_queries * 2 * sizeof(double)) + 8 * sizeof(unsigned long long) +
         (is_cloud(R) ? (size_t)R->r.n_queries * 2 * sizeof(double) : 0);
}

// Staging of R: queries, table, then u, stderr and the counters out.
static double* staging_out(const SrvReq* R) {
  return (double*)(R->h_io + HostArena::round((size_t)R->r.n_queries * R->args.n * sizeof(double)) +
                   HostArena::round(R->table.size() * sizeof(double)));
}

// After u, stderr and the counters: the point-cloud query check.
static double* check_out(const SrvReq* R) {
  return (double*)((char*)staging_out(R) + HostArena::round((size_t)R->r.n_queries * 2 * sizeof(double)) +
                   8 * sizeof(unsigned long long));
}

// Admission without waiting: device memory from the stream-ordered allocator
// and uploads from pinned staging, all on the completion stream, then an
// event that the first launch holding R's walks waits on.  Returns EBUSY
// (nothing done) when the staging block is full for now.
static mpwos_status admit(mpwos_server* s, SrvReq* R) {
  hipStream_t st = s->done_stream;
  R->h_io_bytes = staging_bytes(R);
  if (R->h_io_bytes > kArenaBytes / 4) {
    if (hipHostMalloc((void**)&R->h_io, R->h_io_bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      R->h_io = nullptr;
      return fail(MPWOS_ENOMEM, "server: pinned staging allocation failed");
    }
    R->h_io_own = true;
  } else {
    R->h_io = s->arena.alloc(R->h_io_bytes);
    if (!R->h_io) return MPWOS_EBUSY;
  }
  R->ready_ev = take_event(s);
  R->done_ev = take_event(s);
  if (!R->ready_ev || !R->done_ev) return fail(MPWOS_EDEVICE, "server: event creation failed");
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
  if (R->rec_bytes) R->d_state = take((size_t)R->total * R->rec_bytes);
  double* d_check = is_cloud(R) ? (double*)take((size_t)R->r.n_queries * 2 * sizeof(double)) : nullptr;
  const size_t qb = (size_t)R->r.n_queries * n * sizeof(double);
  std::memcpy(R->h_io, R->r.queries, qb);
  char* ht = R->h_io + HostArena::round(qb);
  if (!R->table.empty()) std::memcpy(ht, R->table.data(), R->table.size() * sizeof(double));
  e = hipMemcpyAsync(R->d_queries, R->h_io, qb, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && R->d_table)
    e = hipMemcpyAsync(R->d_table, ht, R->table.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_zero_u64(R->d_stats, 8, st);
  // a point-cloud request's queries are checked here, on the completion
  // stream (a check at submit would wait for the device): the verdict is
  // read when the request completes
  if (e == hipSuccess && d_check) {
    e = launch_cloud_check(R->args, R->d_queries, d_check, R->r.n_queries, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(check_out(R), d_check, (size_t)R->r.n_queries * 2 * sizeof(double), hipMemcpyDeviceToHost,
                         st);
  }
  if (e == hipSuccess) e = hipEventRecord(R->ready_ev, st);
  if (e != hipSuccess) return hip_fail(e, "server: admission copies");
  WalkArgs& a = R->args;
  a.queries = R->d_queries;
  a.nq = R->r.n_queries;
  a.nw = R->r.n_walks;
  a.q_offset = 0;
  a.walk_S = R->d_S;
  a.walk_K = R->d_K;
  if (R->d_table) a.f.values = R->d_table;
  // the batch class: every launch argument except those an entry carries
  WalkArgs k = a;
  k.queries = nullptr;
  k.nq = k.nw = k.q_offset = k.idx_base = k.count = 0;
  k.seed = 0;
  k.seed_dev = nullptr;
  k.walk_S = nullptr;
  k.walk_K = nullptr;
  k.queue = nullptr;
  k.chunk = 0;
  k.persistent = 0;
  k.batch = nullptr;
  k.n_batch = 0;
  const int32_t shape[2] = {R->opt.block_size, R->opt.lanes_per_walk};
  R->cls.assign((const char*)&k, sizeof(k));
  R->cls.append((const char*)shape, sizeof(shape));
  R->unit = batch_unit(a, R->opt);
  R->min_walks = (int64_t)s->n_cu * 16 * R->unit;   // walks that fill the device
  return MPWOS_OK;
}

// Every launch holding walks of R has completed (their events were
// observed): the reduction and the copies out are enqueued on the completion
// stream, followed by R's done event; nothing waits here.
static mpwos_status begin_finish(mpwos_server* s, SrvReq* R) {
  hipStream_t st = s->done_stream;
  double* out = staging_out(R);
  const size_t nq = (size_t)R->r.n_queries;
  hipError_t e = launch_reduce(R->d_S, R->d_K, R->r.n_queries, R->r.n_walks, R->opt.max_steps, R->d_u, R->d_se,
                               R->d_stats + 0, (int32_t*)(R->d_stats + 1), R->d_stats + 2, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, R->d_u, nq * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out + nq, R->d_se, nq * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out + 2 * nq, R->d_stats, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(R->done_ev, st);
  if (e != hipSuccess) return hip_fail(e, "server: completion");
  R->completing = true;
  return MPWOS_OK;
}

// R's done event completed: results to the caller's buffers, unless a
// point-cloud query lies farther than two local spacings from the
// reconstruction (then the request fails with EOFFMANIFOLD and its outputs
// stay untouched).
static void end_finish(SrvReq* R) {
  const double* out = staging_out(R);
  const size_t nq = (size_t)R->r.n_queries;
  if (is_cloud(R)) {
    const double* chk = check_out(R);
    for (size_t i = 0; i < nq; ++i)
      if (!(chk[2 * i] <= 2.0 * chk[2 * i + 1])) {
        R->status = MPWOS_EOFFMANIFOLD;
        return;
      }
  }
  std::memcpy(R->r.u_out, out, nq * sizeof(double));
  if (R->r.stderr_out) std::memcpy(R->r.stderr_out, out + nq, nq * sizeof(double));
  unsigned long long hs[8];
  std::memcpy(hs, out + 2 * nq, sizeof(hs));
  R->walk_steps = (int64_t)hs[0];
  if (R->status == MPWOS_OK && hs[2]) R->status = MPWOS_WTRUNC;
}

// Device memory, staging and events back; the manifold reference dropped.
// Runs after R's done event completed, or after a failure (then the device
// may still use R's memory: the completion stream is drained first).
static void release(mpwos_server* s, SrvReq* R, bool failed) {
  if (failed) (void)hipStreamSynchronize(s->done_stream);
  if (R->dev) {
    if (R->async_alloc) (void)hipFreeAsync(R->dev, s->done_stream);
    else (void)hipFree(R->dev);
  }
  R->dev = nullptr;
  if (R->h_io) {
    if (R->h_io_own) (void)hipHostFree(R->h_io);
    else s->arena.release(R->h_io, R->h_io_bytes);
  }
  R->h_io = nullptr;
  for (hipEvent_t* ev : {&R->ready_ev, &R->done_ev}) {
    if (*ev) s->events.push_back(*ev);
    *ev = nullptr;
  }
  manifold_ref(R->r.manifold, -1);
}

static int64_t walks_left(const SrvReq* R) {
  int64_t n = R->total - R->next;
  for (const auto& rg : R->resume) n += rg.second;
  return n;
}

// Walks per launch for a class: the larger of the slice budget (in Philox
// blocks; a time-sliced walk costs at most its step budget per launch) and
// what fills the device, shared out over the class's requests in arrival
// order; a request that needs less than its share leaves the rest to the
// later ones.  Every request with walks left gets at least one batch unit.
static std::vector<int64_t> batch_walks(const mpwos_server* s, const std::vector<SrvReq*>& cls) {
  const SrvReq* R0 = cls.front();
  const double k = R0->args.step_budget > 0 ? std::min(R0->k_est, (double)R0->args.step_budget) : R0->k_est;
  const double cost = std::max(1.0, k * R0->step_cost);
  int64_t cap = std::max<int64_t>((int64_t)((double)s->slice / cost), R0->min_walks);
  std::vector<int64_t> take(cls.size(), 0);
  size_t left = cls.size();
  for (size_t i = 0; i < cls.size(); ++i) {
    const SrvReq* R = cls[i];
    const int64_t share = std::max<int64_t>(cap / (int64_t)left, R->unit);
    take[i] = std::min<int64_t>(walks_left(R), share);
    cap = std::max<int64_t>(0, cap - take[i]);
    left -= 1;
  }
  return take;
}

// One batched launch of the class `cls` on slot `sl`: per request, ranges of
// unfinished time-sliced walks first (resumed from their records), then new
// walks.
static mpwos_status launch_batch(mpwos_server* s, Slot& sl, const std::vector<SrvReq*>& cls, hipStream_t st) {
  const std::vector<int64_t> take = batch_walks(s, cls);
  const int64_t unit = cls.front()->unit;
  int64_t pos = 0;
  int nb = 0;
  sl.members.clear();
  auto add = [&](SrvReq* R, int64_t idx0, int64_t count, bool resume) {
    BatchEntry& E = sl.h_tab[nb++];
    E.begin = pos;
    E.count = count;
    E.idx0 = idx0;
    E.nw = R->r.n_walks;
    E.queries = R->d_queries;
    E.walk_S = R->d_S;
    E.walk_K = R->d_K;
    E.seed = R->r.seed;
    E.state = R->d_state;
    E.resume = resume ? 1 : 0;
    E.pad = 0;
    E.pending = 0;
    pos += (count + unit - 1) / unit * unit;
    sl.members.push_back(R);
  };
  for (size_t i = 0; i < cls.size() && nb < kMaxBatch; ++i) {
    SrvReq* R = cls[i];
    int64_t want = take[i];
    while (want > 0 && !R->resume.empty() && nb < kMaxBatch) {
      const auto rg = R->resume.front();
      R->resume.pop_front();
      add(R, rg.first, rg.second, true);
      want -= rg.second;
    }
    if (want > 0 && R->next < R->total && nb < kMaxBatch) {
      const int64_t c = std::min<int64_t>(want, R->total - R->next);
      add(R, R->next, c, false);
      R->next += c;
    }
  }
  WalkArgs a = cls.front()->args;
  a.batch = sl.d_tab;
  a.n_batch = nb;
  a.count = pos;
  a.idx_base = 0;
  a.persistent = 1;
  hipError_t e = hipSuccess;
  const double now = since(s);
  for (SrvReq* R : sl.members) {
    R->inflight += 1;
    if (R->times[2] < 0) R->times[2] = now;
  }
  // members whose uploads are not known to be done: the launch waits for them
  for (SrvReq* R : sl.members)
    if (!R->ready && e == hipSuccess) e = hipStreamWaitEvent(st, R->ready_ev, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.d_tab, sl.h_tab, (size_t)nb * sizeof(BatchEntry), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(sl.t0, st);
  if (e != hipSuccess) return hip_fail(e, "server: batch table upload");
  mpwos_status ls = launch_walks(a, cls.front()->opt, st, sl.d_queue);
  if (ls) return ls;
  // the entries come back with their counts of unfinished walks
  e = hipMemcpyAsync(sl.h_tab, sl.d_tab, (size_t)nb * sizeof(BatchEntry), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(sl.ev, st);
  if (e != hipSuccess) return hip_fail(e, "server: launch event");
  return MPWOS_OK;
}

static void worker_main(mpwos_server* s) {
  (void)hipSetDevice(s->device);
  Slot* slots = s->slots;
  const int n_slots = s->n_streams * kDepth;
  std::map<std::string, ClassInfo> cinfo;   // per class: launches in flight, last launch time, launch duration
  auto last = std::chrono::steady_clock::now();
  for (;;) {
    std::vector<SrvReq*> active;
    bool busy_slot = false;
    for (int k = 0; k < n_slots; ++k) busy_slot = busy_slot || !slots[k].members.empty();
    {
      const auto now = std::chrono::steady_clock::now();
      if (busy_slot) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.busy_seconds += std::chrono::duration<double>(now - last).count();
      }
      last = now;
    }
    bool progress = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (!busy_slot)
        s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
      if (s->stop && s->pending.empty() && s->active.empty() && !busy_slot) break;
      // admission in arrival order while the budget allows
      while (!s->pending.empty()) {
        SrvReq* R = s->pending.front();
        if (!s->active.empty() && s->in_flight + R->bytes > s->budget) break;
        const mpwos_status st = admit(s, R);
        if (st == MPWOS_EBUSY) break;   // staging full: retried once completions free it
        s->pending.pop_front();
        R->times[1] = since(s);
        s->in_flight += R->bytes;
        s->active.push_back(R);
        s->st.admitted += 1;
        progress = true;
        if (st) {
          R->status = st;
          R->next = R->total;
        }
      }
      active = s->active;
      s->st.in_flight_bytes = (int64_t)s->in_flight;
    }
    // completed launches free their slots
    for (int k = 0; k < n_slots; ++k) {
      Slot& sl = slots[k];
      if (sl.members.empty()) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      auto ci = cinfo.find(sl.cls);
      float ms = 0.f;
      if (ci != cinfo.end() && q == hipSuccess && hipEventElapsedTime(&ms, sl.t0, sl.ev) == hipSuccess)
        ci->second.ms = ci->second.ms < 0 ? ms : 0.7 * ci->second.ms + 0.3 * ms;
      if (ci != cinfo.end() && --ci->second.inflight <= 0 && ci->second.last < since(s) - 60.0) cinfo.erase(ci);
      for (size_t i = 0; i < sl.members.size(); ++i) {
        SrvReq* R = sl.members[i];
        if (q != hipSuccess && R->status >= 0) R->status = hip_fail(q, "server: batched launch");
        if (q == hipSuccess && sl.h_tab[i].pending > 0) R->resume.emplace_back(sl.h_tab[i].idx0, sl.h_tab[i].count);
        R->inflight -= 1;
      }
      sl.members.clear();
      progress = true;
    }
    // uploads observed done; requests whose walks have all completed start
    // their reduction; those whose copies out are done finish
    std::vector<SrvReq*> done;
    for (SrvReq* R : active) {
      if (!R->ready && R->ready_ev && hipEventQuery(R->ready_ev) == hipSuccess) R->ready = true;
      if (R->status >= 0 && (R->next < R->total || !R->resume.empty())) continue;
      if (R->inflight > 0) continue;
      if (R->times[3] < 0) R->times[3] = since(s);
      if (!R->completing && R->status >= 0) {
        const mpwos_status st = begin_finish(s, R);
        if (st) R->status = st;
        else continue;
      }
      if (R->completing && R->status >= 0) {
        const hipError_t q = hipEventQuery(R->done_ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) R->status = hip_fail(q, "server: completion");
        else end_finish(R);
      }
      release(s, R, R->status < 0);
      done.push_back(R);
      progress = true;
    }
    // classes of the requests with walks left, in order of their oldest request
    std::vector<std::vector<SrvReq*>> classes;
    {
      std::map<std::string, size_t> where;
      for (SrvReq* R : active) {
        if (R->status < 0 || walks_left(R) == 0) continue;
        auto it = where.find(R->cls);
        if (it == where.end()) {
          where.emplace(R->cls, classes.size());
          classes.push_back({R});
        } else if (classes[it->second].size() < (size_t)kMaxBatch) {
          classes[it->second].push_back(R);
        }
      }
    }
    // Free slots go to the classes least recently served: those with fewer
    // launches in flight first, then the one whose last launch is oldest.  A
    // long class (launches above kLongMs) runs on the long streams only; a
    // short one on the other streams, or on an idle long stream, never behind
    // a long launch.  Among the streams allowed, an idle one first (for a
    // short class an idle short stream before an idle long one), then the one
    // whose launch in flight was issued first.
    std::vector<char> skip(classes.size(), 0);
    for (;;) {
      int best = -1;
      for (size_t t = 0; t < classes.size(); ++t) {
        auto& c = classes[t];
        c.erase(std::remove_if(c.begin(), c.end(), [](SrvReq* R) { return walks_left(R) == 0; }), c.end());
        if (c.empty() || skip[t]) continue;
        if (best < 0) {
          best = (int)t;
          continue;
        }
        const ClassInfo& a = cinfo[c.front()->cls];
        const ClassInfo& b = cinfo[classes[best].front()->cls];
        if (a.inflight < b.inflight || (a.inflight == b.inflight && a.last < b.last)) best = (int)t;
      }
      if (best < 0) break;
      auto& c = classes[best];
      const bool want_long = cinfo[c.front()->cls].ms > kLongMs;
      int k = -1, best_rank = 3;
      double best_issued = 1e300;
      for (int sx = 0; sx < s->n_streams; ++sx) {
        int free_slot = -1, busy = 0;
        bool has_long = false;
        double issued = 1e300;
        for (int d = 0; d < kDepth; ++d) {
          const Slot& sl = slots[sx + d * s->n_streams];
          if (sl.members.empty()) {
            if (free_slot < 0) free_slot = sx + d * s->n_streams;
            continue;
          }
          busy += 1;
          has_long = has_long || sl.is_long;
          issued = std::min(issued, sl.issued);
        }
        const bool long_stream = sx < s->n_long;
        if (free_slot < 0 || (want_long && !long_stream) || (!want_long && (has_long || (long_stream && busy))))
          continue;
        const int rank = busy ? 2 : (long_stream == want_long ? 0 : 1);
        if (rank < best_rank || (rank == best_rank && issued < best_issued)) {
          best_rank = rank;
          best_issued = issued;
          k = free_slot;
        }
      }
      if (k < 0) {
        skip[best] = 1;
        continue;
      }
      Slot& sl = slots[k];
      mpwos_status ls = launch_batch(s, sl, c, s->streams[k % s->n_streams]);
      ClassInfo& ci = cinfo[c.front()->cls];
      ci.last = since(s);
      if (ls) {
        for (SrvReq* R : c) {
          if (R->status >= 0) R->status = ls;
          R->next = R->total;
          R->resume.clear();
        }
        for (SrvReq* R : sl.members) R->inflight -= 1;
        sl.members.clear();
        continue;
      }
      sl.cls = c.front()->cls;
      sl.issued = ci.last;
      sl.is_long = want_long;
      ci.inflight += 1;
      progress = true;
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.rounds += 1;
    }
    if (!done.empty()) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        const double now = since(s);
        for (SrvReq* R : done) {
          R->times[4] = now;
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
      // launches still running: look again shortly, or sooner when work arrives
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(100));
    }
  }
}

}  // namespace mpwos

using namespace mpwos;

// Streams, slot tables and the server object (the worker has ended).
static void free_server(mpwos_server* s) {
  for (auto& st : s->streams)
    if (st) (void)hipStreamSynchronize(st);
  if (s->done_stream) (void)hipStreamSynchronize(s->done_stream);
  for (int k = 0; k < kSlots; ++k) {
    Slot& sl = s->slots[k];
    if (sl.t0) (void)hipEventDestroy(sl.t0);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.h_tab) (void)hipHostFree(sl.h_tab);
    if (sl.d_tab) (void)hipFree(sl.d_tab);
    if (sl.d_queue) (void)hipFree(sl.d_queue);
  }
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  if (s->arena.base) (void)hipHostFree(s->arena.base);
  for (auto& st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->done_stream) (void)hipStreamDestroy(s->done_stream);
  delete s;
}

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
  // The runtime shares hardware queues between streams beyond
  // GPU_MAX_HW_QUEUES (default 4), and kernels of streams that share a queue
  // run one after another.  With queues for at least six walk streams beside
  // the null stream and the completion stream, the walk streams are ordinary
  // ones (up to eight); with fewer, six streams are created with a CU mask
  // covering every CU, which the runtime gives queues of their own.
  int hwq = 4;
  if (const char* v = std::getenv("GPU_MAX_HW_QUEUES"))
    if (std::atoi(v) > 0) hwq = std::atoi(v);
  bool masked = false;
  if (hwq - 2 >= kMinStreams) {
    s->n_streams = std::min(kMaxStreams, hwq - 2);
    for (int i = 0; e == hipSuccess && i < s->n_streams; ++i)
      e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
  } else {
    s->n_streams = kMinStreams;
    uint32_t all[16];
    for (uint32_t& w : all) w = 0xFFFFFFFFu;
    masked = true;
    for (int i = 0; masked && i < s->n_streams; ++i)
      masked = hipExtStreamCreateWithCUMask(&s->streams[i], 16, all) == hipSuccess;
    if (!masked) {
      // ordinary streams on the queues there are
      (void)hipGetLastError();
      for (auto& st : s->streams)
        if (st) (void)hipStreamDestroy(st);
      for (auto& st : s->streams) st = nullptr;
      s->n_streams = std::max(2, std::min(kMaxStreams, hwq - 2));
      for (int i = 0; e == hipSuccess && i < s->n_streams; ++i)
        e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    }
  }
  s->n_long = std::max(1, s->n_streams / 2);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->done_stream, hipStreamNonBlocking);
  for (int k = 0; e == hipSuccess && k < s->n_streams * kDepth; ++k) {
    Slot& sl = s->slots[k];
    e = hipEventCreateWithFlags(&sl.t0, hipEventDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_tab, kMaxBatch * sizeof(BatchEntry), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_tab, kMaxBatch * sizeof(BatchEntry));
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_queue, 256);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->arena.base, kArenaBytes, hipHostMallocDefault);
  if (e == hipSuccess) {
    s->arena.size = kArenaBytes;
    s->arena.free_[0] = kArenaBytes;
  }
  if (e != hipSuccess) {
    free_server(s);
    return hip_fail(e, "server: streams and launch tables");
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
  if (fn_has_values(req->f.kind) && req->f.values && req->f.n_values > 0)
    R->table.assign(req->f.values, req->f.values + req->f.n_values);
  mpwos_status st = prepare_solve(req->manifold, &R->r.f, g, req->c, req->n_queries, req->n_walks, req->eps,
                                  req->seed, R->opt, R->args);
  // analytic manifolds: the host check; point clouds are checked on the
  // device at admission (see admit)
  if (!st && manifold_desc(req->manifold).kind != MPWOS_POINT_CLOUD)
    st = check_queries_host(req->manifold, R->args, req->queries, req->n_queries);
  if (st) {
    delete R;
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected += 1;
    return st;
  }
  const int n = R->args.n;
  R->total = req->n_queries * req->n_walks;
  R->bytes = request_bytes(*req, n, R->args.kind == kCloud);
  if (R->bytes > s->budget) {
    delete R;
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected += 1;
    return fail(MPWOS_ENOMEM, "request needs " + std::to_string(R->bytes) + " bytes, above the HBM budget");
  }
  if (R->args.const_r) R->k_est = std::ceil(std::log(R->opt.tau_w) / std::log(R->args.c0));
  R->step_cost = philox_blocks_per_step(n, R->opt.n_v);
  // Long lane-group walks are time-sliced: a launch runs each for at most
  // kSliceBlocks Philox blocks of work, so that no launch holds a stream (and
  // whatever shares its hardware queue) for long.  Point-cloud lane walks
  // (every step is nearest-point lookups: a walk of 1601 steps holds a launch
  // for about half a second) run kCloudSliceSteps steps per launch when their
  // length is not known to stay below kCloudWholeSteps: a radius that varies
  // per step (the spacing rule gives walks of about 1e6 steps on a dense
  // cloud), or a constant one with longer walks.  Shorter cloud walks run
  // whole: slicing them only adds launches between the slices.  The state
  // records must fit an eighth of the budget; otherwise the walks run to the
  // end in one launch.
  if (n >= 4) {
    const double budget = std::max(256.0, kSliceBlocks / R->step_cost);
    const int64_t rec = group_record_bytes(n, R->opt.lanes_per_walk, R->args.precision == 0);
    if (R->k_est > 1.5 * budget && rec > 0 && (size_t)(R->total * rec) <= s->budget / 8) {
      R->args.step_budget = (int32_t)budget;
      R->rec_bytes = rec;
      R->bytes += align256((size_t)R->total * rec);
    }
  } else if (R->args.kind == kCloud && (!R->args.const_r || R->k_est > kCloudWholeSteps) &&
             (size_t)(R->total * kLaneRecordBytes) <= s->budget / 8) {
    R->args.step_budget = kCloudSliceSteps;
    R->rec_bytes = kLaneRecordBytes;
    R->bytes += align256((size_t)R->total * kLaneRecordBytes);
  }
  manifold_ref(req->manifold, +1);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      manifold_ref(req->manifold, -1);
      delete R;
      return fail(MPWOS_EBUSY, "server is shutting down");
    }
    R->ticket = s->next_ticket++;
    R->times[0] = since(s);
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

mpwos_status mpwos_request_times(mpwos_server* s, uint64_t ticket, double times[5]) {
  if (!s || !times) return fail(MPWOS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(MPWOS_EINVAL, "unknown ticket");
  for (int i = 0; i < 5; ++i) times[i] = it->second->times[i];
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
  free_server(s);
  return MPWOS_OK;
}

}  // extern "C"
