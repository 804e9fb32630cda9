// Internal interfaces between the host translation units of the solver.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "kernel_args.h"
#include "mpwos.h"

namespace mpwos {

struct CloudState;

mpwos_status fail(mpwos_status st, const std::string& msg);
// Families whose host `values` array is copied to the device with the solve.
inline bool fn_has_values(int kind) {
  return kind == MPWOS_FN_TABLE_S1 || kind == MPWOS_FN_DUMBBELL_POLY || kind == MPWOS_FN_TORUS_SINE;
}
mpwos_status hip_fail(hipError_t e, const char* what);
int device_cu_count();
void manifold_ref(const mpwos_manifold* m, int d);
const mpwos_manifold_desc& manifold_desc(const mpwos_manifold* m);

struct TableSink;
// Validates a solve and fills the kernel arguments (except buffers).  With a
// sink, an inverse table that is not cached goes to the sink's device region
// instead of a new allocation.
mpwos_status prepare_solve(const mpwos_manifold* man, const mpwos_fn* f, const mpwos_fn* g, double sigma,
                           int64_t nq, int64_t nw, double eps, uint64_t seed, const mpwos_options& o,
                           WalkArgs& a, TableSink* sink = nullptr);
mpwos_status launch_walks(WalkArgs& a, const mpwos_options& o, hipStream_t s, unsigned long long* queue);
// Walks per batch unit of a batched launch: every entry begins on a multiple.
int64_t batch_unit(const WalkArgs& a, const mpwos_options& o);
// Philox blocks one walk-step draws (a cost estimate for sizing work): one
// per sub-stream for n <= 3, the normal pairs and radius word for n >= 4.
double philox_blocks_per_step(int n, int n_v);
// Every point-cloud query within two local spacings of the reconstruction.
// With a device buffer (out, out_cap doubles) the check runs in batches in
// it and allocates no device memory.
mpwos_status cloud_check_queries(const WalkArgs& a, const double* dq, int64_t nq, hipStream_t s,
                                 double* out = nullptr, int64_t out_cap = 0);
mpwos_status check_queries_host(const mpwos_manifold* man, const WalkArgs& a, const double* q, int64_t nq);
// The point-cloud query check on a stream, without waiting: per query the
// distance to its FP64 projection and the local spacing there (2 doubles).
hipError_t launch_cloud_check(const WalkArgs& a, const double* dq, double* out, int64_t nq, hipStream_t s);

// query_check.hip: the analytic manifolds' query check on the device; slot
// (zeroed by the caller) ends at n_q - (first failing query), or 0
bool device_query_check(int kind);
hipError_t launch_query_check(const mpwos_manifold_desc& d, const double* q, int64_t nq, unsigned long long* slot,
                              hipStream_t s);

// khist.hip: histogram of the per-walk K^i (exact below kKHistExact, then
// 128 bins per octave up to 2^31) and its nearest-rank p50 / p99
constexpr int kKHistExact = 2048;
constexpr int kKHistBins = kKHistExact + 20 * 128;
hipError_t launch_khist(const int32_t* K, int64_t n, unsigned long long* hist, hipStream_t s);
int32_t khist_lower(int bin);
void khist_quantiles(const unsigned long long* hist, int32_t& p50, int32_t& p99);

// walk_lane.hip
hipError_t launch_walk_lane(const WalkArgs& a, int grid, int block, hipStream_t s);
int lane_occupancy(const WalkArgs& a, int block);
hipError_t launch_reduce(const double* walk_S, const int32_t* walk_K, int64_t nq, int64_t nw, int64_t max_steps,
                         double* u, double* se, unsigned long long* ksum, int32_t* kmax,
                         unsigned long long* ntrunc, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_set_u64(unsigned long long* p, unsigned long long v, hipStream_t s);
hipError_t launch_cp_points(const WalkArgs& a, const double* x, double* y, int64_t m, hipStream_t s);
hipError_t launch_radial_inv(const WalkArgs& a, const double* u, double* s_out, int64_t m, int fp64,
                             hipStream_t s);
hipError_t launch_philox(const uint32_t* c, uint64_t seed, uint32_t* out, int64_t m, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);
hipError_t launch_valu_probe(int op, uint32_t seed, int32_t iters, uint32_t* out, int blocks, hipStream_t s);

// walk_group.hip
mpwos_status launch_group_walks(WalkArgs& a, const mpwos_options& o, hipStream_t s, unsigned long long* queue);
void group_shape(int n, int lanes_req, int& L, int& mb, int& nblk, int& rblk, int& rword);
hipError_t launch_cp_group(const WalkArgs& a, const double* x, double* y, int64_t m, hipStream_t s);
hipError_t launch_ct_nodes(double R, double a, double cut_c, double cut_s, int nt, int ns, double* out,
                           hipStream_t s);
hipError_t launch_ts_fit(const double* U, int nt, int ns, int kt, int ks, double* coef, hipStream_t s);
// Bytes of the state record of one time-sliced walk (0 for an unsupported shape).
int64_t group_record_bytes(int n, int lanes_req, bool fp64);

// cloud.hip
mpwos_status cloud_create(const mpwos_manifold_desc& d, hipStream_t s, CloudState** out);
void cloud_destroy(CloudState* c);
double cloud_spacing_rmax(const CloudState* c, const mpwos_options& o);
void cloud_fill_args(const CloudState* c, const mpwos_options& o, WalkArgs& a);
int64_t cloud_fallback_points(const CloudState* c);
double cloud_max_spacing(const CloudState* c);
int cloud_nn_only(const CloudState* c);

}  // namespace mpwos
