// One lane per walk (n <= 3): the whole walk state (Y, W, S, k) lives in
// registers; each iteration of the loop is one step of Algorithm 1.
//
// Two launch forms share the step code:
//   plain      - one walk per lane, grid covers every walk, one launch per solve;
//   persistent - a grid sized to the device; a lane whose walk stops takes the
//                next walk index from a per-wave chunk of a global queue, so
//                uneven walk lengths (boundary problems) keep lanes busy.
#include <hip/hip_runtime.h>

#include "cloud_dev.h"
#include "kernel_args.h"
#include "mpwos_dev.h"

namespace mpwos {

template <class T, int N>
struct LaneState {
  T Y[N];
  double W, S, C;
  T rg;                // point cloud: rho_geo from the reconstruction that produced Y; cap: delta_Gamma(Y)
  int32_t pidx;        // point cloud: the patch that holds Y (start of the next projections)
  uint32_t k, q, w;
  int64_t idx;
};

// ---- geometry of the sphere cap (n <= 3) ----------------------------------
// Gamma = S_R cap {x_n = h}; y_Gamma is the nearest point of Gamma; the
// effective distance is the distance to the normal disk of radius ell at
// y_Gamma (eq. extended_boundary_disk, eq. delta_Gamma_general).
// The uniform constants (sqrt(R^2 - h^2), 1/R, ell) come precomputed.
template <class T, int N>
__device__ __forceinline__ void cap_gamma_point(const WalkArgs& a, const T* y, T* yg) {
  const T rg = (T)a.cap_rg;
  T s = (T)0;
  for (int i = 0; i < N - 1; ++i) s += y[i] * y[i];
  const T is = rsqrt_(s);
  for (int i = 0; i < N - 1; ++i) yg[i] = rg * y[i] * is;
  yg[N - 1] = (T)a.p[1];
}

template <class T, int N>
__device__ __forceinline__ T cap_delta(const WalkArgs& a, const T* y, T* yg) {
  cap_gamma_point<T, N>(a, y, yg);
  // r = y_Gamma - y splits into rn along the normal y_Gamma / R and the
  // tangential rest, |r^T|^2 = |r|^2 - rn^2 (rn^2 is the smaller term: no
  // cancellation)
  T rr = (T)0, rn = (T)0;
  for (int i = 0; i < N; ++i) {
    const T d = yg[i] - y[i];
    rr += d * d;
    rn += d * yg[i];
  }
  rn *= (T)a.inv_R;
  T rt2 = rr - rn * rn;
  rt2 = rt2 > (T)0 ? rt2 : (T)0;
  // ell = c_kappa / (1 + kappa) with kappa = 1/R, the same as rho_geo
  const T ell = (T)a.rho_geo;
  T tn = abs_(rn) - ell;
  tn = tn > (T)0 ? tn : (T)0;
  return sqrt_(rt2 + tn * tn);
}

// Membership of the boundary layer, in the walk's precision; dg receives
// delta_Gamma(y) when y is above the cutting plane (the next step's radius
// reuses it), yg the nearest point of Gamma when y is in the layer (the
// boundary datum is taken there).
template <class T, int N>
__device__ __forceinline__ bool cap_in_layer(const WalkArgs& a, const T* y, T& dg, T* yg) {
  if (y[N - 1] <= (T)a.p[1]) {
    cap_gamma_point<T, N>(a, y, yg);
    return true;
  }
  dg = cap_delta<T, N>(a, y, yg);
  return dg < (T)a.eps;
}

// ---- geometry of the torus with a planar cut --------------------------------
// Omega = {0 < s < pi}, s = phi - phi_c; Gamma is the two tube circles s = 0
// and s = pi.  y_Gamma is the nearer of the two circles' nearest points; the
// torus normal there is the unit vector from the circle's centre.  FP64 in
// both precisions (a handful of operations per step).
__device__ __forceinline__ void ct_gamma_point(const WalkArgs& a, const double* y, double* yg, double* ng) {
  const double R = a.p[0], tube = a.p[1];
  double best = 0.0;
  for (int b = 0; b < 2; ++b) {
    const double ex = b ? -a.cut_c : a.cut_c, ey = b ? -a.cut_s : a.cut_s;
    const double pe = y[0] * ex + y[1] * ey - R, pz = y[2];
    const double d = sqrt(pe * pe + pz * pz);
    const double n0 = ex * pe / d, n1 = ey * pe / d, n2 = pz / d;
    const double q0 = R * ex + tube * n0, q1 = R * ey + tube * n1, q2 = tube * n2;
    const double dd = (q0 - y[0]) * (q0 - y[0]) + (q1 - y[1]) * (q1 - y[1]) + (q2 - y[2]) * (q2 - y[2]);
    if (b == 0 || dd < best) {
      best = dd;
      yg[0] = q0; yg[1] = q1; yg[2] = q2;
      ng[0] = n0; ng[1] = n1; ng[2] = n2;
    }
  }
}

// effective distance to the normal segment of half-length ell = rho_geo(y_Gamma)
// (the manifold's constant curvature indicator 1/a)
__device__ __forceinline__ double ct_delta(const WalkArgs& a, const double* y) {
  double yg[3], ng[3];
  ct_gamma_point(a, y, yg, ng);
  const double r0 = yg[0] - y[0], r1 = yg[1] - y[1], r2 = yg[2] - y[2];
  const double rn = r0 * ng[0] + r1 * ng[1] + r2 * ng[2];
  const double t0 = r0 - rn * ng[0], t1 = r1 - rn * ng[1], t2 = r2 - rn * ng[2];
  double tn = fabs(rn) - a.rho_geo;
  tn = tn > 0.0 ? tn : 0.0;
  return sqrt(t0 * t0 + t1 * t1 + t2 * t2 + tn * tn);
}

// Membership of the boundary layer; the far side of the cut (sin s <= 0)
// counts as inside.  dg receives delta_Gamma(y) otherwise.
template <class T>
__device__ __forceinline__ bool ct_in_layer(const WalkArgs& a, const T* y, T& dg) {
  const double yd[3] = {(double)y[0], (double)y[1], (double)y[2]};
  if (!(yd[1] * a.cut_c - yd[0] * a.cut_s > 0.0)) return true;
  const double d = ct_delta(a, yd);
  dg = (T)d;
  return d < a.eps;
}

// Boundary layer test, by manifold: true when y is in the layer, with g the
// boundary datum at y's nearest point of Gamma; dg as for the tests above.
template <class T, int N, int KIND>
__device__ __forceinline__ bool layer_stop(const WalkArgs& a, const T* y, T& dg, double& g) {
  T yg[N];
  if constexpr (KIND == kCutTorus) {
    if (!ct_in_layer<T>(a, y, dg)) return false;
    const double yd[3] = {(double)y[0], (double)y[1], (double)y[2]};
    double gd[3], nd[3];
    ct_gamma_point(a, yd, gd, nd);
    for (int i = 0; i < 3; ++i) yg[i] = (T)gd[i];
  } else {
    if (!cap_in_layer<T, N>(a, y, dg, yg)) return false;
  }
  g = boundary_value<T>(a, yg, N);
  return true;
}

// ---- closest point ----------------------------------------------------------
// (point clouds: `start` is the patch the search for x's patch starts from,
// the walker's, or -1 for the cloud point nearest to x)
template <class T, int N, int KIND>
__device__ __forceinline__ void closest_point(const WalkArgs& a, const T* x, T* y, int32_t start = -1) {
  if constexpr (KIND == kCutTorus) {
    // the parametrized torus of the cut example: the nearest point of the
    // core circle, then the tube radius along the offset (closed form)
    const T R = (T)a.p[0], tube = (T)a.p[1];
    const T f = R * rsqrt_(x[0] * x[0] + x[1] * x[1]);
    const T c0 = x[0] * f, c1 = x[1] * f;
    const T d0 = x[0] - c0, d1 = x[1] - c1, d2 = x[2];
    const T g = tube * rsqrt_(d0 * d0 + d1 * d1 + d2 * d2);
    y[0] = c0 + g * d0;
    y[1] = c1 + g * d1;
    y[2] = g * d2;
  } else if constexpr (KIND == kTorus) {
    torus_cp_newton<T>((T)a.p[0], (T)a.p[1], x, y);
  } else if constexpr (KIND == kCloud) {
    const CloudProj<T> p = cloud_cp<T>(a.cloud, x, start);
    for (int i = 0; i < 3; ++i) y[i] = p.y[i];
  } else {
    T s = (T)0;
    for (int i = 0; i < N; ++i) s += x[i] * x[i];
    const T f = (T)a.p[0] * rsqrt_(s);
    for (int i = 0; i < N; ++i) y[i] = x[i] * f;
  }
}

// ---- one walk ---------------------------------------------------------------
// Walk idx (= q_local * nw + w) of a launch whose queries start at global
// query q_offset.
template <class T, int N, int KIND>
__device__ __forceinline__ bool walk_init(const WalkArgs& a, const double* queries, int64_t nw, int64_t q_offset,
                                          int64_t idx, LaneState<T, N>& st) {
  st.idx = idx;
  const int64_t ql = idx / nw;
  st.q = (uint32_t)(ql + q_offset);
  st.w = (uint32_t)(idx - ql * nw);
  const double* y0 = queries + ql * N;
  for (int i = 0; i < N; ++i) st.Y[i] = (T)y0[i];
  st.W = 1.0;
  st.S = 0.0;
  st.C = 0.0;
  st.k = 0;
  st.rg = (T)0;
  st.pidx = -1;
  if constexpr (KIND == kCloud) {
    // the walk starts from the query's projection onto the reconstruction
    const CloudProj<T> p = cloud_cp<T>(a.cloud, st.Y);
    for (int i = 0; i < N; ++i) st.Y[i] = p.y[i];
    st.pidx = p.patch;
    if (!a.const_r) st.rg = (T)cloud_rho_geo(a, p);
  }
  if constexpr (KIND == kCap || KIND == kCutTorus) {
    double g;
    if (layer_stop<T, N, KIND>(a, st.Y, st.rg, g)) {
      st.S = g;
      return true;
    }
  }
  return false;
}

// S += x in FP64: with Neumaier compensation in the FP64 mode (the oracle's
// summation); a plain FP64 sum in the FP32 mode, whose rounding (K eps
// relative) is far below the FP32 walk arithmetic's.
template <class T, class St>
__device__ __forceinline__ void score_add(St& st, double x) {
  if constexpr (sizeof(T) == 8) kahan_add(st.S, st.C, x);
  else st.S += x;
}

template <class T, int N>
__device__ __forceinline__ void walk_store(double* walk_S, int32_t* walk_K, const LaneState<T, N>& st) {
  walk_S[st.idx] = st.S + st.C;
  walk_K[st.idx] = (int32_t)st.k;
}

// Record of a time-sliced lane walk (serving), kLaneRecord bytes per request
// walk: W, S, C; k and the finished flag; the patch index; Y and rg in the
// walk's precision (kLaneRecordBytes in all).  The step sequence continues
// unchanged from a record, so a sliced walk ends with the bits of an
// unsliced one.
constexpr int64_t kLaneRecord = kLaneRecordBytes;
static_assert(40 + 3 * 8 <= 64 && 64 + 8 <= kLaneRecord, "lane record layout");

template <class T, int N>
__device__ __forceinline__ void lane_save(char* rec, const LaneState<T, N>& st, uint32_t finished) {
  double* d = (double*)rec;
  uint32_t* u = (uint32_t*)(rec + 24);
  u[1] = finished;
  if (finished) return;
  d[0] = st.W;
  d[1] = st.S;
  d[2] = st.C;
  u[0] = st.k;
  ((int32_t*)(rec + 32))[0] = st.pidx;
  T* y = (T*)(rec + 40);
  for (int i = 0; i < N; ++i) y[i] = st.Y[i];
  *(T*)(rec + 64) = st.rg;
}

// false when the walk finished in an earlier launch
template <class T, int N>
__device__ __forceinline__ bool lane_load(const char* rec, int64_t nw, int64_t idx, LaneState<T, N>& st) {
  const uint32_t* u = (const uint32_t*)(rec + 24);
  if (u[1]) return false;
  st.idx = idx;
  const int64_t ql = idx / nw;
  st.q = (uint32_t)ql;
  st.w = (uint32_t)(idx - ql * nw);
  const double* d = (const double*)rec;
  st.W = d[0];
  st.S = d[1];
  st.C = d[2];
  st.k = u[0];
  st.pidx = ((const int32_t*)(rec + 32))[0];
  const T* y = (const T*)(rec + 40);
  for (int i = 0; i < N; ++i) st.Y[i] = y[i];
  st.rg = *(const T*)(rec + 64);
  return true;
}

// One Green sample Z = Y + t zeta' (t = r s, s from the radial law for the
// uniform word ux, zeta' from words x, y of block b) and (f + m)(Z).
template <class T, int N, int KIND, bool RICH>
__device__ __forceinline__ T green_sample(const WalkArgs& a, const T* Y, uint4 b, uint32_t ux, T rT, T X2,
                                          double norm, const float4* tab, int32_t pidx) {
  T s;
  if constexpr (sizeof(T) == 8) s = radial_inv64(a, u01_64(ux), X2, norm);
  else s = radial_inv32(a, u01_32(ux), X2);
  const T t = rT * s;
  T Z[N], Zc[N];
  lane_point<N>(b.x, b.y, t, Y, Z);
  closest_point<T, N, KIND>(a, Z, Zc, pidx);
  if constexpr (KIND == kCutTorus) {
    // the cut torus takes the series family (from the workgroup's staged
    // table when there is one) or ZERO / CONST: no other family is compiled in
    if constexpr (RICH) {
      if (a.f.kind == kFnTorusSine) return torus_sine_source<T>(a, Z, Zc, tab);
    }
    return source<T, false>(a, Z, Zc, N);
  }
  return source<T, RICH>(a, Z, Zc, N);
}

template <class T, int N, int KIND, bool RICH>
__device__ __forceinline__ bool walk_step(const WalkArgs& a, LaneState<T, N>& st, uint64_t seed,
                                          const float4* tab = nullptr) {
  const Stream rs{st.q, st.w, (uint32_t)seed, (uint32_t)(seed >> 32)};
  // (i) radius r(Y) = theta min(delta_Gamma, rho_geo) and the weights; a
  // per-step radius is computed in the walk's precision (its step factors c
  // and omega too), the constant one comes from the host in FP64
  double r, c, om, norm = 0.0;
  T X2;
  constexpr bool kStepRadius = KIND == kCap || KIND == kCutTorus || KIND == kCloud;
  if (kStepRadius && (KIND != kCloud || !a.const_r)) {
    T rs;
    if constexpr (KIND == kCloud) {
      rs = (T)a.theta * st.rg;
    } else {
      // delta_Gamma(Y) from the previous step's stop test (or the start)
      const T rg = (T)a.rho_geo;
      rs = (T)a.theta * (st.rg < rg ? st.rg : rg);
    }
    if constexpr (sizeof(T) == 4) {
      float cf, omf;
      weights32<N>(a, rs, cf, omf);
      c = (double)cf;
      om = (double)omf;
      X2 = (float)a.sigma * rs * rs;
    } else {
      weights(a, rs, c, om);
      X2 = a.sigma * rs * rs;
      norm = radial_norm(a.law, X2);
    }
    r = (double)rs;
  } else {
    r = a.r0;
    c = a.c0;
    om = a.om0;
    X2 = (T)(a.X0 * a.X0);
  }
  const T rT = (T)r;
  // Each Philox block is drawn where it is used.  (Drawing the first Green
  // sample's block together with the direction block, to interleave their
  // rounds, changed FP64 cap results with this toolchain although the values
  // are the same by construction; the multiple-Green-sample parity test
  // guards the form kept here.)
  const uint4 bd = rs.block(st.k, 0, 0);
  // (ii) Theta = Y + r zeta and Y' = cp(Theta)
  T Yn[N];
  T rg_next = (T)0;
  int32_t pidx_next = -1;
  {
    T Th[N];
    lane_point<N>(bd.x, bd.y, rT, st.Y, Th);
    if constexpr (KIND == kCloud) {
      const CloudProj<T> p = cloud_cp<T>(a.cloud, Th, st.pidx);
      for (int i = 0; i < N; ++i) Yn[i] = p.y[i];
      pidx_next = p.patch;
      if (!a.const_r) rg_next = (T)cloud_rho_geo(a, p);
    } else {
      closest_point<T, N, KIND>(a, Th, Yn);
    }
  }
  // Green samples Z ~ rho(Y, .): radius from the radial law, direction uniform
  T Fsum = (T)0;
  for (int l = 1; l <= a.n_v; ++l) {
    const uint4 b = rs.block(st.k, (uint32_t)l, 0);
    Fsum += green_sample<T, N, KIND, RICH>(a, st.Y, b, b.w, rT, X2, norm, tab, st.pidx);
  }
  // the mean over the N_V samples (times 1/N_V: exact for N_V = 1 and powers
  // of two, within an ulp of the quotient otherwise)
  const double F = (double)Fsum * a.inv_nv;
  score_add<T>(st, (st.W * om) * F);
  st.W = st.W * c;
  for (int i = 0; i < N; ++i) st.Y[i] = Yn[i];
  if constexpr (KIND == kCloud) {
    st.rg = rg_next;
    st.pidx = pidx_next;
  }
  st.k += 1;
  if constexpr (KIND == kCap || KIND == kCutTorus) {
    double g;
    if (layer_stop<T, N, KIND>(a, st.Y, st.rg, g)) {
      score_add<T>(st, st.W * g);
      return true;
    }
  } else {
    // a non-finite weight (NaN from a degenerate projection) also ends the walk
    if (!(st.W >= a.tau_w)) return true;
  }
  // a non-finite state ends the walk instead of running it to max_steps
  if (!(st.Y[0] == st.Y[0])) return true;
  return (int64_t)st.k >= a.max_steps;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// The cap kernel is held to 80 VGPRs (6 waves per SIMD instead of 5): its
// walks are short, and the refill and stop paths want the latency hiding.
template <class T, int N, int KIND, bool PERSIST, bool RICH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KIND == kCap && sizeof(T) == 4 ? 6 : 1)))
void walk_lane_kernel(WalkArgs a) {
  const int64_t total = a.count;
  const uint64_t seed = a.seed_dev ? *a.seed_dev : a.seed;
  LaneState<T, N> st;
  // cut torus, FP32: the source series staged in LDS once per workgroup
  // (before any lane leaves)
  const float4* tab = nullptr;
  if constexpr (KIND == kCutTorus && RICH && sizeof(T) == 4) {
    __shared__ float4 ts_tab[kTsLds];
    if (ts_stage(a, ts_tab)) tab = ts_tab;
  }
  if constexpr (!PERSIST) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    if (walk_init<T, N, KIND>(a, a.queries, a.nw, a.q_offset, a.idx_base + idx, st)) {
      walk_store(a.walk_S, a.walk_K, st);
      return;
    }
    while (!walk_step<T, N, KIND, RICH>(a, st, seed, tab)) {
    }
    walk_store(a.walk_S, a.walk_K, st);
    return;
  } else {
    // persistent form: per-wave chunks of the global queue.  A refill pass
    // costs the whole wave the issue of a walk's start (and the steps in
    // between carry its stop), so idle lanes are refilled together once at
    // least kRefillIdle of them wait (or the wave is empty): with walks of
    // 28 steps on average (the cap) a wave otherwise refills on almost
    // every step.
    constexpr int kRefillIdle = 12;
    const uint32_t lane = lane_id();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool active = false;
    bool exhausted = false;
    int64_t next = 0, end = 0;
    for (;;) {
      const uint64_t idle = __ballot(!active);
      if (!exhausted && (__popcll(idle) >= kRefillIdle || idle == ~0ull)) {
        // the idle lanes take their walk indices first (from the wave's chunk,
        // and further chunks while it runs out), then start those walks
        // together: the loop over chunks carries indices only, not the walk
        // state.  A walk that starts in the boundary layer ends here; its lane
        // waits for the next pass.
        int64_t mine = -1;
        bool need = !active;
        for (;;) {
          const uint64_t want = __ballot(need);
          if (want == 0) break;
          if (next >= end) {
            const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)want) - 1);
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)a.chunk);
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)base, leader);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), leader);
            const int64_t b = (int64_t)(((uint64_t)hi << 32) | lo);
            if (b >= total) {
              exhausted = true;
              break;
            }
            next = b;
            end = b + a.chunk < total ? b + a.chunk : total;
          }
          const int rank = __popcll(want & lt_mask);
          const int64_t avail = end - next;
          const int64_t cnt = (int64_t)__popcll(want) < avail ? (int64_t)__popcll(want) : avail;
          if (need && rank < cnt) {
            mine = next + rank;
            need = false;
          }
          next += cnt;
        }
        if (mine >= 0) {
          if (walk_init<T, N, KIND>(a, a.queries, a.nw, a.q_offset, a.idx_base + mine, st))
            walk_store(a.walk_S, a.walk_K, st);
          else active = true;
        }
      }
      if (__ballot(active) == 0) {
        if (exhausted) break;
        continue;
      }
      if (active) {
        if (walk_step<T, N, KIND, RICH>(a, st, seed, tab)) {
          walk_store(a.walk_S, a.walk_K, st);
          active = false;
        }
      }
    }
  }
}

// Batched persistent form (serving): the launch holds the walks of several
// requests (a.batch), each starting on a whole chunk of 64 launch walks, so a
// chunk belongs to one request.  A wave runs walks of one request at a time:
// its seed, queries and outputs stay wave-uniform.  Free lanes refill from
// the wave's chunk; a used-up chunk is replaced from the global counter, and
// a new chunk of another request waits until the wave's running walks end.
// Every wave leaves once the counter passes the last chunk and its lanes are
// idle.
template <class T, int N, int KIND, bool RICH>
__global__ __launch_bounds__(256) void walk_lane_batch_kernel(WalkArgs a) {
  constexpr int64_t kChunk = 64;
  const int64_t nchunks = a.count / kChunk;
  const uint32_t lane = lane_id();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  LaneState<T, N> st;
  const float4* tab = nullptr;
  if constexpr (KIND == kCutTorus && RICH && sizeof(T) == 4) {
    __shared__ float4 ts_tab[kTsLds];
    if (ts_stage(a, ts_tab)) tab = ts_tab;
  }
  bool active = false;
  bool exhausted = false;
  int cur = -1;                // entry of the walks the wave runs
  int64_t held = -1;           // chunk of another entry, started once the wave is idle
  int64_t next = 0, end = 0;
  // entry fields of `cur` (uniform)
  int64_t e_begin = 0, e_end = 0, e_idx0 = 0, e_nw = 1;
  const double* e_q = nullptr;
  double* e_S = nullptr;
  int32_t* e_K = nullptr;
  uint64_t e_seed = 0;
  char* e_rec = nullptr;       // time slicing: the entry's walk records (null: walks run to the end)
  bool e_resume = false;
  unsigned long long* e_pending = nullptr;
  int32_t steps = 0;           // steps of the lane's walk in this launch
  auto enter = [&](int64_t c) {
    cur = batch_entry(a, c * kChunk);
    const BatchEntry& E = a.batch[cur];
    e_begin = E.begin;
    e_idx0 = E.idx0;
    e_nw = E.nw;
    e_q = E.queries;
    e_S = E.walk_S;
    e_K = E.walk_K;
    e_seed = E.seed;
    e_end = E.begin + E.count;
    e_rec = (E.state && a.step_budget > 0) ? E.state : nullptr;
    e_resume = e_rec && E.resume != 0;
    e_pending = const_cast<unsigned long long*>(&a.batch[cur].pending);
    next = c * kChunk;
    end = next + kChunk < e_end ? next + kChunk : e_end;
  };
  for (;;) {
    for (;;) {
      const uint64_t want = __ballot(!active);
      if (want == 0 || exhausted || held >= 0) break;
      if (next >= end) {
        const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)want) - 1);
        unsigned long long c = 0;
        if (lane == leader) c = atomicAdd(a.queue, 1ull);
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)c, leader);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(c >> 32), leader);
        const int64_t cb = (int64_t)(((uint64_t)hi << 32) | lo);
        if (cb >= nchunks) {
          exhausted = true;
          break;
        }
        if (cur >= 0 && cb * kChunk < e_end) {
          // chunks are handed out in increasing order: cb lies past the wave's
          // earlier chunks, hence at or after e_begin
          next = cb * kChunk;
          end = next + kChunk < e_end ? next + kChunk : e_end;
        } else if (__ballot(active) != 0) {
          held = cb;
          break;
        } else {
          enter(cb);
        }
      }
      const int rank = __popcll(want & lt_mask);
      const int64_t avail = end - next;
      const int64_t cnt = (int64_t)__popcll(want) < avail ? (int64_t)__popcll(want) : avail;
      if (!active && rank < cnt) {
        const int64_t widx = e_idx0 + (next + rank - e_begin);
        steps = 0;
        if (e_resume) {
          // a walk finished in an earlier launch keeps its outputs
          active = lane_load<T, N>(e_rec + widx * kLaneRecord, e_nw, widx, st);
        } else if (walk_init<T, N, KIND>(a, e_q, e_nw, 0, widx, st)) {
          walk_store(e_S, e_K, st);
          if (e_rec) lane_save<T, N>(e_rec + widx * kLaneRecord, st, 1u);
        } else {
          active = true;
        }
      }
      next += cnt;
    }
    if (__ballot(active) == 0) {
      if (held < 0) break;
      enter(held);
      held = -1;
      continue;
    }
    if (active) {
      if (walk_step<T, N, KIND, RICH>(a, st, e_seed, tab)) {
        walk_store(e_S, e_K, st);
        if (e_rec) lane_save<T, N>(e_rec + st.idx * kLaneRecord, st, 1u);
        active = false;
      } else if (e_rec && ++steps >= a.step_budget) {
        // the slice is used up: the walk continues in a later launch
        lane_save<T, N>(e_rec + st.idx * kLaneRecord, st, 0u);
        atomicAdd(e_pending, 1ull);
        active = false;
      }
    }
  }
}

// ---- per-query estimator (eq. mc_estimator) --------------------------------
// One 256-thread block per query: compensated sums per thread over a fixed
// stride, then a fixed-order tree, so the result does not depend on timing.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ __launch_bounds__(256) void reduce_queries_kernel(const double* __restrict__ walk_S,
                                                             const int32_t* __restrict__ walk_K, int64_t nq,
                                                             int64_t nw, int64_t max_steps, double* u_out,
                                                             double* se_out, unsigned long long* ksum,
                                                             int32_t* kmax, unsigned long long* ntrunc) {
  __shared__ double sh_s[256], sh_c[256];
  __shared__ long long sh_k[256];
  __shared__ int sh_m[256], sh_t[256];
  const int t = threadIdx.x;
  for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const double* S = walk_S + q * nw;
    const int32_t* K = walk_K + q * nw;
    double s = 0.0, c = 0.0;
    long long ks = 0;
    int km = 0, tr = 0;
    for (int64_t w = t; w < nw; w += 256) {
      kahan_add(s, c, S[w]);
      const int kk = K[w];
      ks += kk;
      km = kk > km ? kk : km;
      tr += (kk >= max_steps) ? 1 : 0;
    }
    sh_s[t] = s;
    sh_c[t] = c;
    sh_k[t] = ks;
    sh_m[t] = km;
    sh_t[t] = tr;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) {
        double ss, ee;
        two_sum(sh_s[t], sh_s[t + o], ss, ee);
        sh_s[t] = ss;
        sh_c[t] = sh_c[t] + sh_c[t + o] + ee;
        sh_k[t] += sh_k[t + o];
        sh_m[t] = sh_m[t] > sh_m[t + o] ? sh_m[t] : sh_m[t + o];
        sh_t[t] += sh_t[t + o];
      }
      __syncthreads();
    }
    const double mean = (sh_s[0] + sh_c[0]) / (double)nw;
    if (t == 0) {
      atomicAdd(ksum, (unsigned long long)sh_k[0]);
      atomicMax(kmax, sh_m[0]);
      if (sh_t[0]) atomicAdd(ntrunc, (unsigned long long)sh_t[0]);
    }
    __syncthreads();
    double v = 0.0, vc = 0.0;
    for (int64_t w = t; w < nw; w += 256) {
      const double d = S[w] - mean;
      kahan_add(v, vc, d * d);
    }
    sh_s[t] = v + vc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) sh_s[t] += sh_s[t + o];
      __syncthreads();
    }
    if (t == 0) {
      u_out[q] = mean;
      if (se_out) se_out[q] = nw > 1 ? sqrt(sh_s[0] / (double)(nw - 1) / (double)nw) : 0.0;
    }
    __syncthreads();
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void set_u64_kernel(unsigned long long* p, unsigned long long v) {
  if (threadIdx.x == 0) p[0] = v;
}

// ---- inspection kernels -------------------------------------------------------
template <class T, int N, int KIND>
__global__ void cp_points_kernel(WalkArgs a, const double* x, double* y, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  T xi[N], yi[N];
  for (int d = 0; d < N; ++d) xi[d] = (T)x[i * N + d];
  closest_point<T, N, KIND>(a, xi, yi);
  for (int d = 0; d < N; ++d) y[i * N + d] = (double)yi[d];
}

__global__ void radial_inv_kernel(WalkArgs a, const double* u, double* s, int64_t m, int fp64) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double X2 = a.X0 * a.X0;
  if (fp64) s[i] = radial_inv64(a, u[i], X2, a.fixed.norm);
  else s[i] = (double)radial_inv32(a, (float)u[i], (float)X2);
}

__global__ void philox_kernel(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                              uint32_t* out, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint4 v = philox(c0 + (uint32_t)i, c1, c2, c3, k0, k1);
  out[4 * i + 0] = v.x;
  out[4 * i + 1] = v.y;
  out[4 * i + 2] = v.z;
  out[4 * i + 3] = v.w;
}

// Plain streaming copy, 16 B per lane per iteration: the reference kernel for
// calibrating HBM byte counters.
__global__ __launch_bounds__(256) void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t m) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// VALU throughput probe: 8 independent dependency chains of one operation per
// lane, so the issue rate of that operation (not its latency) bounds the run.
// OP: 0 fma_f32, 1 fma_f64, 2 mad_u64_u32, 3 mul_hi_u32, 4 log_f32, 5 sin_f32,
//     6 sqrt_f32, 7 rsq_f32, 8 rcp_f32, 9 xor_b32, 10 add_f64,
//     11 sin_f32 + 3 fma_f32, 12 mad_u64_u32 + 3 fma_f32 (mixed streams).
template <int OP>
__global__ __launch_bounds__(256) void valu_probe_kernel(uint32_t seed, int32_t iters, uint32_t* out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  if constexpr (OP == 0 || (OP >= 4 && OP <= 8)) {
    float a[8];
    const float b = 0.999f + (float)(seed & 7) * 1e-6f, c = 1e-3f;
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = 1.0f + (float)((t + 3 * i + seed) & 1023) * 1e-4f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if constexpr (OP == 0) a[i] = fmaf(a[i], b, c);
        if constexpr (OP == 4) a[i] = __builtin_amdgcn_logf(fabsf(a[i]));
        if constexpr (OP == 5) a[i] = __builtin_amdgcn_sinf(a[i]);
        if constexpr (OP == 6) a[i] = __builtin_amdgcn_sqrtf(a[i]);
        if constexpr (OP == 7) a[i] = __builtin_amdgcn_rsqf(a[i]);
        if constexpr (OP == 8) a[i] = __builtin_amdgcn_rcpf(a[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) acc ^= __float_as_uint(a[i]);
  } else if constexpr (OP == 11 || OP == 12) {
    // a transcendental (11: sin_f32) or a 64-bit multiply-add (12: mad_u64_u32)
    // per chain step, beside three independent fma_f32: does it overlap them?
    float a[8], b[8];
    uint32_t x[8], y[8];
    const float bb = 0.999f + (float)(seed & 7) * 1e-6f, cc = 1e-3f;
    const uint32_t m = 0xD2511F53u ^ (seed & 0xF0u);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = 1.0f + (float)((t + 3 * i + seed) & 1023) * 1e-4f;
      b[i] = a[i] * 0.5f;
      x[i] = t * 0x85EBCA6Bu + (uint32_t)i * 0xC2B2AE35u + seed;
      y[i] = x[i] * 0x9E3779B9u;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if constexpr (OP == 11) {
          a[i] = __builtin_amdgcn_sinf(a[i]);
        } else {
          uint64_t p = ((uint64_t)y[i] << 32) | x[i];
          p = (uint64_t)(uint32_t)(p >> 32) * m + p;
          x[i] = (uint32_t)p;
          y[i] = (uint32_t)(p >> 32);
        }
        b[i] = fmaf(b[i], bb, cc);
        b[i] = fmaf(b[i], bb, cc);
        b[i] = fmaf(b[i], bb, cc);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) acc ^= __float_as_uint(a[i]) ^ __float_as_uint(b[i]) ^ x[i] ^ y[i];
  } else if constexpr (OP == 1 || OP == 10) {
    double a[8];
    const double b = 0.999 + (double)(seed & 7) * 1e-9, c = 1e-3;
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = 1.0 + (double)((t + 3 * i + seed) & 1023) * 1e-4;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if constexpr (OP == 1) a[i] = fma(a[i], b, c);
        if constexpr (OP == 10) a[i] = a[i] + b;
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) acc ^= (uint32_t)__double_as_longlong(a[i]);
  } else {
    uint32_t x[8], y[8];
    const uint32_t m = 0xD2511F53u ^ (seed & 0xF0u);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      x[i] = t * 0x85EBCA6Bu + (uint32_t)i * 0xC2B2AE35u + seed;
      y[i] = x[i] * 0x9E3779B9u;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if constexpr (OP == 2) {
          // 32x32->64 multiply plus a 64-bit addend: the previous product, so
          // the chain needs no register moves
          uint64_t p = ((uint64_t)y[i] << 32) | x[i];
          p = (uint64_t)(uint32_t)(p >> 32) * m + p;
          x[i] = (uint32_t)p;
          y[i] = (uint32_t)(p >> 32);
        }
        if constexpr (OP == 3) x[i] = __umulhi(x[i], m);
        if constexpr (OP == 9) {
          x[i] = x[i] ^ y[(i + 1) & 7];
          y[i] = y[i] ^ x[(i + 3) & 7];
        }
        if constexpr (OP == 13) {
          x[i] = __builtin_amdgcn_bitop3_b32(x[i], y[(i + 1) & 7], m, 0x96);
          y[i] = __builtin_amdgcn_bitop3_b32(y[i], x[(i + 3) & 7], m, 0x96);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) acc ^= x[i] ^ y[i];
  }
  out[t] = acc;
}

hipError_t launch_valu_probe(int op, uint32_t seed, int32_t iters, uint32_t* out, int blocks, hipStream_t s) {
  switch (op) {
#define MPWOS_PROBE_CASE(K) \
  case K: hipLaunchKernelGGL(valu_probe_kernel<K>, dim3(blocks), dim3(256), 0, s, seed, iters, out); break;
    MPWOS_PROBE_CASE(0) MPWOS_PROBE_CASE(1) MPWOS_PROBE_CASE(2) MPWOS_PROBE_CASE(3) MPWOS_PROBE_CASE(4)
    MPWOS_PROBE_CASE(5) MPWOS_PROBE_CASE(6) MPWOS_PROBE_CASE(7) MPWOS_PROBE_CASE(8) MPWOS_PROBE_CASE(9)
    MPWOS_PROBE_CASE(10) MPWOS_PROBE_CASE(11) MPWOS_PROBE_CASE(12) MPWOS_PROBE_CASE(13)
#undef MPWOS_PROBE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define MPWOS_LANE_DISPATCH(FN, ...)                                                   \
  do {                                                                               \
    if (fp64) {                                                                      \
      if (kind == kSphere && n == 2) return FN<double, 2, kSphere>(__VA_ARGS__);     \
      if (kind == kSphere && n == 3) return FN<double, 3, kSphere>(__VA_ARGS__);     \
      if (kind == kCap && n == 3) return FN<double, 3, kCap>(__VA_ARGS__);           \
      if (kind == kCap && n == 2) return FN<double, 2, kCap>(__VA_ARGS__);           \
      if (kind == kTorus && n == 3) return FN<double, 3, kTorus>(__VA_ARGS__);       \
      if (kind == kCloud && n == 3) return FN<double, 3, kCloud>(__VA_ARGS__);       \
      if (kind == kCutTorus && n == 3) return FN<double, 3, kCutTorus>(__VA_ARGS__); \
    } else {                                                                         \
      if (kind == kSphere && n == 2) return FN<float, 2, kSphere>(__VA_ARGS__);      \
      if (kind == kSphere && n == 3) return FN<float, 3, kSphere>(__VA_ARGS__);      \
      if (kind == kCap && n == 3) return FN<float, 3, kCap>(__VA_ARGS__);            \
      if (kind == kCap && n == 2) return FN<float, 2, kCap>(__VA_ARGS__);            \
      if (kind == kTorus && n == 3) return FN<float, 3, kTorus>(__VA_ARGS__);        \
      if (kind == kCloud && n == 3) return FN<float, 3, kCloud>(__VA_ARGS__);        \
      if (kind == kCutTorus && n == 3) return FN<float, 3, kCutTorus>(__VA_ARGS__);  \
    }                                                                                \
  } while (0)

// ---- host launchers -----------------------------------------------------------
template <class T, int N, int KIND>
static hipError_t launch_cp_t(const WalkArgs& a, const double* x, double* y, int64_t m, hipStream_t s) {
  hipLaunchKernelGGL((cp_points_kernel<T, N, KIND>), dim3((unsigned)((m + 127) / 128)), dim3(128), 0, s, a, x, y, m);
  return hipGetLastError();
}

hipError_t launch_cp_points(const WalkArgs& a, const double* x, double* y, int64_t m, hipStream_t s) {
  const bool fp64 = a.precision == 0;
  const int kind = a.kind, n = a.n;
  MPWOS_LANE_DISPATCH(launch_cp_t, a, x, y, m, s);
  return hipErrorInvalidValue;
}

hipError_t launch_radial_inv(const WalkArgs& a, const double* u, double* s_out, int64_t m, int fp64,
                             hipStream_t s) {
  hipLaunchKernelGGL(radial_inv_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, u, s_out, m, fp64);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* c, uint64_t seed, uint32_t* out, int64_t m, hipStream_t s) {
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, c[0], c[1], c[2], c[3],
                     (uint32_t)seed, (uint32_t)(seed >> 32), out, m);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t m = bytes / 16;
  hipLaunchKernelGGL(copy_kernel, dim3(2048), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, m);
  return hipGetLastError();
}

// Sources outside ZERO, CONST, SPH_PAIR and TORUS_MODE take the kernels that
// carry every family.
static bool rich_source(const WalkArgs& a) {
  const int k = a.f.kind;
  return !(k == kFnZero || k == kFnConst || k == kFnSphPair || k == kFnTorus);
}

template <class T, int N, int KIND>
static hipError_t launch_lane_t(const WalkArgs& a, int grid, int block, hipStream_t s) {
  const dim3 g(grid), b(block);
  if (rich_source(a)) {
    if (a.n_batch) hipLaunchKernelGGL((walk_lane_batch_kernel<T, N, KIND, true>), g, b, 0, s, a);
    else if (a.persistent) hipLaunchKernelGGL((walk_lane_kernel<T, N, KIND, true, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((walk_lane_kernel<T, N, KIND, false, true>), g, b, 0, s, a);
  } else {
    if (a.n_batch) hipLaunchKernelGGL((walk_lane_batch_kernel<T, N, KIND, false>), g, b, 0, s, a);
    else if (a.persistent) hipLaunchKernelGGL((walk_lane_kernel<T, N, KIND, true, false>), g, b, 0, s, a);
    else hipLaunchKernelGGL((walk_lane_kernel<T, N, KIND, false, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

template <class T, int N, int KIND>
static int occupancy_t(int block, bool rich, bool batch) {
  int nb = 0;
  hipError_t e;
  if (batch)
    e = rich ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_lane_batch_kernel<T, N, KIND, true>, block, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_lane_batch_kernel<T, N, KIND, false>, block, 0);
  else
    e = rich ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_lane_kernel<T, N, KIND, true, true>, block, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_lane_kernel<T, N, KIND, true, false>, block, 0);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

hipError_t launch_walk_lane(const WalkArgs& a, int grid, int block, hipStream_t s) {
  const bool fp64 = a.precision == 0;
  const int kind = a.kind, n = a.n;
  MPWOS_LANE_DISPATCH(launch_lane_t, a, grid, block, s);
  return hipErrorInvalidValue;
}

int lane_occupancy(const WalkArgs& a, int block) {
  const bool fp64 = a.precision == 0, rich = rich_source(a), batch = a.n_batch > 0;
  const int kind = a.kind, n = a.n;
  MPWOS_LANE_DISPATCH(occupancy_t, block, rich, batch);
  return 1;
}

bool lane_supported(int kind, int n) {
  return (n == 2 || n == 3) &&
         (kind == kSphere || kind == kCap || ((kind == kTorus || kind == kCloud || kind == kCutTorus) && n == 3));
}

hipError_t launch_reduce(const double* walk_S, const int32_t* walk_K, int64_t nq, int64_t nw, int64_t max_steps,
                         double* u, double* se, unsigned long long* ksum, int32_t* kmax,
                         unsigned long long* ntrunc, hipStream_t s) {
  const int64_t g = nq < 65536 ? nq : 65536;
  hipLaunchKernelGGL(reduce_queries_kernel, dim3((unsigned)g), dim3(256), 0, s, walk_S, walk_K, nq, nw, max_steps,
                     u, se, ksum, kmax, ntrunc);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long* p, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace mpwos
