// One lane group per walk on S^{n-1}_R for n >= 4 (up to n = 4092): the n
// coordinates of a walk are spread over L lanes of a wavefront (L = 4 .. 64).
// Philox block b of a sub-stream (coordinates 4b .. 4b+3) belongs to lane
// b mod L, slot b / L, so every lane draws its own normals; the norms |g|,
// |Theta|, |g'| and |Z| are butterfly sums across the group (commutative, so
// every lane ends with the same bits).  W, S and the radial inverse are
// computed redundantly by all lanes of the group.
#include <hip/hip_runtime.h>

#include "host_internal.h"
#include "kernel_args.h"
#include "mpwos_dev.h"

namespace mpwos {

template <int L, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
  return v;
}

template <class T, int L, int MB>
struct GroupWalk {
  T Y[4 * MB];
  double W, S, C;
  uint32_t k, q, w;
  int64_t idx;
};

// n normals of one sub-stream into this lane's slots (zeros past n).  Returns
// the radius uniform word if this lane owns it.
template <class T, int L, int MB>
__device__ __forceinline__ void group_normals(const WalkArgs& a, const Stream& rs, uint32_t step, uint32_t sub,
                                              int gl, T* g, bool want_u, uint32_t& uword) {
  const int n = a.n;
  const int npairs = (n + 1) / 2;
  const int nbd = (n + 3) / 4;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int b = gl + L * m;
    T* gm = g + 4 * m;
    gm[0] = gm[1] = gm[2] = gm[3] = (T)0;
    const bool dir = b < nbd;
    const bool rad = want_u && b == a.rblk;
    if (dir || rad) {
      const uint4 x = rs.block(step, sub, (uint32_t)b);
      if (dir) {
        T g0, g1;
        if (2 * b < npairs) {
          box_muller(x.x, x.y, g0, g1);
          gm[0] = g0;
          gm[1] = (4 * b + 1 < n) ? g1 : (T)0;
        }
        if (2 * b + 1 < npairs) {
          box_muller(x.z, x.w, g0, g1);
          gm[2] = g0;
          gm[3] = (4 * b + 3 < n) ? g1 : (T)0;
        }
      }
      if (rad) {
        const uint32_t ws[4] = {x.x, x.y, x.z, x.w};
        uword = ws[a.rword];
      }
    }
  }
}

template <class T, int L, int MB>
__device__ __forceinline__ T coord_of(const T* v, int i, int gl) {
  // value of coordinate i, broadcast from its owner lane
  const int b = i >> 2;
  const int owner = b % L;
  const int slot = b / L;
  T mine = (T)0;
#pragma unroll
  for (int m = 0; m < MB; ++m)
    if (m == slot) mine = v[4 * m + (i & 3)];
  return __shfl(mine, owner, L);
}

template <class T, int L, int MB>
__device__ __forceinline__ bool group_step(const WalkArgs& a, GroupWalk<T, L, MB>& st, int gl, uint64_t seed) {
  const Stream rs{st.q, st.w, (uint32_t)seed, (uint32_t)(seed >> 32)};
  const double r = a.r0;
  const T rT = (T)r;
  const T R = (T)a.p[0];
  uint32_t dummy = 0;
  // sphere sample and projection: Theta = Y + r g/|g|, Y' = R Theta/|Theta|
  T Yn[4 * MB];
  {
    T g[4 * MB];
    group_normals<T, L, MB>(a, rs, st.k, 0, gl, g, false, dummy);
    T gg = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) gg += g[i] * g[i];
    gg = group_sum<L>(gg);
    const T ig = rsqrt_(gg);
    T tt = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) {
      Yn[i] = st.Y[i] + rT * (g[i] * ig);
      tt += Yn[i] * Yn[i];
    }
    tt = group_sum<L>(tt);
    const T f = R * rsqrt_(tt);
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) Yn[i] *= f;
  }
  // Green samples
  T Fsum = (T)0;
  for (int l = 1; l <= a.n_v; ++l) {
    T g[4 * MB];
    uint32_t uw = 0;
    group_normals<T, L, MB>(a, rs, st.k, (uint32_t)l, gl, g, true, uw);
    uw = __shfl(uw, a.rblk % L, L);
    T s;
    if constexpr (sizeof(T) == 8) s = radial_inv64(a, u01_64(uw), a.X0 * a.X0, a.fixed.norm);
    else s = radial_inv32(a, u01_32(uw), (float)(a.X0 * a.X0));
    T gg = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) gg += g[i] * g[i];
    gg = group_sum<L>(gg);
    const T ig = rsqrt_(gg);
    const T t = rT * s;
    T Z[4 * MB];
    T zz = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) {
      Z[i] = st.Y[i] + t * (g[i] * ig);
      zz += Z[i] * Z[i];
    }
    zz = group_sum<L>(zz);
    const FnDev& f = a.f;
    T v;
    if (f.kind == kFnSphPair) {
      const T zi = coord_of<T, L, MB>(Z, f.idx[0], gl);
      const T zj = coord_of<T, L, MB>(Z, f.idx[1], gl);
      // cp(Z) = R Z/|Z|; f_Omega(cp Z) = coef (Z_i/|Z|)(Z_j/|Z|)
      const T fv = (T)f.coef[0] * (zi * zj / zz);
      v = fv;
      if (a.comp) v += (T)(f.lam * f.u_scale) * fv * (over_(R * R, zz) - (T)1);
    } else if (f.kind == kFnConst) {
      v = (T)f.coef[0];
    } else {
      v = (T)0;
    }
    Fsum += v;
  }
  const double F = a.n_v == 1 ? (double)Fsum : (double)Fsum / (double)a.n_v;
  kahan_add(st.S, st.C, (st.W * a.om0) * F);
  st.W = st.W * a.c0;
#pragma unroll
  for (int i = 0; i < 4 * MB; ++i) st.Y[i] = Yn[i];
  st.k += 1;
  if (!(st.W >= a.tau_w)) return true;  // NaN ends the walk too
  return (int64_t)st.k >= a.max_steps;
}

template <class T, int L, int MB>
__device__ __forceinline__ void group_init(const WalkArgs& a, const double* queries, int64_t nw, int64_t q_offset,
                                           int64_t idx, GroupWalk<T, L, MB>& st, int gl) {
  st.idx = idx;
  const int64_t ql = idx / nw;
  st.q = (uint32_t)(ql + q_offset);
  st.w = (uint32_t)(idx - ql * nw);
  const double* y0 = queries + ql * a.n;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int b = gl + L * m;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * b + j;
      st.Y[4 * m + j] = (i < a.n) ? (T)y0[i] : (T)0;
    }
  }
  st.W = 1.0;
  st.S = 0.0;
  st.C = 0.0;
  st.k = 0;
}

// State record of a time-sliced walk: W, S, C, k and a done flag (written by
// the group's lane 0), then each lane's 4 MB coordinates.
template <class T, int L, int MB>
struct GroupRecord {
  static constexpr int64_t kBytes = (32 + (int64_t)L * 4 * MB * (int64_t)sizeof(T) + 63) / 64 * 64;
};

template <class T, int L, int MB>
__device__ __forceinline__ void group_save(char* rec, const GroupWalk<T, L, MB>& st, int gl, uint32_t flag) {
  if (gl == 0) {
    double* d = (double*)rec;
    d[0] = st.W;
    d[1] = st.S;
    d[2] = st.C;
    uint32_t* u = (uint32_t*)(rec + 24);
    u[0] = st.k;
    u[1] = flag;
  }
  if (flag) return;
  T* y = (T*)(rec + 32) + gl * 4 * MB;
#pragma unroll
  for (int i = 0; i < 4 * MB; ++i) y[i] = st.Y[i];
}

template <class T, int L, int MB>
__device__ __forceinline__ void group_load(const char* rec, int64_t idx, int64_t nw, GroupWalk<T, L, MB>& st,
                                           int gl) {
  st.idx = idx;
  const int64_t ql = idx / nw;
  st.q = (uint32_t)ql;
  st.w = (uint32_t)(idx - ql * nw);
  const double* d = (const double*)rec;
  st.W = d[0];
  st.S = d[1];
  st.C = d[2];
  st.k = ((const uint32_t*)(rec + 24))[0];
  const T* y = (const T*)(rec + 32) + gl * 4 * MB;
#pragma unroll
  for (int i = 0; i < 4 * MB; ++i) st.Y[i] = y[i];
}

// plain: group id -> walk; persistent: grid-stride over walks (closed
// spheres have one deterministic walk length, so a static split is balanced).
// Batched launches (serving) take the grid-stride form; every entry begins on
// a whole wavefront of groups and the stride is a whole number of wavefronts,
// so the groups of a wavefront always share one request (its seed stays
// uniform); launch walks past an entry's count are padding.
template <class T, int L, int MB>
__global__ __launch_bounds__(256) void walk_group_kernel(WalkArgs a) {
  const int64_t total = a.count;
  const int gl = threadIdx.x % L;
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / L;
  GroupWalk<T, L, MB> st;
  for (int64_t idx = gid; idx < total; idx += (a.persistent ? ngroups : total)) {
    const double* queries = a.queries;
    int64_t nw = a.nw, q_offset = a.q_offset, widx = a.idx_base + idx;
    uint64_t seed;
    double* walk_S = a.walk_S;
    int32_t* walk_K = a.walk_K;
    char* rec = nullptr;
    bool resume = false;
    unsigned long long* pending = nullptr;
    if (a.n_batch) {
      const int64_t first = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)idx) |
                            ((int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(idx >> 32)) << 32);
      const int e = batch_entry(a, first);
      const BatchEntry& E = a.batch[e];
      if (idx >= E.begin + E.count) continue;
      queries = E.queries;
      nw = E.nw;
      q_offset = 0;
      widx = E.idx0 + (idx - E.begin);
      seed = E.seed;
      walk_S = E.walk_S;
      walk_K = E.walk_K;
      if (E.state && a.step_budget > 0) {
        rec = E.state + widx * GroupRecord<T, L, MB>::kBytes;
        resume = E.resume != 0;
        pending = const_cast<unsigned long long*>(&a.batch[e].pending);
      }
    } else {
      seed = a.seed_dev ? *a.seed_dev : a.seed;
    }
    if (resume) {
      if (((const uint32_t*)(rec + 24))[1]) continue;   // finished in an earlier launch
      group_load<T, L, MB>(rec, widx, nw, st, gl);
    } else {
      group_init<T, L, MB>(a, queries, nw, q_offset, widx, st, gl);
    }
    bool done = false;
    if (rec) {
      for (int32_t j = 0; j < a.step_budget && !done; ++j) done = group_step<T, L, MB>(a, st, gl, seed);
    } else {
      while (!group_step<T, L, MB>(a, st, gl, seed)) {
      }
      done = true;
    }
    if (done) {
      if (gl == 0) {
        walk_S[st.idx] = st.S + st.C;
        walk_K[st.idx] = (int32_t)st.k;
      }
      if (rec) group_save<T, L, MB>(rec, st, gl, 1u);
    } else {
      group_save<T, L, MB>(rec, st, gl, 0u);
      if (gl == 0) atomicAdd(pending, 1ull);
    }
  }
}

template <class T, int L, int MB>
static hipError_t launch_group_t(const WalkArgs& a, int64_t grid, int block, hipStream_t s) {
  hipLaunchKernelGGL((walk_group_kernel<T, L, MB>), dim3((unsigned)grid), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <class T, int L, int MB>
static int group_occ_t(int block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_group_kernel<T, L, MB>, block, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

#define MPWOS_GROUP_MB(T, LL, FN, ...)                 \
  switch (mb) {                                        \
    case 1: return FN<T, LL, 1>(__VA_ARGS__);          \
    case 2: return FN<T, LL, 2>(__VA_ARGS__);          \
    case 4: return FN<T, LL, 4>(__VA_ARGS__);          \
    case 8: return FN<T, LL, 8>(__VA_ARGS__);          \
  }
#define MPWOS_GROUP_L(T, FN, ...)                                       \
  switch (L) {                                                          \
    case 4: MPWOS_GROUP_MB(T, 4, FN, __VA_ARGS__) break;                \
    case 8: MPWOS_GROUP_MB(T, 8, FN, __VA_ARGS__) break;                \
    case 16: MPWOS_GROUP_MB(T, 16, FN, __VA_ARGS__) break;              \
    case 32: MPWOS_GROUP_MB(T, 32, FN, __VA_ARGS__) break;              \
    case 64:                                                            \
      if (mb == 16) return FN<T, 64, 16>(__VA_ARGS__);                  \
      MPWOS_GROUP_MB(T, 64, FN, __VA_ARGS__) break;                     \
  }

static hipError_t group_launch(bool fp64, int L, int mb, const WalkArgs& a, int64_t grid, int block, hipStream_t s) {
  if (fp64) {
    MPWOS_GROUP_L(double, launch_group_t, a, grid, block, s)
  } else {
    MPWOS_GROUP_L(float, launch_group_t, a, grid, block, s)
  }
  return hipErrorInvalidValue;
}

static int group_occ(bool fp64, int L, int mb, int block) {
  if (fp64) {
    MPWOS_GROUP_L(double, group_occ_t, block)
  } else {
    MPWOS_GROUP_L(float, group_occ_t, block)
  }
  return 1;
}

// Group shape for dimension n: Philox blocks per Green sub-stream (direction
// blocks plus the block that holds the radius word) spread over L lanes.
void group_shape(int n, int lanes_req, int& L, int& mb, int& nblk, int& rblk, int& rword) {
  const int nbd = (n + 3) / 4;
  const int rw = 2 * ((n + 1) / 2);
  rblk = rw / 4;
  rword = rw % 4;
  nblk = nbd > rblk + 1 ? nbd : rblk + 1;
  L = lanes_req > 1 ? lanes_req : 0;
  if (!L) {
    L = 64;
    for (int c : {4, 8, 16, 32, 64}) {
      if ((nblk + c - 1) / c <= 4) { L = c; break; }
    }
  }
  const int per = (nblk + L - 1) / L;
  mb = 1;
  while (mb < per) mb *= 2;
}

template <class T, int L, int MB>
static int64_t group_record_t() {
  return GroupRecord<T, L, MB>::kBytes;
}

int64_t group_record_bytes(int n, int lanes_req, bool fp64) {
  int L, mb, nblk, rblk, rword;
  group_shape(n, lanes_req, L, mb, nblk, rblk, rword);
  if (fp64) {
    MPWOS_GROUP_L(double, group_record_t)
  } else {
    MPWOS_GROUP_L(float, group_record_t)
  }
  return 0;
}

mpwos_status launch_group_walks(WalkArgs& a, const mpwos_options& o, hipStream_t s, unsigned long long* queue) {
  (void)queue;
  if (a.kind != kSphere) return fail(MPWOS_EINVAL, "n >= 4 is supported on the closed sphere only");
  if (a.f.kind != kFnSphPair && a.f.kind != kFnConst && a.f.kind != kFnZero)
    return fail(MPWOS_EINVAL, "n >= 4 supports the ZERO, CONST and SPH_PAIR sources");
  int L, mb, nblk, rblk, rword;
  group_shape(a.n, o.lanes_per_walk, L, mb, nblk, rblk, rword);
  if (L < 4) return fail(MPWOS_EINVAL, "lanes_per_walk must be >= 4 for n >= 4");
  if (mb > 8 && !(L == 64 && mb == 16)) return fail(MPWOS_EINVAL, "n too large for the lane group");
  a.lanes = L;
  a.nblk = nblk;
  a.rblk = rblk;
  a.rword = rword;
  const int block = o.block_size ? o.block_size : 256;
  const bool fp64 = a.precision == 0;
  const int64_t total = a.count;
  const int64_t need = (total * L + block - 1) / block;
  int64_t grid = need;
  if (a.persistent) {
    const int64_t gmax = (int64_t)group_occ(fp64, L, mb, block) * device_cu_count();
    grid = std::max<int64_t>(1, std::min(need, gmax));
  }
  if (grid > 0x7FFFFFFF) return fail(MPWOS_EINVAL, "too many walks for one launch");
  hipError_t e = group_launch(fp64, L, mb, a, grid, block, s);
  if (e != hipSuccess) return hip_fail(e, "group walk kernel launch");
  return MPWOS_OK;
}

}  // namespace mpwos
