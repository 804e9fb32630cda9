// Host side of the lane-group walks (n >= 4): the group shape, the state
// record size for time slicing, and dispatch to the kernels of each manifold
// kind.  The kernels are templates in walk_group_dev.h, instantiated per kind
// in walk_group_sphere.hip, walk_group_dumbbell.hip and
// walk_group_product.hip, so that each kind's kernel carries only its own
// projection and source (registers and occupancy) and the three compile in
// parallel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "host_internal.h"
#include "kernel_args.h"
#include "walk_group_dev.h"

namespace mpwos {

hipError_t group_launch_sphere(bool fp64, int L, int mb, const WalkArgs& a, int64_t grid, int block, hipStream_t s);
hipError_t group_launch_dumbbell(bool fp64, int L, int mb, const WalkArgs& a, int64_t grid, int block,
                                 hipStream_t s);
hipError_t group_launch_product(bool fp64, int L, int mb, const WalkArgs& a, int64_t grid, int block,
                                hipStream_t s);
int group_occ_sphere(bool fp64, int L, int mb, int block);
int group_occ_dumbbell(bool fp64, int L, int mb, int block);
int group_occ_product(bool fp64, int L, int mb, int block);
hipError_t launch_cp_group_sphere(bool fp64, int L, int mb, const WalkArgs& a, const double* x, double* y,
                                  int64_t m, hipStream_t s);
hipError_t launch_cp_group_dumbbell(bool fp64, int L, int mb, const WalkArgs& a, const double* x, double* y,
                                    int64_t m, hipStream_t s);
hipError_t launch_cp_group_product(bool fp64, int L, int mb, const WalkArgs& a, const double* x, double* y,
                                   int64_t m, hipStream_t s);

static hipError_t group_launch(int kind, bool fp64, int L, int mb, const WalkArgs& a, int64_t grid, int block,
                               hipStream_t s) {
  if (kind == kDumbbell) return group_launch_dumbbell(fp64, L, mb, a, grid, block, s);
  if (kind == kProduct) return group_launch_product(fp64, L, mb, a, grid, block, s);
  return group_launch_sphere(fp64, L, mb, a, grid, block, s);
}

static int group_occ(int kind, bool fp64, int L, int mb, int block) {
  if (kind == kDumbbell) return group_occ_dumbbell(fp64, L, mb, block);
  if (kind == kProduct) return group_occ_product(fp64, L, mb, block);
  return group_occ_sphere(fp64, L, mb, block);
}

hipError_t launch_cp_group(const WalkArgs& a, const double* x, double* y, int64_t m, hipStream_t s) {
  int L, mb, nblk, rblk, rword;
  group_shape(a.n, 0, L, mb, nblk, rblk, rword);
  const bool fp64 = a.precision == 0;
  if (a.kind == kDumbbell) return launch_cp_group_dumbbell(fp64, L, mb, a, x, y, m, s);
  if (a.kind == kProduct) return launch_cp_group_product(fp64, L, mb, a, x, y, m, s);
  return launch_cp_group_sphere(fp64, L, mb, a, x, y, m, s);
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
  const int ll = L;
  auto pick = [&](auto tag) -> int64_t {
    using T = decltype(tag);
    switch (ll) {
      case 4: return mb == 1 ? group_record_t<T, 4, 1>() : mb == 2 ? group_record_t<T, 4, 2>()
                   : mb == 4 ? group_record_t<T, 4, 4>() : group_record_t<T, 4, 8>();
      case 8: return mb == 1 ? group_record_t<T, 8, 1>() : mb == 2 ? group_record_t<T, 8, 2>()
                   : mb == 4 ? group_record_t<T, 8, 4>() : group_record_t<T, 8, 8>();
      case 16: return mb == 1 ? group_record_t<T, 16, 1>() : mb == 2 ? group_record_t<T, 16, 2>()
                    : mb == 4 ? group_record_t<T, 16, 4>() : group_record_t<T, 16, 8>();
      case 32: return mb == 1 ? group_record_t<T, 32, 1>() : mb == 2 ? group_record_t<T, 32, 2>()
                    : mb == 4 ? group_record_t<T, 32, 4>() : group_record_t<T, 32, 8>();
      case 64: return mb == 1 ? group_record_t<T, 64, 1>() : mb == 2 ? group_record_t<T, 64, 2>()
                    : mb == 4 ? group_record_t<T, 64, 4>() : mb == 8 ? group_record_t<T, 64, 8>()
                    : group_record_t<T, 64, 16>();
    }
    return 0;
  };
  return fp64 ? pick(0.0) : pick(0.0f);
}

mpwos_status launch_group_walks(WalkArgs& a, const mpwos_options& o, hipStream_t s, unsigned long long* queue) {
  (void)queue;
  if (a.kind != kSphere && a.kind != kDumbbell && a.kind != kProduct)
    return fail(MPWOS_EINVAL, "n >= 4 is supported on the closed sphere, the dumbbell and the product manifold");
  if (a.kind == kProduct && a.f.kind != kFnProduct && a.f.kind != kFnConst && a.f.kind != kFnZero)
    return fail(MPWOS_EINVAL, "the product manifold supports the ZERO, CONST and PRODUCT_MODES sources");
  if (a.kind == kSphere && a.f.kind != kFnSphPair && a.f.kind != kFnConst && a.f.kind != kFnZero)
    return fail(MPWOS_EINVAL, "n >= 4 spheres support the ZERO, CONST and SPH_PAIR sources");
  if (a.kind == kDumbbell && a.f.kind != kFnDumbbell && a.f.kind != kFnConst && a.f.kind != kFnZero)
    return fail(MPWOS_EINVAL, "the dumbbell supports the ZERO, CONST and DUMBBELL_POLY sources");
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
    const int64_t gmax = (int64_t)group_occ(a.kind, fp64, L, mb, block) * device_cu_count();
    grid = std::max<int64_t>(1, std::min(need, gmax));
  }
  if (grid > 0x7FFFFFFF) return fail(MPWOS_EINVAL, "too many walks for one launch");
  hipError_t e = group_launch(a.kind, fp64, L, mb, a, grid, block, s);
  if (e != hipSuccess) return hip_fail(e, "group walk kernel launch");
  return MPWOS_OK;
}

}  // namespace mpwos
