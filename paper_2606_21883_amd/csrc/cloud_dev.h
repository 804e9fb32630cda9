// Device side of the point-cloud closest-point map (Sec. 2.3.2: nearest-
// neighbour search with local reconstruction).  cp_h(x) is the Newton foot
// point of x on the local quadratic patch (built once per manifold) of the
// cloud point nearest to that foot point: a fixed point found from a start
// patch by alternating the foot point on the current patch and the nearest
// cloud point of the foot (ties to the lower original index; a grid of small
// cells answers when it can show the answer exact, else a KD-tree search),
// at most kCloudRounds times.  The start patch is that of the cloud point
// nearest to x for a query, and for a walk point x near the walker's Y the
// one nearest to x's foot on the osculating quadratic of Y's patch (not
// clamped to its support).  Every search is then of a point near the
// surface; a search from x itself, up to a walk radius away, has to visit
// the boxes of every sample nearly as close as the nearest when x lies near
// a focal point of the surface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_args.h"
#include "mpwos_dev.h"

namespace mpwos {

// |x - p|^2 evaluated as ((dx dx + dy dy) + dz dz) without contraction in FP64,
// so that equal inputs give equal bits on every path that compares distances.
__device__ __forceinline__ double dist2_exact(const double* x, float px, float py, float pz) {
  const double dx = (double)px - x[0], dy = (double)py - x[1], dz = (double)pz - x[2];
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}
__device__ __forceinline__ float dist2_exact(const float* x, float px, float py, float pz) {
  const float dx = px - x[0], dy = py - x[1], dz = pz - x[2];
  return dx * dx + dy * dy + dz * dz;
}

template <class T>
__device__ __forceinline__ T box_dist2(const float* lo, const float* hi, const T* x) {
  T s = (T)0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T e = (T)0;
    if (x[d] < (T)lo[d]) e = (T)lo[d] - x[d];
    else if (x[d] > (T)hi[d]) e = x[d] - (T)hi[d];
    s += e * e;
  }
  return s;
}

// A leaf reference packs its first point and its size (at most 8 points):
// ref = -(start * 16 + count) - 1.
__device__ __forceinline__ int32_t leaf_start(int32_t ref) { return (-ref - 1) >> 4; }
__device__ __forceinline__ int32_t leaf_count(int32_t ref) { return (-ref - 1) & 15; }

// Median splits give leaves at depth at most ceil(log2(n / 8)) <= 24 for
// n <= 2^27 points, and the search defers at most one far child per internal
// node on its current path: 24 entries always suffice.
constexpr int kKdStack = 24;
// Workgroups of the kernels that search the cloud hold at most this many lanes.
constexpr int kCloudBlock = 128;

// Distance stored on the stack: rounded down, so a deferred box is never
// pruned when its exact distance is within the best one.
__device__ __forceinline__ float stack_dist(float d) { return d; }
__device__ __forceinline__ float stack_dist(double d) { return __double2float_rd(d); }

// Nearest cloud point of x: depth-first search that descends into the nearer
// child and defers the farther one with its box distance, pruning boxes
// farther than the best distance (a box at exactly the best distance is still
// visited, so the index tie-break is exact).  Returns the original index.
// The deferred nodes live in LDS: column threadIdx.x of kKdStack x
// kCloudBlock arrays (24 KB per workgroup).
template <class T>
__device__ __forceinline__ int32_t kd_nearest(const CloudDev& c, const T* x) {
  __shared__ int32_t sref[kKdStack][kCloudBlock];
  __shared__ float sdist[kKdStack][kCloudBlock];
  const int lane = threadIdx.x;
  // a non-finite x matches no point: skip the search (it would visit every node)
  if (!(abs_(x[0]) + abs_(x[1]) + abs_(x[2]) < (T)3.0e38)) return 0;
  T best = (T)3.0e38;
  int32_t bidx = 0x7fffffff;
  int sp = 0;
  int32_t ref = c.root;
  for (;;) {
    if (ref < 0) {
      const int32_t start = leaf_start(ref), end = start + leaf_count(ref);
      for (int32_t i = start; i < end; ++i) {
        const float4 p = c.kd_pts[i];
        const T d2 = dist2_exact(x, p.x, p.y, p.z);
        const int32_t id = __float_as_int(p.w);
        if (d2 < best || (d2 == best && id < bidx)) {
          best = d2;
          bidx = id;
        }
      }
    } else {
      const KdNode nd = c.nodes[ref];
      const T d0 = box_dist2<T>(nd.lo[0], nd.hi[0], x);
      const T d1 = box_dist2<T>(nd.lo[1], nd.hi[1], x);
      const bool first = d0 <= d1;
      const T dn = first ? d0 : d1, df = first ? d1 : d0;
      const int32_t cn = first ? nd.child[0] : nd.child[1], cf = first ? nd.child[1] : nd.child[0];
      if (df <= best && sp < kKdStack) {
        sref[sp][lane] = cf;
        sdist[sp][lane] = stack_dist(df);
        ++sp;
      }
      if (dn <= best) {
        ref = cn;
        continue;
      }
    }
    bool more = false;
    while (sp > 0) {
      --sp;
      if ((T)sdist[sp][lane] <= best) {
        ref = sref[sp][lane];
        more = true;
        break;
      }
    }
    if (!more) break;
  }
  // a non-finite x matches no point: fall back to point 0 so the caller's
  // patch read stays in bounds (the walk then ends on its non-finite state)
  return (uint32_t)bidx < (uint32_t)c.n_points ? bidx : 0;
}

// Nearest cloud point of x from the walk grid, or -1 when the grid cannot
// show its answer exact.  The 3x3x3 block of cells around x's cell is
// scanned plane by plane: three rows of three cells, each row one contiguous
// run of points whose six bounds are loaded before any point, the points
// eight at a time (independent loads, one latency per batch).  The answer (ties to the lower original index) is accepted when its
// distance lies below the distance from x to the block's boundary less the
// binning allowance, with a relative margin far above the rounding of a
// squared distance: every point outside the block is then farther, so the
// block's minimum is the global one, the KD-tree's answer.  A side of the
// block at the grid's edge has no points beyond it.
template <class T>
__device__ __forceinline__ int32_t grid_nearest(const CloudDev& c, const T* x) {
  constexpr int W = 8;         // points loaded together
  if (!c.g_start) return -1;
  double g[3];
  int ic[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g[d] = ((double)x[d] - c.g_lo[d]) * c.g_inv;
    // outside the grid, or not finite
    if (!(g[d] >= 0.0 && g[d] < (double)c.g_n[d])) return -1;
    ic[d] = (int)g[d];
  }
  const int nx = c.g_n[0], ny = c.g_n[1], nz = c.g_n[2];
  const int x0 = ic[0] > 0 ? ic[0] - 1 : 0, x1 = ic[0] + 1 < nx ? ic[0] + 1 : nx - 1;
  T best = (T)3.0e38;
  int32_t bidx = 0x7fffffff;
#pragma unroll
  for (int pz = 0; pz < 3; ++pz) {
    int32_t rs[3], re[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int yy = ic[1] + r - 1, zz = ic[2] + pz - 1;
      const bool in = yy >= 0 && yy < ny && zz >= 0 && zz < nz;
      const int64_t row = ((int64_t)(in ? zz : 0) * ny + (in ? yy : 0)) * nx;
      const int32_t a = c.g_start[row + x0], b = c.g_start[row + x1 + 1];
      rs[r] = in ? a : 0;
      re[r] = in ? b : 0;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int32_t e = re[r];
      for (int32_t i = rs[r]; i < e; i += W) {
        float4 q[W];
#pragma unroll
        for (int j = 0; j < W; ++j) q[j] = c.g_pts[i + j < e ? i + j : e - 1];
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const T d2 = dist2_exact(x, q[j].x, q[j].y, q[j].z);
          const int32_t id = __float_as_int(q[j].w);
          if (d2 < best || (d2 == best && id < bidx)) {
            best = d2;
            bidx = id;
          }
        }
      }
    }
  }
  if (bidx == 0x7fffffff) return -1;
  double m = 3.0e300;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (ic[d] >= 1) m = fmin(m, (g[d] - (double)(ic[d] - 1)) * c.g_h);
    if (ic[d] + 2 <= c.g_n[d]) m = fmin(m, ((double)(ic[d] + 2) - g[d]) * c.g_h);
  }
  m -= c.g_slack;
  if (m > 0.0 && (double)best < m * m * (1.0 - 1e-5)) return bidx;
  return -1;
}

// Nearest cloud point of a point near the surface: the walk grid, else the
// KD-tree (the same answer either way).
template <class T>
__device__ __forceinline__ int32_t near_surface_nearest(const CloudDev& c, const T* x) {
  const int32_t g = grid_nearest<T>(c, x);
  return g >= 0 ? g : kd_nearest<T>(c, x);
}

template <class T>
struct CloudProj {
  T y[3];
  T kappa;   // largest |principal curvature| of the patch at the foot point
  T hmean;   // local spacing of the nearest cloud point
  int32_t patch;  // original index of the cloud point whose patch holds y
};

// Rounds of the fixed-point search for the patch (foot point, then nearest
// cloud point of the foot).
constexpr int kCloudRounds = 4;

// Foot point of x on patch P: minimise E = (a - ax)^2 + (b - bx)^2 +
// (h(a,b) - hx)^2 over the support square |a|, |b| <= ext from (ax, bx)
// clamped to it, by Newton steps that fall back to the Gauss-Newton matrix
// I + J^T J where the Newton Hessian is not positive definite (x beyond the
// focal distance of the fitted quadratic), each iterate clamped; then the
// curvature of the patch there (eigenvalues of the shape operator I^-1 II).
// Without `clamp` the support square is unbounded: the foot point on the
// patch's whole quadratic (its osculating extension).
template <class T>
__device__ __forceinline__ CloudProj<T> patch_project(const Patch<T>& P, const T* x, int iters, bool clamp = true) {
  const T d0 = x[0] - P.cen[0], d1 = x[1] - P.cen[1], d2 = x[2] - P.cen[2];
  const T ax = d0 * P.e1[0] + d1 * P.e1[1] + d2 * P.e1[2];
  const T bx = d0 * P.e2[0] + d1 * P.e2[1] + d2 * P.e2[2];
  const T hx = d0 * P.n[0] + d1 * P.n[1] + d2 * P.n[2];
  const T* c = P.c;
  const T ext = clamp ? P.ext : (T)3.0e38;
  T a = fmin(fmax(ax, -ext), ext), b = fmin(fmax(bx, -ext), ext);
  for (int it = 0; it < iters; ++it) {
    const T h = c[0] + c[1] * a + c[2] * b + c[3] * a * a + c[4] * a * b + c[5] * b * b;
    const T ha = c[1] + (T)2 * c[3] * a + c[4] * b;
    const T hb = c[2] + c[4] * a + (T)2 * c[5] * b;
    const T res = h - hx;
    const T ga = (a - ax) + res * ha;
    const T gb = (b - bx) + res * hb;
    T Haa = (T)1 + ha * ha + res * (T)2 * c[3];
    T Hab = ha * hb + res * c[4];
    T Hbb = (T)1 + hb * hb + res * (T)2 * c[5];
    T det = Haa * Hbb - Hab * Hab;
    if (!(Haa > (T)0 && det > (T)0)) {
      Haa = (T)1 + ha * ha;
      Hab = ha * hb;
      Hbb = (T)1 + hb * hb;
      det = Haa * Hbb - Hab * Hab;
    }
    a = fmin(fmax(a - (Hbb * ga - Hab * gb) / det, -ext), ext);
    b = fmin(fmax(b - (Haa * gb - Hab * ga) / det, -ext), ext);
  }
  CloudProj<T> out;
  const T h = c[0] + c[1] * a + c[2] * b + c[3] * a * a + c[4] * a * b + c[5] * b * b;
  for (int i = 0; i < 3; ++i) out.y[i] = P.cen[i] + a * P.e1[i] + b * P.e2[i] + h * P.n[i];
  const T ha = c[1] + (T)2 * c[3] * a + c[4] * b;
  const T hb = c[2] + c[4] * a + (T)2 * c[5] * b;
  const T gf = sqrt_((T)1 + ha * ha + hb * hb);
  const T I11 = (T)1 + ha * ha, I12 = ha * hb, I22 = (T)1 + hb * hb;
  const T L11 = (T)2 * c[3] / gf, L12 = c[4] / gf, L22 = (T)2 * c[5] / gf;
  const T dI = I11 * I22 - I12 * I12;
  const T S11 = (I22 * L11 - I12 * L12) / dI, S12 = (I22 * L12 - I12 * L22) / dI;
  const T S21 = (I11 * L12 - I12 * L11) / dI, S22 = (I11 * L22 - I12 * L12) / dI;
  const T tr = S11 + S22, dt = S11 * S22 - S12 * S21;
  T disc = tr * tr / (T)4 - dt;
  disc = disc > (T)0 ? disc : (T)0;
  const T sq = sqrt_(disc);
  const T k1 = abs_(tr / (T)2 + sq), k2 = abs_(tr / (T)2 - sq);
  out.kappa = k1 > k2 ? k1 : k2;
  out.hmean = P.hmean;
  return out;
}

template <class T>
__device__ __forceinline__ const Patch<T>& patch_of(const CloudDev& c, int32_t i);
template <>
__device__ __forceinline__ const Patch<double>& patch_of<double>(const CloudDev& c, int32_t i) { return c.patch64[i]; }
template <>
__device__ __forceinline__ const Patch<float>& patch_of<float>(const CloudDev& c, int32_t i) { return c.patch32[i]; }

// cp_h(x) from a start patch (start < 0: the cloud point nearest to x).
template <class T>
__device__ __forceinline__ CloudProj<T> cloud_cp(const CloudDev& c, const T* x, int32_t start = -1) {
  if (c.nn_only) {
    // the nearest cloud point itself; its patch supplies only the spacing
    const int32_t nn = kd_nearest<T>(c, x);
    const float4 p = c.pts[nn];
    CloudProj<T> r;
    r.y[0] = (T)p.x;
    r.y[1] = (T)p.y;
    r.y[2] = (T)p.z;
    r.kappa = (T)0;
    r.hmean = patch_of<T>(c, nn).hmean;
    r.patch = nn;
    return r;
  }
  int32_t p;
  if (start < 0) {
    p = near_surface_nearest<T>(c, x);
  } else {
    const CloudProj<T> y0 = patch_project<T>(patch_of<T>(c, start), x, c.newton_iters, false);
    p = near_surface_nearest<T>(c, y0.y);
  }
  CloudProj<T> r;
  for (int j = 0; j < kCloudRounds; ++j) {
    r = patch_project<T>(patch_of<T>(c, p), x, c.newton_iters);
    if (j == kCloudRounds - 1) break;
    const int32_t q = near_surface_nearest<T>(c, r.y);
    if (q == p) break;
    p = q;
  }
  r.patch = p;
  return r;
}

// rho_geo of a projected point: curvature rule on the fitted patch, or c_h h.
template <class T>
__device__ __forceinline__ double cloud_rho_geo(const WalkArgs& a, const CloudProj<T>& p) {
  if (a.cloud.radius_rule == 1) return a.c_h * (double)p.hmean;
  return a.c_kappa / (1.0 + (double)p.kappa);
}

}  // namespace mpwos
