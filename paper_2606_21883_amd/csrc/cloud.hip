// Point-cloud manifolds: the resident data structures and their one-time build.
//
// At creation the cloud is copied to the device with
//   - a uniform grid (points sorted by cell), used to find, for every cloud
//     point, its k nearest cloud points: one wavefront per tile of up to 32
//     points of a cell; candidates from the 3x3x3 block of cells are staged
//     32 at a time and their dot products with the tile's points computed by
//     one v_mfma_f32_32x32x16_bf16 on coordinates centred on the cell (each
//     coordinate split in two bf16 parts, three of the four cross products
//     kept), giving approximate squared distances with a bound delta; the
//     best 32 by approximate distance are re-ranked exactly in FP64.  The
//     result is exact whenever the k-th exact distance is below both the
//     32nd approximate distance minus delta and the radius the 3x3x3 block
//     covers; other points are recomputed by an exact search.
//   - the local quadratic patch of every point (centroid, PCA frame,
//     least-squares height field), in FP64 and FP32;
//   - a KD-tree for the nearest-point query of the walk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "cloud_dev.h"
#include "host_internal.h"
#include "kernel_args.h"

namespace mpwos {

struct CloudState {
  int64_t n = 0;
  int k = 16;
  KdNode* nodes = nullptr;
  float4* kd_pts = nullptr;
  Patch<double>* patch64 = nullptr;
  Patch<float>* patch32 = nullptr;
  int32_t n_nodes = 0;
  int32_t root = 0;
  double hmean_max = 0.0;
  int64_t fallback_points = 0;
  int32_t nn_only = 0;
  float4* pts = nullptr;       // nn_only: the points by original index (kept from the build)
  // the walk grid (patch reconstruction only)
  int32_t* g_start = nullptr;
  float4* g_pts = nullptr;
  int32_t g_n[3] = {0, 0, 0};
  double g_lo[3] = {0, 0, 0};
  double g_h = 0.0, g_slack = 0.0;
};

struct GridArgs {
  const float4* pts;       // sorted by cell: x, y, z, original index bits
  const float4* orig;      // by original index
  const int32_t* cell_start;
  const int4* tiles;       // cell, first sorted index, count, unused
  int32_t nx, ny, nz;
  float lox, loy, loz, h;
  double slack;            // rounding allowance of the cell binning
  int32_t k;
  int32_t* knn;            // n x k original indices
  uint8_t* flag;           // 1: recompute exactly
  int64_t n;
};

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // round to nearest even
}
__device__ __forceinline__ float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ __bf16 as_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

constexpr int kKeep = 32;

__global__ __launch_bounds__(64) void knn_tile_kernel(GridArgs g) {
  __shared__ float tile_d[32][33];
  __shared__ int32_t tile_id[32];
  __shared__ float qnorm[32];
  const int lane = threadIdx.x;
  const int r = lane & 31, half = lane >> 5;
  const int4 tl = g.tiles[blockIdx.x];
  const int cell = tl.x, first = tl.y, cnt = tl.z;
  const int cx = cell % g.nx, cy = (cell / g.nx) % g.ny, cz = cell / (g.nx * g.ny);
  const float ccx = g.lox + ((float)cx + 0.5f) * g.h;
  const float ccy = g.loy + ((float)cy + 0.5f) * g.h;
  const float ccz = g.loz + ((float)cz + 0.5f) * g.h;
  const bool has_q = r < cnt;
  float4 q = has_q ? g.pts[first + r] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float qx = q.x - ccx, qy = q.y - ccy, qz = q.z - ccz;
  const uint16_t qxh = bf16_bits(qx), qyh = bf16_bits(qy), qzh = bf16_bits(qz);
  const uint16_t qxl = bf16_bits(qx - bf16_value(qxh)), qyl = bf16_bits(qy - bf16_value(qyh));
  const uint16_t qzl = bf16_bits(qz - bf16_value(qzh));
  bf16x8 A;
  if (half == 0) {
    A[0] = as_bf16(qxh); A[1] = as_bf16(qyh); A[2] = as_bf16(qzh);
    A[3] = as_bf16(qxh); A[4] = as_bf16(qyh); A[5] = as_bf16(qzh);
    A[6] = as_bf16(qxl); A[7] = as_bf16(qyl);
  } else {
    A[0] = as_bf16(qzl);
    for (int t = 1; t < 8; ++t) A[t] = as_bf16(0);
  }
  if (!has_q)
    for (int t = 0; t < 8; ++t) A[t] = as_bf16(0);
  if (half == 0) qnorm[r] = qx * qx + qy * qy + qz * qz;
  float ld[kKeep];
  int32_t li[kKeep];
  int nk = 0;
  __syncthreads();
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int ax = cx + dx, ay = cy + dy, az = cz + dz;
        if (ax < 0 || ay < 0 || az < 0 || ax >= g.nx || ay >= g.ny || az >= g.nz) continue;
        const int nc = (az * g.ny + ay) * g.nx + ax;
        const int cs = g.cell_start[nc], ce = g.cell_start[nc + 1];
        for (int cb = cs; cb < ce; cb += 32) {
          const int j = cb + r;
          const bool valid = j < ce;
          const float4 p = valid ? g.pts[j] : make_float4(0.f, 0.f, 0.f, 0.f);
          const float px = p.x - ccx, py = p.y - ccy, pz = p.z - ccz;
          const uint16_t pxh = bf16_bits(px), pyh = bf16_bits(py), pzh = bf16_bits(pz);
          bf16x8 B;
          if (half == 0) {
            B[0] = as_bf16(pxh); B[1] = as_bf16(pyh); B[2] = as_bf16(pzh);
            B[3] = as_bf16(bf16_bits(px - bf16_value(pxh)));
            B[4] = as_bf16(bf16_bits(py - bf16_value(pyh)));
            B[5] = as_bf16(bf16_bits(pz - bf16_value(pzh)));
            B[6] = as_bf16(pxh); B[7] = as_bf16(pyh);
          } else {
            B[0] = as_bf16(pzh);
            for (int t = 1; t < 8; ++t) B[t] = as_bf16(0);
          }
          const float pn = px * px + py * py + pz * pz;
          f32x16 acc = {};
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc, 0, 0, 0);
          // lane holds column r (candidate), rows 8*(t/4) + 4*half + t%4
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            const int i = 8 * (t / 4) + 4 * half + (t % 4);
            tile_d[i][r] = qnorm[i] + pn - 2.0f * acc[t];
          }
          if (half == 0) tile_id[r] = valid ? __float_as_int(p.w) : -1;
          __syncthreads();
          if (half == 0 && has_q) {
            for (int jj = 0; jj < 32; ++jj) {
              const int32_t id = tile_id[jj];
              if (id < 0) continue;
              const float d = tile_d[r][jj];
              if (nk < kKeep || d < ld[kKeep - 1]) {
                int pos = nk < kKeep ? nk : kKeep - 1;
                while (pos > 0 && ld[pos - 1] > d) {
                  ld[pos] = ld[pos - 1];
                  li[pos] = li[pos - 1];
                  --pos;
                }
                ld[pos] = d;
                li[pos] = id;
                if (nk < kKeep) ++nk;
              }
            }
          }
          __syncthreads();
        }
      }
  if (half != 0 || !has_q) return;
  // exact FP64 re-rank of the kept candidates, ordered by (distance^2, index)
  const double xq[3] = {(double)q.x, (double)q.y, (double)q.z};
  double ed[kKeep];
  int32_t ei[kKeep];
  for (int m = 0; m < nk; ++m) {
    const float4 p = g.orig[li[m]];
    const double d2 = dist2_exact(xq, p.x, p.y, p.z);
    int pos = m;
    while (pos > 0 && (ed[pos - 1] > d2 || (ed[pos - 1] == d2 && ei[pos - 1] > li[m]))) {
      ed[pos] = ed[pos - 1];
      ei[pos] = ei[pos - 1];
      --pos;
    }
    ed[pos] = d2;
    ei[pos] = li[m];
  }
  const int32_t self = __float_as_int(q.w);
  bool ok = nk >= g.k;
  if (ok && nk == kKeep) {
    const double delta = 1e-3 * (double)g.h * (double)g.h;
    ok = ed[g.k - 1] < (double)ld[kKeep - 1] - delta;
  }
  if (ok) {
    // radius the 3x3x3 block covers around q (faces at the grid edge hold no points)
    double gr = 1e300;
    const double hb = 1.5 * (double)g.h;
    const double cc[3] = {(double)ccx, (double)ccy, (double)ccz};
    const int ci[3] = {cx, cy, cz}, nd[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
      if (ci[d] > 0) gr = fmin(gr, xq[d] - (cc[d] - hb));
      if (ci[d] < nd[d] - 1) gr = fmin(gr, (cc[d] + hb) - xq[d]);
    }
    gr -= g.slack;
    ok = gr > 0.0 && ed[g.k - 1] < gr * gr;
  }
  g.flag[self] = ok ? 0 : 1;
  if (ok)
    for (int t = 0; t < g.k; ++t) g.knn[(int64_t)self * g.k + t] = ei[t];
}

// Exact k nearest points of each flagged point: the depth-first KD-tree
// search of the walk's nearest-point query, keeping the k best (ordered by
// distance^2, then original index) and pruning boxes strictly farther than the
// current k-th distance.
__global__ void knn_kd_kernel(const KdNode* __restrict__ nodes, int32_t root, const float4* __restrict__ kd_pts,
                              const float4* __restrict__ orig, int32_t k, const int32_t* list, int32_t nlist,
                              int32_t* knn) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlist) return;
  const int32_t self = list[t];
  const float4 q = orig[self];
  const double xq[3] = {(double)q.x, (double)q.y, (double)q.z};
  double ed[kMaxK];
  int32_t ei[kMaxK];
  int nk = 0;
  int32_t sref[kKdStack];
  double sdist[kKdStack];
  int sp = 0;
  int32_t ref = root;
  auto bound = [&]() { return nk == k ? ed[k - 1] : 1e300; };
  for (;;) {
    if (ref < 0) {
      const int32_t start = leaf_start(ref), end = start + leaf_count(ref);
      for (int32_t i = start; i < end; ++i) {
        const float4 p = kd_pts[i];
        const double d2 = dist2_exact(xq, p.x, p.y, p.z);
        const int32_t id = __float_as_int(p.w);
        if (nk == k && !(d2 < ed[k - 1] || (d2 == ed[k - 1] && id < ei[k - 1]))) continue;
        int pos = nk < k ? nk : k - 1;
        while (pos > 0 && (ed[pos - 1] > d2 || (ed[pos - 1] == d2 && ei[pos - 1] > id))) {
          ed[pos] = ed[pos - 1];
          ei[pos] = ei[pos - 1];
          --pos;
        }
        ed[pos] = d2;
        ei[pos] = id;
        if (nk < k) ++nk;
      }
    } else {
      const KdNode nd = nodes[ref];
      const double d0 = box_dist2<double>(nd.lo[0], nd.hi[0], xq);
      const double d1 = box_dist2<double>(nd.lo[1], nd.hi[1], xq);
      const bool first = d0 <= d1;
      const double dn = first ? d0 : d1, df = first ? d1 : d0;
      if (df <= bound() && sp < kKdStack) {
        sref[sp] = first ? nd.child[1] : nd.child[0];
        sdist[sp] = df;
        ++sp;
      }
      if (dn <= bound()) {
        ref = first ? nd.child[0] : nd.child[1];
        continue;
      }
    }
    bool more = false;
    while (sp > 0) {
      --sp;
      if (sdist[sp] <= bound()) {
        ref = sref[sp];
        more = true;
        break;
      }
    }
    if (!more) break;
  }
  for (int m = 0; m < k; ++m) knn[(int64_t)self * k + m] = ei[m];
}

// Symmetric 3x3 eigenvectors by cyclic Jacobi rotations; columns of V sorted
// by ascending eigenvalue.
__device__ void eig3(double A[3][3], double V[3][3], double w[3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off == 0.0 || off <= 1e-34 * dg) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  w[0] = A[0][0]; w[1] = A[1][1]; w[2] = A[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (w[j] < w[i]) {
        const double tw = w[i]; w[i] = w[j]; w[j] = tw;
        for (int k = 0; k < 3; ++k) { const double tv = V[k][i]; V[k][i] = V[k][j]; V[k][j] = tv; }
      }
}

// Height-field coefficients from the normal equations M c = rhs of the scaled
// basis 1, a/sc, b/sc, (a/sc)^2, ab/sc^2, (b/sc)^2 (Cholesky), then the patch in
// FP64 and FP32.
__device__ void finish_patch(const double cen[3], const double e1[3], const double e2[3], const double nn[3],
                             double M[6][6], double rhs[6], double sc, double ext, double hmean,
                             Patch<double>& P64, Patch<float>& P32) {
  double L[6][6];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c <= r; ++c) {
      double s = M[r][c];
      for (int t = 0; t < c; ++t) s -= L[r][t] * L[c][t];
      L[r][c] = (r == c) ? sqrt(fmax(s, 1e-300)) : s / L[c][c];
    }
  double y[6], cf[6];
  for (int r = 0; r < 6; ++r) {
    double s = rhs[r];
    for (int t = 0; t < r; ++t) s -= L[r][t] * y[t];
    y[r] = s / L[r][r];
  }
  for (int r = 5; r >= 0; --r) {
    double s = y[r];
    for (int t = r + 1; t < 6; ++t) s -= L[t][r] * cf[t];
    cf[r] = s / L[r][r];
  }
  // undo the scaling of a and b
  cf[1] /= sc; cf[2] /= sc; cf[3] /= sc * sc; cf[4] /= sc * sc; cf[5] /= sc * sc;
  Patch<double> P;
  for (int d = 0; d < 3; ++d) {
    P.cen[d] = cen[d]; P.e1[d] = e1[d]; P.e2[d] = e2[d]; P.n[d] = nn[d];
  }
  for (int t = 0; t < 6; ++t) P.c[t] = cf[t];
  P.ext = ext;
  P.hmean = hmean;
  P64 = P;
  Patch<float> Q;
  for (int d = 0; d < 3; ++d) {
    Q.cen[d] = (float)cen[d]; Q.e1[d] = (float)e1[d]; Q.e2[d] = (float)e2[d]; Q.n[d] = (float)nn[d];
  }
  for (int t = 0; t < 6; ++t) Q.c[t] = (float)cf[t];
  Q.ext = (float)ext;
  Q.hmean = (float)hmean;
  P32 = Q;
}

// Local quadratic patch of every point from its k nearest points: centroid,
// PCA frame (normal = least-variance direction), height field by least
// squares on the scaled basis 1, a, b, a^2, a b, b^2 (Cholesky on the normal
// equations), and the mean distance to the other k-1 neighbours.
__global__ void fit_kernel(GridArgs g, Patch<double>* P64, Patch<float>* P32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int k = g.k;
  const int32_t* nb = g.knn + i * k;
  const float4 pi = g.orig[i];
  const double xi[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
  double cen[3] = {0, 0, 0}, hs = 0.0;
  for (int j = 0; j < k; ++j) {
    const float4 p = g.orig[nb[j]];
    cen[0] += (double)p.x; cen[1] += (double)p.y; cen[2] += (double)p.z;
    if (j > 0) hs += sqrt(dist2_exact(xi, p.x, p.y, p.z));
  }
  for (int d = 0; d < 3; ++d) cen[d] /= (double)k;
  double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int j = 0; j < k; ++j) {
    const float4 p = g.orig[nb[j]];
    const double d[3] = {(double)p.x - cen[0], (double)p.y - cen[1], (double)p.z - cen[2]};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[r][c] += d[r] * d[c];
  }
  double V[3][3], w[3];
  eig3(C, V, w);
  const double e1[3] = {V[0][2], V[1][2], V[2][2]};
  const double e2[3] = {V[0][1], V[1][1], V[2][1]};
  const double nn[3] = {V[0][0], V[1][0], V[2][0]};
  double sc = 0.0;
  for (int j = 0; j < k; ++j) {
    const float4 p = g.orig[nb[j]];
    const double d[3] = {(double)p.x - cen[0], (double)p.y - cen[1], (double)p.z - cen[2]};
    sc = fmax(sc, fabs(d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2]));
    sc = fmax(sc, fabs(d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2]));
  }
  const double ext = sc;
  sc = sc > 0.0 ? sc : 1.0;
  double M[6][6], rhs[6];
  for (int r = 0; r < 6; ++r) {
    rhs[r] = 0.0;
    for (int c = 0; c < 6; ++c) M[r][c] = 0.0;
  }
  for (int j = 0; j < k; ++j) {
    const float4 p = g.orig[nb[j]];
    const double d[3] = {(double)p.x - cen[0], (double)p.y - cen[1], (double)p.z - cen[2]};
    const double a = (d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2]) / sc;
    const double b = (d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2]) / sc;
    const double h = d[0] * nn[0] + d[1] * nn[1] + d[2] * nn[2];
    const double ph[6] = {1.0, a, b, a * a, a * b, b * b};
    for (int r = 0; r < 6; ++r) {
      rhs[r] += ph[r] * h;
      for (int c = 0; c < 6; ++c) M[r][c] += ph[r] * ph[c];
    }
  }
  finish_patch(cen, e1, e2, nn, M, rhs, sc, ext, hs / (double)(k - 1), P64[i], P32[i]);
}

// The patch of every point fitted to the cloud points within fit_scale r_k of
// it (r_k: the distance to its k-th nearest point; ball membership
// |p - x_i|^2 <= (fit_scale^2) r_k^2 in exact FP64 products and sums), found
// on the uniform grid: the cells within the ball's bounding box (one cell of
// margin for the binning's rounding).  Two passes over the ball: moments about
// x_i give the centroid and covariance (PCA frame); then the normal
// equations of the height field on the basis scaled by the ball radius, and
// the patch support.  The spacing stays the mean distance to the k-1 nearest.
__global__ void fit_ball_kernel(GridArgs g, double fit_scale, Patch<double>* P64, Patch<float>* P32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int k = g.k;
  const int32_t* nb = g.knn + i * k;
  const float4 pi = g.orig[i];
  const double xi[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
  double hs = 0.0;
  for (int j = 1; j < k; ++j) {
    const float4 p = g.orig[nb[j]];
    hs += sqrt(dist2_exact(xi, p.x, p.y, p.z));
  }
  const float4 pk = g.orig[nb[k - 1]];
  const double rho2 = __dmul_rn(__dmul_rn(fit_scale, fit_scale), dist2_exact(xi, pk.x, pk.y, pk.z));
  const double rho = sqrt(rho2);
  const double lo[3] = {(double)g.lox, (double)g.loy, (double)g.loz};
  const int nc[3] = {g.nx, g.ny, g.nz};
  int ca[3], cb[3];
  for (int d = 0; d < 3; ++d) {
    ca[d] = max(0, (int)floor((xi[d] - rho - lo[d]) / (double)g.h) - 1);
    cb[d] = min(nc[d] - 1, (int)floor((xi[d] + rho - lo[d]) / (double)g.h) + 1);
  }
  // visit(f): f(offset from x_i) for every point of the ball
  auto visit = [&](auto&& f) {
    for (int cz = ca[2]; cz <= cb[2]; ++cz)
      for (int cy = ca[1]; cy <= cb[1]; ++cy) {
        const int row = (cz * g.ny + cy) * g.nx;
        const int s0 = g.cell_start[row + ca[0]], s1 = g.cell_start[row + cb[0] + 1];
        for (int t = s0; t < s1; ++t) {
          const float4 p = g.pts[t];
          if (dist2_exact(xi, p.x, p.y, p.z) <= rho2) {
            const double d[3] = {(double)p.x - xi[0], (double)p.y - xi[1], (double)p.z - xi[2]};
            f(d);
          }
        }
      }
  };
  double cnt = 0.0, m1[3] = {0, 0, 0}, m2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  visit([&](const double* d) {
    cnt += 1.0;
    for (int r = 0; r < 3; ++r) {
      m1[r] += d[r];
      for (int c = 0; c < 3; ++c) m2[r][c] += d[r] * d[c];
    }
  });
  double mu[3], cen[3], C[3][3];
  for (int r = 0; r < 3; ++r) {
    mu[r] = m1[r] / cnt;
    cen[r] = xi[r] + mu[r];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) C[r][c] = m2[r][c] - cnt * mu[r] * mu[c];
  double V[3][3], w[3];
  eig3(C, V, w);
  const double e1[3] = {V[0][2], V[1][2], V[2][2]};
  const double e2[3] = {V[0][1], V[1][1], V[2][1]};
  const double nn[3] = {V[0][0], V[1][0], V[2][0]};
  const double sc = rho > 0.0 ? rho : 1.0;
  double M[6][6], rhs[6], ext = 0.0;
  for (int r = 0; r < 6; ++r) {
    rhs[r] = 0.0;
    for (int c = 0; c < 6; ++c) M[r][c] = 0.0;
  }
  visit([&](const double* d0) {
    const double d[3] = {d0[0] - mu[0], d0[1] - mu[1], d0[2] - mu[2]};
    const double a = d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2];
    const double b = d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2];
    const double h = d[0] * nn[0] + d[1] * nn[1] + d[2] * nn[2];
    ext = fmax(ext, fmax(fabs(a), fabs(b)));
    const double as = a / sc, bs = b / sc;
    const double ph[6] = {1.0, as, bs, as * as, as * bs, bs * bs};
    for (int r = 0; r < 6; ++r) {
      rhs[r] += ph[r] * h;
      for (int c = 0; c < 6; ++c) M[r][c] += ph[r] * ph[c];
    }
  });
  finish_patch(cen, e1, e2, nn, M, rhs, sc, ext, hs / (double)(k - 1), P64[i], P32[i]);
}

// Distance from each query to its FP64 projection, and the local spacing there.
__global__ void cloud_query_check_kernel(CloudDev c, const double* __restrict__ q, double* __restrict__ out,
                                         int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double x[3] = {q[3 * i], q[3 * i + 1], q[3 * i + 2]};
  const CloudProj<double> p = cloud_cp<double>(c, x);
  const double d0 = p.y[0] - x[0], d1 = p.y[1] - x[1], d2 = p.y[2] - x[2];
  out[2 * i] = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  out[2 * i + 1] = p.hmean;
}

// ---------------------------------------------------------------------------
// host: grid, KD-tree, build sequence
// ---------------------------------------------------------------------------
namespace {

struct HostKd {
  std::vector<KdNode> nodes;
  std::vector<int32_t> order;
};

struct HostBox {
  float lo[3], hi[3];
};

// Median split on the widest axis of the subtree's box, leaves of at most 8
// points.  Returns the subtree's reference (internal node index, or a leaf
// reference) and its box.
int32_t kd_build(HostKd& t, const std::vector<float>& P, int lo, int hi, HostBox& bx) {
  for (int d = 0; d < 3; ++d) { bx.lo[d] = 3e38f; bx.hi[d] = -3e38f; }
  for (int i = lo; i < hi; ++i)
    for (int d = 0; d < 3; ++d) {
      bx.lo[d] = std::min(bx.lo[d], P[3 * t.order[i] + d]);
      bx.hi[d] = std::max(bx.hi[d], P[3 * t.order[i] + d]);
    }
  if (hi - lo <= 8) return -(lo * 16 + (hi - lo)) - 1;
  int dim = 0;
  for (int d = 1; d < 3; ++d)
    if (bx.hi[d] - bx.lo[d] > bx.hi[dim] - bx.lo[dim]) dim = d;
  const int mid = (lo + hi) / 2;
  std::nth_element(t.order.begin() + lo, t.order.begin() + mid, t.order.begin() + hi, [&](int a, int b) {
    const float va = P[3 * a + dim], vb = P[3 * b + dim];
    return va < vb || (va == vb && a < b);
  });
  const int id = (int)t.nodes.size();
  t.nodes.emplace_back();
  HostBox bl, br;
  const int32_t l = kd_build(t, P, lo, mid, bl);
  const int32_t r = kd_build(t, P, mid, hi, br);
  KdNode& nd = t.nodes[id];
  for (int d = 0; d < 3; ++d) {
    nd.lo[0][d] = bl.lo[d]; nd.hi[0][d] = bl.hi[d];
    nd.lo[1][d] = br.lo[d]; nd.hi[1][d] = br.hi[d];
  }
  nd.child[0] = l;
  nd.child[1] = r;
  nd.count[0] = l < 0 ? mid - lo : 0;
  nd.count[1] = r < 0 ? hi - mid : 0;
  return id;
}

template <class T>
T* upload(const std::vector<T>& v, hipError_t& e) {
  T* p = nullptr;
  if (e != hipSuccess || v.empty()) return nullptr;
  e = hipMalloc((void**)&p, v.size() * sizeof(T));
  if (e == hipSuccess) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return p;
}

}  // namespace

mpwos_status cloud_create(const mpwos_manifold_desc& d, hipStream_t s, CloudState** out) {
  const int64_t n = d.n_points;
  const int k = d.k_nn;
  std::vector<float> P((size_t)n * 3);
  hipError_t e = hipSuccess;
  if (d.points_on_device) e = hipMemcpy(P.data(), d.points, P.size() * sizeof(float), hipMemcpyDeviceToHost);
  else memcpy(P.data(), d.points, P.size() * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "point cloud copy");
  float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      const float v = P[3 * i + c];
      if (!std::isfinite(v)) return fail(MPWOS_EINVAL, "point cloud holds a non-finite coordinate");
      lo[c] = std::min(lo[c], v);
      hi[c] = std::max(hi[c], v);
    }
  // cell size: about k points per non-empty cell, so the 3x3x3 block reaches
  // past the k-th neighbour of almost every point
  double ext = std::max({(double)hi[0] - lo[0], (double)hi[1] - lo[1], (double)hi[2] - lo[2], 1e-30});
  double h = ext / std::cbrt((double)n);
  for (int it = 0; it < 4; ++it) {
    std::unordered_map<int64_t, int> occ;
    occ.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t a = (int64_t)((P[3 * i] - lo[0]) / h), b = (int64_t)((P[3 * i + 1] - lo[1]) / h),
                    c = (int64_t)((P[3 * i + 2] - lo[2]) / h);
      occ[(a * 1000003 + b) * 1000033 + c] += 1;
    }
    const double mean = (double)n / (double)occ.size();
    h *= std::sqrt((double)k / mean);
  }
  auto cells = [&](int c) { return std::floor(((double)hi[c] - (double)lo[c]) / h) + 1.0; };
  while (cells(0) * cells(1) * cells(2) > (double)(1 << 24)) h *= 1.25;
  const int nx = (int)cells(0), ny = (int)cells(1), nz = (int)cells(2);
  const int64_t ncell = (int64_t)nx * ny * nz;
  std::vector<int32_t> cell((size_t)n), ord((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    const int a = std::min(nx - 1, (int)((P[3 * i] - lo[0]) / h));
    const int b = std::min(ny - 1, (int)((P[3 * i + 1] - lo[1]) / h));
    const int c = std::min(nz - 1, (int)((P[3 * i + 2] - lo[2]) / h));
    cell[i] = (int32_t)(((int64_t)c * ny + b) * nx + a);
  }
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cell[a] < cell[b]; });
  std::vector<int32_t> cstart((size_t)ncell + 1, 0);
  for (int64_t i = 0; i < n; ++i) cstart[cell[i] + 1] += 1;
  for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  std::vector<float4> sorted((size_t)n), orig((size_t)n);
  std::vector<int4> tiles;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t o = ord[i];
    int32_t ob;
    memcpy(&ob, &o, 4);
    float w;
    memcpy(&w, &ob, 4);
    sorted[i] = make_float4(P[3 * o], P[3 * o + 1], P[3 * o + 2], w);
  }
  for (int64_t i = 0; i < n; ++i) {
    const int32_t o = (int32_t)i;
    float w;
    memcpy(&w, &o, 4);
    orig[i] = make_float4(P[3 * i], P[3 * i + 1], P[3 * i + 2], w);
  }
  for (int64_t c = 0; c < ncell; ++c)
    for (int32_t s0 = cstart[c]; s0 < cstart[c + 1]; s0 += 32)
      tiles.push_back(make_int4((int)c, s0, std::min(32, cstart[c + 1] - s0), 0));
  HostKd kd;
  kd.order.resize((size_t)n);
  std::iota(kd.order.begin(), kd.order.end(), 0);
  kd.nodes.reserve((size_t)(n / 4 + 16));
  HostBox root_box;
  const int32_t root = kd_build(kd, P, 0, (int)n, root_box);
  std::vector<float4> kdp((size_t)n);
  for (int64_t i = 0; i < n; ++i) kdp[i] = orig[kd.order[i]];

  auto* C = new CloudState;
  C->n = n;
  C->k = k;
  C->n_nodes = (int32_t)kd.nodes.size();
  C->root = root;
  float4 *d_sorted = upload(sorted, e), *d_orig = upload(orig, e);
  int32_t* d_cstart = upload(cstart, e);
  int4* d_tiles = upload(tiles, e);
  C->nodes = upload(kd.nodes, e);
  C->kd_pts = upload(kdp, e);
  // The walk grid of the patch reconstruction: cells with about one and a
  // half points each where the surface crosses them (the build grid's cells
  // hold about k), so a near-surface lookup scans a few dozen points; at most
  // 2^26 cells.  (On the 1e6-point torus, cells of about three points ran
  // 7% slower, one point 2% slower: fewer points per lookup against a larger
  // table of cell starts.)  Points are binned in FP64 as the device locates
  // a query.
  if (e == hipSuccess && d.reconstruction == 0) {
    double hw = h * std::min(1.0, std::sqrt(1.5 / (double)std::max(k, 1)));
    auto wcells = [&](int c) { return std::floor(((double)hi[c] - (double)lo[c]) / hw) + 1.0; };
    while (wcells(0) * wcells(1) * wcells(2) > (double)(1 << 26)) hw *= 1.25;
    const int wn[3] = {(int)wcells(0), (int)wcells(1), (int)wcells(2)};
    const int64_t ncw = (int64_t)wn[0] * wn[1] * wn[2];
    std::vector<int32_t> wcell((size_t)n), wstart((size_t)ncw + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      int64_t cc[3];
      for (int c = 0; c < 3; ++c)
        cc[c] = std::min<int64_t>(wn[c] - 1, (int64_t)(((double)P[3 * i + c] - (double)lo[c]) / hw));
      wcell[i] = (int32_t)((cc[2] * wn[1] + cc[1]) * wn[0] + cc[0]);
      wstart[wcell[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncw; ++c) wstart[c + 1] += wstart[c];
    std::vector<int32_t> fill(wstart.begin(), wstart.end() - 1);
    std::vector<float4> wpts((size_t)n);
    for (int64_t i = 0; i < n; ++i) wpts[fill[wcell[i]]++] = orig[i];
    C->g_start = upload(wstart, e);
    C->g_pts = upload(wpts, e);
    double amax = 0.0;
    for (int c = 0; c < 3; ++c) {
      C->g_n[c] = wn[c];
      C->g_lo[c] = (double)lo[c];
      amax = std::max({amax, std::fabs((double)lo[c]), std::fabs((double)hi[c])});
    }
    C->g_h = hw;
    C->g_slack = 1e-6 * hw + 1e-12 * amax;
  }
  int32_t* d_knn = nullptr;
  uint8_t* d_flag = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&d_knn, (size_t)n * k * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&d_flag, (size_t)n);
  if (e == hipSuccess) e = hipMalloc((void**)&C->patch64, (size_t)n * sizeof(Patch<double>));
  if (e == hipSuccess) e = hipMalloc((void**)&C->patch32, (size_t)n * sizeof(Patch<float>));
  GridArgs g;
  g.pts = d_sorted; g.orig = d_orig; g.cell_start = d_cstart; g.tiles = d_tiles;
  g.nx = nx; g.ny = ny; g.nz = nz; g.lox = lo[0]; g.loy = lo[1]; g.loz = lo[2]; g.h = (float)h;
  g.k = k; g.knn = d_knn; g.flag = d_flag; g.n = n;
  {
    double amax = 0.0;
    for (int c = 0; c < 3; ++c) amax = std::max({amax, std::fabs((double)lo[c]), std::fabs((double)hi[c])});
    g.slack = 1e-4 * h + 1e-6 * amax;
  }
  if (e == hipSuccess && k <= kKeep - 8 && !tiles.empty()) {
    hipLaunchKernelGGL(knn_tile_kernel, dim3((unsigned)tiles.size()), dim3(64), 0, s, g);
    e = hipGetLastError();
  } else if (e == hipSuccess) {
    e = hipMemsetAsync(d_flag, 1, (size_t)n, s);
  }
  std::vector<uint8_t> flag((size_t)n);
  if (e == hipSuccess) e = hipMemcpyAsync(flag.data(), d_flag, (size_t)n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  std::vector<int32_t> redo;
  for (int64_t i = 0; i < n; ++i)
    if (flag[i]) redo.push_back((int32_t)i);
  C->fallback_points = (int64_t)redo.size();
  int32_t* d_redo = upload(redo, e);
  if (e == hipSuccess && !redo.empty()) {
    hipLaunchKernelGGL(knn_kd_kernel, dim3((unsigned)((redo.size() + 63) / 64)), dim3(64), 0, s, C->nodes,
                       C->root, C->kd_pts, d_orig, k, d_redo, (int32_t)redo.size(), d_knn);
    e = hipGetLastError();
  }
  if (e == hipSuccess && d.fit_scale > 1.0 && d.reconstruction == 0) {
    hipLaunchKernelGGL(fit_ball_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, g, d.fit_scale,
                       C->patch64, C->patch32);
    e = hipGetLastError();
  } else if (e == hipSuccess) {
    hipLaunchKernelGGL(fit_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, g, C->patch64, C->patch32);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  // the nearest-point projection reads the points by original index
  if (d.reconstruction == 1) {
    C->nn_only = 1;
    C->pts = d_orig;
    d_orig = nullptr;
  }
  for (void* p : {(void*)d_sorted, (void*)d_orig, (void*)d_cstart, (void*)d_tiles, (void*)d_knn, (void*)d_flag,
                  (void*)d_redo})
    if (p) (void)hipFree(p);
  if (e != hipSuccess) {
    cloud_destroy(C);
    return hip_fail(e, "point cloud build");
  }
  // largest local spacing (bounds the spacing-rule radius)
  {
    std::vector<Patch<double>> host((size_t)n);
    if (hipMemcpy(host.data(), C->patch64, host.size() * sizeof(Patch<double>), hipMemcpyDeviceToHost) == hipSuccess)
      for (auto& q : host) C->hmean_max = std::max(C->hmean_max, q.hmean);
  }
  *out = C;
  return MPWOS_OK;
}

void cloud_destroy(CloudState* c) {
  if (!c) return;
  for (void* p : {(void*)c->nodes, (void*)c->kd_pts, (void*)c->patch64, (void*)c->patch32, (void*)c->pts,
                  (void*)c->g_start, (void*)c->g_pts})
    if (p) (void)hipFree(p);
  delete c;
}

double cloud_spacing_rmax(const CloudState* c, const mpwos_options& o) { return o.theta * o.c_h * c->hmean_max; }

void cloud_fill_args(const CloudState* c, const mpwos_options& o, WalkArgs& a) {
  a.cloud.nodes = c->nodes;
  a.cloud.kd_pts = c->kd_pts;
  a.cloud.patch64 = c->patch64;
  a.cloud.patch32 = c->patch32;
  a.cloud.n_points = c->n;
  a.cloud.n_nodes = c->n_nodes;
  a.cloud.root = c->root;
  a.cloud.k = c->k;
  a.cloud.newton_iters = o.newton_iters;
  a.cloud.radius_rule = o.radius_rule == MPWOS_RADIUS_SPACING ? 1 : 0;
  a.cloud.nn_only = c->nn_only;
  a.cloud.pts = c->pts;
  a.cloud.g_start = c->g_start;
  a.cloud.g_pts = c->g_pts;
  for (int d = 0; d < 3; ++d) {
    a.cloud.g_n[d] = c->g_n[d];
    a.cloud.g_lo[d] = c->g_lo[d];
  }
  a.cloud.g_h = c->g_h;
  a.cloud.g_inv = c->g_h > 0.0 ? 1.0 / c->g_h : 0.0;
  a.cloud.g_slack = c->g_slack;
}

int cloud_nn_only(const CloudState* c) { return c->nn_only; }

int64_t cloud_fallback_points(const CloudState* c) { return c->fallback_points; }
double cloud_max_spacing(const CloudState* c) { return c->hmean_max; }

// A point-cloud query is an ambient point within two local spacings of the
// reconstructed surface (the walk starts from its projection).
hipError_t launch_cloud_check(const WalkArgs& a, const double* dq, double* out, int64_t nq, hipStream_t s) {
  hipLaunchKernelGGL(cloud_query_check_kernel, dim3((unsigned)((nq + kCloudBlock - 1) / kCloudBlock)),
                     dim3(kCloudBlock), 0, s, a.cloud, dq, out, nq);
  return hipGetLastError();
}

mpwos_status cloud_check_queries(const WalkArgs& a, const double* dq, int64_t nq, hipStream_t s, double* out_dev,
                                 int64_t out_cap) {
  double* dout = out_dev;
  int64_t batch = out_cap / 2;
  if (!dout) {
    const size_t bytes = (size_t)nq * 2 * sizeof(double);
    hipError_t e = hipMalloc((void**)&dout, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(MPWOS_ENOMEM, "query check buffer");
    }
    batch = nq;
  }
  if (batch < 1) return fail(MPWOS_EINVAL, "query check buffer too small");
  std::vector<double> out((size_t)std::min(batch, nq) * 2);
  hipError_t e = hipSuccess;
  mpwos_status st = MPWOS_OK;
  for (int64_t q0 = 0; q0 < nq && e == hipSuccess && !st; q0 += batch) {
    const int64_t nb = std::min(batch, nq - q0);
    hipLaunchKernelGGL(cloud_query_check_kernel, dim3((unsigned)((nb + kCloudBlock - 1) / kCloudBlock)),
                       dim3(kCloudBlock), 0, s, a.cloud, dq + q0 * 3, dout, nb);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), dout, (size_t)nb * 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    for (int64_t i = 0; i < nb; ++i)
      if (!(out[2 * i] <= 2.0 * out[2 * i + 1])) {
        st = fail(MPWOS_EOFFMANIFOLD, "query " + std::to_string(q0 + i) + " is farther than two local spacings "
                                      "from the reconstructed surface");
        break;
      }
  }
  if (!out_dev) (void)hipFree(dout);
  if (e != hipSuccess) return hip_fail(e, "query check");
  return st;
}

}  // namespace mpwos
