// Plain-old-data arguments shared by the host orchestration and the gfx950
// walk kernels.  Passed by value as kernel arguments.
#pragma once
#include <stdint.h>

namespace mpwos {

constexpr int kMaxJ = 32;       // series terms kept for the radial law
constexpr int kMaxK = 32;       // point-cloud neighbours

enum Kind : int32_t { kSphere = 0, kCap = 1, kTorus = 2, kCloud = 3, kDumbbell = 4, kProduct = 5, kCutTorus = 6 };
enum FnKind : int32_t {
  kFnZero = 0, kFnConst = 1, kFnSphPair = 2, kFnCircle = 3, kFnLegendre = 4, kFnTorus = 5, kFnTableS1 = 6,
  kFnDumbbell = 7, kFnProduct = 8, kFnTorusSine = 9
};
// compensation modes (WalkArgs::comp)
enum Comp : int32_t { kCompNone = 0, kCompExact = 1, kCompSecondOrder = 2 };

// A source / boundary family as the device sees it.
struct FnDev {
  int32_t kind;
  int32_t idx[3];
  double coef[8];
  const double* values;   // device copy of a TABLE_S1 table (2M doubles), the dumbbell diagonal (n-1),
                          // or a TORUS_SINE series (idx[0] rows of 2 idx[1] + 1, then idx[2] predictor rows)
  int64_t m;              // M (table length of one half); n - 1 for the dumbbell diagonal
  double lam;             // eigenvalue of the family (sphere families); trace of the dumbbell diagonal
  double u_scale;         // u = u_scale * f for eigen families
};

// Coefficients of the radial law of the normalised Green density for one
// dimension n (independent of the radius).
//   S_nu(x)      = sum_j alpha[j]  z^j, z = x^2
//   S_{nu+1}(x)  = sum_j alpha1[j] z^j
//   D(s)         = sum_{j != nu} bd[j] X^{2j} (s^{2j} - s^{2 nu}) - beta_nu X^{2 nu} s^{2 nu} ln s
struct RadialLaw {
  int32_t n;
  int32_t nu_int;         // nu when n is even (log term index), else -1
  int32_t js;             // terms used for S_nu and S_{nu+1}
  int32_t jd;             // terms used for D
  double nu;
  double inv_2nu1;        // 1 / (2 (nu + 1))
  double alpha[kMaxJ];
  double alpha1[kMaxJ];
  double bd[kMaxJ];       // beta_j / (2 (nu - j)); at j == nu_int: beta_nu
};

// The same law with a fixed X = sqrt(sigma) r folded in.
struct RadialFixed {
  double X2;
  double A[kMaxJ];        // alpha[j] X^{2j} (A[0] unused)
  double A1[kMaxJ];       // alpha1[j] X^{2j}
  double B[kMaxJ];        // bd[j] X^{2j} (0 at the log index)
  double Q1;              // sum_j B[j]
  double L;               // beta_nu X^{2nu} (log term), 0 when n is odd
  double norm;            // 1 / (1 - c)
};

// Inverse-CDF guess table.  For each of mx radius slices, two halves of mu
// points each: the lower half holds s at u = w^2, the upper half s at
// u = 1 - w^2, with w = sqrt(1/2) i/(mu-1); s is close to linear in w at both
// ends of the law (s ~ sqrt(u) near 0, 1 - s ~ sqrt(1 - u) near 1).
struct InvTable {
  const double* s64;      // mx * 2 * mu doubles (FP64 guesses / brackets)
  const float* s32;       // mx * 2 * mu floats
  int32_t mu;             // points per half
  int32_t mx;             // slices in X^2 (1 when X is fixed)
  double x2max;           // X^2 of the last slice
  double x2scale;         // (mx - 1) / x2max: X^2 -> slice position
};

// Internal node of the KD-tree over the cloud, holding its two children's
// bounding boxes (so a visit costs one 64-byte load): child[c] >= 0 is an
// internal node; child[c] < 0 is a leaf, the points kd_pts[-child[c] - 1 ..
// -child[c] - 1 + count[c]).
struct KdNode {
  float lo[2][3], hi[2][3];
  int32_t child[2];
  int32_t count[2];
};

// Local quadratic patch of one cloud point: centroid, tangent frame e1, e2,
// unit normal n, height field h(a,b) = c0 + c1 a + c2 b + c3 a^2 + c4 a b + c5 b^2
// over (a, b) = ((x - cen).e1, (x - cen).e2), the support half-width ext (the
// largest |a| or |b| of the k points) and the mean distance from the point to
// its other k-1 neighbours.
template <class T>
struct Patch {
  T cen[3], e1[3], e2[3], n[3], c[6], ext, hmean;
};

struct CloudDev {
  const KdNode* nodes;
  const float4* kd_pts;        // x, y, z, original index (bit pattern of an int32)
  const Patch<double>* patch64; // indexed by original point index
  const Patch<float>* patch32;
  int64_t n_points;
  int32_t n_nodes;
  int32_t root;                // internal node 0, or the leaf reference of a one-leaf cloud
  int32_t k;                   // neighbours of the reconstruction
  int32_t newton_iters;
  int32_t radius_rule;         // 1 = spacing, otherwise curvature of the fitted patch
  int32_t nn_only;             // 1: cp is the nearest cloud point itself (no patch)
  const float4* pts;           // nn_only: the points by original index
  // The walk's nearest-point lookups of points near the surface: a uniform
  // grid of cells holding a few points each (null: the KD-tree only).  Cell
  // (i, j, l) = (l g_n[1] + j) g_n[0] + i holds g_pts[g_start[c] ..
  // g_start[c + 1]); a point sits in the cell floor((p - g_lo) / g_h).
  const int32_t* g_start;
  const float4* g_pts;         // x, y, z, original index bits, sorted by cell
  int32_t g_n[3];
  double g_lo[3];
  double g_h, g_inv;
  double g_slack;              // bound on the host's cell-binning rounding (ambient units)
};

// One request of a batched launch (serving).  Launch walks [begin, begin +
// count) are the request's walks idx0 .. idx0 + count - 1, where a request
// walk index is q * nw + w.  Entries are sorted by begin, and each begins on a
// whole batch unit (64 walks for lane kernels, the walks of one wavefront for
// group kernels): a wavefront then never holds walks of two requests at once.
//
// Time slicing: with a state buffer, a walk runs at most step_budget steps
// per launch; an unfinished walk saves its state (one record per request
// walk: kLaneRecordBytes for lane kernels, the group record for lane-group
// kernels) and counts itself in `pending`, and a later launch of the same
// range with `resume` set continues it (finished walks of the range are
// marked in their records and skipped).
constexpr int64_t kLaneRecordBytes = 80;
struct BatchEntry {
  int64_t begin, count, idx0, nw;
  const double* queries;       // the request's queries (device)
  double* walk_S;              // the request's per-walk outputs, indexed by request walk index
  int32_t* walk_K;
  uint64_t seed;
  char* state;                 // per-walk records, or null (the walks run to the end)
  int32_t resume;              // 1: continue the walks from their records
  int32_t pad;
  unsigned long long pending;  // walks of the entry saved unfinished (written by the kernel)
};

struct WalkArgs {
  // problem
  int32_t kind, n;
  double p[4];
  double sigma, lam_sqrt, eps, theta, c_kappa, c_h, tau_w;
  int32_t n_v, comp, precision, persistent;
  double inv_R;                // 1 / p[0] (the radius the source families scale by)
  double inv_sigma;            // 1 / sigma
  double inv_nv;               // 1 / N_V (the mean over the Green samples of a step)
  double rho_geo;              // c_kappa / (1 + kappa) with the manifold's constant curvature bound
  double cap_rg;               // sphere cap: radius sqrt(R^2 - h^2) of the boundary circle
  double cut_c, cut_s;         // cut torus: cos and sin of the cut angle phi_c
  int64_t max_steps;
  FnDev f, g;
  // constant-radius data (closed analytic manifolds)
  int32_t const_r;
  double r0, c0, om0, X0;
  RadialLaw law;
  // FP32 walks whose radius varies per step: the screening series'
  // coefficients alpha_j in float (wcoef[0] unused) and the number of terms
  // that can exceed 1e-10 over the solve's radii; w32n terms j = 1..w32n
  // keep the first dropped term below 2^-30 of the leading one there
  float wcoef[kMaxJ];
  int32_t wjs, w32n;
  RadialFixed fixed;
  InvTable tab;
  CloudDev cloud;
  // work
  const double* queries;       // this launch's queries (q_offset .. q_offset + nq)
  int64_t nq, nw;
  int64_t q_offset;            // global index of queries[0] in the solve (Philox counter word 0)
  int64_t idx_base;            // first walk (linear index q_local * nw + w) of this launch
  int64_t count;               // walks in this launch
  uint64_t seed;
  const uint64_t* seed_dev;    // non-null: the seed is read from device memory (graph replays)
  double* walk_S;
  int32_t* walk_K;
  unsigned long long* queue;   // persistent work counter
  int32_t chunk;               // walks taken per queue grab
  int32_t lanes;               // lanes per walk (group kernels)
  int32_t nblk;                // Philox blocks per Green sub-stream (group kernels)
  int32_t rblk, rword;         // block / word of the Green radius uniform
  // batched launches: count is the padded launch size; queries, nw, seed,
  // idx_base, q_offset and the per-walk outputs come from the entries
  const BatchEntry* batch;
  int32_t n_batch;
  int32_t step_budget;         // steps per launch of walks with a state record (0: no limit)
};

}  // namespace mpwos
