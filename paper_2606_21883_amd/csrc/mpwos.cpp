// Host side of the C ABI (include/mpwos.h): argument validation, the
// per-dimension coefficients of the radial Green law and its inverse tables,
// device workspaces, and the launch sequence of a solve:
//   queries -> walk kernel (per-walk S^i, K^i) -> per-query reduction -> u, stderr.
#include "mpwos.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "host_internal.h"
#include "kernel_args.h"

namespace mpwos {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

mpwos_status fail(mpwos_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

mpwos_status hip_fail(hipError_t e, const char* what) {
  return fail(MPWOS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return hip_fail(_e, #call);   \
  } while (0)

// ---------------------------------------------------------------------------
// device context: stream, events, grow-only workspace
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Context {
  std::mutex lock;
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  hipEvent_t ev[4] = {};
  DevBuf queries, walkS, walkK, u, se, stats, tmp, khist;
  // pinned host words for a solve's read-back: the statistics words, then
  // the K histogram
  unsigned long long* hpin = nullptr;
  bool ready = false;
};

static Context g_ctx;

static mpwos_status ensure(DevBuf& b, size_t bytes) {
  if (b.cap >= bytes) return MPWOS_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  const size_t want = std::max<size_t>(bytes, 256);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MPWOS_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  b.cap = want;
  return MPWOS_OK;
}

static mpwos_status context_init(Context& c) {
  if (c.ready) return MPWOS_OK;
  HIP_TRY(hipGetDevice(&c.device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, c.device));
  c.n_cu = prop.multiProcessorCount;
  HIP_TRY(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
  for (auto& e : c.ev) HIP_TRY(hipEventCreate(&e));
  HIP_TRY(hipHostMalloc((void**)&c.hpin, (8 + kKHistBins) * sizeof(unsigned long long), hipHostMallocDefault));
  c.ready = true;
  return MPWOS_OK;
}

int device_cu_count() { return g_ctx.ready ? g_ctx.n_cu : 256; }

// ---------------------------------------------------------------------------
// radial law of the Green density: coefficients for dimension n
//   S_nu(x) = sum_j (x^2/4)^j / (j! (nu+1)_j),  sum_j beta_j y^{2j} = S_nu(y)^{-2}
// ---------------------------------------------------------------------------
static constexpr int kHostJ = 96;

struct HostLaw {
  int n = 0;
  double nu = 0;
  int nu_int = -1;
  double alpha[kHostJ], alpha1[kHostJ], beta[kHostJ];
};

static void host_law(int n, HostLaw& h) {
  h.n = n;
  h.nu = 0.5 * (n - 2);
  h.nu_int = (n % 2 == 0) ? (n - 2) / 2 : -1;
  // alpha_j = 1/(4^j j! (nu+1)_j); the S_{nu+1} coefficients follow from
  // (nu+2)_j = (nu+1)_j (nu+1+j)/(nu+1).
  h.alpha[0] = 1.0;
  for (int j = 1; j < kHostJ; ++j) h.alpha[j] = h.alpha[j - 1] * (0.25 / j) / (h.nu + j);
  for (int j = 0; j < kHostJ; ++j) h.alpha1[j] = h.alpha[j] * ((h.nu + 1.0) / (h.nu + 1.0 + j));
  // S_nu^-2 as the square of the reciprocal series P = 1/S_nu:
  // p_0 = 1, p_j = -sum_{i=1..j} alpha_i p_{j-i}; beta_j = sum_i p_i p_{j-i}.
  double p[kHostJ];
  p[0] = 1.0;
  for (int j = 1; j < kHostJ; ++j) {
    double acc = 0.0;
    for (int i = j; i >= 1; --i) acc -= h.alpha[i] * p[j - i];
    p[j] = acc;
  }
  for (int j = 0; j < kHostJ; ++j) {
    double acc = 0.0;
    for (int i = 0; 2 * i < j; ++i) acc += 2.0 * p[i] * p[j - i];
    if (j % 2 == 0) acc += p[j / 2] * p[j / 2];
    h.beta[j] = acc;
  }
}

static double bd_of(const HostLaw& h, int j) {
  if (j == h.nu_int) return h.beta[j];
  return h.beta[j] / (2.0 * (h.nu - j));
}

// Series lengths for X^2 <= x2max: S_nu / S_{nu+1} keep terms until they drop
// below 1e-18; D keeps every beta term above 1e-20 (the log term at j = nu is
// dropped when it is below that too).  False when more than kMaxJ are needed.
static bool law_terms(const HostLaw& h, double x2max, int& js, int& jd) {
  js = kMaxJ + 1;
  for (int j = 1; j <= kMaxJ; ++j) {
    if (h.alpha[j] * std::pow(x2max, j) < 1e-18) { js = j; break; }
  }
  jd = 1;
  for (int j = kHostJ - 1; j >= 1; --j) {
    if (std::fabs(h.beta[j]) * std::pow(x2max, j) >= 1e-20) { jd = j + 1; break; }
  }
  return js <= kMaxJ && jd <= kMaxJ;
}

static void fill_law(const HostLaw& h, int js, int jd, RadialLaw& L) {
  memset(&L, 0, sizeof(L));
  L.n = h.n;
  L.nu = h.nu;
  L.nu_int = (h.nu_int >= 0 && h.nu_int < jd) ? h.nu_int : -1;
  L.js = js;
  L.jd = jd;
  L.inv_2nu1 = 1.0 / (2.0 * (h.nu + 1.0));
  for (int j = 0; j < kMaxJ; ++j) {
    L.alpha[j] = h.alpha[j];
    L.alpha1[j] = h.alpha1[j];
    L.bd[j] = bd_of(h, j);
  }
}

static void fill_fixed(const HostLaw& h, const RadialLaw& L, double X, RadialFixed& R) {
  memset(&R, 0, sizeof(R));
  const double X2 = X * X;
  R.X2 = X2;
  double xp = 1.0, q1 = 0.0, s1 = 0.0;
  for (int j = 0; j < kMaxJ; ++j) {
    if (j > 0) xp *= X2;
    R.A[j] = h.alpha[j] * xp;
    R.A1[j] = h.alpha1[j] * xp;
    if (j == L.nu_int) {
      R.L = h.beta[j] * xp;
      R.B[j] = 0.0;
    } else if (j < L.jd) {
      R.B[j] = bd_of(h, j) * xp;
      q1 += R.B[j];
    }
  }
  R.Q1 = q1;
  xp = 1.0;
  for (int j = 1; j < kHostJ; ++j) {
    xp *= X2;
    s1 += h.alpha[j] * xp;
  }
  R.norm = (1.0 + s1) / s1;
}

// exact F(s) and F'(s) on the host (full-length series)
static void host_F(const HostLaw& h, double X2, double s, double& F, double& pdf) {
  if (s <= 0.0) { F = 0.0; pdf = 0.0; return; }
  if (s >= 1.0) { F = 1.0; pdf = 0.0; return; }
  const double z = s * s;
  double t1 = 0, S1 = 0, Dz = 0, Q1 = 0, Lg = 0, s1X = 0;
  double xp = 1.0, zp = 1.0;
  for (int j = 0; j < kHostJ; ++j) {
    if (j > 0) { xp *= X2; zp *= z; }
    if (j > 0) { t1 += h.alpha[j] * xp * zp; s1X += h.alpha[j] * xp; }
    S1 += h.alpha1[j] * xp * zp;
    const double b = bd_of(h, j) * xp;
    if (j == h.nu_int) Lg = b;
    else { Dz += b * zp; Q1 += b; }
  }
  const double s2nu = std::pow(s, (double)(h.n - 2));
  double D = Dz - s2nu * Q1;
  if (h.nu_int >= 0) D -= Lg * s2nu * std::log(s);
  const double norm = (1.0 + s1X) / s1X;
  F = norm * (t1 / (1.0 + t1) + X2 * z * S1 / (2.0 * (h.nu + 1.0)) * D);
  pdf = norm * X2 * s * (1.0 + t1) * D;
}

static double host_inv(const HostLaw& h, double X2, double u, double lo, double hi) {
  double s = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double F, p;
    host_F(h, X2, s, F, p);
    if (F == u) break;
    if (F < u) lo = s; else hi = s;
    double sn = s - (F - u) / p;
    if (!(sn >= lo && sn <= hi)) sn = 0.5 * (lo + hi);
    const double ds = std::fabs(sn - s);
    s = sn;
    if (ds <= 0x1p-51 * s || hi - lo <= 0x1p-52 * hi) break;
  }
  return s;
}

// Inverse tables, cached per (n, slices, X^2 range).
struct TableKey {
  int n, mx;
  double x2max;
  bool operator<(const TableKey& o) const { return std::tie(n, mx, x2max) < std::tie(o.n, o.mx, o.x2max); }
};
struct TableVal {
  double* d64 = nullptr;
  float* d32 = nullptr;
  int mu = 0;
};
static std::mutex g_tab_lock;
static std::map<TableKey, TableVal> g_tables;

// 1025 points per half keep linear interpolation in w within 1.1e-6 of the
// root for every n (the worst case is n = 2 near u = 0, where s ~ sqrt(u / ln(1/u)))
static constexpr int kTableMu = 1025;

// The inverse radial law at the table points, on the host: mx slices in X^2,
// two halves (u = w^2 and 1 - w^2, w uniform in [0, sqrt(1/2)]) of kTableMu
// points each, FP64 and FP32 copies.
static void fill_table_host(const HostLaw& h, int mx, double x2max, double* s64, float* s32) {
  const int mu = kTableMu;
  const double wmax = std::sqrt(0.5);
  for (int k = 0; k < mx; ++k) {
    const double X2 = (mx == 1) ? x2max : (k == 0 ? x2max * 1e-6 : x2max * k / (mx - 1));
    for (int half = 0; half < 2; ++half) {
      double* row = s64 + ((size_t)k * 2 + half) * mu;
      for (int i = 0; i < mu; ++i) {
        const double w = wmax * (double)i / (mu - 1);
        const double u = half == 0 ? w * w : 1.0 - w * w;
        double sv;
        if (half == 0 && i == 0) sv = 0.0;
        else if (half == 1 && i == 0) sv = 1.0;
        else sv = host_inv(h, X2, u, 0.0, 1.0);
        row[i] = sv;
      }
      for (int i = 0; i < mu; ++i) s32[((size_t)k * 2 + half) * mu + i] = (float)row[i];
    }
  }
}

static void set_table_view(const double* d64, const float* d32, int mx, double x2max, InvTable& t) {
  t.s64 = d64;
  t.s32 = d32;
  t.mu = kTableMu;
  t.mx = mx;
  t.x2max = x2max;
  t.x2scale = mx > 1 ? (double)(mx - 1) / x2max : 0.0;
}

// A device region the allocation-free solve keeps one inverse table in
// (instead of the cache below, which allocates), and the key of the table it
// holds.
struct TableSink {
  double* d64 = nullptr;
  float* d32 = nullptr;
  size_t bytes = 0;
  TableKey* held = nullptr;
  hipStream_t stream = nullptr;
  bool use_cache = false;  // the cache's tables live on the calling device
};

static mpwos_status get_table(const HostLaw& h, int mx, double x2max, InvTable& t, TableSink* sink = nullptr) {
  const int mu = kTableMu;
  TableKey key{h.n, mx, x2max};
  std::lock_guard<std::mutex> g(g_tab_lock);
  auto it = g_tables.find(key);
  if (it != g_tables.end() && (!sink || sink->use_cache)) {
    set_table_view(it->second.d64, it->second.d32, mx, x2max, t);
    return MPWOS_OK;
  }
  std::vector<double> s64((size_t)mx * 2 * mu);
  std::vector<float> s32((size_t)mx * 2 * mu);
  if (sink) {
    const size_t b64 = s64.size() * sizeof(double), b32 = s32.size() * sizeof(float);
    if (b64 + b32 > sink->bytes) return fail(MPWOS_EINVAL, "inverse table exceeds the allocation-free scratch");
    sink->d32 = (float*)((char*)sink->d64 + b64);
    if (!(sink->held && !(*sink->held < key) && !(key < *sink->held))) {
      fill_table_host(h, mx, x2max, s64.data(), s32.data());
      hipError_t e = hipMemcpyAsync(sink->d64, s64.data(), b64, hipMemcpyHostToDevice, sink->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(sink->d32, s32.data(), b32, hipMemcpyHostToDevice, sink->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(sink->stream);
      if (e != hipSuccess) return hip_fail(e, "inverse table upload to the scratch");
      if (sink->held) *sink->held = key;
    }
    set_table_view(sink->d64, sink->d32, mx, x2max, t);
    return MPWOS_OK;
  }
  fill_table_host(h, mx, x2max, s64.data(), s32.data());
  TableVal v;
  v.mu = mu;
  hipError_t e = hipMalloc(&v.d64, s64.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&v.d32, s32.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(v.d64, s64.data(), s64.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(v.d32, s32.data(), s32.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "inverse table upload");
  it = g_tables.emplace(key, v).first;
  set_table_view(it->second.d64, it->second.d32, mx, x2max, t);
  return MPWOS_OK;
}

// Screening factor c and volume weight omega for a constant radius (Lemma
// 3.1 series, eq. omega_explicit_formula): s1 = S_nu(X) - 1 by Horner in
// z = X^2 = sigma r^2 over the law's coefficients alpha_j (the same form the
// device uses for per-step radii), with every coefficient the host keeps.
static void host_weights(const HostLaw& h, double sigma, double r, double& c, double& om) {
  const double z = sigma * r * r;
  double s1 = 0.0;
  for (int j = kHostJ - 1; j >= 1; --j) s1 = (s1 + h.alpha[j]) * z;
  c = 1.0 / (1.0 + s1);
  om = s1 * c / sigma;
}

// ---------------------------------------------------------------------------
// manifolds
// ---------------------------------------------------------------------------
}  // namespace mpwos

struct mpwos_manifold {
  mpwos_manifold_desc desc;
  mpwos::CloudState* cloud = nullptr;
  std::atomic<int> refs{0};
};

namespace mpwos {

static mpwos_status check_manifold_desc(const mpwos_manifold_desc* d) {
  if (!d) return fail(MPWOS_EINVAL, "manifold descriptor is NULL");
  switch (d->kind) {
    case MPWOS_SPHERE:
      if (d->n < 2 || d->n > 4096) return fail(MPWOS_EINVAL, "sphere: n must be in [2, 4096]");
      if (!(d->p[0] > 0) || !std::isfinite(d->p[0])) return fail(MPWOS_EINVAL, "sphere: radius p[0] must be > 0");
      return MPWOS_OK;
    case MPWOS_SPHERE_CAP:
      if (d->n < 2 || d->n > 3) return fail(MPWOS_EINVAL, "sphere cap: n must be 2 or 3");
      if (!(d->p[0] > 0)) return fail(MPWOS_EINVAL, "sphere cap: radius p[0] must be > 0");
      if (!(std::fabs(d->p[1]) < d->p[0])) return fail(MPWOS_EINVAL, "sphere cap: |h| must be < R");
      return MPWOS_OK;
    case MPWOS_TORUS_IMPLICIT:
      if (d->n != 3) return fail(MPWOS_EINVAL, "torus: n must be 3");
      if (!(d->p[1] > 0 && d->p[1] <= 0.5 * d->p[0]))
        return fail(MPWOS_EINVAL, "torus: need 0 < a <= R/2 (constant curvature indicator 1/a)");
      return MPWOS_OK;
    case MPWOS_CUT_TORUS:
      if (d->n != 3) return fail(MPWOS_EINVAL, "cut torus: n must be 3");
      if (!(d->p[1] > 0 && d->p[1] <= 0.5 * d->p[0]))
        return fail(MPWOS_EINVAL, "cut torus: need 0 < a <= R/2 (constant curvature indicator 1/a)");
      if (!std::isfinite(d->p[2])) return fail(MPWOS_EINVAL, "cut torus: the cut angle p[2] must be finite");
      return MPWOS_OK;
    case MPWOS_PRODUCT:
      if (d->n != 9) return fail(MPWOS_EINVAL, "product manifold: n must be 9");
      if (!(d->p[0] > 0.0) || !(d->p[1] > 0.0) || !std::isfinite(d->p[0]) || !std::isfinite(d->p[1]))
        return fail(MPWOS_EINVAL, "product manifold: R = p[0] and a = p[1] must be > 0");
      return MPWOS_OK;
    case MPWOS_DUMBBELL:
      if (d->n < 4 || d->n > 4096) return fail(MPWOS_EINVAL, "dumbbell: n must be in [4, 4096]");
      if (!(d->p[0] >= 0.0 && d->p[0] < 0.5)) return fail(MPWOS_EINVAL, "dumbbell: a = p[0] must be in [0, 1/2)");
      if (!(d->p[1] > 0.0) || !std::isfinite(d->p[1])) return fail(MPWOS_EINVAL, "dumbbell: k = p[1] must be > 0");
      return MPWOS_OK;
    case MPWOS_POINT_CLOUD:
      if (d->n != 3) return fail(MPWOS_EINVAL, "point cloud: n must be 3");
      if (!d->points) return fail(MPWOS_EINVAL, "point cloud: points is NULL");
      if (d->k_nn < 6 || d->k_nn > kMaxK) return fail(MPWOS_EINVAL, "point cloud: k_nn must be in [6, 32]");
      if (d->n_points < d->k_nn || d->n_points > (int64_t)1 << 27)
        return fail(MPWOS_EINVAL, "point cloud: n_points must be in [k_nn, 2^27]");
      if (d->reconstruction != 0 && d->reconstruction != 1)
        return fail(MPWOS_EINVAL, "point cloud: reconstruction must be 0 (patch) or 1 (nearest point)");
      if (!(d->fit_scale >= 0.0 && d->fit_scale <= 16.0))
        return fail(MPWOS_EINVAL, "point cloud: fit_scale must be in [0, 16]");
      return MPWOS_OK;
  }
  return fail(MPWOS_EINVAL, "unknown manifold kind");
}

// curvature indicator kappa (largest |principal curvature|) when constant
static double const_kappa(const mpwos_manifold_desc& d) {
  switch (d.kind) {
    case MPWOS_SPHERE:
    case MPWOS_SPHERE_CAP: return 1.0 / d.p[0];
    case MPWOS_TORUS_IMPLICIT:
    case MPWOS_CUT_TORUS: return 1.0 / d.p[1];
    // the Fourier curve's curvature (|C''|^2 = 14, speed sqrt 3) and the sphere's
    case MPWOS_PRODUCT: return std::max(std::sqrt(14.0) / (3.0 * d.p[0]), 1.0 / d.p[1]);
  }
  return 0.0;
}

static mpwos_status check_fn(const mpwos_fn* f, const mpwos_manifold_desc& d, bool is_g) {
  if (!f) return MPWOS_OK;
  const char* which = is_g ? "g" : "f";
  auto bad = [&](const char* m) { return fail(MPWOS_EINVAL, std::string(which) + ": " + m); };
  const bool sph = d.kind == MPWOS_SPHERE || d.kind == MPWOS_SPHERE_CAP;
  switch (f->kind) {
    case MPWOS_FN_ZERO:
    case MPWOS_FN_CONST: return MPWOS_OK;
    case MPWOS_FN_SPH_PAIR:
      if (!sph) return bad("SPH_PAIR needs a sphere");
      if (f->idx[0] < 0 || f->idx[1] < 0 || f->idx[0] >= d.n || f->idx[1] >= d.n || f->idx[0] == f->idx[1])
        return bad("SPH_PAIR needs distinct indices in [0, n)");
      return MPWOS_OK;
    case MPWOS_FN_CIRCLE_MODE:
      if (!sph || d.n != 2 || is_g) return bad("CIRCLE_MODE is a source on S^1");
      if (f->idx[0] < 0 || f->idx[0] > 64) return bad("CIRCLE_MODE: k must be in [0, 64]");
      return MPWOS_OK;
    case MPWOS_FN_LEGENDRE:
      if (!((sph || d.kind == MPWOS_POINT_CLOUD) && d.n == 3)) return bad("LEGENDRE needs S^2 or a cloud of it");
      return MPWOS_OK;
    case MPWOS_FN_TORUS_MODE:
      if (is_g || (d.kind != MPWOS_TORUS_IMPLICIT && d.kind != MPWOS_POINT_CLOUD))
        return bad("TORUS_MODE is a source on a torus");
      return MPWOS_OK;
    case MPWOS_FN_TABLE_S1:
      if (!sph || d.n != 2 || is_g) return bad("TABLE_S1 is a source on S^1");
      if (!f->values || f->n_values < 4 || (f->n_values % 2)) return bad("TABLE_S1 needs 2M >= 4 values");
      return MPWOS_OK;
    case MPWOS_FN_PRODUCT_MODES:
      if (d.kind != MPWOS_PRODUCT || is_g) return bad("PRODUCT_MODES is a source on the product manifold");
      return MPWOS_OK;
    case MPWOS_FN_DUMBBELL_POLY:
      if (d.kind != MPWOS_DUMBBELL || is_g) return bad("DUMBBELL_POLY is a source on the dumbbell");
      if (!f->values || f->n_values != d.n - 1) return bad("DUMBBELL_POLY needs n - 1 values");
      return MPWOS_OK;
    case MPWOS_FN_TORUS_SINE:
      if (d.kind != MPWOS_CUT_TORUS || is_g) return bad("TORUS_SINE is a source on the cut torus");
      if (f->idx[0] < 1 || f->idx[0] > 64 || f->idx[1] < 0 || f->idx[1] > 64 || f->idx[2] < 0 || f->idx[2] > 64)
        return bad("TORUS_SINE: idx[0] in [1, 64], idx[1] and idx[2] in [0, 64]");
      if (!f->values || f->n_values != (int64_t)(f->idx[0] + f->idx[2]) * (2 * f->idx[1] + 1))
        return bad("TORUS_SINE needs (idx[0] + idx[2]) (2 idx[1] + 1) values");
      for (int64_t i = 0; i < f->n_values; ++i)
        if (!std::isfinite(f->values[i])) return bad("TORUS_SINE: non-finite coefficient");
      return MPWOS_OK;
  }
  return bad("unknown function kind");
}

static void fill_fn(const mpwos_fn* f, const mpwos_manifold_desc& d, double sigma, FnDev& o) {
  memset(&o, 0, sizeof(o));
  if (!f) return;
  o.kind = f->kind;
  for (int i = 0; i < 3; ++i) o.idx[i] = f->idx[i];
  for (int i = 0; i < 8; ++i) o.coef[i] = f->coef[i];
  const double R = d.p[0];
  if (f->kind == MPWOS_FN_SPH_PAIR) o.lam = 2.0 * d.n / (R * R);
  if (f->kind == MPWOS_FN_CIRCLE_MODE) o.lam = (double)f->idx[0] * f->idx[0] / (R * R);
  o.u_scale = 1.0 / (o.lam + sigma);
  if (f->kind == MPWOS_FN_TABLE_S1) o.m = f->n_values / 2;
  if (f->kind == MPWOS_FN_DUMBBELL_POLY) {
    o.m = f->n_values;
    double tr = 0.0;
    for (int64_t i = 0; i < f->n_values; ++i) tr += f->values[i];
    o.lam = tr;
  }
}

// Distance from (|x_h|, x_n) = (rho, zs) to the dumbbell's profile
// {(R(x*), x*) : |x*| <= kc}, R(x*) = sqrt(1 - (x*/kc)^2) (1 - a + 2a (x*/kc)^2)
// (Example 2's level set), as far as the query check needs it: a profile
// point within tol of (rho, zs) has |x* - zs| <= tol, so the minimum of the
// distance over that window decides whether the query lies within tol of
// the manifold.  The window is far shorter than any radius of curvature of
// the profile, so the distance is unimodal on it and a golden-section search
// finds its minimum.
static double dumbbell_window_distance(double a, double kc, double rho, double zs, double tol) {
  const double lo0 = std::max(-kc, zs - tol), hi0 = std::min(kc, zs + tol);
  if (lo0 > hi0) return INFINITY;
  // 1 - (x*/kc)^2 as (kc - x*)(kc + x*)/kc^2: no cancellation at the tips
  auto dist2 = [&](double xs) {
    const double q = xs / kc;
    const double w = std::max(0.0, (kc - xs) * (kc + xs)) / (kc * kc);
    const double R = std::sqrt(w) * (1.0 - a + 2.0 * a * q * q);
    return (rho - R) * (rho - R) + (zs - xs) * (zs - xs);
  };
  const double gr = 0.6180339887498949;
  double lo = lo0, hi = hi0;
  double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
  double f1 = dist2(x1), f2 = dist2(x2);
  double best = std::min({dist2(lo0), dist2(hi0), f1, f2});
  for (int it = 0; it < 200 && hi - lo > 1e-17 * (1.0 + std::fabs(hi)); ++it) {
    if (f1 <= f2) {
      hi = x2; x2 = x1; f2 = f1;
      x1 = hi - gr * (hi - lo); f1 = dist2(x1);
    } else {
      lo = x1; x1 = x2; f1 = f2;
      x2 = lo + gr * (hi - lo); f2 = dist2(x2);
    }
    best = std::min({best, f1, f2});
  }
  return std::sqrt(best);
}

// on-manifold test of a query (host side, analytic manifolds)
// (the dumbbell's: the distance to its nearest point)
static bool query_on_manifold(const mpwos_manifold_desc& d, const double* y) {
  const int n = d.n;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += y[i] * y[i];
  const double tol = 1e-9 * (1.0 + std::sqrt(s));
  switch (d.kind) {
    case MPWOS_SPHERE: return std::fabs(std::sqrt(s) - d.p[0]) <= tol;
    case MPWOS_SPHERE_CAP: return std::fabs(std::sqrt(s) - d.p[0]) <= tol && y[n - 1] > d.p[1];
    case MPWOS_TORUS_IMPLICIT: {
      const double rho = std::hypot(y[0], y[1]);
      const double dc = std::hypot(rho - d.p[0], y[2]);
      return std::fabs(dc - d.p[1]) <= tol;
    }
    case MPWOS_CUT_TORUS: {
      // on the torus and on the open half 0 < phi - phi_c < pi
      const double rho = std::hypot(y[0], y[1]);
      const double dc = std::hypot(rho - d.p[0], y[2]);
      return std::fabs(dc - d.p[1]) <= tol && y[1] * std::cos(d.p[2]) - y[0] * std::sin(d.p[2]) > 0.0;
    }
    case MPWOS_PRODUCT: {
      // nearest point of the Fourier curve: maximise x_c . C(phi) (fine grid, Newton)
      auto g = [&](double t, double* d) {
        d[0] = d[1] = d[2] = 0.0;
        for (int k = 1; k <= 3; ++k) {
          const double c = std::cos(k * t), s = std::sin(k * t), ak = y[2 * k - 2], bk = y[2 * k - 1];
          d[0] += (ak * c + bk * s) / k;
          d[1] += -ak * s + bk * c;
          d[2] += -k * (ak * c + bk * s);
        }
      };
      const int G = 1024;
      const double h = 6.283185307179586 / G;
      double best = -INFINITY, t = 0.0, v[3];
      for (int j = 0; j < G; ++j) {
        g(j * h, v);
        if (v[0] > best) { best = v[0]; t = j * h; }
      }
      double lo = t - h, hi = t + h;
      for (int it = 0; it < 100; ++it) {
        g(t, v);
        if (v[1] > 0.0) lo = t; else hi = t;
        double nx = v[2] < 0.0 ? t - v[1] / v[2] : lo - 1.0;
        if (!(nx >= lo && nx <= hi)) nx = 0.5 * (lo + hi);
        const double step = std::fabs(nx - t);
        t = nx;
        if (step <= 1e-16 * (1.0 + std::fabs(t)) || hi - lo <= 1e-16 * (1.0 + std::fabs(t))) break;
      }
      double d2 = 0.0;
      for (int k = 1; k <= 3; ++k) {
        const double ex = y[2 * k - 2] - d.p[0] * std::cos(k * t) / k, ey = y[2 * k - 1] - d.p[0] * std::sin(k * t) / k;
        d2 += ex * ex + ey * ey;
      }
      const double ns = std::sqrt(y[6] * y[6] + y[7] * y[7] + y[8] * y[8]);
      return std::sqrt(d2) + std::fabs(ns - d.p[1]) <= tol;
    }
    case MPWOS_DUMBBELL: {
      double hh = 0.0;
      for (int i = 0; i < n - 1; ++i) hh += y[i] * y[i];
      const double rho = std::sqrt(hh), zs = y[n - 1];
      return dumbbell_window_distance(d.p[0], d.p[1], rho, zs, tol) <= tol;
    }
  }
  return true;
}

}  // namespace mpwos

using namespace mpwos;

extern "C" {

const char* mpwos_last_error(void) { return g_last_error.c_str(); }

const char* mpwos_version(void) { return "mpwos-gfx950 0.1"; }

void mpwos_options_default(mpwos_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->theta = 0.95;
  o->c_kappa = 1.2;
  o->c_h = 2.4;
  o->tau_w = 1e-8;
  o->n_v = 1;
  o->precision = MPWOS_FP64_PLAIN;
  o->compensation = MPWOS_COMP_EXACT;
  o->radius_rule = MPWOS_RADIUS_CURVATURE;
  o->max_steps = 10000000;
  o->persistent = 0;
  o->newton_iters = 6;
}

mpwos_status mpwos_manifold_create(const mpwos_manifold_desc* desc, mpwos_manifold** out) {
  g_last_error.clear();
  if (!out) return fail(MPWOS_EINVAL, "out is NULL");
  mpwos_status st = check_manifold_desc(desc);
  if (st) return st;
  {
    std::lock_guard<std::mutex> g(g_ctx.lock);
    st = context_init(g_ctx);
    if (st) return st;
  }
  auto* m = new (std::nothrow) mpwos_manifold;
  if (!m) return fail(MPWOS_ENOMEM, "host allocation");
  m->desc = *desc;
  if (desc->kind == MPWOS_POINT_CLOUD) {
    st = cloud_create(*desc, g_ctx.stream, &m->cloud);
    if (st) {
      delete m;
      return st;
    }
  }
  m->desc.points = nullptr;
  *out = m;
  return MPWOS_OK;
}

mpwos_status mpwos_manifold_destroy(mpwos_manifold* m) {
  g_last_error.clear();
  if (!m) return fail(MPWOS_EINVAL, "manifold is NULL");
  if (m->refs.load() > 0) return fail(MPWOS_EBUSY, "manifold is referenced by a queued request");
  if (m->cloud) cloud_destroy(m->cloud);
  delete m;
  return MPWOS_OK;
}

}  // extern "C"

namespace mpwos {

void manifold_ref(const mpwos_manifold* m, int d) { const_cast<mpwos_manifold*>(m)->refs += d; }
const mpwos_manifold_desc& manifold_desc(const mpwos_manifold* m) { return m->desc; }

// Validates a solve and fills the kernel arguments (except buffers).
mpwos_status prepare_solve(const mpwos_manifold* man, const mpwos_fn* f, const mpwos_fn* g, double sigma,
                           int64_t nq, int64_t nw, double eps, uint64_t seed, const mpwos_options& o,
                           WalkArgs& a, TableSink* sink) {
  if (!man) return fail(MPWOS_EINVAL, "manifold is NULL");
  const mpwos_manifold_desc& d = man->desc;
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(MPWOS_EINVAL, "c (sigma) must be finite and > 0");
  if (nq < 1 || nq > 0xFFFFFFFFll) return fail(MPWOS_EINVAL, "n_queries must be in [1, 2^32)");
  if (nw < 1 || nw > 0xFFFFFFFFll) return fail(MPWOS_EINVAL, "n_walks must be in [1, 2^32)");
  const bool boundary = d.kind == MPWOS_SPHERE_CAP || d.kind == MPWOS_CUT_TORUS;
  if (boundary && !g) return fail(MPWOS_EINVAL, "g is required on a manifold with boundary");
  if (!boundary && g) return fail(MPWOS_EINVAL, "g must be NULL on a closed manifold");
  if (boundary && !(eps > 0.0 && std::isfinite(eps))) return fail(MPWOS_EINVAL, "eps must be > 0");
  if (!f) return fail(MPWOS_EINVAL, "f is NULL");
  if (!(o.theta > 0.0 && o.theta < 1.0)) return fail(MPWOS_EINVAL, "theta must be in (0, 1)");
  if (!(o.c_kappa > 0.0)) return fail(MPWOS_EINVAL, "c_kappa must be > 0");
  if (!(o.c_h > 0.0)) return fail(MPWOS_EINVAL, "c_h must be > 0");
  if (!boundary && !(o.tau_w > 0.0 && o.tau_w < 1.0)) return fail(MPWOS_EINVAL, "tau_w must be in (0, 1)");
  if (o.n_v < 1 || o.n_v > 255) return fail(MPWOS_EINVAL, "n_v must be in [1, 255]");
  if (o.max_steps < 1) return fail(MPWOS_EINVAL, "max_steps must be >= 1");
  if (o.precision != MPWOS_FP64_PLAIN && o.precision != MPWOS_FP32_MIXED)
    return fail(MPWOS_EINVAL, "unknown precision");
  if (o.compensation != MPWOS_COMP_NONE && o.compensation != MPWOS_COMP_EXACT &&
      o.compensation != MPWOS_COMP_SECOND_ORDER)
    return fail(MPWOS_EINVAL, "unknown compensation");
  if (o.compensation == MPWOS_COMP_SECOND_ORDER) {
    if (d.kind != MPWOS_CUT_TORUS || f->kind != MPWOS_FN_TORUS_SINE)
      return fail(MPWOS_EINVAL, "the second-order compensation takes a TORUS_SINE source on the cut torus");
    if (f->idx[2] < 1) return fail(MPWOS_EINVAL, "the second-order compensation needs predictor rows (idx[2] >= 1)");
    if (!(f->coef[0] > 0.0 && f->coef[0] < 0.5 * d.p[1]))
      return fail(MPWOS_EINVAL, "the second-order compensation needs h_eta = coef[0] in (0, a/2)");
  }
  if (d.kind == MPWOS_CUT_TORUS) {
    if (f->kind != MPWOS_FN_ZERO && f->kind != MPWOS_FN_CONST && f->kind != MPWOS_FN_TORUS_SINE)
      return fail(MPWOS_EINVAL, "f: the cut torus takes ZERO, CONST or TORUS_SINE");
    if (g && g->kind != MPWOS_FN_ZERO && g->kind != MPWOS_FN_CONST)
      return fail(MPWOS_EINVAL, "g: the cut torus takes ZERO or CONST boundary data");
  }
  if (o.radius_rule < MPWOS_RADIUS_CURVATURE || o.radius_rule > MPWOS_RADIUS_CURVATURE_BOUND)
    return fail(MPWOS_EINVAL, "unknown radius_rule");
  if (d.kind == MPWOS_PRODUCT && o.compensation != MPWOS_COMP_NONE)
    return fail(MPWOS_EINVAL, "the product manifold has no exact compensation: set compensation NONE");
  if ((d.kind == MPWOS_DUMBBELL || d.kind == MPWOS_PRODUCT) && f->kind != MPWOS_FN_ZERO &&
      f->kind != MPWOS_FN_CONST && f->kind != MPWOS_FN_DUMBBELL_POLY && f->kind != MPWOS_FN_PRODUCT_MODES)
    return fail(MPWOS_EINVAL, "f: this manifold takes ZERO, CONST or its own source family");
  if (d.kind == MPWOS_DUMBBELL) {
    if (o.radius_rule != MPWOS_RADIUS_CURVATURE_BOUND)
      return fail(MPWOS_EINVAL, "the dumbbell takes the CURVATURE_BOUND radius rule");
    if (o.compensation != MPWOS_COMP_NONE)
      return fail(MPWOS_EINVAL, "the dumbbell has no exact compensation: set compensation NONE");
  } else if (d.kind != MPWOS_POINT_CLOUD && o.radius_rule != MPWOS_RADIUS_CURVATURE) {
    return fail(MPWOS_EINVAL, "radius rules other than CURVATURE apply to point clouds and the dumbbell");
  }
  if (d.kind == MPWOS_POINT_CLOUD && man->cloud && cloud_nn_only(man->cloud) &&
      o.radius_rule != MPWOS_RADIUS_SPACING && o.radius_rule != MPWOS_RADIUS_CURVATURE_BOUND)
    return fail(MPWOS_EINVAL, "the nearest-point projection has no fitted curvature: use SPACING or CURVATURE_BOUND");
  if (o.radius_rule == MPWOS_RADIUS_CURVATURE_BOUND && !(o.kappa_bound >= 0.0 && std::isfinite(o.kappa_bound)))
    return fail(MPWOS_EINVAL, "kappa_bound must be finite and >= 0");
  if (o.block_size != 0 && (o.block_size < 64 || o.block_size > 256 || o.block_size % 64))
    return fail(MPWOS_EINVAL, "block_size must be 0 or a multiple of 64 in [64, 256]");
  {
    const int l = o.lanes_per_walk;
    if (!(l == 0 || l == 1 || l == 4 || l == 8 || l == 16 || l == 32 || l == 64))
      return fail(MPWOS_EINVAL, "lanes_per_walk must be 0, 1, 4, 8, 16, 32 or 64");
  }
  mpwos_status st = check_fn(f, d, false);
  if (st) return st;
  st = check_fn(g, d, true);
  if (st) return st;
  if (o.compensation == MPWOS_COMP_EXACT && f->kind == MPWOS_FN_TABLE_S1 && !f->values)
    return fail(MPWOS_EINVAL, "TABLE_S1 needs values");

  memset(&a, 0, sizeof(a));
  a.kind = d.kind;
  a.n = d.n;
  for (int i = 0; i < 4; ++i) a.p[i] = d.p[i];
  a.sigma = sigma;
  a.inv_R = 1.0 / d.p[0];
  a.lam_sqrt = std::sqrt(sigma);
  a.inv_sigma = 1.0 / sigma;
  a.inv_nv = 1.0 / (double)o.n_v;
  a.rho_geo = o.c_kappa / (1.0 + const_kappa(d));
  if (d.kind == MPWOS_SPHERE_CAP) a.cap_rg = std::sqrt(d.p[0] * d.p[0] - d.p[1] * d.p[1]);
  if (d.kind == MPWOS_CUT_TORUS) {
    a.cut_c = std::cos(d.p[2]);
    a.cut_s = std::sin(d.p[2]);
  }
  a.eps = eps;
  a.theta = o.theta;
  a.c_kappa = o.c_kappa;
  a.c_h = o.c_h;
  a.tau_w = o.tau_w;
  a.n_v = o.n_v;
  a.comp = o.compensation;
  a.precision = o.precision;
  a.persistent = o.persistent;
  a.max_steps = o.max_steps;
  a.seed = seed;
  fill_fn(f, d, sigma, a.f);
  fill_fn(g, d, sigma, a.g);

  HostLaw h;
  host_law(d.n, h);
  // largest X^2 = sigma r^2 the walk can reach
  double rmax;
  const bool cloud_bound = d.kind == MPWOS_POINT_CLOUD && o.radius_rule == MPWOS_RADIUS_CURVATURE_BOUND;
  if (cloud_bound || d.kind == MPWOS_DUMBBELL) {
    rmax = o.theta * o.c_kappa / (1.0 + o.kappa_bound);
  } else if (d.kind == MPWOS_POINT_CLOUD) {
    rmax = o.radius_rule == MPWOS_RADIUS_SPACING ? cloud_spacing_rmax(man->cloud, o) : o.theta * o.c_kappa;
  } else {
    rmax = o.theta * o.c_kappa / (1.0 + const_kappa(d));
  }
  const double x2max = sigma * rmax * rmax;
  int js, jd;
  if (!law_terms(h, x2max, js, jd))
    return fail(MPWOS_EINVAL, "sqrt(sigma) r_max = " + std::to_string(std::sqrt(x2max)) +
                                  " is beyond the range of the series radial law for this n");
  fill_law(h, js, jd, a.law);
  // FP32 screening series for per-step radii: alpha_j in float, the terms
  // whose alpha_j X^2j can reach 1e-10 (far below FP32 rounding of
  // c = 1/(1+s1)); never more than the FP64 series keeps
  a.wjs = js;
  for (int j = 1; j < js; ++j) {
    if (h.alpha[j] * std::pow(x2max, j) < 1e-10) { a.wjs = j; break; }
  }
  memset(a.wcoef, 0, sizeof(a.wcoef));
  for (int j = 1; j < a.wjs; ++j) a.wcoef[j] = (float)h.alpha[j];
  // terms for FP32 relative accuracy: the series is alpha_1 X^2 (1 + ...),
  // so the truncation error relative to s1 is about the first dropped term
  // over the leading one
  a.w32n = kMaxJ - 1;
  for (int j = 1; j + 1 < kMaxJ; ++j) {
    if (h.alpha[j + 1] / h.alpha[1] * std::pow(x2max, j) < 0x1p-30) { a.w32n = j; break; }
  }
  a.const_r = (d.kind == MPWOS_SPHERE || d.kind == MPWOS_TORUS_IMPLICIT || d.kind == MPWOS_DUMBBELL ||
               d.kind == MPWOS_PRODUCT || cloud_bound)
                  ? 1 : 0;
  if (a.const_r) {
    a.r0 = rmax;
    host_weights(h, sigma, a.r0, a.c0, a.om0);
    a.X0 = std::sqrt(sigma) * a.r0;
    fill_fixed(h, a.law, a.X0, a.fixed);
    st = get_table(h, 1, a.X0 * a.X0, a.tab, sink);
  } else {
    st = get_table(h, 17, x2max, a.tab, sink);
  }
  if (st) return st;
  if (d.kind == MPWOS_POINT_CLOUD) cloud_fill_args(man->cloud, o, a);
  return MPWOS_OK;
}

// Every query on the manifold, for a host array of queries.
mpwos_status check_queries_host(const mpwos_manifold* man, const WalkArgs& a, const double* q, int64_t nq) {
  const mpwos_manifold_desc& d = man->desc;
  if (d.kind != MPWOS_POINT_CLOUD) {
    for (int64_t i = 0; i < nq; ++i)
      if (!query_on_manifold(d, q + i * d.n))
        return fail(MPWOS_EOFFMANIFOLD, "query " + std::to_string(i) + " is not on the manifold");
    return MPWOS_OK;
  }
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "query check stream");
  double* dq = nullptr;
  const size_t bytes = (size_t)nq * 3 * sizeof(double);
  e = hipMalloc((void**)&dq, bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(dq, q, bytes, hipMemcpyHostToDevice, s);
  mpwos_status st = e == hipSuccess ? cloud_check_queries(a, dq, nq, s) : hip_fail(e, "query check upload");
  if (dq) (void)hipFree(dq);
  (void)hipStreamDestroy(s);
  return st;
}

// Walk kernel launch for a batch (queries/outputs already on the device).
mpwos_status launch_walks(WalkArgs& a, const mpwos_options& o, hipStream_t s, unsigned long long* queue) {
  const int64_t total = a.count;
  const int n_cu = device_cu_count();
  if (a.n <= 3) {
    // the point-cloud search keeps a per-lane stack in LDS sized for 128-lane workgroups
    const int block = a.kind == MPWOS_POINT_CLOUD ? (o.block_size ? o.block_size : 128) : (o.block_size ? o.block_size : 256);
    if (a.kind == MPWOS_POINT_CLOUD && block > 128)
      return fail(MPWOS_EINVAL, "point clouds take block_size 0, 64 or 128");
    hipError_t e;
    if (a.persistent || a.n_batch) {
      const int occ = lane_occupancy(a, block);
      const int64_t grid_max = (int64_t)occ * n_cu;
      const int64_t need = (total + block - 1) / block;
      const int64_t grid = std::max<int64_t>(1, std::min(grid_max, need));
      const int64_t waves = grid * (block / 64);
      int64_t chunk = total / (waves * 8);
      chunk = std::max<int64_t>(64, std::min<int64_t>(4096, (chunk / 64) * 64));
      a.chunk = (int32_t)chunk;
      a.queue = queue;
      e = launch_zero_u64(queue, 1, s);
      if (e == hipSuccess) e = launch_walk_lane(a, (int)grid, block, s);
    } else {
      const int64_t grid = (total + block - 1) / block;
      if (grid > 0x7FFFFFFF) return fail(MPWOS_EINVAL, "too many walks for one launch");
      e = launch_walk_lane(a, (int)grid, block, s);
    }
    if (e != hipSuccess) return hip_fail(e, "walk kernel launch");
    return MPWOS_OK;
  }
  if (a.n_batch) a.persistent = 1;
  return launch_group_walks(a, o, s, queue);
}

double philox_blocks_per_step(int n, int n_v) {
  if (n <= 3) return 1.0 + n_v;
  return (double)((n + 3) / 4) + (double)n_v * ((n + 3) / 4 + 1);
}

int64_t batch_unit(const WalkArgs& a, const mpwos_options& o) {
  if (a.n <= 3) return 64;
  int L, mb, nblk, rblk, rword;
  group_shape(a.n, o.lanes_per_walk, L, mb, nblk, rblk, rword);
  return L >= 4 && L <= 64 ? 64 / L : 1;
}

}  // namespace mpwos

extern "C" mpwos_status mpwos_solve(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g, double c,
                                    const double* queries, int64_t n_queries, int64_t n_walks, double eps,
                                    uint64_t seed, const mpwos_options* opt, double* u_out, double* stderr_out,
                                    mpwos_stats* stats) {
  g_last_error.clear();
  const auto t0 = std::chrono::steady_clock::now();
  mpwos_options o;
  if (opt) o = *opt;
  else mpwos_options_default(&o);
  if (!queries || !u_out) return fail(MPWOS_EINVAL, "queries and u_out must not be NULL");
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  mpwos_status st = context_init(g_ctx);
  if (st) return st;
  WalkArgs a;
  st = prepare_solve(manifold, f, g, c, n_queries, n_walks, eps, seed, o, a);
  if (st) return st;
  const mpwos_manifold_desc& d = manifold->desc;
  const int n = d.n;
  hipStream_t s = o.stream ? (hipStream_t)o.stream : g_ctx.stream;

  // host view of the queries for validation; device queries on an analytic
  // manifold are checked on the device instead, beside the walks, and the
  // solve returns EOFFMANIFOLD before writing any output
  const bool dev_check = o.device_io && device_query_check(d.kind);
  std::vector<double> hq;
  const double* qhost = queries;
  if (o.device_io && !dev_check) {
    hq.resize((size_t)n_queries * n);
    HIP_TRY(hipMemcpyAsync(hq.data(), queries, hq.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    qhost = hq.data();
  }
  if (d.kind != MPWOS_POINT_CLOUD && !dev_check) {
    for (int64_t q = 0; q < n_queries; ++q)
      if (!query_on_manifold(d, qhost + q * n))
        return fail(MPWOS_EOFFMANIFOLD, "query " + std::to_string(q) + " is not on the manifold");
  }

  // TABLE_S1 / DUMBBELL_POLY values to the device
  DevBuf& tmp = g_ctx.tmp;
  if (fn_has_values(f->kind)) {
    st = ensure(tmp, (size_t)f->n_values * sizeof(double));
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(tmp.p, f->values, (size_t)f->n_values * sizeof(double), hipMemcpyHostToDevice, s));
    a.f.values = (const double*)tmp.p;
  }

  // batches of queries, bounded by the per-walk buffer size
  const int64_t walk_budget = (int64_t)1 << 27;
  int64_t qb = std::max<int64_t>(1, walk_budget / n_walks);
  qb = std::min(qb, n_queries);
  const bool user_walk_dev = o.device_io && o.walk_S && o.walk_K;
  if (user_walk_dev) qb = n_queries;

  st = ensure(g_ctx.queries, (size_t)n_queries * n * sizeof(double));
  if (!st) st = ensure(g_ctx.u, (size_t)n_queries * sizeof(double));
  if (!st) st = ensure(g_ctx.se, (size_t)n_queries * sizeof(double));
  if (!st) st = ensure(g_ctx.stats, 8 * sizeof(unsigned long long));
  if (!st && !user_walk_dev) st = ensure(g_ctx.walkS, (size_t)qb * n_walks * sizeof(double));
  if (!st && !user_walk_dev) st = ensure(g_ctx.walkK, (size_t)qb * n_walks * sizeof(int32_t));
  if (st) return st;
  double* dq = (double*)g_ctx.queries.p;
  if (o.device_io) HIP_TRY(hipMemcpyAsync(dq, queries, (size_t)n_queries * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  else HIP_TRY(hipMemcpyAsync(dq, queries, (size_t)n_queries * n * sizeof(double), hipMemcpyHostToDevice, s));
  if (d.kind == MPWOS_POINT_CLOUD) {
    st = cloud_check_queries(a, dq, n_queries, s);
    if (st) return st;
  }
  unsigned long long* dstat = (unsigned long long*)g_ctx.stats.p;
  HIP_TRY(launch_zero_u64(dstat, 8, s));
  if (dev_check) HIP_TRY(launch_query_check(d, dq, n_queries, dstat + 7, s));
  // the K histogram, for the statistics only
  unsigned long long* dhist = nullptr;
  if (stats) {
    st = ensure(g_ctx.khist, kKHistBins * sizeof(unsigned long long));
    if (st) return st;
    dhist = (unsigned long long*)g_ctx.khist.p;
    HIP_TRY(launch_zero_u64(dhist, kKHistBins, s));
  }
  double* du = (double*)g_ctx.u.p;
  double* dse = (double*)g_ctx.se.p;
  float kernel_ms = 0.f, reduce_ms = 0.f;
  for (int64_t q0 = 0; q0 < n_queries; q0 += qb) {
    const int64_t nb = std::min(qb, n_queries - q0);
    double* wS = user_walk_dev ? o.walk_S : (double*)g_ctx.walkS.p;
    int32_t* wK = user_walk_dev ? o.walk_K : (int32_t*)g_ctx.walkK.p;
    a.queries = dq + q0 * n;
    a.nq = nb;
    a.nw = n_walks;
    a.q_offset = q0;
    a.idx_base = 0;
    a.count = nb * n_walks;
    a.walk_S = wS;
    a.walk_K = wK;
    HIP_TRY(hipEventRecord(g_ctx.ev[0], s));
    st = launch_walks(a, o, s, dstat + 4);
    if (st) return st;
    HIP_TRY(hipEventRecord(g_ctx.ev[1], s));
    HIP_TRY(launch_reduce(wS, wK, nb, n_walks, o.max_steps, du + q0, dse + q0, dstat + 0, (int32_t*)(dstat + 1),
                          dstat + 2, s));
    HIP_TRY(hipEventRecord(g_ctx.ev[2], s));
    if (dhist) HIP_TRY(launch_khist(wK, nb * n_walks, dhist, s));
    if (!o.device_io && o.walk_S)
      HIP_TRY(hipMemcpyAsync(o.walk_S + q0 * n_walks, wS, (size_t)nb * n_walks * sizeof(double), hipMemcpyDeviceToHost, s));
    if (!o.device_io && o.walk_K)
      HIP_TRY(hipMemcpyAsync(o.walk_K + q0 * n_walks, wK, (size_t)nb * n_walks * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventSynchronize(g_ctx.ev[2]));
    float ms1 = 0.f, ms2 = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms1, g_ctx.ev[0], g_ctx.ev[1]));
    HIP_TRY(hipEventElapsedTime(&ms2, g_ctx.ev[1], g_ctx.ev[2]));
    kernel_ms += ms1;
    reduce_ms += ms2;
  }
  const hipMemcpyKind dk = o.device_io ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (!dev_check) {
    HIP_TRY(hipMemcpyAsync(u_out, du, (size_t)n_queries * sizeof(double), dk, s));
    if (stderr_out) HIP_TRY(hipMemcpyAsync(stderr_out, dse, (size_t)n_queries * sizeof(double), dk, s));
  }
  unsigned long long* hs = g_ctx.hpin;
  unsigned long long* hh = g_ctx.hpin + 8;
  HIP_TRY(hipMemcpyAsync(hs, dstat, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if (dhist) HIP_TRY(hipMemcpyAsync(hh, dhist, kKHistBins * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (dev_check) {
    if (hs[7])
      return fail(MPWOS_EOFFMANIFOLD, "query " + std::to_string(n_queries - (int64_t)hs[7]) + " is not on the manifold");
    HIP_TRY(hipMemcpyAsync(u_out, du, (size_t)n_queries * sizeof(double), dk, s));
    if (stderr_out) HIP_TRY(hipMemcpyAsync(stderr_out, dse, (size_t)n_queries * sizeof(double), dk, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  const int64_t ksum = (int64_t)hs[0];
  const int32_t kmax = (int32_t)(uint32_t)hs[1];
  const int64_t ntr = (int64_t)hs[2];
  if (stats) {
    stats->walk_steps = ksum;
    stats->truncated = ntr;
    stats->k_max = kmax;
    stats->k_mean = (double)ksum / ((double)n_queries * (double)n_walks);
    stats->kernel_ms = kernel_ms;
    stats->reduce_ms = reduce_ms;
    khist_quantiles(hh, stats->k_p50, stats->k_p99);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return ntr ? MPWOS_WTRUNC : MPWOS_OK;
}

// ---------------------------------------------------------------------------
// allocation-free solve
// ---------------------------------------------------------------------------
// One fixed array per device holds everything mpwos_solve would allocate:
//   [0, 4 KiB)        statistics words and the persistent queue counter
//   [4 KiB, 260 KiB)  the source family's values (at most 32768 doubles)
//   [384 KiB, 420 KiB) the K histogram (when statistics are asked for)
//   [512 KiB, 1 MiB)  one inverse radial table (at most 17 slices)
//   [1 MiB, end)      per-walk scores and lengths of a batch of queries, the
//                     discarded standard errors when stderr_out is NULL, or
//                     the point-cloud query check's output
// In host code `scratch` names a host-side stand-in: only the address from
// hipGetSymbolAddress is passed to kernels and copies.
namespace mpwos {
static constexpr size_t kScratchBytes = (size_t)MPWOS_NOALLOC_SCRATCH_BYTES;
static constexpr size_t kScratchValuesOff = 4096, kScratchValuesMax = 32768;
static constexpr size_t kScratchTableOff = 512 * 1024, kScratchTableBytes = 512 * 1024;
static constexpr size_t kScratchWalkOff = 1024 * 1024;
static constexpr size_t kScratchHistOff = 384 * 1024;
static_assert(kScratchValuesOff + kScratchValuesMax * sizeof(double) <= kScratchHistOff &&
                  kScratchHistOff + kKHistBins * sizeof(unsigned long long) <= kScratchTableOff,
              "scratch layout");
static_assert(kScratchTableOff + kScratchTableBytes <= kScratchWalkOff && kScratchWalkOff < kScratchBytes,
              "scratch layout");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
struct ScratchSlot {
  unsigned char* ptr = nullptr;  // device address of this device's array
  TableKey table{0, 0, 0.0};     // inverse table the array holds (n = 0: none)
};
static ScratchSlot g_scratch[kMaxDevices];
static std::mutex g_scratch_lock;

// The device address of the current device's array, looked up once per device.
static mpwos_status scratch_slot(int dev, ScratchSlot*& slot) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MPWOS_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_lock);
  ScratchSlot& sl = g_scratch[dev];
  if (!sl.ptr) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol address");
    sl.ptr = (unsigned char*)p;
  }
  slot = &sl;
  return MPWOS_OK;
}
}  // namespace mpwos

extern "C" mpwos_status mpwos_solve_noalloc(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g,
                                            double c, const double* queries, int64_t n_queries, int64_t n_walks,
                                            double eps, uint64_t seed, const mpwos_options* opt, double* u_out,
                                            double* stderr_out, mpwos_stats* stats) {
  g_last_error.clear();
  const auto t0 = std::chrono::steady_clock::now();
  mpwos_options o;
  if (opt) o = *opt;
  else mpwos_options_default(&o);
  o.device_io = 1;
  if (!queries || !u_out) return fail(MPWOS_EINVAL, "queries and u_out must not be NULL");
  if ((o.walk_S == nullptr) != (o.walk_K == nullptr))
    return fail(MPWOS_EINVAL, "walk_S and walk_K are given together or not at all");
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  mpwos_status st = context_init(g_ctx);
  if (st) return st;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  ScratchSlot* slot = nullptr;
  st = scratch_slot(dev, slot);
  if (st) return st;
  unsigned char* base = slot->ptr;
  hipStream_t s = o.stream ? (hipStream_t)o.stream : (dev == g_ctx.device ? g_ctx.stream : nullptr);

  TableSink sink;
  sink.d64 = (double*)(base + kScratchTableOff);
  sink.bytes = kScratchTableBytes;
  sink.held = &slot->table;
  sink.stream = s;
  sink.use_cache = dev == g_ctx.device;
  WalkArgs a;
  st = prepare_solve(manifold, f, g, c, n_queries, n_walks, eps, seed, o, a, &sink);
  if (st) return st;
  const mpwos_manifold_desc& d = manifold->desc;
  const int n = d.n;

  // sizes against the array
  const bool user_walk = o.walk_S && o.walk_K;
  const size_t walk_region = kScratchBytes - kScratchWalkOff;
  const int64_t max_walks = (int64_t)((walk_region - sizeof(double)) / 12);
  if (!user_walk && n_walks > max_walks)
    return fail(MPWOS_EINVAL, "n_walks = " + std::to_string(n_walks) + " exceeds the allocation-free limit of " +
                                  std::to_string(max_walks) + " walks per query");
  const size_t per_query = (user_walk ? 0 : (size_t)n_walks * 12) + (stderr_out ? 0 : sizeof(double));
  const int64_t qb =
      user_walk ? n_queries : (int64_t)std::min<size_t>((size_t)n_queries, walk_region / per_query);
  if (user_walk && !stderr_out && (size_t)n_queries * sizeof(double) > walk_region)
    return fail(MPWOS_EINVAL, "n_queries exceeds the allocation-free limit without stderr_out");
  if (fn_has_values(f->kind) && (size_t)f->n_values > kScratchValuesMax)
    return fail(MPWOS_EINVAL, "f has more than " + std::to_string(kScratchValuesMax) +
                                  " values, beyond the allocation-free limit");

  // queries on the manifold
  if (d.kind != MPWOS_POINT_CLOUD) {
    std::vector<double> hq((size_t)n_queries * n);
    HIP_TRY(hipMemcpyAsync(hq.data(), queries, hq.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t q = 0; q < n_queries; ++q)
      if (!query_on_manifold(d, hq.data() + q * n))
        return fail(MPWOS_EOFFMANIFOLD, "query " + std::to_string(q) + " is not on the manifold");
  } else {
    st = cloud_check_queries(a, queries, n_queries, s, (double*)(base + kScratchWalkOff),
                             (int64_t)(walk_region / sizeof(double)));
    if (st) return st;
  }
  if (fn_has_values(f->kind)) {
    double* dv = (double*)(base + kScratchValuesOff);
    HIP_TRY(hipMemcpyAsync(dv, f->values, (size_t)f->n_values * sizeof(double), hipMemcpyHostToDevice, s));
    a.f.values = dv;
  }

  unsigned long long* dstat = (unsigned long long*)base;
  HIP_TRY(launch_zero_u64(dstat, 8, s));
  unsigned long long* dhist = stats ? (unsigned long long*)(base + kScratchHistOff) : nullptr;
  if (dhist) HIP_TRY(launch_zero_u64(dhist, kKHistBins, s));
  double* wS = user_walk ? o.walk_S : (double*)(base + kScratchWalkOff);
  int32_t* wK = user_walk ? o.walk_K : (int32_t*)(base + kScratchWalkOff + (size_t)qb * n_walks * sizeof(double));
  double* se_discard =
      user_walk ? (double*)(base + kScratchWalkOff) : (double*)((unsigned char*)wK + (size_t)qb * n_walks * 4);
  for (int64_t q0 = 0; q0 < n_queries; q0 += qb) {
    const int64_t nb = std::min(qb, n_queries - q0);
    a.queries = queries + q0 * n;
    a.nq = nb;
    a.nw = n_walks;
    a.q_offset = q0;
    a.idx_base = 0;
    a.count = nb * n_walks;
    a.walk_S = user_walk ? wS + q0 * n_walks : wS;
    a.walk_K = user_walk ? wK + q0 * n_walks : wK;
    st = launch_walks(a, o, s, dstat + 4);
    if (st) return st;
    HIP_TRY(launch_reduce(a.walk_S, a.walk_K, nb, n_walks, o.max_steps, u_out + q0,
                          stderr_out ? stderr_out + q0 : se_discard, dstat + 0, (int32_t*)(dstat + 1), dstat + 2, s));
    if (dhist) HIP_TRY(launch_khist(a.walk_K, nb * n_walks, dhist, s));
  }
  unsigned long long hs[8];
  unsigned long long hh[kKHistBins];
  HIP_TRY(hipMemcpyAsync(hs, dstat, sizeof(hs), hipMemcpyDeviceToHost, s));
  if (dhist) HIP_TRY(hipMemcpyAsync(hh, dhist, sizeof(hh), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t ntr = (int64_t)hs[2];
  if (stats) {
    stats->walk_steps = (int64_t)hs[0];
    stats->truncated = ntr;
    stats->k_max = (int32_t)(uint32_t)hs[1];
    stats->k_mean = (double)hs[0] / ((double)n_queries * (double)n_walks);
    stats->kernel_ms = 0.0;
    stats->reduce_ms = 0.0;
    khist_quantiles(hh, stats->k_p50, stats->k_p99);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return ntr ? MPWOS_WTRUNC : MPWOS_OK;
}

// ---------------------------------------------------------------------------
// inspection entry points
// ---------------------------------------------------------------------------
extern "C" mpwos_status mpwos_debug_cp(const mpwos_manifold* m, const double* x, int64_t n_points, int32_t precision,
                                       double* y) {
  g_last_error.clear();
  if (!m || !x || !y || n_points < 1) return fail(MPWOS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  mpwos_status st = context_init(g_ctx);
  if (st) return st;
  WalkArgs a;
  memset(&a, 0, sizeof(a));
  a.kind = m->desc.kind;
  a.n = m->desc.n;
  for (int i = 0; i < 4; ++i) a.p[i] = m->desc.p[i];
  a.precision = precision ? 1 : 0;
  mpwos_options o;
  mpwos_options_default(&o);
  o.precision = a.precision;
  if (m->cloud) cloud_fill_args(m->cloud, o, a);
  const size_t bytes = (size_t)n_points * a.n * sizeof(double);
  st = ensure(g_ctx.tmp, 2 * bytes);
  if (st) return st;
  hipStream_t s = g_ctx.stream;
  double* dx = (double*)g_ctx.tmp.p;
  double* dy = dx + (size_t)n_points * a.n;
  HIP_TRY(hipMemcpyAsync(dx, x, bytes, hipMemcpyHostToDevice, s));
  hipError_t e = a.n >= 4 ? launch_cp_group(a, dx, dy, n_points, s) : launch_cp_points(a, dx, dy, n_points, s);
  if (e != hipSuccess) return hip_fail(e, "cp kernel");
  HIP_TRY(hipMemcpyAsync(y, dy, bytes, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MPWOS_OK;
}

// grid limits shared by the predictor fit and its inspection entry point
static mpwos_status check_fit_grid(int32_t nt, int32_t ns, int32_t ks, int32_t kt) {
  if (nt < 1 || ns < 2 || (int64_t)nt * (ns - 1) > ((int64_t)1 << 20))
    return fail(MPWOS_EINVAL, "predictor grid: nt >= 1, ns >= 2 and nt (ns - 1) <= 2^20");
  if (ks < 1 || ks >= ns || kt < 0 || 2 * kt >= nt || ks > 64 || kt > 64)
    return fail(MPWOS_EINVAL, "predictor series: 1 <= ks < ns, 0 <= kt, 2 kt < nt, both <= 64");
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_predictor_fit(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g,
                                            double c, double eps, uint64_t seed, const mpwos_options* opt, int32_t nt,
                                            int32_t ns, int64_t n_walks, int32_t ks, int32_t kt, double* coef_out,
                                            mpwos_stats* stats) {
  g_last_error.clear();
  if (!manifold || !coef_out) return fail(MPWOS_EINVAL, "manifold and coef_out must not be NULL");
  const mpwos_manifold_desc& d = manifold->desc;
  if (d.kind != MPWOS_CUT_TORUS) return fail(MPWOS_EINVAL, "the predictor fit is defined on the cut torus");
  mpwos_status st = check_fit_grid(nt, ns, ks, kt);
  if (st) return st;
  mpwos_options o;
  if (opt) o = *opt;
  else mpwos_options_default(&o);
  o.compensation = MPWOS_COMP_NONE;
  o.device_io = 1;
  o.walk_S = nullptr;
  o.walk_K = nullptr;
  hipStream_t s = (hipStream_t)o.stream;
  hipStream_t own = nullptr;
  if (!s) {
    HIP_TRY(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    s = own;
  }
  o.stream = s;
  const int64_t m = (int64_t)nt * (ns - 1);
  const int64_t nc = (int64_t)ks * (2 * kt + 1);
  double* buf = nullptr;
  hipError_t e = hipMalloc((void**)&buf, (size_t)(4 * m + nc) * sizeof(double));
  if (e != hipSuccess) {
    if (own) (void)hipStreamDestroy(own);
    return hip_fail(e, "predictor buffers");
  }
  double *nodes = buf, *u = buf + 3 * m, *coef = buf + 4 * m;
  e = launch_ct_nodes(d.p[0], d.p[1], std::cos(d.p[2]), std::sin(d.p[2]), nt, ns, nodes, s);
  if (e != hipSuccess) st = hip_fail(e, "predictor nodes");
  // the coarse solve: every node is a query of the baseline estimator
  if (!st) st = mpwos_solve(manifold, f, g, c, nodes, m, n_walks, eps, seed, &o, u, nullptr, stats);
  if (st >= 0) {
    const mpwos_status solve_st = st;
    e = launch_ts_fit(u, nt, ns, kt, ks, coef, s);
    if (e == hipSuccess) e = hipMemcpyAsync(coef_out, coef, (size_t)nc * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = e == hipSuccess ? solve_st : hip_fail(e, "predictor fit");
  } else {
    (void)hipStreamSynchronize(s);
  }
  (void)hipFree(buf);
  if (own) (void)hipStreamDestroy(own);
  return st;
}

extern "C" mpwos_status mpwos_debug_ts_fit(const double* U, int32_t nt, int32_t ns, int32_t ks, int32_t kt,
                                           double* coef_out) {
  g_last_error.clear();
  if (!U || !coef_out) return fail(MPWOS_EINVAL, "bad arguments");
  mpwos_status st = check_fit_grid(nt, ns, ks, kt);
  if (st) return st;
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  st = context_init(g_ctx);
  if (st) return st;
  const int64_t m = (int64_t)nt * (ns - 1);
  const int64_t nc = (int64_t)ks * (2 * kt + 1);
  st = ensure(g_ctx.tmp, (size_t)(m + nc) * sizeof(double));
  if (st) return st;
  hipStream_t s = g_ctx.stream;
  double* du = (double*)g_ctx.tmp.p;
  double* dc = du + m;
  HIP_TRY(hipMemcpyAsync(du, U, (size_t)m * sizeof(double), hipMemcpyHostToDevice, s));
  hipError_t e = launch_ts_fit(du, nt, ns, kt, ks, dc, s);
  if (e != hipSuccess) return hip_fail(e, "fit kernel");
  HIP_TRY(hipMemcpyAsync(coef_out, dc, (size_t)nc * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_debug_cloud_info(const mpwos_manifold* m, int64_t* knn_fallback_points,
                                               double* max_spacing) {
  g_last_error.clear();
  if (!m || !m->cloud) return fail(MPWOS_EINVAL, "not a point-cloud manifold");
  if (knn_fallback_points) *knn_fallback_points = cloud_fallback_points(m->cloud);
  if (max_spacing) *max_spacing = cloud_max_spacing(m->cloud);
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_debug_radial_inv(int32_t n, double X, const double* u, int64_t count, int32_t precision,
                                               double* s_out) {
  g_last_error.clear();
  if (n < 2 || n > 4096 || !(X > 0) || !u || !s_out || count < 1) return fail(MPWOS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  mpwos_status st = context_init(g_ctx);
  if (st) return st;
  WalkArgs a;
  memset(&a, 0, sizeof(a));
  HostLaw h;
  host_law(n, h);
  int js, jd;
  if (!law_terms(h, X * X, js, jd)) return fail(MPWOS_EINVAL, "X beyond the series radial law");
  fill_law(h, js, jd, a.law);
  a.const_r = 1;
  a.X0 = X;
  fill_fixed(h, a.law, X, a.fixed);
  st = get_table(h, 1, X * X, a.tab);
  if (st) return st;
  st = ensure(g_ctx.tmp, 2 * (size_t)count * sizeof(double));
  if (st) return st;
  hipStream_t s = g_ctx.stream;
  double* du = (double*)g_ctx.tmp.p;
  double* ds = du + count;
  HIP_TRY(hipMemcpyAsync(du, u, (size_t)count * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_radial_inv(a, du, ds, count, precision ? 0 : 1, s));
  HIP_TRY(hipMemcpyAsync(s_out, ds, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_debug_philox(const uint32_t ctr[4], uint64_t seed, int64_t count, uint32_t* out) {
  g_last_error.clear();
  if (!ctr || !out || count < 1) return fail(MPWOS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  mpwos_status st = context_init(g_ctx);
  if (st) return st;
  st = ensure(g_ctx.tmp, (size_t)count * 16);
  if (st) return st;
  hipStream_t s = g_ctx.stream;
  HIP_TRY(launch_philox(ctr, seed, (uint32_t*)g_ctx.tmp.p, count, s));
  HIP_TRY(hipMemcpyAsync(out, g_ctx.tmp.p, (size_t)count * 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_copy_probe(int64_t bytes, int32_t reps, double* ms) {
  g_last_error.clear();
  if (bytes < 16 || reps < 1 || !ms) return fail(MPWOS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  mpwos_status st = context_init(g_ctx);
  if (st) return st;
  void *src = nullptr, *dst = nullptr;
  hipStream_t s = g_ctx.stream;
  hipError_t e = hipMalloc(&src, (size_t)bytes);
  if (e == hipSuccess) e = hipMalloc(&dst, (size_t)bytes);
  if (e == hipSuccess) e = hipMemsetAsync(src, 1, (size_t)bytes, s);
  if (e == hipSuccess) e = launch_copy(src, dst, bytes, s);
  if (e == hipSuccess) e = hipEventRecord(g_ctx.ev[0], s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(src, dst, bytes, s);
  if (e == hipSuccess) e = hipEventRecord(g_ctx.ev[1], s);
  if (e == hipSuccess) e = hipEventSynchronize(g_ctx.ev[1]);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, g_ctx.ev[0], g_ctx.ev[1]);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  if (e != hipSuccess) return hip_fail(e, "copy probe");
  *ms = t / reps;
  return MPWOS_OK;
}

extern "C" mpwos_status mpwos_valu_probe(int32_t op, double* lane_ops_per_s) {
  g_last_error.clear();
  if (op < 0 || op > 13 || !lane_ops_per_s) return fail(MPWOS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> guard(g_ctx.lock);
  mpwos_status st = context_init(g_ctx);
  if (st) return st;
  const int blocks = g_ctx.n_cu * 16;
  const int32_t iters = 4096;
  uint32_t* out = nullptr;
  hipStream_t s = g_ctx.stream;
  hipError_t e = hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(uint32_t));
  // warm-up launches (clocks settle), then the best of seven timed ones
  for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_valu_probe(op, 1u, iters, out, blocks, s);
  float best = 1e30f;
  for (int r = 0; r < 7 && e == hipSuccess; ++r) {
    e = hipEventRecord(g_ctx.ev[0], s);
    if (e == hipSuccess) e = launch_valu_probe(op, (uint32_t)(r + 2), iters, out, blocks, s);
    if (e == hipSuccess) e = hipEventRecord(g_ctx.ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(g_ctx.ev[1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, g_ctx.ev[0], g_ctx.ev[1]);
    best = std::min(best, t);
  }
  if (out) (void)hipFree(out);
  if (e != hipSuccess) return hip_fail(e, "valu probe");
  // operations per chain step: the xor and bitop3 chains issue two, the mixed streams four
  const double per_chain = (op == 9 || op == 13) ? 2.0 : (op == 11 || op == 12 ? 4.0 : 1.0);
  *lane_ops_per_s = (double)blocks * 256.0 * 8.0 * per_chain * (double)iters / (best * 1e-3);
  return MPWOS_OK;
}
