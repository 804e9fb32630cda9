/*
 * mpwos_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle for the modified projected Walk on Spheres
 * (MPWoS) estimator of the screened Poisson equation -Lap_Omega u + sigma u = f
 * on an embedded manifold (Sec. 2.1, eq. surface_pde / surface_bc).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * constant generator with the GPU path; it is written from the paper's
 * formulas and from the published definitions it names:
 *   - Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 *     as easy as 1, 2, 3", SC'11.
 *   - Box-Muller transform (Box & Muller 1958).
 *   - Archimedes' hat-box theorem for uniform directions on S^2.
 *   - Jacobi eigenvalue iteration (textbook) for the point-cloud frame.
 *
 * Floating point: IEEE binary64, built with -ffp-contract=off and no
 * fast-math, so every multiply-add is rounded twice, as written.
 *
 * Parity status of each function is stated in its comment; every function
 * here is pinned by a CPU test unless it says "parity unpinned".
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Codes (numeric values fixed by the solver's public interface).             */
/* ------------------------------------------------------------------------- */
enum { ORC_SPHERE = 0, ORC_SPHERE_CAP = 1, ORC_TORUS = 2, ORC_POINT_CLOUD = 3, ORC_DUMBBELL = 4, ORC_PRODUCT = 5,
       ORC_CUT_TORUS = 6 };
enum {
  ORC_FN_ZERO = 0, ORC_FN_CONST = 1, ORC_FN_SPH_PAIR = 2, ORC_FN_CIRCLE_MODE = 3,
  ORC_FN_LEGENDRE = 4, ORC_FN_TORUS_MODE = 5, ORC_FN_TABLE_S1 = 6, ORC_FN_DUMBBELL_POLY = 7,
  ORC_FN_PRODUCT_MODES = 8, ORC_FN_TORUS_SINE = 9
};
enum { ORC_COMP_NONE = 0, ORC_COMP_EXACT = 1, ORC_COMP_SECOND_ORDER = 2 };
enum { ORC_RADIUS_CURVATURE = 0, ORC_RADIUS_SPACING = 1, ORC_RADIUS_CURVATURE_FIT = 2,
       ORC_RADIUS_CURVATURE_BOUND = 3 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EOFFMANIFOLD = -2, ORC_ENOMEM = -3, ORC_WTRUNC = 1 };

#define ORC_MAXN 4096
#define ORC_NSERIES 160
#define ORC_MAXK 64

typedef struct {
  int32_t manifold;      /* ORC_SPHERE ... */
  int32_t n;             /* ambient dimension */
  double p[4];           /* sphere: R; cap: R, h; torus: R, a; dumbbell: alpha, kappa (half-length);
                            product: R (Fourier curve), a (sphere); cut torus: R, a, phi_c */
  const double* points;  /* point cloud, n_points x 3, row-major */
  int64_t n_points;
  int32_t k_nn;          /* neighbours used by the local reconstruction */
  int32_t radius_rule;   /* ORC_RADIUS_* */
  int32_t f_kind; int32_t f_idx[3]; double f_coef[8];
  const double* f_values; int64_t f_nvalues;
  int32_t g_kind; int32_t g_idx[3]; double g_coef[8];
  double sigma, eps, theta, c_kappa, c_h, tau_w;
  int32_t n_v, compensation;
  int64_t max_steps;
  int32_t k_spacing;     /* neighbours for the spacing rule h(y) */
  int32_t newton_iters;  /* foot-point Newton iterations on the fitted patch */
  double kappa_bound;    /* point cloud, CURVATURE_BOUND rule: a bound of kappa over M */
  int32_t reconstruction; /* point cloud: 0 = quadratic patch, 1 = the nearest cloud point */
  /* second-order compensation: coefficients of the predictor u_* as a
   * Fourier-sine series (layout of ORC_FN_TORUS_SINE), and the normal step */
  const double* pred_coef; int32_t pred_ks, pred_kt; double h_eta;
  /* point cloud: the patch of a cloud point p is fitted to the cloud points
   * within fit_scale r_k of p, r_k the distance to its k_nn-th nearest
   * point; fit_scale <= 1 fits the k_nn nearest points themselves */
  double fit_scale;
  const struct orc_grid* grid;  /* optional exact grid index of the points (orc_grid_build) */
} orc_problem;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 Philox S-box,  */
/* multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 /      */
/* 0xBB67AE85, key bumped between rounds.                                     */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Random stream of one walk: Philox block `block` of sub-stream `sub` at step
 * k of walk w of query q.  counter = (q, w, k, sub<<24 | block),
 * key = (seed_lo, seed_hi).  sub 0 = sphere direction, sub l = Green sample l. */
static void orc_block(uint64_t seed, uint32_t q, uint32_t w, uint32_t k, uint32_t sub,
                      uint32_t block, uint32_t out[4]) {
  uint32_t ctr[4] = {q, w, k, (sub << 24) | block};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* 32-bit word -> uniform in (0,1): (x + 1/2) 2^-32. */
double orc_uniform(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

/* Box-Muller on one word pair. */
void orc_box_muller(uint32_t x0, uint32_t x1, double out[2]) {
  double u0 = orc_uniform(x0), u1 = orc_uniform(x1);
  double rad = sqrt(-2.0 * log(u0));
  double ang = 6.283185307179586 * u1;
  out[0] = rad * cos(ang);
  out[1] = rad * sin(ang);
}

/* n standard normals of sub-stream `sub`: normal i comes from words
 * (2*floor(i/2), 2*floor(i/2)+1) of the sub-stream, word j being word j%4
 * of block j/4. */
void orc_normals(uint64_t seed, uint32_t q, uint32_t w, uint32_t k, uint32_t sub, int n,
                 double* g) {
  int nblocks = (n + 3) / 4;
  for (int b = 0; b < nblocks; ++b) {
    uint32_t x[4];
    orc_block(seed, q, w, k, sub, (uint32_t)b, x);
    double pr[2];
    orc_box_muller(x[0], x[1], pr);
    if (4 * b + 0 < n) g[4 * b + 0] = pr[0];
    if (4 * b + 1 < n) g[4 * b + 1] = pr[1];
    orc_box_muller(x[2], x[3], pr);
    if (4 * b + 2 < n) g[4 * b + 2] = pr[0];
    if (4 * b + 3 < n) g[4 * b + 3] = pr[1];
  }
}

/* Uniform direction on S^{n-1} from sub-stream `sub` (the zeta of eq.
 * projected_chain_update and the direction of a Green sample).
 *   n = 2: angle 2 pi u0 (word 0): zeta = (cos, sin).
 *   n = 3: Archimedes' hat-box theorem: the last coordinate z = 1 - 2 u0 is
 *          uniform on [-1, 1] and the azimuth 2 pi u1 is uniform and
 *          independent of it (words 0, 1): zeta = (rho cos, rho sin, z) with
 *          rho = sqrt(1 - z^2) = 2 sqrt(u0 (1 - u0)).
 *   n >= 4: n standard normals (orc_normals) divided by their norm.
 * Every form is an exact sample of the uniform law. */
void orc_direction(uint64_t seed, uint32_t q, uint32_t w, uint32_t k, uint32_t sub, int n, double* zeta) {
  if (n == 2 || n == 3) {
    uint32_t x[4];
    orc_block(seed, q, w, k, sub, 0, x);
    if (n == 2) {
      double ang = 6.283185307179586 * orc_uniform(x[0]);
      zeta[0] = cos(ang);
      zeta[1] = sin(ang);
    } else {
      double u = orc_uniform(x[0]);
      double ang = 6.283185307179586 * orc_uniform(x[1]);
      double rho = 2.0 * sqrt(u * (1.0 - u));
      zeta[0] = rho * cos(ang);
      zeta[1] = rho * sin(ang);
      zeta[2] = 1.0 - 2.0 * u;
    }
    return;
  }
  orc_normals(seed, q, w, k, sub, n, zeta);
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += zeta[i] * zeta[i];
  s = sqrt(s);
  for (int i = 0; i < n; ++i) zeta[i] = zeta[i] / s;
}

/* The uniform that picks the radius of Green sample `sub`: word 3 of the
 * sub-stream for n <= 3 (after the direction words); for n >= 4 the first
 * word after the normal pairs, word index 2*ceil(n/2). */
double orc_radius_uniform(uint64_t seed, uint32_t q, uint32_t w, uint32_t k, uint32_t sub, int n) {
  int word = n <= 3 ? 3 : 2 * ((n + 1) / 2);
  uint32_t x[4];
  orc_block(seed, q, w, k, sub, (uint32_t)(word / 4), x);
  return orc_uniform(x[word % 4]);
}

/* ------------------------------------------------------------------------- */
/* Screening factor c_{sigma,r} and omega = (1-c)/sigma.                      */
/* Lemma 3.1 series: c = [sum_j (sigma r^2/4)^j / (j! (nu+1)_j)]^-1,          */
/* nu = (n-2)/2 (eq. def_c_sigma_r); omega from Theorem 2.2                   */
/* (eq. omega_explicit_formula).  s1 = sum_{j>=1}, so 1-c = s1/(1+s1) has no  */
/* cancellation.                                                              */
/* ------------------------------------------------------------------------- */
static double orc_s1(int n, double sigma, double r) {
  double nu = 0.5 * (double)(n - 2);
  double q = sigma * r * r / 4.0;
  double term = 1.0, s1 = 0.0;
  for (int j = 1; j < 100000; ++j) {
    term = term * q / ((double)j * (nu + (double)j));
    s1 += term;
    if (term <= 1e-18 * s1) break;
  }
  return s1;
}
double orc_c_sigma_r(int n, double sigma, double r) { return 1.0 / (1.0 + orc_s1(n, sigma, r)); }
double orc_omega(int n, double sigma, double r) {
  double s1 = orc_s1(n, sigma, r);
  return s1 / (sigma * (1.0 + s1));
}

/* ------------------------------------------------------------------------- */
/* Radial law of the normalised Green density rho = G/omega (eq. omega_of_y,  */
/* eq. Z_sampling_density).  With lambda = sqrt(sigma), X = lambda r,         */
/* s = t/r, x = X s, S_nu(x) = Gamma(nu+1)(2/x)^nu I_nu(x) = sum_j            */
/* (x^2/4)^j/(j!(nu+1)_j) and sum_j b_j y^{2j} = S_nu(y)^-2, the flux of G    */
/* through the sphere of radius t gives the CDF of |Z-Y|/r:                    */
/*   (1-c) F(s) = (1 - 1/S_nu(x)) + x^2 S_{nu+1}(x)/(2(nu+1)) D(s),           */
/*   (1-c) F'(s) = X^2 s S_nu(x) D(s),                                        */
/*   D(s) = sum_{j != nu} b_j X^{2j} (s^{2j} - s^{2nu})/(2(nu-j))             */
/*          + [nu integer] b_nu X^{2nu} (-s^{2nu} ln s).                      */
/* Derived from the Green function of the Remark after Lemma 2.1 by reduction */
/* of order on the regular radial solution (proof of Lemma 2.1).              */
/* ------------------------------------------------------------------------- */
typedef struct {
  int n;
  double nu;
  int nu_int;            /* nu is an integer (n even): index of the log term, else -1 */
  double alpha[ORC_NSERIES];   /* S_nu coefficients in z = y^2 */
  double alpha1[ORC_NSERIES];  /* S_{nu+1} coefficients */
  double beta[ORC_NSERIES];    /* coefficients of S_nu^-2 */
} orc_radial;

static void orc_radial_init(orc_radial* R, int n) {
  R->n = n;
  R->nu = 0.5 * (double)(n - 2);
  R->nu_int = (n % 2 == 0) ? (n - 2) / 2 : -1;
  R->alpha[0] = 1.0;
  R->alpha1[0] = 1.0;
  for (int j = 1; j < ORC_NSERIES; ++j) {
    R->alpha[j] = R->alpha[j - 1] / (4.0 * (double)j * (R->nu + (double)j));
    R->alpha1[j] = R->alpha1[j - 1] / (4.0 * (double)j * (R->nu + 1.0 + (double)j));
  }
  double gam[ORC_NSERIES];
  for (int j = 0; j < ORC_NSERIES; ++j) {
    double acc = 0.0;
    for (int i = 0; i <= j; ++i) acc += R->alpha[i] * R->alpha[j - i];
    gam[j] = acc;
  }
  R->beta[0] = 1.0;
  for (int j = 1; j < ORC_NSERIES; ++j) {
    double acc = 0.0;
    for (int i = 1; i <= j; ++i) acc += gam[i] * R->beta[j - i];
    R->beta[j] = -acc;
  }
}

/* Largest X for which the b_j series is used: 0.8 sqrt((nu+1)(nu+5)), a lower
 * bound of the first zero j_{nu,1} of J_nu (the radius of convergence). */
double orc_radial_xmax(int n) {
  double nu = 0.5 * (double)(n - 2);
  return 0.8 * sqrt((nu + 1.0) * (nu + 5.0));
}

/* sum_{j>=1} a_j z^j */
static double orc_series_tail(const double* a, double z) {
  double zp = 1.0, acc = 0.0;
  for (int j = 1; j < ORC_NSERIES; ++j) {
    zp *= z;
    double t = a[j] * zp;
    acc += t;
    if (fabs(t) <= 1e-19 * fabs(acc)) break;
  }
  return acc;
}
static double orc_series(const double* a, double z) { return 1.0 + orc_series_tail(a, z); }

static double orc_radial_D(const orc_radial* R, double X, double s) {
  double X2 = X * X;
  double s2 = s * s;
  double s2nu = (R->n == 2) ? 1.0 : pow(s, (double)(R->n - 2));
  /* Each term is at most |b_j| X^{2j} in size (|s^{2j} - s^{2nu}| <= 1,
   * |2(nu - j)| >= 1), and the b_j X^{2j} decay geometrically inside the
   * series' disc, so the sum stops after three terms below 1e-19 of it. */
  double acc = 0.0, Xp = 1.0, sp = 1.0;
  int small = 0;
  for (int j = 0; j < ORC_NSERIES; ++j) {
    if (j > 0) { Xp *= X2; sp *= s2; }
    if (!isfinite(Xp)) break;
    double bx = R->beta[j] * Xp;
    double t;
    if (j == R->nu_int) t = bx * (-s2nu * log(s));
    else t = bx * (sp - s2nu) / (2.0 * (R->nu - (double)j));
    acc += t;
    if (fabs(bx) <= 1e-19 * fabs(acc)) {
      if (++small >= 3 && j >= 2) break;
    } else {
      small = 0;
    }
  }
  return acc;
}

static double orc_radial_cdf_r(const orc_radial* R, double X, double s) {
  if (s <= 0.0) return 0.0;
  if (s >= 1.0) return 1.0;
  double z = X * X * s * s;
  double s1x = orc_series_tail(R->alpha, z);
  double S1 = orc_series(R->alpha1, z);
  double s1X = orc_series_tail(R->alpha, X * X);
  double D = orc_radial_D(R, X, s);
  double num = s1x / (1.0 + s1x) + z * S1 / (2.0 * (R->nu + 1.0)) * D;
  return num * (1.0 + s1X) / s1X;
}

static double orc_radial_pdf_r(const orc_radial* R, double X, double s) {
  if (s <= 0.0 || s >= 1.0) return 0.0;
  double z = X * X * s * s;
  double Sx = orc_series(R->alpha, z);
  double s1X = orc_series_tail(R->alpha, X * X);
  double D = orc_radial_D(R, X, s);
  return X * X * s * Sx * D * (1.0 + s1X) / s1X;
}

/* Inverse CDF by bisection on [0,1] until the bracket cannot shrink. */
static double orc_radial_inv_r(const orc_radial* R, double X, double u) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (orc_radial_cdf_r(R, X, mid) < u) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

double orc_radial_cdf(int n, double X, double s) {
  orc_radial R; orc_radial_init(&R, n);
  return orc_radial_cdf_r(&R, X, s);
}
double orc_radial_pdf(int n, double X, double s) {
  orc_radial R; orc_radial_init(&R, n);
  return orc_radial_pdf_r(&R, X, s);
}
double orc_radial_inv(int n, double X, double u) {
  orc_radial R; orc_radial_init(&R, n);
  return orc_radial_inv_r(&R, X, u);
}

/* ------------------------------------------------------------------------- */
/* Small vector helpers.                                                      */
/* ------------------------------------------------------------------------- */
static double orc_dot(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}
static double orc_norm(const double* a, int n) { return sqrt(orc_dot(a, a, n)); }

/* ------------------------------------------------------------------------- */
/* Point cloud: exact kNN by brute force, ties by index, then the local       */
/* reconstruction (centroid, PCA frame, least-squares quadratic height field, */
/* Newton foot point).  The paper names "nearest-neighbour search with local  */
/* reconstruction" for point clouds (Sec. 2.3.2); the reconstruction used is  */
/* this quadratic patch.                                                      */
/* ------------------------------------------------------------------------- */
typedef struct { double d2; int64_t idx; } orc_nb;

static int orc_nb_less(const orc_nb* a, const orc_nb* b) {
  return (a->d2 < b->d2) || (a->d2 == b->d2 && a->idx < b->idx);
}

/* k nearest points of x (sorted by (distance^2, index)). */
int orc_knn(const double* pts, int64_t np, const double* x, int k, int64_t* idx_out, double* d2_out) {
  if (k > ORC_MAXK || k > np || k < 1) return ORC_EINVAL;
  orc_nb best[ORC_MAXK];
  int cnt = 0;
  for (int64_t i = 0; i < np; ++i) {
    double dx = pts[3 * i] - x[0], dy = pts[3 * i + 1] - x[1], dz = pts[3 * i + 2] - x[2];
    orc_nb c = {dx * dx + dy * dy + dz * dz, i};
    if (cnt < k) {
      int j = cnt++;
      while (j > 0 && orc_nb_less(&c, &best[j - 1])) { best[j] = best[j - 1]; --j; }
      best[j] = c;
    } else if (orc_nb_less(&c, &best[k - 1])) {
      int j = k - 1;
      while (j > 0 && orc_nb_less(&c, &best[j - 1])) { best[j] = best[j - 1]; --j; }
      best[j] = c;
    }
  }
  for (int j = 0; j < k; ++j) { idx_out[j] = best[j].idx; d2_out[j] = best[j].d2; }
  return ORC_OK;
}

/* Exact search on a uniform grid of cubic cells of side h: point i lies in
 * cell floor((p_i - lo) / h) (clamped to the grid), the cells' point lists in
 * ascending index.  A k-nearest search visits the cells in shells of growing
 * Chebyshev distance L from the cell of x; every point outside the shells
 * visited so far lies beyond the slab faces of the visited block, so the search
 * stops once the k-th distance is below the nearest face (less a rounding
 * allowance for the binning).  The results equal orc_knn's brute force. */
typedef struct orc_grid {
  const double* pts;
  int64_t np;
  double lo[3], h, slack;
  int64_t nc[3];
  int64_t* start;  /* ncell + 1 offsets into idx */
  int64_t* idx;    /* point indices by cell */
} orc_grid;

static int64_t orc_grid_axis(const orc_grid* G, int d, double v) {
  double c = floor((v - G->lo[d]) / G->h);
  if (!(c >= 0.0)) return 0;
  if (c > (double)(G->nc[d] - 1)) return G->nc[d] - 1;
  return (int64_t)c;
}

orc_grid* orc_grid_build(const double* pts, int64_t np) {
  if (!pts || np < 1) return NULL;
  orc_grid* G = (orc_grid*)calloc(1, sizeof(orc_grid));
  if (!G) return NULL;
  G->pts = pts;
  G->np = np;
  double hi[3];
  for (int d = 0; d < 3; ++d) { G->lo[d] = pts[d]; hi[d] = pts[d]; }
  for (int64_t i = 0; i < np; ++i)
    for (int d = 0; d < 3; ++d) {
      G->lo[d] = fmin(G->lo[d], pts[3 * i + d]);
      hi[d] = fmax(hi[d], pts[3 * i + d]);
    }
  double vol = 1.0, amax = 0.0;
  for (int d = 0; d < 3; ++d) {
    vol *= fmax(hi[d] - G->lo[d], 1e-12);
    amax = fmax(amax, fmax(fabs(G->lo[d]), fabs(hi[d])));
  }
  /* about one cell per point of the bounding box, coarsened until at most
   * 2^24 cells */
  G->h = 1.5 * cbrt(vol / (double)np);
  for (;;) {
    double cells = 1.0;
    for (int d = 0; d < 3; ++d) cells *= floor((hi[d] - G->lo[d]) / G->h) + 1.0;
    if (cells <= 16777216.0) break;
    G->h *= 1.25;
  }
  for (int d = 0; d < 3; ++d) G->nc[d] = (int64_t)floor((hi[d] - G->lo[d]) / G->h) + 1;
  G->slack = 1e-13 * (amax + G->h);
  int64_t ncell = G->nc[0] * G->nc[1] * G->nc[2];
  G->start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
  G->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)np);
  int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)np);
  if (!G->start || !G->idx || !cell) {
    free(cell);
    free(G->start);
    free(G->idx);
    free(G);
    return NULL;
  }
  for (int64_t i = 0; i < np; ++i) {
    const double* q = pts + 3 * i;
    cell[i] = (orc_grid_axis(G, 2, q[2]) * G->nc[1] + orc_grid_axis(G, 1, q[1])) * G->nc[0] + orc_grid_axis(G, 0, q[0]);
    G->start[cell[i] + 1] += 1;
  }
  for (int64_t c = 0; c < ncell; ++c) G->start[c + 1] += G->start[c];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
  if (!fill) {
    free(cell);
    free(G->start);
    free(G->idx);
    free(G);
    return NULL;
  }
  memcpy(fill, G->start, sizeof(int64_t) * (size_t)ncell);
  for (int64_t i = 0; i < np; ++i) G->idx[fill[cell[i]]++] = i;
  free(fill);
  free(cell);
  return G;
}

void orc_grid_free(orc_grid* G) {
  if (!G) return;
  free(G->start);
  free(G->idx);
  free(G);
}

/* k nearest points of x on the grid, sorted by (distance^2, index). */
int orc_grid_knn(const orc_grid* G, const double* x, int k, int64_t* idx_out, double* d2_out) {
  if (!G || k > ORC_MAXK || k > G->np || k < 1) return ORC_EINVAL;
  orc_nb best[ORC_MAXK];
  int cnt = 0;
  int64_t c[3];
  for (int d = 0; d < 3; ++d) c[d] = orc_grid_axis(G, d, x[d]);
  int64_t Lmax = 0;
  for (int d = 0; d < 3; ++d) {
    if (c[d] > Lmax) Lmax = c[d];
    if (G->nc[d] - 1 - c[d] > Lmax) Lmax = G->nc[d] - 1 - c[d];
  }
  for (int64_t L = 0; L <= Lmax; ++L) {
    for (int64_t kz = c[2] - L; kz <= c[2] + L; ++kz) {
      if (kz < 0 || kz >= G->nc[2]) continue;
      for (int64_t ky = c[1] - L; ky <= c[1] + L; ++ky) {
        if (ky < 0 || ky >= G->nc[1]) continue;
        for (int64_t kx = c[0] - L; kx <= c[0] + L; ++kx) {
          if (kx < 0 || kx >= G->nc[0]) continue;
          int64_t cheb = llabs(kx - c[0]);
          if (llabs(ky - c[1]) > cheb) cheb = llabs(ky - c[1]);
          if (llabs(kz - c[2]) > cheb) cheb = llabs(kz - c[2]);
          if (cheb != L) continue;
          int64_t cc = (kz * G->nc[1] + ky) * G->nc[0] + kx;
          for (int64_t t = G->start[cc]; t < G->start[cc + 1]; ++t) {
            int64_t i = G->idx[t];
            const double* q = G->pts + 3 * i;
            double dx = q[0] - x[0], dy = q[1] - x[1], dz = q[2] - x[2];
            orc_nb cand = {dx * dx + dy * dy + dz * dz, i};
            if (cnt < k) {
              int j = cnt++;
              while (j > 0 && orc_nb_less(&cand, &best[j - 1])) { best[j] = best[j - 1]; --j; }
              best[j] = cand;
            } else if (orc_nb_less(&cand, &best[k - 1])) {
              int j = k - 1;
              while (j > 0 && orc_nb_less(&cand, &best[j - 1])) { best[j] = best[j - 1]; --j; }
              best[j] = cand;
            }
          }
        }
      }
    }
    if (cnt == k) {
      /* distance from x to the nearest face of the visited block of cells
       * that has cells beyond it */
      double face = INFINITY;
      for (int d = 0; d < 3; ++d) {
        if (c[d] - L > 0) face = fmin(face, x[d] - (G->lo[d] + (double)(c[d] - L) * G->h));
        if (c[d] + L < G->nc[d] - 1) face = fmin(face, (G->lo[d] + (double)(c[d] + L + 1) * G->h) - x[d]);
      }
      face -= G->slack;
      if (face > 0.0 && best[k - 1].d2 < face * face) break;
    }
  }
  for (int j = 0; j < k; ++j) { idx_out[j] = best[j].idx; d2_out[j] = best[j].d2; }
  return ORC_OK;
}

/* Every point within distance^2 <= rho2 of x (ascending index within cells),
 * up to cap of them; returns the count (which may exceed cap), or -1. */
int64_t orc_grid_ball(const orc_grid* G, const double* x, double rho2, int64_t* idx_out, int64_t cap) {
  if (!G || !(rho2 >= 0.0)) return -1;
  double rho = sqrt(rho2) + G->slack;
  int64_t a[3], b[3];
  for (int d = 0; d < 3; ++d) {
    a[d] = orc_grid_axis(G, d, x[d] - rho) - 1;
    b[d] = orc_grid_axis(G, d, x[d] + rho) + 1;
    if (a[d] < 0) a[d] = 0;
    if (b[d] > G->nc[d] - 1) b[d] = G->nc[d] - 1;
  }
  int64_t cnt = 0;
  for (int64_t kz = a[2]; kz <= b[2]; ++kz)
    for (int64_t ky = a[1]; ky <= b[1]; ++ky)
      for (int64_t kx = a[0]; kx <= b[0]; ++kx) {
        int64_t cc = (kz * G->nc[1] + ky) * G->nc[0] + kx;
        for (int64_t t = G->start[cc]; t < G->start[cc + 1]; ++t) {
          int64_t i = G->idx[t];
          const double* q = G->pts + 3 * i;
          double dx = q[0] - x[0], dy = q[1] - x[1], dz = q[2] - x[2];
          if (dx * dx + dy * dy + dz * dz <= rho2) {
            if (cnt < cap) idx_out[cnt] = i;
            ++cnt;
          }
        }
      }
  return cnt;
}

/* The problem's k nearest search: on its grid when it has one. */
static int orc_pc_knn(const orc_problem* P, const double* x, int k, int64_t* idx, double* d2) {
  if (P->grid) return orc_grid_knn(P->grid, x, k, idx, d2);
  return orc_knn(P->points, P->n_points, x, k, idx, d2);
}

static int orc_cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* The cloud points within distance^2 <= rho2 of x, in ascending index order
 * (so that a fit over them is summed in the same order with or without the
 * grid), in a buffer the caller frees; returns the count or -1. */
static int64_t orc_pc_ball(const orc_problem* P, const double* x, double rho2, int64_t** out) {
  int64_t cap = 512;
  for (;;) {
    int64_t* buf = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    if (!buf) return -1;
    int64_t cnt;
    if (P->grid) {
      cnt = orc_grid_ball(P->grid, x, rho2, buf, cap);
    } else {
      cnt = 0;
      for (int64_t i = 0; i < P->n_points; ++i) {
        const double* q = P->points + 3 * i;
        double dx = q[0] - x[0], dy = q[1] - x[1], dz = q[2] - x[2];
        if (dx * dx + dy * dy + dz * dz <= rho2) {
          if (cnt < cap) buf[cnt] = i;
          ++cnt;
        }
      }
    }
    if (cnt < 0 || cnt <= cap) {
      if (cnt > 1) qsort(buf, (size_t)cnt, sizeof(int64_t), orc_cmp_i64);
      *out = buf;
      return cnt;
    }
    free(buf);
    cap = cnt;
  }
}

/* Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (textbook).
 * Eigenvalues ascending in w, eigenvectors as columns of V. */
static void orc_jacobi3(const double A_in[9], double w[3], double V[9]) {
  double A[9];
  memcpy(A, A_in, sizeof(A));
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        double apq = A[3 * p + q];
        if (apq == 0.0) continue;
        double app = A[3 * p + p], aqq = A[3 * q + q];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        /* A <- J^T A J with J the (p,q) rotation */
        for (int k = 0; k < 3; ++k) {
          double akp = A[3 * k + p], akq = A[3 * k + q];
          A[3 * k + p] = c * akp - s * akq;
          A[3 * k + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          double apk = A[3 * p + k], aqk = A[3 * q + k];
          A[3 * p + k] = c * apk - s * aqk;
          A[3 * q + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = V[3 * k + p], vkq = V[3 * k + q];
          V[3 * k + p] = c * vkp - s * vkq;
          V[3 * k + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  int order[3] = {0, 1, 2};
  double d[3] = {A[0], A[4], A[8]};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (d[order[j]] < d[order[i]]) { int t = order[i]; order[i] = order[j]; order[j] = t; }
  double Vs[9];
  for (int c = 0; c < 3; ++c) {
    w[c] = d[order[c]];
    for (int r = 0; r < 3; ++r) Vs[3 * r + c] = V[3 * r + order[c]];
  }
  memcpy(V, Vs, sizeof(Vs));
}

/* Solve the 6x6 SPD system M a = b by Gaussian elimination with partial pivoting. */
static int orc_solve6(double M[36], double b[6], double a[6]) {
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r) if (fabs(M[6 * r + c]) > fabs(M[6 * piv + c])) piv = r;
    if (M[6 * piv + c] == 0.0) return ORC_EINVAL;
    if (piv != c) {
      for (int k = 0; k < 6; ++k) { double t = M[6 * c + k]; M[6 * c + k] = M[6 * piv + k]; M[6 * piv + k] = t; }
      double t = b[c]; b[c] = b[piv]; b[piv] = t;
    }
    for (int r = c + 1; r < 6; ++r) {
      double f = M[6 * r + c] / M[6 * c + c];
      for (int k = c; k < 6; ++k) M[6 * r + k] -= f * M[6 * c + k];
      b[r] -= f * b[c];
    }
  }
  for (int r = 5; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < 6; ++k) s -= M[6 * r + k] * a[k];
    a[r] = s / M[6 * r + r];
  }
  return ORC_OK;
}

typedef struct {
  double y[3];        /* projected point cp_h(x) */
  double kappa;       /* max |principal curvature| of the fitted patch at the foot */
  double h_mean;      /* mean distance from the patch's cloud point to its k-1 neighbours */
  int64_t patch;      /* index of the cloud point whose patch holds y */
} orc_pc_result;

/* The local reconstruction at cloud point i: its k nearest cloud points (i
 * included) or, with fit_scale > 1, the cloud points within fit_scale r_k of
 * it; their centroid and PCA frame; the least-squares quadratic height field
 * h = c0 + c1 a + c2 b + c3 a^2 + c4 a b + c5 b^2 over the tangent plane; the
 * support (largest |a| or |b| of its points); the mean distance from i to its
 * k-1 other neighbours. */
typedef struct {
  double cen[3], e1[3], e2[3], nn[3], coef[6], ext, h_mean;
} orc_patch;

static int orc_pc_fit(const orc_problem* P, int64_t i, orc_patch* pt) {
  int k = P->k_nn;
  const double* pn = P->points + 3 * i;
  int64_t idx[ORC_MAXK];
  double d2[ORC_MAXK];
  int st = orc_pc_knn(P, pn, k, idx, d2);
  if (st) return st;
  double hsum = 0.0;
  for (int j = 1; j < k; ++j) hsum += sqrt(d2[j]);
  pt->h_mean = hsum / (double)(k - 1);
  const int64_t* fit = idx;
  int64_t nfit = k;
  int64_t* ball = NULL;
  if (P->fit_scale > 1.0) {
    double rho2 = P->fit_scale * P->fit_scale * d2[k - 1];
    nfit = orc_pc_ball(P, pn, rho2, &ball);
    if (nfit < 6) { free(ball); return ORC_EINVAL; }
    fit = ball;
  }
  double cen[3] = {0, 0, 0};
  for (int64_t j = 0; j < nfit; ++j)
    for (int c = 0; c < 3; ++c) cen[c] += P->points[3 * fit[j] + c];
  for (int c = 0; c < 3; ++c) cen[c] /= (double)nfit;
  double C[9] = {0};
  for (int64_t j = 0; j < nfit; ++j) {
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = P->points[3 * fit[j] + c] - cen[c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[3 * r + c] += d[r] * d[c];
  }
  double w[3], V[9];
  orc_jacobi3(C, w, V);
  for (int c = 0; c < 3; ++c) {
    pt->cen[c] = cen[c];
    pt->e1[c] = V[c * 3 + 2];
    pt->e2[c] = V[c * 3 + 1];
    pt->nn[c] = V[c * 3 + 0];
  }
  double M[36] = {0}, rhs[6] = {0};
  double ext = 0.0;
  for (int64_t j = 0; j < nfit; ++j) {
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = P->points[3 * fit[j] + c] - cen[c];
    double a = orc_dot(d, pt->e1, 3), b = orc_dot(d, pt->e2, 3), h = orc_dot(d, pt->nn, 3);
    ext = fmax(ext, fmax(fabs(a), fabs(b)));
    double phi[6] = {1.0, a, b, a * a, a * b, b * b};
    for (int r = 0; r < 6; ++r) {
      rhs[r] += phi[r] * h;
      for (int c = 0; c < 6; ++c) M[6 * r + c] += phi[r] * phi[c];
    }
  }
  free(ball);
  pt->ext = ext;
  return orc_solve6(M, rhs, pt->coef);
}

/* Foot point of x on patch pt: minimise E(a,b) = (a-ax)^2 + (b-bx)^2 +
 * (h(a,b)-hx)^2 over the support square |a|, |b| <= ext (unbounded when
 * clamp is 0: the patch's whole quadratic), from (ax,bx) clamped to it, by
 * newton_iters Newton steps; where the Newton Hessian is not positive
 * definite (x beyond the focal distance of the quadratic) the Gauss-Newton
 * matrix I + J^T J replaces it; every iterate is clamped to the square.
 * Then the curvature indicator there: the largest |eigenvalue| of the shape
 * operator I^-1 II of the graph, I = [[1+ha^2, ha hb],[ha hb, 1+hb^2]],
 * II = Hess(h)/sqrt(1+ha^2+hb^2). */
static void orc_patch_foot(const orc_problem* P, const orc_patch* pt, const double* x, int clamp, double* y,
                           double* kappa) {
  const double* coef = pt->coef;
  double dx[3];
  for (int c = 0; c < 3; ++c) dx[c] = x[c] - pt->cen[c];
  double ax = orc_dot(dx, pt->e1, 3), bx = orc_dot(dx, pt->e2, 3), hx = orc_dot(dx, pt->nn, 3);
  double ext = clamp ? pt->ext : 3.0e38;
  double a = fmin(fmax(ax, -ext), ext), b = fmin(fmax(bx, -ext), ext);
  for (int it = 0; it < P->newton_iters; ++it) {
    double h = coef[0] + coef[1] * a + coef[2] * b + coef[3] * a * a + coef[4] * a * b + coef[5] * b * b;
    double ha = coef[1] + 2.0 * coef[3] * a + coef[4] * b;
    double hb = coef[2] + coef[4] * a + 2.0 * coef[5] * b;
    double haa = 2.0 * coef[3], hab = coef[4], hbb = 2.0 * coef[5];
    double r = h - hx;
    double ga = (a - ax) + r * ha;
    double gb = (b - bx) + r * hb;
    double Haa = 1.0 + ha * ha + r * haa;
    double Hab = ha * hb + r * hab;
    double Hbb = 1.0 + hb * hb + r * hbb;
    double det = Haa * Hbb - Hab * Hab;
    if (!(Haa > 0.0 && det > 0.0)) {
      Haa = 1.0 + ha * ha;
      Hab = ha * hb;
      Hbb = 1.0 + hb * hb;
      det = Haa * Hbb - Hab * Hab;
    }
    double da = (Hbb * ga - Hab * gb) / det;
    double db = (Haa * gb - Hab * ga) / det;
    a = fmin(fmax(a - da, -ext), ext);
    b = fmin(fmax(b - db, -ext), ext);
  }
  double h = coef[0] + coef[1] * a + coef[2] * b + coef[3] * a * a + coef[4] * a * b + coef[5] * b * b;
  for (int c = 0; c < 3; ++c) y[c] = pt->cen[c] + a * pt->e1[c] + b * pt->e2[c] + h * pt->nn[c];
  double ha = coef[1] + 2.0 * coef[3] * a + coef[4] * b;
  double hb = coef[2] + coef[4] * a + 2.0 * coef[5] * b;
  double gfac = sqrt(1.0 + ha * ha + hb * hb);
  double I11 = 1.0 + ha * ha, I12 = ha * hb, I22 = 1.0 + hb * hb;
  double II11 = 2.0 * coef[3] / gfac, II12 = coef[4] / gfac, II22 = 2.0 * coef[5] / gfac;
  double detI = I11 * I22 - I12 * I12;
  double S11 = (I22 * II11 - I12 * II12) / detI;
  double S12 = (I22 * II12 - I12 * II22) / detI;
  double S21 = (I11 * II12 - I12 * II11) / detI;
  double S22 = (I11 * II22 - I12 * II12) / detI;
  double tr = S11 + S22, dt = S11 * S22 - S12 * S21;
  double disc = tr * tr / 4.0 - dt;
  if (disc < 0.0) disc = 0.0;
  double l1 = tr / 2.0 + sqrt(disc), l2 = tr / 2.0 - sqrt(disc);
  *kappa = fmax(fabs(l1), fabs(l2));
}

#define ORC_PC_ROUNDS 4

/* Local reconstruction and projection of x onto a point cloud (Sec. 2.3.2,
 * "nearest-neighbour search with local reconstruction"): cp_h(x) is the
 * foot point of x on the patch of the cloud point nearest to that foot
 * point.  It is found from a start patch by alternating the foot point on
 * the current patch and the nearest cloud point of the foot, until the
 * nearest point is the current one, in at most ORC_PC_ROUNDS foot points.
 * Start (start < 0): the cloud point nearest to x.  Otherwise the walker's
 * patch `start`: the cloud point nearest to the foot point of x on that
 * patch's whole quadratic.  The pure nearest-neighbour projection of
 * Example 4 (reconstruction 1) is the cloud point nearest to x. */
int orc_pc_project_from(const orc_problem* P, const double* x, int64_t start, orc_pc_result* res) {
  int64_t p;
  double d2;
  orc_patch pt;
  int st;
  if (P->reconstruction == 1) {
    st = orc_pc_knn(P, x, 1, &p, &d2);
    if (st) return st;
    int64_t idx[ORC_MAXK];
    double dk[ORC_MAXK];
    st = orc_pc_knn(P, P->points + 3 * p, P->k_nn, idx, dk);
    if (st) return st;
    double hsum = 0.0;
    for (int j = 1; j < P->k_nn; ++j) hsum += sqrt(dk[j]);
    for (int c = 0; c < 3; ++c) res->y[c] = P->points[3 * p + c];
    res->kappa = 0.0;
    res->h_mean = hsum / (double)(P->k_nn - 1);
    res->patch = p;
    return ORC_OK;
  }
  if (start < 0) {
    st = orc_pc_knn(P, x, 1, &p, &d2);
    if (st) return st;
  } else {
    double y0[3], kap;
    st = orc_pc_fit(P, start, &pt);
    if (st) return st;
    orc_patch_foot(P, &pt, x, 0, y0, &kap);
    st = orc_pc_knn(P, y0, 1, &p, &d2);
    if (st) return st;
  }
  for (int j = 0; j < ORC_PC_ROUNDS; ++j) {
    st = orc_pc_fit(P, p, &pt);
    if (st) return st;
    orc_patch_foot(P, &pt, x, 1, res->y, &res->kappa);
    res->h_mean = pt.h_mean;
    if (j == ORC_PC_ROUNDS - 1) break;
    int64_t q;
    st = orc_pc_knn(P, res->y, 1, &q, &d2);
    if (st) return st;
    if (q == p) break;
    p = q;
  }
  res->patch = p;
  return ORC_OK;
}

int orc_pc_project(const orc_problem* P, const double* x, orc_pc_result* res) {
  return orc_pc_project_from(P, x, -1, res);
}

/* ------------------------------------------------------------------------- */
/* Manifolds: closest-point map cp (eq. cp_map), curvature indicator kappa    */
/* (eq. rho_geo_curvature), nearest boundary point cp_Gamma and the effective */
/* boundary distance delta_Gamma (eq. delta_Gamma_general).                   */
/* ------------------------------------------------------------------------- */

/* Torus (R, a) around the x3 axis.  Closest point: the nearest point C of the
 * core circle, then the point at distance a from C towards x. */
static int orc_torus_cp(double R, double a, const double* x, double* y) {
  double rho = sqrt(x[0] * x[0] + x[1] * x[1]);
  if (rho == 0.0) return ORC_EINVAL;
  double C[3] = {R * x[0] / rho, R * x[1] / rho, 0.0};
  double d[3] = {x[0] - C[0], x[1] - C[1], x[2]};
  double dn = orc_norm(d, 3);
  if (dn == 0.0) return ORC_EINVAL;
  for (int i = 0; i < 3; ++i) y[i] = C[i] + a * d[i] / dn;
  return ORC_OK;
}

/* Toroidal angle phi, tube angle psi and distance to the core circle. */
static void orc_torus_angles(double R, const double* x, double* phi, double* psi, double* dist) {
  double rho = sqrt(x[0] * x[0] + x[1] * x[1]);
  *phi = atan2(x[1], x[0]);
  *psi = atan2(x[2], rho - R);
  *dist = sqrt((rho - R) * (rho - R) + x[2] * x[2]);
}

/* ------------------------------------------------------------------------- */
/* Torus with a planar cut (Sec. 4, Example 1): the torus of radii R, a cut   */
/* by the plane through its axis at angle phi_c; Omega is the half with       */
/* s = phi - phi_c in (0, pi) (phi the angle about the axis, th the tube      */
/* angle, as in the paper's parametrization X(th, phi)).  Its boundary Gamma  */
/* is the two tube circles s = 0 and s = pi.                                  */
/* ------------------------------------------------------------------------- */

/* Tube angle th, s = phi - phi_c wrapped to (-pi, pi], distance rho to the
 * core circle. */
static void orc_ct_coords(const orc_problem* P, const double* x, double* th, double* s, double* rho) {
  double phi;
  orc_torus_angles(P->p[0], x, &phi, th, rho);
  double d = phi - P->p[2];
  d = d - 6.283185307179586 * floor(d / 6.283185307179586);  /* [0, 2 pi) */
  if (d > 3.141592653589793) d -= 6.283185307179586;
  *s = d;
}

/* u and its derivatives u_th, u_thth, u_ss of a Fourier-sine series
 *   u(th, s) = sum_{k=1..ks} sin(k s) [c_k0 + sum_{j=1..kt} (c_kj cos j th + d_kj sin j th)],
 * coefficients stored per k as (c_k0, c_k1, d_k1, ..., c_kkt, d_kkt). */
typedef struct { double u, ut, utt, uss; } orc_ts_val;

static orc_ts_val orc_ts_eval(const double* c, int ks, int kt, double th, double s) {
  orc_ts_val v = {0.0, 0.0, 0.0, 0.0};
  int stride = 2 * kt + 1;
  for (int k = 1; k <= ks; ++k) {
    const double* ck = c + (size_t)(k - 1) * stride;
    double T = ck[0], T1 = 0.0, T2 = 0.0;
    for (int j = 1; j <= kt; ++j) {
      double cj = cos(j * th), sj = sin(j * th);
      double a = ck[2 * j - 1], b = ck[2 * j];
      T += a * cj + b * sj;
      T1 += (double)j * (b * cj - a * sj);
      T2 -= (double)(j * j) * (a * cj + b * sj);
    }
    double sk = sin(k * s);
    v.u += sk * T;
    v.ut += sk * T1;
    v.utt += sk * T2;
    v.uss -= (double)(k * k) * sk * T;
  }
  return v;
}

/* Ambient Laplacian of the closest-point extension of u at distance rho from
 * the core circle: in toroidal coordinates (rho, th, phi) the extension does
 * not depend on rho, leaving
 *   u_thth / rho^2 - sin(th) u_th / (rho (R + rho cos th)) + u_phiphi / (R + rho cos th)^2;
 * at rho = a this is the Laplace-Beltrami operator of the torus (eq.
 * LB_cp_identity). */
static double orc_ct_lap(double R, double rho, double th, orc_ts_val v) {
  double q = R + rho * cos(th);
  return v.utt / (rho * rho) - sin(th) * v.ut / (rho * q) + v.uss / (q * q);
}

/* Nearest point y_G of Gamma (the nearer of the two cut circles) and the
 * torus normal there. */
static void orc_ct_cp_gamma(const orc_problem* P, const double* y, double* yg, double* ng) {
  double R = P->p[0], a = P->p[1];
  double best = INFINITY;
  for (int b = 0; b < 2; ++b) {
    double ph = P->p[2] + (b ? 3.141592653589793 : 0.0);
    double e[3] = {cos(ph), sin(ph), 0.0};
    /* circle of radius a about R e in the plane spanned by e and the axis:
     * the point of y in that plane, seen from the circle's centre */
    double pe = y[0] * e[0] + y[1] * e[1] - R, pz = y[2];
    double d = sqrt(pe * pe + pz * pz);
    double n[3] = {e[0] * pe / d, e[1] * pe / d, pz / d};
    double q[3] = {R * e[0] + a * n[0], R * e[1] + a * n[1], a * n[2]};
    double dd = 0.0;
    for (int i = 0; i < 3; ++i) dd += (q[i] - y[i]) * (q[i] - y[i]);
    if (dd < best) {
      best = dd;
      for (int i = 0; i < 3; ++i) { yg[i] = q[i]; ng[i] = n[i]; }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Implicit dumbbell hypersurface (Sec. 4, Example 2): x = (xh, xs) with      */
/* xh in R^{n-1}; M = { |xh| = R(xs) },                                       */
/*   R(xs) = sqrt(1 - (xs/kc)^2) (1 - a + 2 a (xs/kc)^2).                     */
/* With xs = kc cos(phi), phi in [0, pi], the profile is                      */
/*   r(phi) = sin(phi) g(phi), g = 1 - a + 2 a cos^2(phi),  z(phi) = kc cos(phi), */
/* smooth up to the poles; M is the surface of revolution of (r, z) about the */
/* xs axis with cross-sections S^{n-2}.                                       */
/* ------------------------------------------------------------------------- */
typedef struct { double r, r1, r2, z, z1, z2, g; } orc_profile;

static orc_profile orc_db_profile(double a, double kc, double phi) {
  orc_profile p;
  double s = sin(phi), c = cos(phi);
  double g = 1.0 - a + 2.0 * a * c * c;
  double g1 = -4.0 * a * c * s;
  double g2 = -4.0 * a * (c * c - s * s);
  p.g = g;
  p.r = s * g;
  p.r1 = c * g + s * g1;
  p.r2 = -s * g + 2.0 * c * g1 + s * g2;
  p.z = kc * c;
  p.z1 = -kc * s;
  p.z2 = -kc * c;
  return p;
}

/* Profile parameter of the point of M nearest to (|xh|, xs) = (rho, zs): the
 * global minimum of D(phi) = (rho - r)^2 + (zs - z)^2 on a 2048-cell grid,
 * then Newton on D' = 0 kept inside the neighbouring cells by bisection. */
double orc_db_phi(double a, double kc, double rho, double zs) {
  const int M = 2048;
  const double pi = 3.141592653589793;
  const double h = pi / M;
  int best = 0;
  double bd = INFINITY;
  for (int i = 0; i <= M; ++i) {
    orc_profile p = orc_db_profile(a, kc, i * h);
    double d = (rho - p.r) * (rho - p.r) + (zs - p.z) * (zs - p.z);
    if (d < bd) { bd = d; best = i; }
  }
  double lo = best > 0 ? (best - 1) * h : 0.0;
  double hi = best < M ? (best + 1) * h : pi;
  double phi = best * h;
  for (int it = 0; it < 200; ++it) {
    orc_profile p = orc_db_profile(a, kc, phi);
    double d1 = -2.0 * ((rho - p.r) * p.r1 + (zs - p.z) * p.z1);
    double d2 = 2.0 * (p.r1 * p.r1 + p.z1 * p.z1) - 2.0 * ((rho - p.r) * p.r2 + (zs - p.z) * p.z2);
    if (d1 > 0.0) hi = phi; else lo = phi;
    double nx = d2 > 0.0 ? phi - d1 / d2 : NAN;
    if (!(nx >= lo && nx <= hi)) nx = 0.5 * (lo + hi);
    double step = fabs(nx - phi);
    phi = nx;
    if (step <= 1e-16 * (1.0 + phi) || hi - lo <= 1e-16 * (1.0 + phi)) break;
  }
  return phi;
}

/* cp onto the dumbbell; phi_out (nullable) receives the profile parameter. */
static int orc_db_cp(const orc_problem* P, const double* x, double* y, double* phi_out) {
  int n = P->n;
  double rho = 0.0;
  for (int i = 0; i < n - 1; ++i) rho += x[i] * x[i];
  rho = sqrt(rho);
  double phi = orc_db_phi(P->p[0], P->p[1], rho, x[n - 1]);
  orc_profile p = orc_db_profile(P->p[0], P->p[1], phi);
  for (int i = 0; i < n - 1; ++i) y[i] = rho > 0.0 ? p.r * (x[i] / rho) : 0.0;
  y[n - 1] = p.z;
  if (phi_out) *phi_out = phi;
  return ORC_OK;
}

/* Principal curvatures of the dumbbell at profile parameter phi, for the
 * outward normal: k1 of the profile curve, k2 (multiplicity n-2) of the
 * cross-section sphere, -z'/(L r) = kc/(g L). */
void orc_db_curvatures(double a, double kc, double phi, double* k1, double* k2) {
  orc_profile p = orc_db_profile(a, kc, phi);
  double L = sqrt(p.r1 * p.r1 + p.z1 * p.z1);
  *k1 = (p.z1 * p.r2 - p.r1 * p.z2) / (L * L * L);
  *k2 = kc / (p.g * L);
}

/* f_Omega = -Lap_M u + sigma u for the polynomial
 *   U(x) = c0 xs + c1 xs^2 + b1 (1.xh)/sqrt(n-1) + b2 xh^T diag(A) xh
 * at the point y of M with profile parameter phi, by the extrinsic formula
 * Lap_M U = Lap U - nu^T Hess(U) nu - H dU/dnu (H = k1 + (n-2) k2, nu the
 * outward unit normal (N_r e, N_z), e = xh/|xh|). */
static double orc_db_f(const orc_problem* P, const double* y, double phi) {
  int n = P->n, m = n - 1;
  const double* c = P->f_coef;
  const double* A = P->f_values;
  orc_profile p = orc_db_profile(P->p[0], P->p[1], phi);
  double L = sqrt(p.r1 * p.r1 + p.z1 * p.z1);
  double Nr = -p.z1 / L, Nz = p.r1 / L;
  double k1, k2;
  orc_db_curvatures(P->p[0], P->p[1], phi, &k1, &k2);
  double rho = 0.0;
  for (int i = 0; i < m; ++i) rho += y[i] * y[i];
  rho = sqrt(rho);
  double s1 = 0.0, sA = 0.0, tr = 0.0;
  for (int i = 0; i < m; ++i) {
    double e = rho > 0.0 ? y[i] / rho : 0.0;
    s1 += e;
    sA += A[i] * e * e;
    tr += A[i];
  }
  double z = y[n - 1];
  double isq = 1.0 / sqrt((double)m);
  double U = c[0] * z + c[1] * z * z + c[2] * rho * s1 * isq + c[3] * rho * rho * sA;
  double lapU = 2.0 * c[1] + 2.0 * c[3] * tr;
  double hess = 2.0 * c[1] * Nz * Nz + 2.0 * c[3] * Nr * Nr * sA;
  double dnu = Nz * (c[0] + 2.0 * c[1] * z) + Nr * (c[2] * s1 * isq + 2.0 * c[3] * rho * sA);
  double H = k1 + (double)(m - 1) * k2;
  double lapM = lapU - hess - H * dnu;
  return -lapM + P->sigma * U;
}

/* ------------------------------------------------------------------------- */
/* Product manifold of Sec. 4, Example 3: M = S^1_Fourier(R) x S^2(a) in R^9, */
/* X(phi, w) = (R C(phi), a w), C(phi) = (cos phi, sin phi, cos 2phi / 2,     */
/* sin 2phi / 2, cos 3phi / 3, sin 3phi / 3).  |C'| = sqrt(3) and            */
/* |C| = const, so the nearest curve point of x_c maximises                   */
/* g(phi) = x_c . C(phi) = sum_k (a_k cos k phi + b_k sin k phi) / k with     */
/* a_k = x_c[2k-2], b_k = x_c[2k-1]; the sphere factor is normalised.         */
/* ------------------------------------------------------------------------- */
static void orc_pr_g(const double* xc, double phi, double* g, double* g1, double* g2) {
  *g = *g1 = *g2 = 0.0;
  for (int k = 1; k <= 3; ++k) {
    double c = cos(k * phi), s = sin(k * phi);
    double ak = xc[2 * k - 2], bk = xc[2 * k - 1];
    *g += (ak * c + bk * s) / k;
    *g1 += -ak * s + bk * c;
    *g2 += -k * (ak * c + bk * s);
  }
}

/* Curve parameter of the point of the Fourier curve nearest to x_c: the best
 * of a 2048-point grid over [0, 2 pi), then Newton on g' = 0 kept inside the
 * neighbouring cells by bisection. */
double orc_pr_phi(const double* xc) {
  const int M = 2048;
  const double h = 6.283185307179586 / M;
  int best = 0;
  double bg = -INFINITY, g, g1, g2;
  for (int i = 0; i < M; ++i) {
    orc_pr_g(xc, i * h, &g, &g1, &g2);
    if (g > bg) { bg = g; best = i; }
  }
  double lo = (best - 1) * h, hi = (best + 1) * h, phi = best * h;
  for (int it = 0; it < 200; ++it) {
    orc_pr_g(xc, phi, &g, &g1, &g2);
    if (g1 > 0.0) lo = phi; else hi = phi;
    double nx = g2 < 0.0 ? phi - g1 / g2 : NAN;
    if (!(nx >= lo && nx <= hi)) nx = 0.5 * (lo + hi);
    double step = fabs(nx - phi);
    phi = nx;
    if (step <= 1e-16 * (1.0 + fabs(phi)) || hi - lo <= 1e-16 * (1.0 + fabs(phi))) break;
  }
  return phi;
}

static int orc_pr_cp(const orc_problem* P, const double* x, double* y, double* phi_out) {
  double R = P->p[0], a = P->p[1];
  double phi = orc_pr_phi(x);
  for (int k = 1; k <= 3; ++k) {
    y[2 * k - 2] = R * cos(k * phi) / k;
    y[2 * k - 1] = R * sin(k * phi) / k;
  }
  double ns = sqrt(x[6] * x[6] + x[7] * x[7] + x[8] * x[8]);
  if (ns == 0.0) return ORC_EINVAL;
  for (int i = 6; i < 9; ++i) y[i] = a * x[i] / ns;
  if (phi_out) *phi_out = phi;
  return ORC_OK;
}

/* f_Omega = -Lap_M u + sigma u for u = c0 cos(phi) w1 + c1 sin(2 phi) w2 +
 * c2 cos(3 phi) (w1^2 - w2^2): Lap_M is the sum of the factors' operators,
 * d^2/ds^2 = (1/(3 R^2)) d^2/dphi^2 on the curve (speed R sqrt 3), and the
 * degree-1 and degree-2 harmonics w1, w2, w1^2 - w2^2 on S^2(a) (eigenvalues
 * 2/a^2, 2/a^2, 6/a^2). */
static double orc_pr_f(const orc_problem* P, const double* y, double phi) {
  const double* c = P->f_coef;
  double R = P->p[0], a = P->p[1], sg = P->sigma;
  double w1 = y[6] / a, w2 = y[7] / a;
  double q = 1.0 / (3.0 * R * R), s2 = 1.0 / (a * a);
  return c[0] * (sg + q + 2.0 * s2) * cos(phi) * w1 + c[1] * (sg + 4.0 * q + 2.0 * s2) * sin(2.0 * phi) * w2 +
         c[2] * (sg + 9.0 * q + 6.0 * s2) * cos(3.0 * phi) * (w1 * w1 - w2 * w2);
}

int orc_cp(const orc_problem* P, const double* x, double* y) {
  int n = P->n;
  switch (P->manifold) {
    case ORC_DUMBBELL: return orc_db_cp(P, x, y, NULL);
    case ORC_PRODUCT: return orc_pr_cp(P, x, y, NULL);
    case ORC_SPHERE:
    case ORC_SPHERE_CAP: {
      double nx = orc_norm(x, n);
      if (nx == 0.0) return ORC_EINVAL;
      for (int i = 0; i < n; ++i) y[i] = P->p[0] * x[i] / nx;
      return ORC_OK;
    }
    case ORC_TORUS:
    case ORC_CUT_TORUS: return orc_torus_cp(P->p[0], P->p[1], x, y);
    case ORC_POINT_CLOUD: {
      orc_pc_result res;
      int st = orc_pc_project(P, x, &res);
      if (st) return st;
      for (int i = 0; i < 3; ++i) y[i] = res.y[i];
      return ORC_OK;
    }
  }
  return ORC_EINVAL;
}

/* Curvature indicator kappa(y): largest |principal curvature|.  On the
 * product: the larger of the curve's curvature sqrt(14)/(3R) (|C''|^2 = 14,
 * C'' normal to C', speed sqrt 3) and the sphere's 1/a, both constant. */
static double orc_kappa(const orc_problem* P, const double* y) {
  switch (P->manifold) {
    case ORC_PRODUCT: {
      double kc = sqrt(14.0) / (3.0 * P->p[0]), ks = 1.0 / P->p[1];
      return kc > ks ? kc : ks;
    }
    case ORC_SPHERE:
    case ORC_SPHERE_CAP: return 1.0 / P->p[0];
    case ORC_TORUS:
    case ORC_CUT_TORUS: {
      double phi, psi, dist;
      orc_torus_angles(P->p[0], y, &phi, &psi, &dist);
      double k1 = 1.0 / P->p[1];
      double k2 = fabs(cos(psi)) / (P->p[0] + P->p[1] * cos(psi));
      return k1 > k2 ? k1 : k2;
    }
  }
  return 0.0;
}

/* Nearest point of the cap boundary Gamma = S^{n-1}_R cap {x_n = h}. */
static void orc_cap_cp_gamma(const orc_problem* P, const double* y, double* yg) {
  int n = P->n;
  double R = P->p[0], h = P->p[1];
  double rg = sqrt(R * R - h * h);
  double ny = 0.0;
  for (int i = 0; i < n - 1; ++i) ny += y[i] * y[i];
  ny = sqrt(ny);
  for (int i = 0; i < n - 1; ++i) yg[i] = rg * y[i] / ny;
  yg[n - 1] = h;
}

/* Nearest boundary point y_G and the unit normal of M there. */
static void orc_gamma_point(const orc_problem* P, const double* y, double* yg, double* nrm) {
  if (P->manifold == ORC_CUT_TORUS) {
    orc_ct_cp_gamma(P, y, yg, nrm);
    return;
  }
  orc_cap_cp_gamma(P, y, yg);
  for (int i = 0; i < P->n; ++i) nrm[i] = yg[i] / P->p[0];
}

static int orc_has_boundary(const orc_problem* P) {
  return P->manifold == ORC_SPHERE_CAP || P->manifold == ORC_CUT_TORUS;
}

/* delta_Gamma(y) = dist(y, E_Gamma(y_Gamma)) with the normal disk of radius
 * ell = rho_geo(y_Gamma) (eq. extended_boundary_disk, eq. delta_Gamma_general).
 * Both boundaries here have codimension one in M and M has codimension one,
 * so the normal space of M at y_G is the line of its unit normal. */
static double orc_bdry_delta(const orc_problem* P, const double* y) {
  int n = P->n;
  double yg[ORC_MAXN], rG[ORC_MAXN], nrm[ORC_MAXN], rT[ORC_MAXN];
  orc_gamma_point(P, y, yg, nrm);
  for (int i = 0; i < n; ++i) rG[i] = yg[i] - y[i];
  double rn = orc_dot(rG, nrm, n);
  for (int i = 0; i < n; ++i) rT[i] = rG[i] - rn * nrm[i];
  double ell = P->c_kappa / (1.0 + orc_kappa(P, yg));
  double tN = fabs(rn) - ell;
  if (tN < 0.0) tN = 0.0;
  return sqrt(orc_dot(rT, rT, n) + tN * tN);
}

/* Membership of the boundary layer Gamma_eps (eq. boundary_layer).  A point
 * on the far side of the cut (at or below the cap's plane, or outside
 * 0 < s < pi on the cut torus) counts as inside the layer. */
static int orc_in_layer(const orc_problem* P, const double* y) {
  if (P->manifold == ORC_CUT_TORUS) {
    double th, sv, rho;
    orc_ct_coords(P, y, &th, &sv, &rho);
    if (!(sv > 0.0 && sv < 3.141592653589793)) return 1;
  } else if (y[P->n - 1] <= P->p[1]) {
    return 1;
  }
  return orc_bdry_delta(P, y) < P->eps;
}

double orc_delta_gamma(const orc_problem* P, const double* y) {
  if (!orc_has_boundary(P)) return INFINITY;
  return orc_bdry_delta(P, y);
}

/* ------------------------------------------------------------------------- */
/* Sources: f(x) = f_Omega(cp(x)) (eq. cp_extension) and the exact            */
/* compensation m(x) = -Lap(Eu)(x) + sigma Eu(x) - f(x) (eq.                  */
/* mismatch_definition) for families whose solution u is known.               */
/* ------------------------------------------------------------------------- */
static double orc_legendre(int l, double t) {
  double p0 = 1.0, p1 = t;
  if (l == 0) return p0;
  for (int k = 1; k < l; ++k) {
    double p2 = ((2.0 * k + 1.0) * t * p1 - (double)k * p0) / (double)(k + 1);
    p0 = p1; p1 = p2;
  }
  return p1;
}

/* -Lap_T of sin(phi) cos(2 psi) on the torus of tube radius `a` (or, with a
 * replaced by the distance to the core circle, the ambient Laplacian of its
 * closest-point extension). */
static double orc_torus_neg_lap(double R, double a, double phi, double psi) {
  double rt = R + a * cos(psi);
  double u = sin(phi) * cos(2.0 * psi);
  return 4.0 * u / (a * a) + u / (rt * rt) - 2.0 * sin(phi) * sin(psi) * sin(2.0 * psi) / (a * rt);
}

/* Linear interpolation of a periodic table over theta in [0, 2 pi). */
static double orc_table_s1(const double* v, int64_t M, double theta) {
  double t = theta / 6.283185307179586;
  t -= floor(t);
  double pos = t * (double)M;
  int64_t i0 = (int64_t)floor(pos);
  double fr = pos - (double)i0;
  i0 %= M;
  int64_t i1 = (i0 + 1) % M;
  return (1.0 - fr) * v[i0] + fr * v[i1];
}

/* f_Omega at a point y of M. */
static double orc_f_omega(const orc_problem* P, const double* y) {
  int n = P->n;
  const double* c = P->f_coef;
  switch (P->f_kind) {
    case ORC_FN_ZERO: return 0.0;
    case ORC_FN_CONST: return c[0];
    case ORC_FN_SPH_PAIR: {
      double R = P->p[0];
      return c[0] * (y[P->f_idx[0]] / R) * (y[P->f_idx[1]] / R);
    }
    case ORC_FN_CIRCLE_MODE: {
      double th = atan2(y[1], y[0]);
      int k = P->f_idx[0];
      return c[0] * cos((double)k * th) + c[1] * sin((double)k * th);
    }
    case ORC_FN_LEGENDRE: {
      double t = y[n - 1] / P->p[0];
      double s = 0.0;
      for (int l = 0; l < 8; ++l) s += c[l] * orc_legendre(l, t);
      return s;
    }
    case ORC_FN_TORUS_MODE: {
      double phi, psi, dist;
      orc_torus_angles(P->p[0], y, &phi, &psi, &dist);
      double u = c[0] * sin(phi) * cos(2.0 * psi);
      return c[0] * orc_torus_neg_lap(P->p[0], P->p[1], phi, psi) + P->sigma * u;
    }
    case ORC_FN_TABLE_S1: {
      double th = atan2(y[1], y[0]);
      return orc_table_s1(P->f_values, P->f_nvalues / 2, th);
    }
    case ORC_FN_TORUS_SINE: {
      /* f = -Lap_T u + sigma u for the series u (Example 1's family) */
      double th, sv, rho;
      orc_ct_coords(P, y, &th, &sv, &rho);
      orc_ts_val v = orc_ts_eval(P->f_values, P->f_idx[0], P->f_idx[1], th, sv);
      return -orc_ct_lap(P->p[0], P->p[1], th, v) + P->sigma * v.u;
    }
  }
  return NAN;
}

/* Second-order compensation from a predictor u_* (Sec. "Approximation of the
 * compensation term"): with y = cp(x), x = y + eta n(y), eta the signed
 * distance along the outward tube normal (eta = rho - a),
 *   R_*(s; y) = -Lap(E u_*)(y + s n(y)) + sigma u_*(y) - f_Omega(y),
 *   m1 = (R_*(h) - R_*(-h)) / (2h),  m2 = (R_*(h) - 2 R_*(0) + R_*(-h)) / h^2,
 *   m_*(x) = eta m1 + eta^2 m2 / 2,  h = h_eta. */
static double orc_m_second_order(const orc_problem* P, const double* x, const double* y) {
  double th, sv, rho;
  orc_ct_coords(P, x, &th, &sv, &rho);
  double R = P->p[0], a = P->p[1], h = P->h_eta;
  orc_ts_val v = orc_ts_eval(P->pred_coef, P->pred_ks, P->pred_kt, th, sv);
  double base = P->sigma * v.u - orc_f_omega(P, y);
  double Rp = -orc_ct_lap(R, a + h, th, v) + base;
  double R0 = -orc_ct_lap(R, a, th, v) + base;
  double Rm = -orc_ct_lap(R, a - h, th, v) + base;
  double m1 = (Rp - Rm) / (2.0 * h);
  double m2 = (Rp - 2.0 * R0 + Rm) / (h * h);
  double eta = rho - a;
  return eta * m1 + 0.5 * eta * eta * m2;
}

/* Predictor fit: the discrete orthogonal projection of node values onto the
 * Fourier-sine series (discrete Fourier transform in th, discrete sine
 * transform in s).  Nodes th_i = 2 pi i / nt (i < nt), s_j = pi j / ns
 * (0 < j < ns; u vanishes at s = 0 and pi), U[i (ns - 1) + j - 1].  A series
 * with ks < ns and 2 kt < nt is reproduced exactly. */
int orc_ts_fit(const double* U, int nt, int ns, int kt, int ks, double* coef) {
  if (nt < 1 || ns < 2 || kt < 0 || ks < 1 || ks >= ns || 2 * kt >= nt) return ORC_EINVAL;
  int stride = 2 * kt + 1;
  for (int k = 1; k <= ks; ++k) {
    for (int c = 0; c < stride; ++c) {
      int j = (c + 1) / 2;
      double acc = 0.0;
      for (int i = 0; i < nt; ++i) {
        double th = 6.283185307179586 * (double)i / (double)nt;
        double wth = (c == 0) ? 1.0 : ((c & 1) ? cos(j * th) : sin(j * th));
        for (int jj = 1; jj < ns; ++jj) {
          double sv = 3.141592653589793 * (double)jj / (double)ns;
          acc += U[(size_t)i * (ns - 1) + (jj - 1)] * wth * sin(k * sv);
        }
      }
      double norm = (c == 0 ? 1.0 : 2.0) * 2.0 / ((double)nt * (double)ns);
      coef[(size_t)(k - 1) * stride + c] = acc * norm;
    }
  }
  return ORC_OK;
}

/* Value and derivatives of a Fourier-sine series, for tests:
 * out = (u, u_th, u_thth, u_ss). */
void orc_ts_value(const double* coef, int ks, int kt, double th, double s, double* out) {
  orc_ts_val v = orc_ts_eval(coef, ks, kt, th, s);
  out[0] = v.u; out[1] = v.ut; out[2] = v.utt; out[3] = v.uss;
}

/* Exact compensation m(x), y = cp(x). */
static double orc_m_exact(const orc_problem* P, const double* x, const double* y) {
  int n = P->n;
  const double* c = P->f_coef;
  double sg = P->sigma;
  switch (P->f_kind) {
    case ORC_FN_ZERO:
    case ORC_FN_CONST: return 0.0;
    case ORC_FN_SPH_PAIR:
    case ORC_FN_CIRCLE_MODE:
    case ORC_FN_LEGENDRE:
    case ORC_FN_TABLE_S1: {
      /* on S^{n-1}_R the degree-0 extension has Lap(Eu)(x) = (R/|x|)^2 Lap_S u,
       * so m(x) = (f - sigma u)(y) ((R/|x|)^2 - 1). */
      double R = P->p[0];
      double rr = orc_dot(x, x, n);
      double fac = R * R / rr - 1.0;
      double lap_part; /* (f - sigma u)(y) = -Lap_S u (y) */
      if (P->f_kind == ORC_FN_SPH_PAIR) {
        double lam = 2.0 * (double)n / (R * R);
        double f = orc_f_omega(P, y);
        lap_part = lam * f / (lam + sg);
      } else if (P->f_kind == ORC_FN_CIRCLE_MODE) {
        int k = P->f_idx[0];
        double lam = (double)(k * k) / (R * R);
        double f = orc_f_omega(P, y);
        lap_part = lam * f / (lam + sg);
      } else if (P->f_kind == ORC_FN_LEGENDRE) {
        double t = y[n - 1] / R;
        lap_part = 0.0;
        for (int l = 0; l < 8; ++l) {
          double lam = (double)(l * (l + 1)) / (R * R);
          lap_part += lam * c[l] / (lam + sg) * orc_legendre(l, t);
        }
      } else {
        double th = atan2(y[1], y[0]);
        int64_t M = P->f_nvalues / 2;
        double f = orc_table_s1(P->f_values, M, th);
        double us = orc_table_s1(P->f_values + M, M, th);
        lap_part = f - sg * us;
      }
      return lap_part * fac;
    }
    case ORC_FN_TORUS_MODE: {
      double phi, psi, dist;
      orc_torus_angles(P->p[0], x, &phi, &psi, &dist);
      return c[0] * (orc_torus_neg_lap(P->p[0], dist, phi, psi) - orc_torus_neg_lap(P->p[0], P->p[1], phi, psi));
    }
    case ORC_FN_TORUS_SINE: {
      /* m(x) = Lap_T u(y) - Lap(Eu)(x): the extension's Laplacian at rho
       * against the intrinsic one at rho = a */
      double th, sv, rho;
      orc_ct_coords(P, x, &th, &sv, &rho);
      orc_ts_val v = orc_ts_eval(P->f_values, P->f_idx[0], P->f_idx[1], th, sv);
      return orc_ct_lap(P->p[0], P->p[1], th, v) - orc_ct_lap(P->p[0], rho, th, v);
    }
  }
  return NAN;
}

/* Dirichlet datum g_Omega at a boundary point. */
static double orc_g_omega(const orc_problem* P, const double* y) {
  const double* c = P->g_coef;
  int n = P->n;
  switch (P->g_kind) {
    case ORC_FN_ZERO: return 0.0;
    case ORC_FN_CONST: return c[0];
    case ORC_FN_SPH_PAIR: {
      double R = P->p[0];
      return c[0] * (y[P->g_idx[0]] / R) * (y[P->g_idx[1]] / R);
    }
    case ORC_FN_LEGENDRE: {
      double t = y[n - 1] / P->p[0];
      double s = 0.0;
      for (int l = 0; l < 8; ++l) s += c[l] * orc_legendre(l, t);
      return s;
    }
  }
  return NAN;
}

/* Source term of one Green sample at ambient point z: f(z) + m(z).  On a
 * point cloud the projection of z starts from patch `start` (the walker's;
 * -1: from the cloud point nearest to z). */
static double orc_source_from(const orc_problem* P, const double* z, int64_t start) {
  double y[ORC_MAXN];
  if (P->manifold == ORC_DUMBBELL) {
    double phi;
    orc_db_cp(P, z, y, &phi);
    if (P->f_kind == ORC_FN_DUMBBELL_POLY) return orc_db_f(P, y, phi);
    return orc_f_omega(P, y);
  }
  if (P->manifold == ORC_PRODUCT) {
    double phi;
    if (orc_pr_cp(P, z, y, &phi)) return NAN;
    if (P->f_kind == ORC_FN_PRODUCT_MODES) return orc_pr_f(P, y, phi);
    return orc_f_omega(P, y);
  }
  if (P->manifold == ORC_POINT_CLOUD) {
    orc_pc_result pc;
    if (orc_pc_project_from(P, z, start, &pc)) return NAN;
    for (int i = 0; i < 3; ++i) y[i] = pc.y[i];
  } else if (orc_cp(P, z, y)) {
    return NAN;
  }
  double v = orc_f_omega(P, y);
  if (P->compensation == ORC_COMP_EXACT) v += orc_m_exact(P, z, y);
  else if (P->compensation == ORC_COMP_SECOND_ORDER) v += orc_m_second_order(P, z, y);
  return v;
}

double orc_source(const orc_problem* P, const double* z) { return orc_source_from(P, z, -1); }

/* ------------------------------------------------------------------------- */
/* Radius rule r(y) = theta min{delta_Gamma(y), rho_geo(y)}                   */
/* (eq. radius_rule_unified, eq. rho_geo_curvature, eq. rho_geo_spacing).     */
/* For point clouds rho_geo comes from the reconstruction that produced y.    */
/* ------------------------------------------------------------------------- */
static double orc_rho_geo(const orc_problem* P, const double* y, const orc_pc_result* pc) {
  /* a bound of kappa over M in eq. rho_geo_curvature: a radius no larger than
   * the local rule gives anywhere */
  if (P->radius_rule == ORC_RADIUS_CURVATURE_BOUND) return P->c_kappa / (1.0 + P->kappa_bound);
  if (P->manifold == ORC_POINT_CLOUD) {
    if (P->radius_rule == ORC_RADIUS_SPACING) return P->c_h * pc->h_mean;
    /* a bound of kappa over M in eq. rho_geo_curvature: a radius no larger
     * than the local rule gives anywhere */
    if (P->radius_rule == ORC_RADIUS_CURVATURE_BOUND) return P->c_kappa / (1.0 + P->kappa_bound);
    return P->c_kappa / (1.0 + pc->kappa);
  }
  return P->c_kappa / (1.0 + orc_kappa(P, y));
}

double orc_radius(const orc_problem* P, const double* y) {
  orc_pc_result pc;
  if (P->manifold == ORC_POINT_CLOUD) {
    if (orc_pc_project(P, y, &pc)) return NAN;
  }
  double rg = orc_rho_geo(P, y, &pc);
  double dg = orc_has_boundary(P) ? orc_bdry_delta(P, y) : INFINITY;
  return P->theta * (dg < rg ? dg : rg);
}

/* ------------------------------------------------------------------------- */
/* One path of Algorithm 1 and its score S (eq. path_score_definition).       */
/* ------------------------------------------------------------------------- */
typedef struct {
  const orc_problem* P;
  orc_radial rad;
  uint64_t seed;
} orc_ctx;

static void orc_sum_add(double* s, double* comp, double x) {
  /* Neumaier compensated summation */
  double t = *s + x;
  if (fabs(*s) >= fabs(x)) *comp += (*s - t) + x;
  else *comp += (x - t) + *s;
  *s = t;
}

static int orc_walk(const orc_ctx* C, const double* y0, uint32_t q, uint32_t w, double* S_out,
                    int32_t* K_out, int* truncated) {
  const orc_problem* P = C->P;
  int n = P->n;
  int boundary = orc_has_boundary(P);
  double* buf = (double*)malloc(sizeof(double) * 7 * (size_t)n);
  if (!buf) return ORC_ENOMEM;
  double *Y = buf, *Yn = buf + n, *Th = buf + 2 * n, *Z = buf + 3 * n, *g = buf + 4 * n, *yg = buf + 5 * n;
  double* ng = buf + 6 * n;
  memcpy(Y, y0, sizeof(double) * (size_t)n);
  double W = 1.0, S = 0.0, comp = 0.0;
  uint32_t k = 0;
  *truncated = 0;
  orc_pc_result pc_cur, pc_next;
  if (P->manifold == ORC_POINT_CLOUD) {
    /* a point-cloud query is an ambient point near the cloud: the walk
     * starts from its projection onto the reconstructed surface */
    if (orc_pc_project(P, Y, &pc_cur)) { free(buf); return ORC_EINVAL; }
    memcpy(Y, pc_cur.y, sizeof(double) * 3);
  }
  if (boundary && orc_in_layer(P, Y)) {
    orc_gamma_point(P, Y, yg, ng);
    *S_out = W * orc_g_omega(P, yg);
    *K_out = 0;
    free(buf);
    return ORC_OK;
  }
  for (;;) {
    /* (i) radius */
    double rg = orc_rho_geo(P, Y, &pc_cur);
    double dg = boundary ? orc_bdry_delta(P, Y) : INFINITY;
    double r = P->theta * (dg < rg ? dg : rg);
    double c = orc_c_sigma_r(n, P->sigma, r);
    double om = orc_omega(n, P->sigma, r);
    double X = sqrt(P->sigma) * r;
    if (!(X <= orc_radial_xmax(n))) { free(buf); return ORC_EINVAL; }
    /* (ii) projected state: Theta = Y + r zeta, zeta uniform on the unit
     * sphere (eq. projected_chain_update) */
    orc_direction(C->seed, q, w, k, 0, n, g);
    for (int i = 0; i < n; ++i) Th[i] = Y[i] + r * g[i];
    if (P->manifold == ORC_POINT_CLOUD) {
      if (orc_pc_project_from(P, Th, pc_cur.patch, &pc_next)) { free(buf); return ORC_EINVAL; }
      for (int i = 0; i < 3; ++i) Yn[i] = pc_next.y[i];
    } else if (orc_cp(P, Th, Yn)) {
      free(buf);
      return ORC_EINVAL;
    }
    /* Green samples Z ~ rho(Y, .) (eq. Z_sampling_density), averaged over N_V
     * (eq. local_average_source) */
    double F = 0.0;
    for (int l = 1; l <= P->n_v; ++l) {
      double u = orc_radius_uniform(C->seed, q, w, k, (uint32_t)l, n);
      double s = orc_radial_inv_r(&C->rad, X, u);
      orc_direction(C->seed, q, w, k, (uint32_t)l, n, g);
      for (int i = 0; i < n; ++i) Z[i] = Y[i] + (r * s) * g[i];
      F += orc_source_from(P, Z, P->manifold == ORC_POINT_CLOUD ? pc_cur.patch : -1);
    }
    F = F / (double)P->n_v;
    orc_sum_add(&S, &comp, (W * om) * F);
    W = W * c;
    memcpy(Y, Yn, sizeof(double) * (size_t)n);
    if (P->manifold == ORC_POINT_CLOUD) pc_cur = pc_next;
    k += 1;
    if (boundary && orc_in_layer(P, Y)) {
      orc_gamma_point(P, Y, yg, ng);
      orc_sum_add(&S, &comp, W * orc_g_omega(P, yg));
      break;
    }
    if (!boundary && !(W >= P->tau_w)) break;
    if ((int64_t)k >= P->max_steps) { *truncated = 1; break; }
  }
  *S_out = S + comp;
  *K_out = (int32_t)k;
  free(buf);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Solve: every walk of every query, then the Monte Carlo estimator           */
/* u ~ N^-1 sum_i S^i (eq. mc_estimator) and its standard error.              */
/* ------------------------------------------------------------------------- */
typedef struct {
  const orc_ctx* C;
  const double* queries;
  int64_t nq, nw;
  double* walk_S;
  int32_t* walk_K;
  int64_t next;
  pthread_mutex_t lock;
  int status;
  int64_t truncated;
} orc_job;

static void* orc_worker(void* arg) {
  orc_job* J = (orc_job*)arg;
  int n = J->C->P->n;
  int64_t total = J->nq * J->nw;
  for (;;) {
    int64_t start = __atomic_fetch_add(&J->next, 64, __ATOMIC_RELAXED);
    if (start >= total) break;
    int64_t end = start + 64 < total ? start + 64 : total;
    for (int64_t i = start; i < end; ++i) {
      int64_t q = i / J->nw, w = i % J->nw;
      int trunc = 0;
      int st = orc_walk(J->C, J->queries + q * n, (uint32_t)q, (uint32_t)w, &J->walk_S[i], &J->walk_K[i], &trunc);
      if (st || trunc) {
        pthread_mutex_lock(&J->lock);
        if (st) J->status = st;
        if (trunc) J->truncated += 1;
        pthread_mutex_unlock(&J->lock);
      }
    }
  }
  return NULL;
}

static int orc_check(const orc_problem* P) {
  if (P->n < 2 || P->n > ORC_MAXN) return ORC_EINVAL;
  if (!(P->sigma > 0.0) || !isfinite(P->sigma)) return ORC_EINVAL;
  if (!(P->theta > 0.0 && P->theta < 1.0)) return ORC_EINVAL;
  if (!(P->c_kappa > 0.0)) return ORC_EINVAL;
  if (P->n_v < 1 || P->n_v > 255) return ORC_EINVAL;
  if (P->max_steps < 1) return ORC_EINVAL;
  if (orc_has_boundary(P)) {
    if (!(P->eps > 0.0)) return ORC_EINVAL;
    if (P->manifold == ORC_SPHERE_CAP && !(fabs(P->p[1]) < P->p[0])) return ORC_EINVAL;
  } else {
    if (!(P->tau_w > 0.0 && P->tau_w < 1.0)) return ORC_EINVAL;
  }
  if ((P->manifold == ORC_TORUS || P->manifold == ORC_CUT_TORUS || P->manifold == ORC_POINT_CLOUD) && P->n != 3)
    return ORC_EINVAL;
  if (P->manifold == ORC_CUT_TORUS) {
    if (!(P->p[1] > 0.0 && P->p[1] < P->p[0]) || !isfinite(P->p[2])) return ORC_EINVAL;
    if (P->radius_rule != ORC_RADIUS_CURVATURE) return ORC_EINVAL;
    if (P->f_kind != ORC_FN_ZERO && P->f_kind != ORC_FN_CONST && P->f_kind != ORC_FN_TORUS_SINE) return ORC_EINVAL;
    if (P->g_kind != ORC_FN_ZERO && P->g_kind != ORC_FN_CONST) return ORC_EINVAL;
    if (P->f_kind == ORC_FN_TORUS_SINE &&
        (!P->f_values || P->f_idx[0] < 1 || P->f_idx[1] < 0 ||
         P->f_nvalues != (int64_t)P->f_idx[0] * (2 * P->f_idx[1] + 1)))
      return ORC_EINVAL;
    if (P->compensation == ORC_COMP_SECOND_ORDER &&
        (P->f_kind != ORC_FN_TORUS_SINE || !P->pred_coef || P->pred_ks < 1 || P->pred_kt < 0 ||
         !(P->h_eta > 0.0 && P->h_eta < 0.5 * P->p[1])))
      return ORC_EINVAL;
  } else if (P->f_kind == ORC_FN_TORUS_SINE || P->compensation == ORC_COMP_SECOND_ORDER) {
    return ORC_EINVAL;
  }
  if (P->manifold == ORC_POINT_CLOUD && (P->k_nn < 6 || P->k_nn > ORC_MAXK || P->n_points < P->k_nn))
    return ORC_EINVAL;
  if (P->manifold == ORC_POINT_CLOUD && !(P->fit_scale >= 0.0 && P->fit_scale <= 16.0)) return ORC_EINVAL;
  /* the nearest point carries no curvature: its radius comes from the spacing or a bound */
  if (P->manifold == ORC_POINT_CLOUD && P->reconstruction == 1 && P->radius_rule != ORC_RADIUS_SPACING &&
      P->radius_rule != ORC_RADIUS_CURVATURE_BOUND)
    return ORC_EINVAL;
  if (P->radius_rule == ORC_RADIUS_CURVATURE_BOUND &&
      ((P->manifold != ORC_POINT_CLOUD && P->manifold != ORC_DUMBBELL) || !(P->kappa_bound >= 0.0) ||
       !isfinite(P->kappa_bound)))
    return ORC_EINVAL;
  if (P->manifold == ORC_DUMBBELL) {
    /* closed; the radius takes a curvature bound; no exact compensation is
     * known for this manifold (the paper sets m = 0 here) */
    if (P->n < 3 || P->radius_rule != ORC_RADIUS_CURVATURE_BOUND || P->compensation != ORC_COMP_NONE)
      return ORC_EINVAL;
    if (!(P->p[0] >= 0.0 && P->p[0] < 0.5) || !(P->p[1] > 0.0)) return ORC_EINVAL;
    if (P->f_kind != ORC_FN_ZERO && P->f_kind != ORC_FN_CONST && P->f_kind != ORC_FN_DUMBBELL_POLY)
      return ORC_EINVAL;
    if (P->f_kind == ORC_FN_DUMBBELL_POLY && (!P->f_values || P->f_nvalues != P->n - 1)) return ORC_EINVAL;
  } else if (P->f_kind == ORC_FN_DUMBBELL_POLY) {
    return ORC_EINVAL;
  }
  if (P->manifold == ORC_PRODUCT) {
    /* R^9; no exact compensation is known here (the paper sets m = 0) */
    if (P->n != 9 || P->compensation != ORC_COMP_NONE || P->radius_rule != ORC_RADIUS_CURVATURE) return ORC_EINVAL;
    if (!(P->p[0] > 0.0) || !(P->p[1] > 0.0)) return ORC_EINVAL;
    if (P->f_kind != ORC_FN_ZERO && P->f_kind != ORC_FN_CONST && P->f_kind != ORC_FN_PRODUCT_MODES)
      return ORC_EINVAL;
  } else if (P->f_kind == ORC_FN_PRODUCT_MODES) {
    return ORC_EINVAL;
  }
  return ORC_OK;
}

/* Largest X = sqrt(sigma) r the solve can reach (constant radius bound). */
static double orc_max_radius(const orc_problem* P) {
  if (P->radius_rule == ORC_RADIUS_CURVATURE_BOUND) return P->theta * P->c_kappa / (1.0 + P->kappa_bound);
  if (P->manifold == ORC_POINT_CLOUD) {
    if (P->radius_rule == ORC_RADIUS_SPACING) return INFINITY;
    if (P->radius_rule == ORC_RADIUS_CURVATURE_BOUND) return P->theta * P->c_kappa / (1.0 + P->kappa_bound);
    return P->theta * P->c_kappa;
  }
  double kmin = 1.0 / P->p[0];
  if (P->manifold == ORC_TORUS || P->manifold == ORC_CUT_TORUS) kmin = 1.0 / P->p[1];
  if (P->manifold == ORC_PRODUCT) kmin = orc_kappa(P, NULL);
  return P->theta * P->c_kappa / (1.0 + kmin);
}

int orc_solve(const orc_problem* P, const double* queries, int64_t nq, int64_t nw, uint64_t seed,
              int n_threads, double* walk_S, int32_t* walk_K, double* u_out, double* stderr_out,
              int64_t* n_truncated) {
  int st = orc_check(P);
  if (st) return st;
  if (nq < 1 || nw < 1 || nq > 0xFFFFFFFFll || nw > 0xFFFFFFFFll) return ORC_EINVAL;
  {
    double rmax = orc_max_radius(P);
    if (isfinite(rmax) && sqrt(P->sigma) * rmax > orc_radial_xmax(P->n)) return ORC_EINVAL;
  }
  int n = P->n;
  /* every query must lie on M */
  double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
  if (!tmp) return ORC_ENOMEM;
  for (int64_t q = 0; q < nq; ++q) {
    const double* y = queries + q * n;
    double tol;
    if (P->manifold == ORC_POINT_CLOUD) {
      /* within two local spacings of the reconstructed surface */
      orc_pc_result pc;
      if (orc_pc_project(P, y, &pc)) { free(tmp); return ORC_EOFFMANIFOLD; }
      for (int i = 0; i < 3; ++i) tmp[i] = pc.y[i];
      tol = 2.0 * pc.h_mean;
    } else {
      if (orc_cp(P, y, tmp)) { free(tmp); return ORC_EOFFMANIFOLD; }
      double sc = 0.0;
      for (int i = 0; i < n; ++i) sc += y[i] * y[i];
      tol = 1e-9 * (1.0 + sqrt(sc));
    }
    double d2 = 0.0;
    for (int i = 0; i < n; ++i) d2 += (tmp[i] - y[i]) * (tmp[i] - y[i]);
    if (!(sqrt(d2) <= tol)) { free(tmp); return ORC_EOFFMANIFOLD; }
  }
  free(tmp);
  orc_ctx C;
  C.P = P;
  C.seed = seed;
  orc_radial_init(&C.rad, n);
  orc_job J;
  J.C = &C; J.queries = queries; J.nq = nq; J.nw = nw;
  J.walk_S = walk_S; J.walk_K = walk_K; J.next = 0; J.status = ORC_OK; J.truncated = 0;
  pthread_mutex_init(&J.lock, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, orc_worker, &J);
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J.lock);
  if (J.status) return J.status;
  for (int64_t q = 0; q < nq; ++q) {
    double s = 0.0, comp = 0.0;
    for (int64_t w = 0; w < nw; ++w) orc_sum_add(&s, &comp, walk_S[q * nw + w]);
    double mean = (s + comp) / (double)nw;
    double v = 0.0;
    for (int64_t w = 0; w < nw; ++w) { double d = walk_S[q * nw + w] - mean; v += d * d; }
    if (u_out) u_out[q] = mean;
    if (stderr_out) stderr_out[q] = nw > 1 ? sqrt(v / (double)(nw - 1) / (double)nw) : 0.0;
  }
  if (n_truncated) *n_truncated = J.truncated;
  return J.truncated ? ORC_WTRUNC : ORC_OK;
}

/* One walk, for tests. */
int orc_walk_one(const orc_problem* P, const double* y0, uint32_t q, uint32_t w, uint64_t seed,
                 double* S_out, int32_t* K_out, int* truncated) {
  int st = orc_check(P);
  if (st) return st;
  orc_ctx C;
  C.P = P;
  C.seed = seed;
  orc_radial_init(&C.rad, P->n);
  return orc_walk(&C, y0, q, w, S_out, K_out, truncated);
}
