/*
 * mpwos.h -- C ABI of the MI355X (gfx950) MPWoS solver.
 *
 * MPWoS (modified projected Walk on Spheres) estimates the solution of the
 * screened Poisson equation
 *      -Lap_Omega u + sigma u = f  on Omega, a patch of an embedded manifold
 *                                  M of R^n                 (Sec. 2.1, eq. surface_pde)
 *      u = g on Gamma = dOmega when Omega has a boundary     (eq. surface_bc)
 * at query points of Omega, from independent random walks in the ambient
 * R^n (Algorithm 1): each step picks the radius r(Y) = theta min(delta_Gamma,
 * rho_geo) (eq. radius_rule_unified), samples a point Theta uniformly on the
 * sphere of radius r around Y and projects it back, Y' = cp(Theta)
 * (eq. projected_chain_update), draws N_V points Z from the normalised Green
 * density of the ball (eq. Z_sampling_density), accumulates
 * W omega(Y) (f + m)(Z) (eq. path_score_definition, eq. local_average_source)
 * and multiplies the screening weight W by c_{sigma,r} (eq. def_c_sigma_r).
 * A walk stops in the eps-shell of the boundary (eq. boundary_layer) or,
 * on a closed manifold, once W < tau_W.  The estimate is the mean score
 * (eq. mc_estimator).
 *
 * Conventions for every entry point:
 *   - Every call returns an mpwos_status; no exception crosses the ABI.
 *   - On failure nothing is written to the outputs, and mpwos_last_error()
 *     returns a message for the calling thread.
 *   - Arrays are row-major.  Pointers named "queries", "u_out" and
 *     "stderr_out" are host pointers unless opt->device_io is 1, in which
 *     case all three (and walk_S / walk_K) are device pointers.
 *   - The library never frees caller memory; caller buffers must stay valid
 *     until the call (or, for a served request, the request) completes.
 *   - Calls are synchronous on opt->stream (a hipStream_t, NULL = the
 *     library's own stream) unless stated otherwise.
 */
#ifndef MPWOS_H
#define MPWOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPWOS_OK = 0,
  MPWOS_EINVAL = -1,        /* an argument is outside the documented domain */
  MPWOS_EOFFMANIFOLD = -2,  /* a query is not on M (|cp(y) - y| > 1e-9 (1 + |y|)) */
  MPWOS_ENOMEM = -3,        /* device or host allocation, or the HBM budget, failed */
  MPWOS_EDEVICE = -4,       /* a HIP runtime error; the message names the call */
  MPWOS_EBUSY = -5,         /* a resource is still referenced (manifold in use, server full) */
  MPWOS_WTRUNC = 1          /* warning: some walks reached max_steps and were cut there */
} mpwos_status;

/* Manifold kinds (Sec. 2.1: parameterised, implicit and point-cloud forms). */
typedef enum {
  MPWOS_SPHERE = 0,          /* S^{n-1}_R, closed; cp(x) = R x/|x| (explicit projection) */
  MPWOS_SPHERE_CAP = 1,      /* Omega = S^{n-1}_R cap {x_n > h}, Gamma = {x_n = h} (boundary case) */
  MPWOS_TORUS_IMPLICIT = 2,  /* {((|x|^2 + R^2 - a^2)^2 - 4R^2(x1^2 + x2^2)) = 0} in R^3; cp by a
                                local Newton solve on the level set (Sec. 2.3.2) */
  MPWOS_POINT_CLOUD = 3,     /* points p_i in R^3; cp by k-nearest-neighbour search and a local
                                quadratic reconstruction (Sec. 2.3.2) */
  MPWOS_DUMBBELL = 4,        /* implicit dumbbell of Sec. 4, Example 2: {|x_h| = R(x_n)} in R^n,
                                x_h = (x_1 .. x_{n-1}), R(s) = sqrt(1 - (s/k)^2)(1 - a + 2a (s/k)^2),
                                a = p[0] in [0, 1/2), k = p[1] > 0; closed; cp by Newton in the
                                profile parameter; n in [4, 4096]; takes the CURVATURE_BOUND rule
                                (kappa_bound >= its largest principal curvature) and no
                                compensation */
  MPWOS_PRODUCT = 5,         /* product manifold of Sec. 4, Example 3: S^1_Fourier(R) x S^2(a) in R^9,
                                X(phi, w) = (R C(phi), a w), C = (cos phi, sin phi, cos 2phi/2,
                                sin 2phi/2, cos 3phi/3, sin 3phi/3); R = p[0], a = p[1]; n = 9;
                                cp by Newton on the curve and normalisation; curvature indicator
                                max(sqrt(14)/(3R), 1/a); no compensation */
  MPWOS_CUT_TORUS = 6        /* torus with a planar cut of Sec. 4, Example 1: the torus of radii
                                R = p[0], a = p[1] (0 < a <= R/2) cut by the plane through its axis at
                                angle phi_c = p[2]; Omega = {0 < phi - phi_c < pi} (phi the angle about
                                the x_3 axis), Gamma the two tube circles of the cut (boundary case;
                                delta_Gamma of eq. delta_Gamma_general with ell = rho_geo); n = 3 */
} mpwos_kind;

/* Source and boundary-data families.  For f the family describes f_Omega;
 * for g it describes g_Omega on Gamma.  Families whose solution u is known
 * in closed form also give the exact compensation m (eq. mismatch_definition). */
typedef enum {
  MPWOS_FN_ZERO = 0,         /* 0 */
  MPWOS_FN_CONST = 1,        /* coef[0] */
  MPWOS_FN_SPH_PAIR = 2,     /* S^{n-1}_R: coef[0] (y_i/R)(y_j/R), i = idx[0] != j = idx[1];
                                eigenvalue 2n/R^2, so u = f/(2n/R^2 + sigma) */
  MPWOS_FN_CIRCLE_MODE = 3,  /* S^1_R: coef[0] cos(k th) + coef[1] sin(k th), k = idx[0] */
  MPWOS_FN_LEGENDRE = 4,     /* S^2_R, or a point cloud of it (R = p[0]): sum_{l<8} coef[l] P_l(y_3/R) */
  MPWOS_FN_TORUS_MODE = 5,   /* torus / point-cloud torus (R = p[0], a = p[1]):
                                u = coef[0] sin(phi) cos(2 psi), f = -Lap_T u + sigma u;
                                as g: g = u */
  MPWOS_FN_TABLE_S1 = 6,     /* S^1_R, f: values[0..M) = f at th_i = 2 pi i/M (linear
                                interpolation), values[M..2M) = predictor u_* used by
                                the compensation; n_values = 2M (host memory) */
  MPWOS_FN_DUMBBELL_POLY = 7, /* dumbbell, f: u = coef[0] x_n + coef[1] x_n^2 + coef[2] (sum x_h)/sqrt(n-1)
                                + coef[3] sum_i values[i] x_i^2 (n_values = n - 1, host memory),
                                f = -Lap_M u + sigma u (Example 2's family; A = diag(values)) */
  MPWOS_FN_PRODUCT_MODES = 8, /* product manifold, f: u = coef[0] cos(phi) w1 + coef[1] sin(2 phi) w2
                                + coef[2] cos(3 phi) (w1^2 - w2^2), f = -Lap_M u + sigma u
                                (Example 3's family) */
  MPWOS_FN_TORUS_SINE = 9    /* cut torus, f: u(th, s) = sum_{k=1..K} sin(k s) T_k(th), s = phi - phi_c,
                                th the tube angle, T_k(th) = c_k0 + sum_{j=1..J} (c_kj cos j th +
                                d_kj sin j th); K = idx[0] in [1, 64], J = idx[1] in [0, 64]; values
                                holds the rows (c_k0, c_k1, d_k1, .., c_kJ, d_kJ), k = 1..K (host
                                memory); f = -Lap_T u + sigma u (Example 1's family; u = 0 on Gamma).
                                With COMP_SECOND_ORDER the predictor u_* follows as idx[2] >= 1 more
                                rows of the same width, and coef[0] = h_eta in (0, a/2) is the normal
                                difference step; n_values = (idx[0] + idx[2]) (2 idx[1] + 1) */
} mpwos_fn_kind;

/* FP64_PLAIN: every operation of the walk in FP64 (the oracle's arithmetic).
 * FP32_MIXED: uniforms, normals, direction, projection (except the implicit
 * torus), radial inverse (table), source and the step factors c and omega of
 * a per-step radius in FP32; the path weight W, the score and the per-query
 * sums in FP64. */
typedef enum { MPWOS_FP64_PLAIN = 0, MPWOS_FP32_MIXED = 1 } mpwos_precision;
/* Compensation m (eq. mismatch_definition) added to the source of each Green sample:
 *   NONE: m_* = 0 (the baseline variant);
 *   EXACT: m from the family's closed-form u;
 *   SECOND_ORDER: m_*(x) = eta m1(cp x) + eta^2 m2(cp x) / 2 from a predictor u_* (the
 *     subsection on approximating the compensation term): R_*(s; y) = -Lap(E u_*)(y + s n(y))
 *     + sigma u_*(y) - f_Omega(y), m1 and m2 its central differences at s = 0, +-h_eta, eta the
 *     signed normal distance of x; TORUS_SINE on CUT_TORUS only (see mpwos_predictor_fit). */
typedef enum { MPWOS_COMP_NONE = 0, MPWOS_COMP_EXACT = 1, MPWOS_COMP_SECOND_ORDER = 2 } mpwos_compensation;
typedef enum {
  MPWOS_RADIUS_CURVATURE = 0,     /* rho_geo = c_kappa/(1 + kappa(y)) (eq. rho_geo_curvature) */
  MPWOS_RADIUS_SPACING = 1,       /* rho_geo = c_h h(y), h = mean kNN distance (eq. rho_geo_spacing) */
  MPWOS_RADIUS_CURVATURE_FIT = 2, /* point cloud: kappa from the fitted patch, then eq. rho_geo_curvature */
  MPWOS_RADIUS_CURVATURE_BOUND = 3 /* point cloud, dumbbell: eq. rho_geo_curvature with a bound kappa_bound of
                                      kappa over M (a constant radius no larger than the local rule's) */
} mpwos_radius_rule;

typedef struct mpwos_manifold mpwos_manifold;

typedef struct {
  int32_t kind;             /* mpwos_kind */
  int32_t n;                /* ambient dimension: >= 2; 3 for torus and point cloud; <= 4096 */
  double p[4];              /* SPHERE: R; SPHERE_CAP: R, h (|h| < R); TORUS / POINT_CLOUD: R, a
                               (the torus the source families refer to) */
  const float* points;      /* POINT_CLOUD: n_points x 3 FP32 */
  int64_t n_points;         /* POINT_CLOUD: k_nn .. 2^27 */
  int32_t k_nn;             /* POINT_CLOUD: neighbours of the local fit and the spacing, 6..32 (default 16) */
  int32_t points_on_device; /* 1: `points` is a device pointer */
  int32_t reconstruction;   /* POINT_CLOUD: 0 = local quadratic patch of the k_nn points (default);
                               1 = the nearest cloud point itself (the pure nearest-neighbour
                               projection of Sec. 4, Example 4), with rho_geo from the spacing or a
                               curvature bound */
  double fit_scale;         /* POINT_CLOUD, patch: the patch of a cloud point p is fitted to the cloud
                               points within fit_scale r_k of p, r_k the distance to its k_nn-th nearest
                               point; 0 or 1 = the k_nn nearest points themselves (default); at most 16.
                               A wider fit resolves the curvature of a noisy cloud whose k_nn-point
                               patches span the noise level */
} mpwos_manifold_desc;

typedef struct {
  int32_t kind;             /* mpwos_fn_kind */
  int32_t idx[3];
  double coef[8];
  const double* values;     /* TABLE_S1 and DUMBBELL_POLY only, host memory, copied at solve time */
  int64_t n_values;
} mpwos_fn;

typedef struct {
  double theta;             /* safety factor, 0 < theta < 1 (default 0.95) */
  double c_kappa;           /* > 0 (default 1.2) */
  double c_h;               /* > 0 (default 2.4) */
  double tau_w;             /* closed manifolds: stop when W < tau_w, 0 < tau_w < 1 (default 1e-8) */
  int32_t n_v;              /* Green samples per step, 1..255 (default 1) */
  int32_t precision;        /* mpwos_precision (default FP64_PLAIN) */
  int32_t compensation;     /* mpwos_compensation (default EXACT) */
  int32_t radius_rule;      /* mpwos_radius_rule (default CURVATURE); SPACING, CURVATURE_FIT and
                               CURVATURE_BOUND apply to POINT_CLOUD only, where CURVATURE means
                               CURVATURE_FIT */
  int64_t max_steps;        /* per-walk step cap, >= 1 (default 1e7); hitting it -> MPWOS_WTRUNC */
  void* stream;             /* hipStream_t or NULL */
  int32_t device_io;        /* 1: queries / outputs / walk_S / walk_K are device pointers */
  int32_t block_size;       /* threads per workgroup, 0 = default (256; 128 on a POINT_CLOUD);
                               else 64, 128, 192 or 256 (at most 128 on a POINT_CLOUD) */
  int32_t lanes_per_walk;   /* 0 = default; 1 for n <= 3; else 8, 16, 32 or 64 */
  int32_t persistent;       /* 1: persistent kernel refilling lanes from a global queue;
                               0: plain launch, one walk per lane (or per lane group) */
  int32_t newton_iters;     /* point-cloud foot-point Newton iterations (default 6) */
  int32_t k_spacing;        /* reserved (spacing rule uses k_nn neighbours) */
  double* walk_S;           /* optional, n_queries x n_walks: per-walk score S^i */
  int32_t* walk_K;          /* optional, n_queries x n_walks: per-walk stopping index K^i */
  double kappa_bound;       /* CURVATURE_BOUND: finite, >= 0 (default 0) */
} mpwos_options;

typedef struct {
  int64_t walk_steps;       /* total walk-steps (sum of K^i) */
  int64_t truncated;        /* walks cut at max_steps */
  int32_t k_max;            /* largest K^i */
  double k_mean;            /* mean K^i */
  double seconds;           /* wall time of the call */
  double kernel_ms;         /* device time of the walk kernel(s), HIP events on the solve stream */
  double reduce_ms;         /* device time of the per-query reduction */
  int32_t k_p50;            /* median K^i (nearest rank); exact below 2048 steps, */
  int32_t k_p99;            /* 99th percentile    above within 1/128 (rounded down) */
} mpwos_stats;

/* Fills `opt` with the defaults listed above. */
void mpwos_options_default(mpwos_options* opt);

/* Creates an immutable manifold (Sec. 2.1).  For POINT_CLOUD (Sec. 2.3.2) the
 * points are copied to the device once and the reconstruction is built there
 * and kept resident until mpwos_manifold_destroy: the k nearest cloud points
 * of every cloud point (grid tiles with BF16 MFMA distance estimates and an
 * exact FP64 re-rank; a KD-tree search where the tile result cannot be shown
 * exact), each point's local quadratic patch, and a KD-tree for the
 * nearest-point queries of the walk.  EINVAL for a bad descriptor or a
 * non-finite coordinate. */
mpwos_status mpwos_manifold_create(const mpwos_manifold_desc* desc, mpwos_manifold** out);

/* Releases a manifold.  EBUSY while a served request still references it. */
mpwos_status mpwos_manifold_destroy(mpwos_manifold* m);

/* Solves at n_queries points of M (Algorithm 1, eq. mc_estimator).
 *   f, g: source and boundary data; g must be NULL exactly when M is closed.
 *   c: the screening constant sigma > 0 of eq. surface_pde.
 *   queries: n_queries x n doubles, each on M (within 1e-9 (1 + |q|)); on a
 *            POINT_CLOUD each within two local spacings of the reconstructed
 *            surface, and the walk starts from its projection cp_h(q), the
 *            point the estimate refers to.  EOFFMANIFOLD otherwise.  Device
 *            queries (opt->device_io) on SPHERE, SPHERE_CAP, TORUS_IMPLICIT
 *            and CUT_TORUS are checked on the device beside the walks:
 *            EOFFMANIFOLD then comes after them, with u_out and stderr_out
 *            left unwritten.
 *   n_walks: paths per query, >= 1.
 *   eps: boundary-layer width (eq. boundary_layer), > 0 on SPHERE_CAP, ignored when closed.
 *   seed: key of the Philox4x32-10 stream; walk w of query q at step k draws
 *         counter (q, w, k, sub << 24 | block), sub 0 = sphere direction,
 *         sub l = Green sample l.
 *   opt: NULL = defaults.
 *   u_out: n_queries estimates; stderr_out (nullable): their standard errors.
 *   stats (nullable).
 * The result depends only on the arguments (not on the stream, timing or
 * other work on the device), for a fixed precision and lanes_per_walk. */
mpwos_status mpwos_solve(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g,
                         double c, const double* queries, int64_t n_queries, int64_t n_walks,
                         double eps, uint64_t seed, const mpwos_options* opt, double* u_out,
                         double* stderr_out, mpwos_stats* stats);

/* ---- allocation-free solve ----------------------------------------------
 * For callers that cannot allocate device memory: tight serving loops and
 * harnesses that forbid hipMalloc (it synchronises on the stream, so it is
 * not for graph capture; mpwos_plan_* is).  The same solve as mpwos_solve
 * with device_io = 1, on the same kernels and with the same results bit for
 * bit, except that everything mpwos_solve would allocate lives in one fixed
 * device array of MPWOS_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends: statistics and queue words, the source's values, one
 * inverse radial table (a table another solve already cached is used from
 * the cache), and the per-walk scores of a batch of queries (12 bytes per
 * walk; queries are processed in batches that fit).
 *   queries, u_out, stderr_out (nullable), opt->walk_S / walk_K (optional,
 *   both or neither, n_queries x n_walks): device pointers, whatever
 *   opt->device_io says.  The manifold must live on the current device.
 * Limits (EINVAL beyond them): n_walks <= (MPWOS_NOALLOC_SCRATCH_BYTES -
 * 1 MiB - 8) / 12 per query (5 505 023); at most 32768 source values;
 * the radial table of 17 slices.
 * Calls on one GPU share its array, which keeps the last call's contents:
 * calls that overlap on one GPU (from several threads, or on several
 * streams) race and must be serialised by the caller.
 * stats->kernel_ms and reduce_ms are 0 (no timing events). */
#define MPWOS_NOALLOC_SCRATCH_BYTES (64u << 20)
mpwos_status mpwos_solve_noalloc(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g,
                                 double c, const double* queries, int64_t n_queries, int64_t n_walks,
                                 double eps, uint64_t seed, const mpwos_options* opt, double* u_out,
                                 double* stderr_out, mpwos_stats* stats);

/* Message of the last failed call on this thread ("" if none). */
const char* mpwos_last_error(void);

/* Coarse predictor u_* for COMP_SECOND_ORDER on a CUT_TORUS (the subsection on
 * approximating the compensation term, where u_* comes from a coarse Monte
 * Carlo solve): the baseline solve (compensation forced to NONE, the other
 * options as given) with n_walks paths at the nt x (ns - 1) interior nodes of
 * the grid th_i = 2 pi i / nt, s_j = pi j / ns (0 < j < ns), then the discrete
 * orthogonal projection of the node estimates onto the Fourier-sine series of
 * MPWOS_FN_TORUS_SINE with ks rows of 2 kt + 1 coefficients (DFT in th, DST
 * in s; exact for a series with ks < ns and 2 kt < nt).  Every step runs on
 * the device.
 *   f, g, c, eps, seed, opt: as for mpwos_solve (opt->device_io is ignored).
 *   nt >= 1, ns >= 2, 1 <= ks < ns, 0 <= kt, 2 kt < nt, ks and kt <= 64;
 *   nt (ns - 1) <= 2^20.
 *   coef_out: ks (2 kt + 1) doubles (host), the rows (c_k0, c_k1, d_k1, ...).
 *   stats (nullable): the baseline solve's statistics.
 * EINVAL for another manifold or an out-of-range grid. */
mpwos_status mpwos_predictor_fit(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g, double c,
                                 double eps, uint64_t seed, const mpwos_options* opt, int32_t nt, int32_t ns,
                                 int64_t n_walks, int32_t ks, int32_t kt, double* coef_out, mpwos_stats* stats);

/* ---- graph-captured solves -----------------------------------------------
 * A plan captures the device work of one solve shape (manifold, f, g, c,
 * n_queries, n_walks, eps, options) in a HIP graph once; each execute then
 * replays it for new device-resident queries and a new seed with a handful of
 * launches.  Results equal mpwos_solve's for the same arguments bit for bit.
 * The plan owns n_queries x n_walks x 12 bytes of per-walk scores plus the
 * queries and estimates, and holds a reference to the manifold. */
typedef struct mpwos_plan mpwos_plan;

/* Validates like mpwos_solve (except the queries, which execute takes) and
 * captures the graph.  opt->stream, device_io and walk_S / walk_K are
 * ignored.  EINVAL above 2^30 walks. */
mpwos_status mpwos_plan_create(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g, double c,
                               int64_t n_queries, int64_t n_walks, double eps, const mpwos_options* opt,
                               mpwos_plan** out);

/* Enqueues one solve on `stream` (a hipStream_t; NULL = the plan's own
 * stream): copies the device array `queries` (n_queries x n, each on M: not
 * checked here) into the plan, replays the graph with `seed`, and copies the
 * estimates to the device arrays u_out and stderr_out (nullable).
 * Asynchronous; executes of one plan must not overlap (use one stream). */
mpwos_status mpwos_plan_execute(mpwos_plan* p, const double* queries, double* u_out, double* stderr_out,
                                uint64_t seed, void* stream);

/* Waits for `stream` and reports the last execute's walk counts (walk_steps,
 * truncated, k_max, k_mean; times are not measured here).  WTRUNC when walks
 * were cut at max_steps. */
mpwos_status mpwos_plan_stats(mpwos_plan* p, void* stream, mpwos_stats* stats);

/* Waits for the plan's own stream and frees the plan. */
mpwos_status mpwos_plan_destroy(mpwos_plan* p);

/* ---- launch autotuner ----------------------------------------------------
 * Times the launch shapes of a solve on a sample of it (up to 2^24 walks;
 * with a constant radius, walks of equal length cut to a step count that keeps
 * a trial to a fraction of a second, otherwise fewer walks) and returns the
 * fastest options: block_size and persistent for n <= 3, also lanes_per_walk
 * for n >= 4.  Other fields are copied from opt.  Walk results do not depend
 * on block_size or persistent; for n >= 4 they depend on lanes_per_walk
 * through the order of the lane-group sums, so a caller that needs
 * reproducible bits keeps the returned options.  best_ms (nullable): kernel
 * time of the best trial. */
mpwos_status mpwos_autotune(const mpwos_manifold* manifold, const mpwos_fn* f, const mpwos_fn* g, double c,
                            const double* queries, int64_t n_queries, int64_t n_walks, double eps,
                            const mpwos_options* opt, mpwos_options* best, double* best_ms);

/* ---- serving: continuous batching of solves (one device) ----------------
 * Requests are admitted in arrival order against an HBM budget.  Admitted
 * requests that run the same kernel on the same problem data (manifold, f,
 * g, c, eps, options; queries, n_walks and seed may differ) form a class, and
 * one launch carries walks of every request of a class, each with its own
 * queries, seed and outputs.  A fixed number of launches is in flight (two
 * per stream on four streams); whenever one completes its slot takes the next
 * class round-robin, so a request that arrives while others run joins the
 * next launch of its class.  A request's result is identical to the same
 * solve run alone. */
typedef struct mpwos_server mpwos_server;

typedef struct {
  const mpwos_manifold* manifold;
  mpwos_fn f, g;
  int32_t has_g;              /* 1 when the manifold has a boundary */
  double c;
  const double* queries;      /* host, n_queries x n; must stay valid until done */
  int64_t n_queries, n_walks;
  double eps;
  uint64_t seed;
  mpwos_options opt;          /* precision, theta, ... (stream, device_io and walk_* ignored) */
  double* u_out;              /* host, n_queries */
  double* stderr_out;         /* host, nullable */
} mpwos_request;

typedef struct {
  int64_t admitted, completed, rejected;
  int64_t walk_steps;
  double busy_seconds;        /* time with at least one request on the device */
  int64_t in_flight_bytes;    /* HBM held by admitted requests */
  int32_t rounds;             /* batched launches */
} mpwos_server_stats;

/* hbm_budget_bytes: device memory the server may hold for admitted requests
 * (queries, per-walk scores, outputs).  slice_walk_steps: work of one launch,
 * shared by the requests of its class, in three-dimensional walk-steps (0 =
 * about 9e7); a launch holds at least the walks that fill the device, or all
 * that its class has left, and at least one wavefront's walks per request.
 * Launches run on six to eight streams, each with a hardware queue of its
 * own: ordinary streams, min(8, GPU_MAX_HW_QUEUES - 2) of them, when the
 * variable (as read at creation, default 4) leaves queues for six beside the
 * null and completion streams; otherwise six streams created with a CU mask
 * of every CU, which the runtime gives queues of their own.  Classes whose
 * launches take above 20 ms of device time run on half of them, and no
 * launch is queued behind such a launch.  The library allocates two launch
 * tables of 512 entries per stream and 64 MiB of pinned staging at creation;
 * admission, uploads, reductions and copies out are
 * asynchronous (events), so the scheduling thread never waits for the
 * device.  A request whose staging does not fit waits for completions to
 * free it; one above 16 MiB takes pinned memory of its own. */
mpwos_status mpwos_server_create(size_t hbm_budget_bytes, int64_t slice_walk_steps, mpwos_server** out);

/* Queues a request (non-blocking); returns its ticket.  EINVAL for bad
 * arguments; ENOMEM when the request alone exceeds the HBM budget;
 * EOFFMANIFOLD for a query off an analytic manifold.  Point-cloud queries
 * are checked on the device at admission (a check at submit would wait for
 * the device): a request with a query farther than two local spacings from
 * the reconstruction completes with EOFFMANIFOLD and writes no output. */
mpwos_status mpwos_submit(mpwos_server* s, const mpwos_request* req, uint64_t* ticket);

/* done = 1 once the request finished; `result` then holds its status. */
mpwos_status mpwos_poll(mpwos_server* s, uint64_t ticket, int32_t* done, int32_t* result);

/* Blocks until the request finished (timeout_ms < 0: no limit); EBUSY on timeout. */
mpwos_status mpwos_wait(mpwos_server* s, uint64_t ticket, int64_t timeout_ms, int32_t* result);

/* Timeline of a request, in seconds since the server was created:
 * times[0] submitted, [1] admitted, [2] first launch holding its walks
 * enqueued, [3] last such launch observed complete, [4] results delivered.
 * Entries not reached yet are -1.  EINVAL for an unknown ticket. */
mpwos_status mpwos_request_times(mpwos_server* s, uint64_t ticket, double times[5]);

mpwos_status mpwos_server_stats_get(mpwos_server* s, mpwos_server_stats* out);

/* Drains outstanding work and frees the server. */
mpwos_status mpwos_server_destroy(mpwos_server* s);

/* ---- inspection entry points (device implementations of single steps) -- */

/* cp (eq. cp_map) of n_points ambient points x (n_points x n doubles, host)
 * into y (host), computed by the device code of the given precision. */
mpwos_status mpwos_debug_cp(const mpwos_manifold* m, const double* x, int64_t n_points,
                            int32_t precision, double* y);

/* Build facts of a POINT_CLOUD manifold (Sec. 2.3.2): how many cloud points
 * took the KD-tree search because the grid-tile kNN result could not be shown
 * exact, and the largest local spacing h (mean distance from a point to its
 * k-1 other neighbours).  EINVAL for another kind. */
mpwos_status mpwos_debug_cloud_info(const mpwos_manifold* m, int64_t* knn_fallback_points, double* max_spacing);

/* Radius fraction s = t/r of a Green sample for uniforms u (host arrays of
 * `count`), dimension n and X = sqrt(sigma) r: the device inverse of the
 * radial law of eq. Z_sampling_density, in the given precision. */
mpwos_status mpwos_debug_radial_inv(int32_t n, double X, const double* u, int64_t count,
                                    int32_t precision, double* s);

/* The device fit of mpwos_predictor_fit alone: node values U (nt x (ns - 1)
 * doubles, host, th-major) to ks (2 kt + 1) series coefficients (host), under
 * the same limits. */
mpwos_status mpwos_debug_ts_fit(const double* U, int32_t nt, int32_t ns, int32_t ks, int32_t kt, double* coef_out);

/* `count` Philox4x32-10 blocks for counters (c0 + i, c1, c2, c3), key
 * (seed_lo, seed_hi), written as 4 x count words (host). */
mpwos_status mpwos_debug_philox(const uint32_t ctr[4], uint64_t seed, int64_t count, uint32_t* out);

/* Times a plain device-to-device copy of `bytes` (device memory owned by the
 * library) repeated `reps` times; average ms per copy in *ms.  Used to
 * calibrate HBM traffic counters. */
mpwos_status mpwos_copy_probe(int64_t bytes, int32_t reps, double* ms);

/* Throughput of one VALU operation, in lane-operations per second, from a
 * kernel of 8 independent dependency chains per lane over 16 blocks of 256
 * lanes per compute unit.  op: 0 fma_f32, 1 fma_f64, 2 mad_u64_u32 (32x32->64
 * multiply-add), 3 mul_hi_u32, 4 log_f32, 5 sin_f32, 6 sqrt_f32, 7 rsq_f32,
 * 8 rcp_f32, 9 xor_b32, 10 add_f64; mixed streams (each step one operation
 * beside three independent fma_f32, all four counted): 11 sin_f32,
 * 12 mad_u64_u32; 13 bitop3_b32 (three-input bitwise operation, here a
 * three-way xor).  Used to weight the operations of the walk-step cost model.
 * EINVAL for another op. */
mpwos_status mpwos_valu_probe(int32_t op, double* lane_ops_per_s);

/* Library version string. */
const char* mpwos_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPWOS_H */
