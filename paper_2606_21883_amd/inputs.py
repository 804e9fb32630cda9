"""Seeded synthetic inputs: query sets, point clouds and problem descriptions.

This module holds none of the walk's arithmetic.  It draws query points and
point clouds with numpy's PCG64 generator (independent of the walk's Philox
stream), describes the benchmark problems as plain dicts, and evaluates the
closed-form solutions u that the estimates are scored against.

Problem shapes follow the paper's experiments (Sec. 4): unit circle and unit
sphere problems with spherical-harmonic solutions, hyperspheres up to
n = 1000, a torus (R = 1, a = 0.3) given implicitly and as a noisy point cloud,
and the 1000-dimensional implicit dumbbell of Example 2 in R^1001.
"""
import math

import numpy as np

# ---------------------------------------------------------------------------
# query sets
# ---------------------------------------------------------------------------


def circle_queries(nq):
    """nq points uniform in angle on the unit circle: theta_p = 2 pi p / nq."""
    th = 2.0 * np.pi * np.arange(nq) / nq
    return np.stack([np.cos(th), np.sin(th)], axis=1)


def sphere_uniform(nq, n, seed=1, radius=1.0):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nq, n))
    return radius * g / np.linalg.norm(g, axis=1, keepdims=True)


def cap_uniform(nq, n=3, h=0.0, seed=1, radius=1.0, margin=0.0):
    """Uniform (area measure) on the cap {x_n > h + margin} of S^{n-1}_R, by rejection."""
    rng = np.random.default_rng(seed)
    out = []
    while sum(len(o) for o in out) < nq:
        g = rng.standard_normal((4 * nq + 16, n))
        g = radius * g / np.linalg.norm(g, axis=1, keepdims=True)
        out.append(g[g[:, -1] > h + margin])
    return np.concatenate(out)[:nq]


def hypersphere_queries(nq, n, seed=1):
    """Half the queries on the (x1, x2) great circle, half uniform on S^{n-1}.

    Uniform points in high dimension give |x1 x2| ~ 1/n; the great circle gives
    values of order one (u = sin(2 alpha)/2 there)."""
    nc = nq // 2
    q = np.zeros((nq, n))
    al = 2.0 * np.pi * (np.arange(nc) + 0.5) / max(nc, 1)
    q[:nc, 0] = np.cos(al)
    q[:nc, 1] = np.sin(al)
    q[nc:] = sphere_uniform(nq - nc, n, seed)
    return q


def torus_point(R, a, phi, psi):
    rt = R + a * np.cos(psi)
    return np.stack([rt * np.cos(phi), rt * np.sin(phi), a * np.sin(psi)], axis=-1)


def torus_area_uniform(nq, R=1.0, a=0.3, seed=1):
    """Area-uniform points on the torus: phi uniform, psi with density ~ R + a cos psi."""
    rng = np.random.default_rng(seed)
    phis, psis = [], []
    cnt = 0
    while cnt < nq:
        m = 2 * (nq - cnt) + 16
        psi = rng.uniform(0.0, 2.0 * np.pi, m)
        acc = rng.uniform(0.0, R + a, m) < R + a * np.cos(psi)
        psi = psi[acc]
        phi = rng.uniform(0.0, 2.0 * np.pi, psi.size)
        phis.append(phi)
        psis.append(psi)
        cnt += psi.size
    phi = np.concatenate(phis)[:nq]
    psi = np.concatenate(psis)[:nq]
    return torus_point(R, a, phi, psi)


def torus_point_cloud(npts, R=1.0, a=0.3, noise=1e-4, seed=1):
    """Area-uniform torus samples plus isotropic Gaussian noise N(0, noise^2 I),
    rounded to FP32 (the precision a cloud is stored in), returned as float64."""
    pts = torus_area_uniform(npts, R, a, seed)
    rng = np.random.default_rng(seed + 1000)
    pts = pts + noise * rng.standard_normal(pts.shape)
    return pts.astype(np.float32).astype(np.float64)


def torus_near_points(m, offset, R=1.0, a=0.3, seed=1):
    """Points at distance up to `offset` from the torus along random directions."""
    base = torus_area_uniform(m, R, a, seed)
    rng = np.random.default_rng(seed + 2000)
    d = rng.standard_normal(base.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return base + offset * rng.uniform(-1.0, 1.0, (m, 1)) * d


# ---------------------------------------------------------------------------
# problem descriptions (plain dicts understood by the solver binding)
# ---------------------------------------------------------------------------

DEFAULTS = dict(theta=0.95, c_kappa=1.2, tau_w=1e-8, n_v=1, compensation="exact",
                max_steps=10_000_000)


def problem(**kw):
    d = dict(DEFAULTS)
    d.update(kw)
    return d


def circle_problem():
    """u = cos(3 theta) on S^1, sigma = 1, f = 10 cos(3 theta)."""
    return problem(manifold="sphere", n=2, p=[1.0], sigma=1.0,
                   f=dict(kind="circle_mode", idx=[3], coef=[10.0, 0.0]))


def sphere_problem():
    """u = x1 x2 on S^2, sigma = 2, f = 8 x1 x2."""
    return problem(manifold="sphere", n=3, p=[1.0], sigma=2.0,
                   f=dict(kind="sph_pair", idx=[0, 1], coef=[8.0]))


def cap_problem(eps=1e-3):
    """Cap x3 > 0 of S^2, u = x1 x2, sigma = 0.5, f = 6.5 x1 x2, g = u."""
    return problem(manifold="sphere_cap", n=3, p=[1.0, 0.0], sigma=0.5, eps=eps,
                   f=dict(kind="sph_pair", idx=[0, 1], coef=[6.5]),
                   g=dict(kind="sph_pair", idx=[0, 1], coef=[1.0]))


def hypersphere_problem(n):
    """u = x1 x2 on S^{n-1}, sigma = 1, f = (2n + 1) x1 x2."""
    return problem(manifold="sphere", n=n, p=[1.0], sigma=1.0,
                   f=dict(kind="sph_pair", idx=[0, 1], coef=[2.0 * n + 1.0]))


def torus_problem(R=1.0, a=0.3):
    """u = sin(phi) cos(2 psi) on the implicit torus, sigma = 1."""
    return problem(manifold="torus", n=3, p=[R, a], sigma=1.0,
                   f=dict(kind="torus_mode", coef=[1.0]))


def point_cloud_problem(points, k_nn=16, radius_rule="curvature_fit", R=1.0, a=0.3, kappa_bound=None, fit_scale=1.0):
    d = problem(manifold="point_cloud", n=3, p=[R, a], sigma=1.0, points=points, k_nn=k_nn,
                radius_rule=radius_rule, c_h=2.4, newton_iters=6, fit_scale=fit_scale,
                f=dict(kind="torus_mode", coef=[1.0]))
    if kappa_bound is not None:
        d["kappa_bound"] = kappa_bound
    return d


# ---------------------------------------------------------------------------
# closed-form solutions u (what the estimates are scored against)
# ---------------------------------------------------------------------------


def _legendre(l, t):
    p0, p1 = np.ones_like(t), t
    if l == 0:
        return p0
    for k in range(1, l):
        p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
    return p1


def exact_u(prob, y):
    """u(y) for the problem's manufactured solution at points y on M."""
    y = np.asarray(y, dtype=np.float64)
    f = prob["f"]
    kind = f["kind"]
    sg = prob["sigma"]
    n = prob["n"]
    R = prob.get("p", [1.0])[0]
    if kind == "zero":
        return np.zeros(len(y))
    if kind == "const":
        return np.full(len(y), f["coef"][0] / sg)
    if kind == "sph_pair":
        i, j = f["idx"][:2]
        lam = 2.0 * n / R ** 2
        return f["coef"][0] / (lam + sg) * (y[:, i] / R) * (y[:, j] / R)
    if kind == "circle_mode":
        k = f["idx"][0]
        lam = k * k / R ** 2
        th = np.arctan2(y[:, 1], y[:, 0])
        c = list(f["coef"]) + [0.0]
        return (c[0] * np.cos(k * th) + c[1] * np.sin(k * th)) / (lam + sg)
    if kind == "legendre":
        t = y[:, -1] / R
        out = np.zeros(len(y))
        for l, c in enumerate(f["coef"]):
            out += c / (l * (l + 1) / R ** 2 + sg) * _legendre(l, t)
        return out
    if kind == "torus_mode":
        Rt = prob["p"][0]
        phi = np.arctan2(y[:, 1], y[:, 0])
        rho = np.hypot(y[:, 0], y[:, 1])
        psi = np.arctan2(y[:, 2], rho - Rt)
        return f["coef"][0] * np.sin(phi) * np.cos(2.0 * psi)
    if kind == "torus_sine":
        ks, kt = f["idx"][:2]
        th, sv = cut_torus_angles(y, prob["p"][0], prob["p"][2])
        return torus_sine_u(np.asarray(f["values"]).reshape(ks, 2 * kt + 1), th, sv)
    if kind == "product_modes":
        c = f["coef"]
        a = prob["p"][1]
        phi = np.arctan2(y[:, 1], y[:, 0])
        w1, w2 = y[:, 6] / a, y[:, 7] / a
        return c[0] * np.cos(phi) * w1 + c[1] * np.sin(2 * phi) * w2 + c[2] * np.cos(3 * phi) * (w1 * w1 - w2 * w2)
    if kind == "dumbbell_poly":
        c = f["coef"]
        a = np.asarray(f["values"])
        xh, xs = y[:, :-1], y[:, -1]
        return (c[0] * xs + c[1] * xs * xs + c[2] * xh.sum(axis=1) / math.sqrt(xh.shape[1])
                + c[3] * (xh * xh * a).sum(axis=1))
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# the product manifold of Example 3: S^1_Fourier(R) x S^2(a) in R^9,
# X(phi, w) = (R C(phi), a w), C = (cos, sin, cos 2/2, sin 2/2, cos 3/3, sin 3/3)
# ---------------------------------------------------------------------------


def product_point(phi, w, R=1.0, a=0.65):
    """X(phi, w) for angles phi (m,) and unit vectors w (m, 3)."""
    phi = np.asarray(phi, dtype=np.float64)
    cols = []
    for k in (1, 2, 3):
        cols += [R * np.cos(k * phi) / k, R * np.sin(k * phi) / k]
    return np.concatenate([np.stack(cols, axis=1), a * np.asarray(w)], axis=1)


def product_points(nq, R=1.0, a=0.65, seed=1):
    """phi uniform on [0, 2 pi), w uniform on S^2."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * np.pi, nq)
    w = rng.standard_normal((nq, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    return product_point(phi, w, R, a)


def product_problem(R=1.0, a=0.65, sigma=1.0, coef=(1.0, 0.3, 0.2)):
    """Example 3: u = cos(phi) w1 + 0.3 sin(2 phi) w2 + 0.2 cos(3 phi) (w1^2 - w2^2)
    on S^1_Fourier(R) x S^2(a) in R^9, no compensation (as in the paper).  sigma
    is not stated in the paper: 1 here."""
    return problem(manifold="product", n=9, p=[R, a], sigma=sigma, compensation="none",
                   f=dict(kind="product_modes", coef=list(coef)))


# ---------------------------------------------------------------------------
# the sphere point cloud of Example 4: 8000 points uniform on S^2, the pure
# nearest-neighbour projection, u = P1 + 0.2 P3 + 0.1 P5 of x3
# ---------------------------------------------------------------------------


def sphere_point_cloud(npts, seed=1):
    """Uniform points on the unit sphere, rounded to binary32 (the library's
    point format)."""
    p = sphere_uniform(npts, 3, seed)
    return p.astype(np.float32).astype(np.float64)


def sphere_cloud_problem(points, sigma=1.0, k_others=6, c_h=2.4):
    """Example 4: f = (sigma + 2) P1 + 0.2 (sigma + 12) P3 + 0.1 (sigma + 30) P5
    of x3 (so u = P1 + 0.2 P3 + 0.1 P5), the spacing rule with h the mean
    distance to the k_others nearest other points (k_nn counts the point
    itself), c_h = 2.4, the nearest cloud point as the projection, no
    compensation.  sigma is not stated in the paper: 1 here."""
    c = [0.0] * 8
    c[1] = sigma + 2.0
    c[3] = 0.2 * (sigma + 12.0)
    c[5] = 0.1 * (sigma + 30.0)
    return problem(manifold="point_cloud", n=3, p=[1.0], sigma=sigma, points=np.asarray(points, dtype=np.float64),
                   k_nn=k_others + 1, radius_rule="spacing", c_h=c_h, reconstruction="nearest",
                   compensation="none", f=dict(kind="legendre", coef=c))


# ---------------------------------------------------------------------------
# the implicit dumbbell of Example 2: |xh| = R(xs) in R^n, xh in R^{n-1},
# R(xs) = sqrt(1 - (xs/kc)^2) (1 - a + 2 a (xs/kc)^2), a = 0.35, kc = 1.2
# ---------------------------------------------------------------------------


def dumbbell_profile_radius(xs, alpha=0.35, kc=1.2):
    """R(xs) as the paper defines it."""
    t = (np.asarray(xs, dtype=np.float64) / kc) ** 2
    return np.sqrt(np.maximum(0.0, 1.0 - t)) * (1.0 - alpha + 2.0 * alpha * t)


def dumbbell_kappa_max(alpha=0.35, kc=1.2, m=400001):
    """Largest principal curvature magnitude over the dumbbell, from the profile
    (sin t g(t), kc cos t), g = 1 - a + 2 a cos^2 t, on a fine grid: the profile
    curvature and kc / (g |profile'|), the curvature of the cross-sections.
    2.9294 for the paper's a = 0.35, kc = 1.2."""
    t = np.linspace(0.0, np.pi, m)
    s, c = np.sin(t), np.cos(t)
    g = 1.0 - alpha + 2.0 * alpha * c * c
    g1 = -4.0 * alpha * c * s
    g2 = -4.0 * alpha * (c * c - s * s)
    r1 = c * g + s * g1
    r2 = -s * g + 2.0 * c * g1 + s * g2
    z1, z2 = -kc * s, -kc * c
    L = np.sqrt(r1 * r1 + z1 * z1)
    k1 = (z1 * r2 - r1 * z2) / L ** 3
    k2 = kc / (g * L)
    return float(max(np.abs(k1).max(), np.abs(k2).max()))


def dumbbell_diag(n):
    """The trace-free diagonal A_2 (the paper leaves its entries open):
    +1, -1, +1, ... over the n-1 coordinates of xh, the last one 0 when n-1 is
    odd."""
    a = np.ones(n - 1)
    a[1::2] = -1.0
    if (n - 1) % 2:
        a[-1] = 0.0
    return a


def dumbbell_problem(n=1001, alpha=0.35, kc=1.2, n_v=1, sigma=None):
    """Example 2: u = 0.15 xs + 0.05 xs^2 + (1.xh)/sqrt(n-1) + 0.2 xh^T A_2 xh on
    the dumbbell in R^n, sigma = 2 d (d = n - 1), theta = 0.95, c_kappa = 1.2, no
    compensation (as in the paper), the radius from the curvature bound."""
    return problem(manifold="dumbbell", n=n, p=[alpha, kc], sigma=2.0 * (n - 1) if sigma is None else sigma,
                   f=dict(kind="dumbbell_poly", coef=[0.15, 0.05, 1.0, 0.2], values=dumbbell_diag(n)),
                   radius_rule="curvature_bound", kappa_bound=dumbbell_kappa_max(alpha, kc),
                   compensation="none", n_v=n_v)


def dumbbell_points(nq, n=1001, alpha=0.35, kc=1.2, seed=1, phi_margin=0.1):
    """Points of the dumbbell: profile angle uniform in [margin, pi - margin],
    cross-section direction uniform on S^{n-2}."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(phi_margin, np.pi - phi_margin, nq)
    e = rng.standard_normal((nq, n - 1))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    xs = kc * np.cos(t)
    r = dumbbell_profile_radius(xs, alpha, kc)
    return np.concatenate([e * r[:, None], xs[:, None]], axis=1)


# ---------------------------------------------------------------------------
# the torus with a planar cut of Example 1: R = 1, a = 0.45, cut by the plane
# through the axis at phi_c = 0.35 pi, Omega = {s = phi - phi_c in (0, pi)}
# ---------------------------------------------------------------------------

# Example 1's solution u = sin(s) A(th) + sin(2s) B(th) + sin(3s) C(th) as a
# Fourier-sine series: per k = 1..3 the row (c_0, c_1, d_1, c_2, d_2, c_3, d_3)
# of T_k(th) = c_0 + sum_j c_j cos(j th) + d_j sin(j th).
#   A = 1 + 0.90 cos th + 0.60 sin 2th + 0.35 cos 3th,  B = 0.45 cos 2th,
#   C = 0.30 (0.5 + sin th)
EX1_COEF = np.array([
    [1.0, 0.90, 0.0, 0.0, 0.60, 0.35, 0.0],
    [0.0, 0.0, 0.0, 0.45, 0.0, 0.0, 0.0],
    [0.15, 0.0, 0.30, 0.0, 0.0, 0.0, 0.0],
])


def cut_torus_point(th, s, R=1.0, a=0.45, phi_c=0.35 * math.pi):
    """X(th, phi) of the paper's parametrization with phi = phi_c + s."""
    return torus_point(R, a, np.asarray(s) + phi_c, np.asarray(th))


def cut_torus_points(nq, R=1.0, a=0.45, phi_c=0.35 * math.pi, seed=1, s_margin=0.0):
    """Area-uniform random points of Omega (s in (s_margin, pi - s_margin))."""
    rng = np.random.default_rng(seed)
    ths = []
    cnt = 0
    while cnt < nq:
        m = 2 * (nq - cnt) + 16
        th = rng.uniform(0.0, 2.0 * np.pi, m)
        th = th[rng.uniform(0.0, R + a, m) < R + a * np.cos(th)]
        ths.append(th)
        cnt += th.size
    th = np.concatenate(ths)[:nq]
    s = rng.uniform(s_margin, np.pi - s_margin, nq)
    return cut_torus_point(th, s, R, a, phi_c)


def cut_torus_nodes(nt, ns, R=1.0, a=0.45, phi_c=0.35 * math.pi):
    """Predictor nodes th_i = 2 pi i / nt, s_j = pi j / ns (0 < j < ns), th-major."""
    th = 2.0 * np.pi * np.arange(nt) / nt
    s = np.pi * np.arange(1, ns) / ns
    T, S = np.meshgrid(th, s, indexing="ij")
    return cut_torus_point(T.ravel(), S.ravel(), R, a, phi_c)


def torus_sine_u(coef, th, s):
    """The series sum_k sin(k s) T_k(th) (coef: ks rows of 2 kt + 1)."""
    coef = np.asarray(coef, dtype=np.float64)
    ks = coef.shape[0]
    kt = (coef.shape[1] - 1) // 2
    th = np.asarray(th)
    s = np.asarray(s)
    out = np.zeros(np.broadcast(th, s).shape)
    for k in range(1, ks + 1):
        T = coef[k - 1, 0] * np.ones_like(th)
        for j in range(1, kt + 1):
            T = T + coef[k - 1, 2 * j - 1] * np.cos(j * th) + coef[k - 1, 2 * j] * np.sin(j * th)
        out = out + np.sin(k * s) * T
    return out


def cut_torus_angles(y, R=1.0, phi_c=0.35 * math.pi):
    """(th, s) of points near the torus; s wrapped to (-pi, pi]."""
    y = np.asarray(y, dtype=np.float64)
    rho = np.hypot(y[:, 0], y[:, 1])
    th = np.arctan2(y[:, 2], rho - R)
    s = np.arctan2(y[:, 1], y[:, 0]) - phi_c
    s = (s + np.pi) % (2.0 * np.pi) - np.pi
    s[s == -np.pi] = np.pi
    return th, s


def cut_torus_problem(R=1.0, a=0.45, phi_c=0.35 * math.pi, sigma=4.0, eps=1e-5, n_v=50, coef=None,
                      compensation="none"):
    """Example 1: screened Poisson (sigma = 4) on the cut torus with the
    paper's u (zero on both cut circles), boundary layer eps = 1e-5, N_V = 50."""
    c = EX1_COEF if coef is None else np.asarray(coef, dtype=np.float64)
    return problem(manifold="cut_torus", n=3, p=[R, a, phi_c], sigma=sigma, eps=eps, n_v=n_v,
                   f=dict(kind="torus_sine", idx=[c.shape[0], (c.shape[1] - 1) // 2], values=c.ravel().copy()),
                   g=dict(kind="zero"), compensation=compensation)


# ---------------------------------------------------------------------------
# the benchmark configurations
# ---------------------------------------------------------------------------


def config(name, scale=1.0, seed=1):
    """Return (problem, queries, n_walks) for a named configuration.

    scale < 1 shrinks queries and walks (for tests); 1 is the full size.  The
    point cloud keeps its 1e6 points at every scale."""
    def sz(v, lo=1):
        return max(lo, int(round(v * scale)))

    if name == "circle":
        return circle_problem(), circle_queries(sz(64)), sz(1000)
    if name == "sphere":
        return sphere_problem(), sphere_uniform(sz(4096), 3, seed), sz(4096)
    if name == "cap":
        return cap_problem(), cap_uniform(sz(4096), 3, 0.0, seed), sz(4096)
    if name == "hyper100":
        return hypersphere_problem(100), hypersphere_queries(sz(1024, 2), 100, seed), sz(2048)
    if name == "hyper1000":
        return hypersphere_problem(1000), hypersphere_queries(sz(1024, 2), 1000, seed), sz(2048)
    if name == "torus":
        return torus_problem(), torus_area_uniform(sz(8192), 1.0, 0.3, seed), sz(1024)
    if name == "cloud":
        # 1e6 noisy torus samples (queries: analytic torus points, within the
        # noise and the fit error of the reconstruction)
        # At this density a 16-point patch spans about 0.008, where the quadratic
        # term (about 1e-4) is at the noise level, so each patch is fitted to the
        # points within 4 r_16 (about 250 points, span 0.03), which resolves the
        # torus's curvature; the radius takes the curvature bound 1/a (constant).
        pts = torus_point_cloud(1_000_000, 1.0, 0.3, 1e-4, seed)
        prob = point_cloud_problem(pts, radius_rule="curvature_bound", kappa_bound=1.0 / 0.3, fit_scale=4.0)
        return prob, torus_area_uniform(sz(8192), 1.0, 0.3, seed + 7), sz(1024)
    if name == "product":
        # Example 3: S^1_Fourier x S^2(0.65) in R^9
        return product_problem(), product_points(sz(4096), seed=seed), sz(1024)
    if name == "sphere_cloud":
        # Example 4: 8000 points on S^2, queries on the sphere
        prob = sphere_cloud_problem(sphere_point_cloud(8000, seed))
        return prob, sphere_uniform(sz(1024), 3, seed + 7), sz(1024)
    if name == "cut_torus":
        # Example 1: N_s = 100 random points of the cut torus, N_V = 50,
        # eps = 1e-5, second-order compensation from a coarse predictor (the
        # baseline solve with 256 paths at 32 x 15 nodes, fitted by a 4 x 9
        # Fourier-sine series), h_eta = 1e-2
        prob = dict(cut_torus_problem(compensation="second_order"), h_eta=1e-2,
                    predictor_grid=dict(nt=32, ns=16, n_walks=sz(256), ks=4, kt=4))
        return prob, cut_torus_points(sz(100), seed=seed), sz(10000)
    if name == "dumbbell":
        # Table 1's setting: 20 points of the 1000-dimensional dumbbell, N = 1000
        # paths each, N_V = 50 Green samples per step, tau_W = 1e-8
        return dumbbell_problem(1001, n_v=50), dumbbell_points(sz(20), 1001, seed=seed), sz(1000)
    raise ValueError(name)


def rmse(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(math.sqrt(np.mean((a - b) ** 2)))
