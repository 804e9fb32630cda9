"""FP64 CPU oracle for MPWoS -- TEST INFRASTRUCTURE ONLY.

Plain ctypes marshalling around ``libmpwos_oracle.so`` (built from
``mpwos_oracle.c`` by ``oracle/build.py``).  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import this module; the
solver itself never does.

Problems are plain dicts (the same dict a test also hands to the GPU binding):

    {"manifold": "sphere" | "sphere_cap" | "torus" | "point_cloud",
     "n": int, "p": [R, h_or_a, ...], "sigma": float,
     "f": {"kind": "sph_pair", "idx": [0, 1], "coef": [8.0]},
     "g": {...} (boundary only), "eps": float, "theta": 0.95, "c_kappa": 1.2,
     "tau_w": 1e-8, "n_v": 1, "compensation": "exact" | "none",
     "max_steps": int, "points": ndarray (point cloud), "k_nn": 16,
     "radius_rule": "curvature" | "spacing" | "curvature_fit" | "curvature_bound", "c_h": 2.4,
     "kappa_bound": float (curvature_bound only),
     "reconstruction": "patch" | "nearest" (point cloud),
     "predictor": {"idx": [ks, kt], "values": coef} and "h_eta" (second_order only)}
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libmpwos_oracle.so")

MANIFOLDS = {"sphere": 0, "sphere_cap": 1, "torus": 2, "point_cloud": 3, "dumbbell": 4, "product": 5,
             "cut_torus": 6}
FN_KINDS = {"zero": 0, "const": 1, "sph_pair": 2, "circle_mode": 3, "legendre": 4,
            "torus_mode": 5, "table_s1": 6, "dumbbell_poly": 7, "product_modes": 8, "torus_sine": 9}
COMP = {"none": 0, "exact": 1, "second_order": 2}
RADIUS_RULES = {"curvature": 0, "spacing": 1, "curvature_fit": 2, "curvature_bound": 3}
STATUS = {0: "OK", -1: "EINVAL", -2: "EOFFMANIFOLD", -3: "ENOMEM", 1: "WTRUNC"}


class _Problem(ctypes.Structure):
    _fields_ = [
        ("manifold", ctypes.c_int32), ("n", ctypes.c_int32), ("p", ctypes.c_double * 4),
        ("points", ctypes.c_void_p), ("n_points", ctypes.c_int64), ("k_nn", ctypes.c_int32),
        ("radius_rule", ctypes.c_int32),
        ("f_kind", ctypes.c_int32), ("f_idx", ctypes.c_int32 * 3), ("f_coef", ctypes.c_double * 8),
        ("f_values", ctypes.c_void_p), ("f_nvalues", ctypes.c_int64),
        ("g_kind", ctypes.c_int32), ("g_idx", ctypes.c_int32 * 3), ("g_coef", ctypes.c_double * 8),
        ("sigma", ctypes.c_double), ("eps", ctypes.c_double), ("theta", ctypes.c_double),
        ("c_kappa", ctypes.c_double), ("c_h", ctypes.c_double), ("tau_w", ctypes.c_double),
        ("n_v", ctypes.c_int32), ("compensation", ctypes.c_int32), ("max_steps", ctypes.c_int64),
        ("k_spacing", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
        ("kappa_bound", ctypes.c_double), ("reconstruction", ctypes.c_int32),
        ("pred_coef", ctypes.c_void_p), ("pred_ks", ctypes.c_int32), ("pred_kt", ctypes.c_int32),
        ("h_eta", ctypes.c_double), ("fit_scale", ctypes.c_double), ("grid", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIBPATH)
        d, i32, u32, i64, u64, vp = (ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                                     ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p)
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_uniform.argtypes = [u32]; L.orc_uniform.restype = d
        L.orc_box_muller.argtypes = [u32, u32, vp]
        L.orc_normals.argtypes = [u64, u32, u32, u32, u32, ctypes.c_int, vp]
        L.orc_direction.argtypes = [u64, u32, u32, u32, u32, ctypes.c_int, vp]
        L.orc_db_phi.argtypes = [d, d, d, d]
        L.orc_db_phi.restype = d
        L.orc_db_curvatures.argtypes = [d, d, d, vp, vp]
        L.orc_pr_phi.argtypes = [vp]
        L.orc_pr_phi.restype = d
        L.orc_radius_uniform.argtypes = [u64, u32, u32, u32, u32, ctypes.c_int]
        L.orc_radius_uniform.restype = d
        for nm in ("orc_c_sigma_r", "orc_omega"):
            getattr(L, nm).argtypes = [ctypes.c_int, d, d]
            getattr(L, nm).restype = d
        for nm in ("orc_radial_cdf", "orc_radial_pdf", "orc_radial_inv"):
            getattr(L, nm).argtypes = [ctypes.c_int, d, d]
            getattr(L, nm).restype = d
        L.orc_radial_xmax.argtypes = [ctypes.c_int]; L.orc_radial_xmax.restype = d
        L.orc_knn.argtypes = [vp, i64, vp, ctypes.c_int, vp, vp]; L.orc_knn.restype = ctypes.c_int
        L.orc_pc_project_from.argtypes = [vp, vp, i64, vp]; L.orc_pc_project_from.restype = ctypes.c_int
        L.orc_grid_build.argtypes = [vp, i64]; L.orc_grid_build.restype = vp
        L.orc_grid_free.argtypes = [vp]; L.orc_grid_free.restype = None
        L.orc_grid_knn.argtypes = [vp, vp, ctypes.c_int, vp, vp]; L.orc_grid_knn.restype = ctypes.c_int
        L.orc_grid_ball.argtypes = [vp, vp, d, vp, i64]; L.orc_grid_ball.restype = i64
        L.orc_cp.argtypes = [vp, vp, vp]; L.orc_cp.restype = ctypes.c_int
        L.orc_delta_gamma.argtypes = [vp, vp]; L.orc_delta_gamma.restype = d
        L.orc_source.argtypes = [vp, vp]; L.orc_source.restype = d
        L.orc_radius.argtypes = [vp, vp]; L.orc_radius.restype = d
        L.orc_solve.argtypes = [vp, vp, i64, i64, u64, ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_solve.restype = ctypes.c_int
        L.orc_walk_one.argtypes = [vp, vp, u32, u32, u64, vp, vp, vp]
        L.orc_walk_one.restype = ctypes.c_int
        L.orc_ts_fit.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
        L.orc_ts_fit.restype = ctypes.c_int
        L.orc_ts_value.argtypes = [vp, ctypes.c_int, ctypes.c_int, d, d, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


GRID_MIN_POINTS = 100_000


class Grid:
    """Exact uniform-grid index of a point cloud (orc_grid_*)."""

    def __init__(self, pts):
        self.pts = np.ascontiguousarray(pts, dtype=np.float64)
        self.handle = lib().orc_grid_build(_ptr(self.pts), self.pts.shape[0])
        if not self.handle:
            raise MemoryError("orc_grid_build")

    def knn(self, x, k):
        x = np.ascontiguousarray(x, dtype=np.float64)
        idx = np.zeros(k, dtype=np.int64)
        d2 = np.zeros(k)
        st = lib().orc_grid_knn(self.handle, _ptr(x), k, _ptr(idx), _ptr(d2))
        if st:
            raise ValueError(st)
        return idx, d2

    def ball(self, x, rho2):
        x = np.ascontiguousarray(x, dtype=np.float64)
        cap = 64
        while True:
            out = np.zeros(cap, dtype=np.int64)
            cnt = lib().orc_grid_ball(self.handle, _ptr(x), float(rho2), _ptr(out), cap)
            if cnt < 0:
                raise ValueError(cnt)
            if cnt <= cap:
                return out[:cnt]
            cap = cnt

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.orc_grid_free(self.handle)
        except Exception:
            pass


class Problem:
    """Marshals a problem dict into the oracle's struct; keeps arrays alive."""

    def __init__(self, d):
        self.d = d
        s = _Problem()
        s.manifold = MANIFOLDS[d["manifold"]]
        s.n = int(d["n"])
        for i, v in enumerate(d.get("p", [1.0])):
            s.p[i] = float(v)
        self._keep = []
        self._grid = None
        if d["manifold"] == "point_cloud":
            pts = np.ascontiguousarray(d["points"], dtype=np.float64)
            self._keep.append(pts)
            s.points = pts.ctypes.data
            s.n_points = pts.shape[0]
            # large clouds are searched on an exact grid (equal to brute force)
            if pts.shape[0] >= GRID_MIN_POINTS:
                self._grid = Grid(pts)
                s.grid = self._grid.handle
        s.fit_scale = float(d.get("fit_scale", 1.0))
        s.k_nn = int(d.get("k_nn", 16))
        s.radius_rule = RADIUS_RULES[d.get("radius_rule", "curvature")]
        f = d.get("f", {"kind": "zero"})
        s.f_kind = FN_KINDS[f["kind"]]
        for i, v in enumerate(f.get("idx", [])):
            s.f_idx[i] = int(v)
        for i, v in enumerate(f.get("coef", [])):
            s.f_coef[i] = float(v)
        if "values" in f:
            vals = np.ascontiguousarray(f["values"], dtype=np.float64)
            self._keep.append(vals)
            s.f_values = vals.ctypes.data
            s.f_nvalues = vals.size
        g = d.get("g", {"kind": "zero"})
        s.g_kind = FN_KINDS[g["kind"]]
        for i, v in enumerate(g.get("idx", [])):
            s.g_idx[i] = int(v)
        for i, v in enumerate(g.get("coef", [])):
            s.g_coef[i] = float(v)
        s.sigma = float(d["sigma"])
        s.eps = float(d.get("eps", 1e-3))
        s.theta = float(d.get("theta", 0.95))
        s.c_kappa = float(d.get("c_kappa", 1.2))
        s.c_h = float(d.get("c_h", 2.4))
        s.tau_w = float(d.get("tau_w", 1e-8))
        s.n_v = int(d.get("n_v", 1))
        s.compensation = COMP[d.get("compensation", "exact")]
        s.max_steps = int(d.get("max_steps", 10_000_000))
        s.k_spacing = int(d.get("k_spacing", d.get("k_nn", 16)))
        s.newton_iters = int(d.get("newton_iters", 6))
        s.kappa_bound = float(d.get("kappa_bound", 0.0))
        s.reconstruction = {"patch": 0, "nearest": 1}[d.get("reconstruction", "patch")]
        if "predictor" in d:
            pc = np.ascontiguousarray(d["predictor"]["values"], dtype=np.float64)
            self._keep.append(pc)
            s.pred_coef = pc.ctypes.data
            s.pred_ks, s.pred_kt = (int(v) for v in d["predictor"]["idx"])
        s.h_eta = float(d.get("h_eta", 1e-2))
        self.s = s

    @property
    def ref(self):
        return ctypes.byref(self.s)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed, q, w, k, sub, n):
    g = np.zeros(n, dtype=np.float64)
    lib().orc_normals(seed, q, w, k, sub, n, _ptr(g))
    return g


def direction(seed, q, w, k, sub, n):
    z = np.zeros(n, dtype=np.float64)
    lib().orc_direction(seed, q, w, k, sub, n, _ptr(z))
    return z


def db_phi(alpha, kc, rho, zs):
    """Profile parameter of the dumbbell point nearest to (|xh|, xs) = (rho, zs)."""
    return lib().orc_db_phi(alpha, kc, rho, zs)


def db_curvatures(alpha, kc, phi):
    """(k1, k2): profile and cross-section principal curvatures at phi."""
    k1, k2 = ctypes.c_double(), ctypes.c_double()
    lib().orc_db_curvatures(alpha, kc, phi, ctypes.byref(k1), ctypes.byref(k2))
    return k1.value, k2.value


def pr_phi(xc):
    """Curve parameter of the Fourier-curve point nearest to x_c (6 coordinates)."""
    x = np.ascontiguousarray(xc, dtype=np.float64)
    return lib().orc_pr_phi(_ptr(x))


def radius_uniform(seed, q, w, k, sub, n):
    return lib().orc_radius_uniform(seed, q, w, k, sub, n)


def uniform(x):
    return lib().orc_uniform(int(x))


def box_muller(x0, x1):
    out = np.zeros(2)
    lib().orc_box_muller(int(x0), int(x1), _ptr(out))
    return out


def c_sigma_r(n, sigma, r):
    return lib().orc_c_sigma_r(n, sigma, r)


def omega(n, sigma, r):
    return lib().orc_omega(n, sigma, r)


def radial_cdf(n, X, s):
    return lib().orc_radial_cdf(n, X, s)


def radial_pdf(n, X, s):
    return lib().orc_radial_pdf(n, X, s)


def radial_inv(n, X, u):
    return lib().orc_radial_inv(n, X, u)


def radial_xmax(n):
    return lib().orc_radial_xmax(n)


def knn(points, x, k):
    pts = np.ascontiguousarray(points, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    idx = np.zeros(k, dtype=np.int64)
    d2 = np.zeros(k, dtype=np.float64)
    st = lib().orc_knn(_ptr(pts), pts.shape[0], _ptr(xx), k, _ptr(idx), _ptr(d2))
    if st:
        raise ValueError(STATUS.get(st, st))
    return idx, d2


def cp(problem, x):
    P = problem if isinstance(problem, Problem) else Problem(problem)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(xx)
    st = lib().orc_cp(P.ref, _ptr(xx), _ptr(y))
    if st:
        raise ValueError(STATUS.get(st, st))
    return y


class _PcResult(ctypes.Structure):
    _fields_ = [("y", ctypes.c_double * 3), ("kappa", ctypes.c_double), ("h_mean", ctypes.c_double),
                ("patch", ctypes.c_int64)]


def pc_project(problem, x, start=-1):
    """Point-cloud projection from a start patch (-1: from the cloud point
    nearest to x): (y, kappa, h_mean, patch)."""
    P = problem if isinstance(problem, Problem) else Problem(problem)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    r = _PcResult()
    st = lib().orc_pc_project_from(P.ref, _ptr(xx), int(start), ctypes.byref(r))
    if st:
        raise ValueError(STATUS.get(st, st))
    return np.array(r.y[:]), r.kappa, r.h_mean, r.patch


def delta_gamma(problem, y):
    P = problem if isinstance(problem, Problem) else Problem(problem)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_delta_gamma(P.ref, _ptr(yy))


def source(problem, z):
    P = problem if isinstance(problem, Problem) else Problem(problem)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    return lib().orc_source(P.ref, _ptr(zz))


def radius(problem, y):
    P = problem if isinstance(problem, Problem) else Problem(problem)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_radius(P.ref, _ptr(yy))


def walk(problem, y0, q, w, seed):
    P = problem if isinstance(problem, Problem) else Problem(problem)
    yy = np.ascontiguousarray(y0, dtype=np.float64)
    S = ctypes.c_double()
    K = ctypes.c_int32()
    tr = ctypes.c_int()
    st = lib().orc_walk_one(P.ref, _ptr(yy), q, w, seed, ctypes.byref(S), ctypes.byref(K),
                            ctypes.byref(tr))
    if st:
        raise ValueError(STATUS.get(st, st))
    return S.value, K.value, bool(tr.value)


def solve(problem, queries, n_walks, seed, threads=None):
    """Run every walk; returns dict(u, stderr, walk_S (nq, nw), walk_K, status, truncated)."""
    P = problem if isinstance(problem, Problem) else Problem(problem)
    Q = np.ascontiguousarray(queries, dtype=np.float64)
    nq = Q.shape[0]
    nw = int(n_walks)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    wS = np.zeros((nq, nw), dtype=np.float64)
    wK = np.zeros((nq, nw), dtype=np.int32)
    u = np.zeros(nq, dtype=np.float64)
    se = np.zeros(nq, dtype=np.float64)
    ntr = ctypes.c_int64(0)
    st = lib().orc_solve(P.ref, _ptr(Q), nq, nw, seed, int(threads), _ptr(wS), _ptr(wK), _ptr(u),
                         _ptr(se), ctypes.byref(ntr))
    if st < 0:
        raise ValueError(STATUS.get(st, st))
    return {"u": u, "stderr": se, "walk_S": wS, "walk_K": wK, "status": STATUS[st],
            "truncated": ntr.value, "threads": int(threads)}


def ts_fit(U, kt, ks):
    """Fourier-sine coefficients (ks rows of 2 kt + 1) of node values U (nt, ns - 1)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    nt, ns = U.shape[0], U.shape[1] + 1
    coef = np.zeros(ks * (2 * kt + 1), dtype=np.float64)
    st = lib().orc_ts_fit(_ptr(U), nt, ns, kt, ks, _ptr(coef))
    if st:
        raise ValueError(STATUS.get(st, st))
    return coef


def ts_value(coef, ks, kt, th, s):
    """(u, u_th, u_thth, u_ss) of the Fourier-sine series at (th, s)."""
    c = np.ascontiguousarray(coef, dtype=np.float64)
    out = np.zeros(4)
    lib().orc_ts_value(_ptr(c), ks, kt, float(th), float(s), _ptr(out))
    return out
