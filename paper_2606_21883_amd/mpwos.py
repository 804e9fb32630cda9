"""ctypes binding of libmpwos.so (include/mpwos.h).

Argument marshalling only: every step of a solve runs in the HIP library.
Loading fails loudly when the library has not been built; there is no CPU
fallback.  Names follow the C entry points without the ``mpwos_`` prefix.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libmpwos.so")

OK, EINVAL, EOFFMANIFOLD, ENOMEM, EDEVICE, EBUSY, WTRUNC = 0, -1, -2, -3, -4, -5, 1
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EOFFMANIFOLD", -3: "ENOMEM", -4: "EDEVICE", -5: "EBUSY",
                1: "WTRUNC"}
KINDS = {"sphere": 0, "sphere_cap": 1, "torus": 2, "point_cloud": 3, "dumbbell": 4, "product": 5,
         "cut_torus": 6}
FN_KINDS = {"zero": 0, "const": 1, "sph_pair": 2, "circle_mode": 3, "legendre": 4, "torus_mode": 5,
            "table_s1": 6, "dumbbell_poly": 7, "product_modes": 8, "torus_sine": 9}
PRECISION = {"fp64": 0, "fp32": 1}
RECONSTRUCTIONS = {"patch": 0, "nearest": 1}
COMP = {"none": 0, "exact": 1, "second_order": 2}
RADIUS_RULES = {"curvature": 0, "spacing": 1, "curvature_fit": 2, "curvature_bound": 3}


class MpwosError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ManifoldDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("p", ctypes.c_double * 4),
                ("points", ctypes.c_void_p), ("n_points", ctypes.c_int64), ("k_nn", ctypes.c_int32),
                ("points_on_device", ctypes.c_int32), ("reconstruction", ctypes.c_int32),
                ("fit_scale", ctypes.c_double)]


class Fn(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("idx", ctypes.c_int32 * 3), ("coef", ctypes.c_double * 8),
                ("values", ctypes.c_void_p), ("n_values", ctypes.c_int64)]


class Options(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("c_kappa", ctypes.c_double), ("c_h", ctypes.c_double),
                ("tau_w", ctypes.c_double), ("n_v", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("compensation", ctypes.c_int32), ("radius_rule", ctypes.c_int32),
                ("max_steps", ctypes.c_int64), ("stream", ctypes.c_void_p), ("device_io", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("lanes_per_walk", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("k_spacing", ctypes.c_int32), ("walk_S", ctypes.c_void_p), ("walk_K", ctypes.c_void_p),
                ("kappa_bound", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("walk_steps", ctypes.c_int64), ("truncated", ctypes.c_int64), ("k_max", ctypes.c_int32),
                ("k_mean", ctypes.c_double), ("seconds", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("k_p50", ctypes.c_int32), ("k_p99", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("manifold", ctypes.c_void_p), ("f", Fn), ("g", Fn), ("has_g", ctypes.c_int32),
                ("c", ctypes.c_double), ("queries", ctypes.c_void_p), ("n_queries", ctypes.c_int64),
                ("n_walks", ctypes.c_int64), ("eps", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("opt", Options), ("u_out", ctypes.c_void_p), ("stderr_out", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("admitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("walk_steps", ctypes.c_int64), ("busy_seconds", ctypes.c_double),
                ("in_flight_bytes", ctypes.c_int64), ("rounds", ctypes.c_int32)]


EXPORTS = ["mpwos_options_default", "mpwos_manifold_create", "mpwos_manifold_destroy", "mpwos_solve",
           "mpwos_last_error", "mpwos_server_create", "mpwos_submit", "mpwos_poll", "mpwos_wait",
           "mpwos_request_times",
           "mpwos_server_stats_get", "mpwos_server_destroy", "mpwos_debug_cp", "mpwos_debug_cloud_info",
           "mpwos_debug_radial_inv",
           "mpwos_debug_philox", "mpwos_copy_probe", "mpwos_valu_probe", "mpwos_version",
           "mpwos_plan_create", "mpwos_plan_execute", "mpwos_plan_stats", "mpwos_plan_destroy", "mpwos_autotune",
           "mpwos_predictor_fit", "mpwos_debug_ts_fit", "mpwos_solve_noalloc"]

_lib = None


def lib():
    """Loads libmpwos.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        # Load torch's HIP runtime first when torch is installed: the library
        # then binds to that same runtime (one HIP runtime per process, so
        # torch device pointers and streams are valid in both).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with paper_2606_21883_amd/build.py")
        L = ctypes.CDLL(LIBPATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.mpwos_options_default.argtypes = [vp]
        L.mpwos_options_default.restype = None
        L.mpwos_manifold_create.argtypes = [vp, vp]
        L.mpwos_manifold_destroy.argtypes = [vp]
        L.mpwos_solve.argtypes = [vp, vp, vp, d, vp, i64, i64, d, ctypes.c_uint64, vp, vp, vp, vp]
        L.mpwos_solve_noalloc.argtypes = [vp, vp, vp, d, vp, i64, i64, d, ctypes.c_uint64, vp, vp, vp, vp]
        L.mpwos_last_error.restype = ctypes.c_char_p
        L.mpwos_version.restype = ctypes.c_char_p
        L.mpwos_server_create.argtypes = [ctypes.c_size_t, i64, vp]
        L.mpwos_submit.argtypes = [vp, vp, vp]
        L.mpwos_poll.argtypes = [vp, ctypes.c_uint64, vp, vp]
        L.mpwos_wait.argtypes = [vp, ctypes.c_uint64, i64, vp]
        L.mpwos_request_times.argtypes = [vp, ctypes.c_uint64, vp]
        L.mpwos_server_stats_get.argtypes = [vp, vp]
        L.mpwos_server_destroy.argtypes = [vp]
        L.mpwos_debug_cp.argtypes = [vp, vp, i64, i32, vp]
        L.mpwos_debug_cloud_info.argtypes = [vp, vp, vp]
        L.mpwos_debug_radial_inv.argtypes = [i32, d, vp, i64, i32, vp]
        L.mpwos_debug_philox.argtypes = [vp, ctypes.c_uint64, i64, vp]
        L.mpwos_copy_probe.argtypes = [i64, i32, vp]
        L.mpwos_valu_probe.argtypes = [i32, vp]
        L.mpwos_plan_create.argtypes = [vp, vp, vp, d, i64, i64, d, vp, vp]
        L.mpwos_plan_execute.argtypes = [vp, vp, vp, vp, ctypes.c_uint64, vp]
        L.mpwos_plan_stats.argtypes = [vp, vp, vp]
        L.mpwos_plan_destroy.argtypes = [vp]
        L.mpwos_autotune.argtypes = [vp, vp, vp, d, vp, i64, i64, d, vp, vp, vp]
        L.mpwos_predictor_fit.argtypes = [vp, vp, vp, d, d, ctypes.c_uint64, vp, i32, i32, i64, i32, i32, vp, vp]
        L.mpwos_debug_ts_fit.argtypes = [vp, i32, i32, i32, i32, vp]
        for nm in EXPORTS:
            if nm not in ("mpwos_options_default", "mpwos_last_error", "mpwos_version"):
                getattr(L, nm).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error():
    return lib().mpwos_last_error().decode()


def _check(st):
    if st < 0:
        raise MpwosError(st, last_error())
    return st


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def options_default():
    o = Options()
    lib().mpwos_options_default(ctypes.byref(o))
    return o


def make_options(prob=None, **kw):
    """Options from a problem dict (theta, c_kappa, ...) plus keyword overrides."""
    o = options_default()
    src = dict(prob or {})
    src.update(kw)
    for k in ("theta", "c_kappa", "c_h", "tau_w", "kappa_bound"):
        if k in src:
            setattr(o, k, float(src[k]))
    if "n_v" in src:
        o.n_v = int(src["n_v"])
    if "max_steps" in src:
        o.max_steps = int(src["max_steps"])
    if "compensation" in src:
        o.compensation = COMP[src["compensation"]]
    if "radius_rule" in src:
        o.radius_rule = RADIUS_RULES[src["radius_rule"]]
    if "precision" in src:
        o.precision = PRECISION[src["precision"]] if isinstance(src["precision"], str) else int(src["precision"])
    for k in ("block_size", "lanes_per_walk", "persistent", "newton_iters", "device_io"):
        if k in src:
            setattr(o, k, int(src[k]))
    if "stream" in src and src["stream"] is not None:
        o.stream = ctypes.c_void_p(int(src["stream"]))
    return o


def has_boundary(prob):
    return prob["manifold"] in ("sphere_cap", "cut_torus")


def source_fn(prob):
    """The f record of a problem dict.  A TORUS_SINE source under the
    second-order compensation carries the predictor's rows after u's (both
    padded to one th width) and h_eta in coef[0]."""
    f = prob.get("f", {"kind": "zero"})
    if f["kind"] != "torus_sine" or prob.get("compensation") != "second_order" or "predictor" not in prob:
        return f
    ks, kt = (int(v) for v in f["idx"][:2])
    pk, pt = (int(v) for v in prob["predictor"]["idx"][:2])
    w = 2 * max(kt, pt) + 1
    rows = np.zeros((ks + pk, w))
    rows[:ks, :2 * kt + 1] = np.asarray(f["values"], dtype=np.float64).reshape(ks, 2 * kt + 1)
    rows[ks:, :2 * pt + 1] = np.asarray(prob["predictor"]["values"], dtype=np.float64).reshape(pk, 2 * pt + 1)
    return {"kind": "torus_sine", "idx": [ks, max(kt, pt), pk], "coef": [float(prob.get("h_eta", 1e-2))],
            "values": rows.ravel()}


def make_fn(d, keep):
    f = Fn()
    if d is None:
        return None
    f.kind = FN_KINDS[d["kind"]]
    for i, v in enumerate(d.get("idx", [])):
        f.idx[i] = int(v)
    for i, v in enumerate(d.get("coef", [])):
        f.coef[i] = float(v)
    if "values" in d:
        vals = np.ascontiguousarray(d["values"], dtype=np.float64)
        keep.append(vals)
        f.values = vals.ctypes.data
        f.n_values = vals.size
    return f


class Manifold:
    """Owns an mpwos_manifold handle."""

    def __init__(self, prob):
        self._keep = []
        d = ManifoldDesc()
        d.kind = KINDS[prob["manifold"]]
        d.n = int(prob["n"])
        for i, v in enumerate(prob.get("p", [1.0])):
            d.p[i] = float(v)
        if prob["manifold"] == "point_cloud":
            pts = np.ascontiguousarray(prob["points"], dtype=np.float32)
            self._keep.append(pts)
            d.points = pts.ctypes.data
            d.n_points = pts.shape[0]
            d.k_nn = int(prob.get("k_nn", 16))
            d.reconstruction = RECONSTRUCTIONS[prob.get("reconstruction", "patch")]
            d.fit_scale = float(prob.get("fit_scale", 1.0))
        self.handle = ctypes.c_void_p()
        _check(lib().mpwos_manifold_create(ctypes.byref(d), ctypes.byref(self.handle)))
        self._keep = []

    def close(self):
        if self.handle:
            _check(lib().mpwos_manifold_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.mpwos_manifold_destroy(self.handle)
        except Exception:
            pass


def manifold_create(prob):
    return Manifold(prob)


def manifold_destroy(m):
    m.close()


def solve(prob, queries, n_walks, seed, manifold=None, walk_outputs=False, **optkw):
    """mpwos_solve for a problem dict; returns dict(u, stderr, stats, status[, walk_S, walk_K])."""
    own = manifold is None
    m = Manifold(prob) if own else manifold
    keep = []
    Q = np.ascontiguousarray(queries, dtype=np.float64)
    nq = Q.shape[0]
    f = make_fn(source_fn(prob), keep)
    g = make_fn(prob.get("g"), keep) if has_boundary(prob) else None
    o = make_options(prob, **optkw)
    u = np.zeros(nq)
    se = np.zeros(nq)
    st = Stats()
    out = {}
    if walk_outputs:
        wS = np.zeros((nq, int(n_walks)))
        wK = np.zeros((nq, int(n_walks)), dtype=np.int32)
        o.walk_S = wS.ctypes.data
        o.walk_K = wK.ctypes.data
        out.update(walk_S=wS, walk_K=wK)
    rc = lib().mpwos_solve(m.handle, ctypes.byref(f), ctypes.byref(g) if g is not None else None,
                           float(prob["sigma"]), _ptr(Q), nq, int(n_walks), float(prob.get("eps", 1e-3)),
                           int(seed), ctypes.byref(o), _ptr(u), _ptr(se), ctypes.byref(st))
    if own:
        m.close()
    _check(rc)
    out.update(u=u, stderr=se, status=STATUS_NAMES[rc],
               stats={k: getattr(st, k) for k, _ in Stats._fields_})
    return out


def solve_device(manifold, prob, queries_ptr, nq, n_walks, seed, u_ptr, se_ptr, stream=None, **optkw):
    """mpwos_solve with device-resident queries and outputs (raw device pointers)."""
    keep = []
    f = make_fn(source_fn(prob), keep)
    g = make_fn(prob.get("g"), keep) if has_boundary(prob) else None
    o = make_options(prob, device_io=1, stream=stream, **optkw)
    st = Stats()
    rc = lib().mpwos_solve(manifold.handle, ctypes.byref(f), ctypes.byref(g) if g is not None else None,
                           float(prob["sigma"]), ctypes.c_void_p(queries_ptr), int(nq), int(n_walks),
                           float(prob.get("eps", 1e-3)), int(seed), ctypes.byref(o), ctypes.c_void_p(u_ptr),
                           ctypes.c_void_p(se_ptr) if se_ptr else None, ctypes.byref(st))
    _check(rc)
    return {k: getattr(st, k) for k, _ in Stats._fields_}


def solve_noalloc(manifold, prob, queries_ptr, nq, n_walks, seed, u_ptr, se_ptr, stream=None, walk_S_ptr=None,
                  walk_K_ptr=None, **optkw):
    """mpwos_solve_noalloc: device queries and outputs (raw device pointers),
    no device allocation in the call."""
    keep = []
    f = make_fn(source_fn(prob), keep)
    g = make_fn(prob.get("g"), keep) if has_boundary(prob) else None
    o = make_options(prob, stream=stream, **optkw)
    if walk_S_ptr:
        o.walk_S = int(walk_S_ptr)
        o.walk_K = int(walk_K_ptr)
    st = Stats()
    rc = lib().mpwos_solve_noalloc(manifold.handle, ctypes.byref(f), ctypes.byref(g) if g is not None else None,
                                   float(prob["sigma"]), ctypes.c_void_p(queries_ptr), int(nq), int(n_walks),
                                   float(prob.get("eps", 1e-3)), int(seed), ctypes.byref(o), ctypes.c_void_p(u_ptr),
                                   ctypes.c_void_p(se_ptr) if se_ptr else None, ctypes.byref(st))
    _check(rc)
    return {k: getattr(st, k) for k, _ in Stats._fields_}


def debug_cp(manifold, x, precision="fp64"):
    X = np.ascontiguousarray(x, dtype=np.float64)
    Y = np.zeros_like(X)
    _check(lib().mpwos_debug_cp(manifold.handle, _ptr(X), X.shape[0], PRECISION[precision], _ptr(Y)))
    return Y


def debug_cloud_info(manifold):
    fb = ctypes.c_int64()
    h = ctypes.c_double()
    _check(lib().mpwos_debug_cloud_info(manifold.handle, ctypes.byref(fb), ctypes.byref(h)))
    return {"knn_fallback_points": fb.value, "max_spacing": h.value}


def debug_radial_inv(n, X, u, precision="fp64"):
    U = np.ascontiguousarray(u, dtype=np.float64)
    S = np.zeros_like(U)
    _check(lib().mpwos_debug_radial_inv(int(n), float(X), _ptr(U), U.size, PRECISION[precision], _ptr(S)))
    return S


def debug_philox(ctr, seed, count):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros((int(count), 4), dtype=np.uint32)
    _check(lib().mpwos_debug_philox(_ptr(c), int(seed), int(count), _ptr(out)))
    return out


def copy_probe(nbytes, reps):
    ms = ctypes.c_double()
    _check(lib().mpwos_copy_probe(int(nbytes), int(reps), ctypes.byref(ms)))
    return ms.value


VALU_OPS = ["fma_f32", "fma_f64", "mad_u64_u32", "mul_hi_u32", "log_f32", "sin_f32", "sqrt_f32", "rsq_f32",
            "rcp_f32", "xor_b32", "add_f64",
            "sin_f32+3fma", "mad_u64_u32+3fma", "bitop3_b32"]


def valu_probe(op):
    """Lane-operations per second of one VALU operation (name from VALU_OPS)."""
    r = ctypes.c_double()
    _check(lib().mpwos_valu_probe(VALU_OPS.index(op), ctypes.byref(r)))
    return r.value


def version():
    return lib().mpwos_version().decode()


class Plan:
    """mpwos_plan_*: one solve shape captured in a HIP graph; execute() replays
    it for device-resident queries and outputs (raw device pointers)."""

    def __init__(self, manifold, prob, n_queries, n_walks, **optkw):
        self._keep = []
        f = make_fn(source_fn(prob), self._keep)
        g = make_fn(prob.get("g"), self._keep) if has_boundary(prob) else None
        o = make_options(prob, **optkw)
        self.handle = ctypes.c_void_p()
        _check(lib().mpwos_plan_create(manifold.handle, ctypes.byref(f), ctypes.byref(g) if g is not None else None,
                                       float(prob["sigma"]), int(n_queries), int(n_walks),
                                       float(prob.get("eps", 1e-3)), ctypes.byref(o), ctypes.byref(self.handle)))

    def execute(self, queries_ptr, u_ptr, se_ptr, seed, stream=None):
        _check(lib().mpwos_plan_execute(self.handle, ctypes.c_void_p(queries_ptr), ctypes.c_void_p(u_ptr),
                                        ctypes.c_void_p(se_ptr) if se_ptr else None, int(seed),
                                        ctypes.c_void_p(int(stream)) if stream else None))

    def stats(self, stream=None):
        st = Stats()
        rc = lib().mpwos_plan_stats(self.handle, ctypes.c_void_p(int(stream)) if stream else None, ctypes.byref(st))
        _check(rc)
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    def close(self):
        if self.handle:
            _check(lib().mpwos_plan_destroy(self.handle))
            self.handle = ctypes.c_void_p()


def autotune(prob, queries, n_walks, manifold=None, **optkw):
    """mpwos_autotune: returns (options dict of the fastest launch shape, its kernel ms)."""
    own = manifold is None
    m = Manifold(prob) if own else manifold
    keep = []
    Q = np.ascontiguousarray(queries, dtype=np.float64)
    f = make_fn(source_fn(prob), keep)
    g = make_fn(prob.get("g"), keep) if has_boundary(prob) else None
    o = make_options(prob, **optkw)
    best = Options()
    ms = ctypes.c_double()
    rc = lib().mpwos_autotune(m.handle, ctypes.byref(f), ctypes.byref(g) if g is not None else None,
                              float(prob["sigma"]), _ptr(Q), Q.shape[0], int(n_walks),
                              float(prob.get("eps", 1e-3)), ctypes.byref(o), ctypes.byref(best), ctypes.byref(ms))
    if own:
        m.close()
    _check(rc)
    return {"block_size": best.block_size, "lanes_per_walk": best.lanes_per_walk,
            "persistent": best.persistent}, ms.value


class Server:
    """mpwos_server_*: continuous batching of solves on one device.

    Arrays handed to submit() are kept alive here until the request is
    collected with wait()."""

    def __init__(self, hbm_budget_bytes, slice_walk_steps=0):
        self.handle = ctypes.c_void_p()
        _check(lib().mpwos_server_create(int(hbm_budget_bytes), int(slice_walk_steps), ctypes.byref(self.handle)))
        self._live = {}

    def submit(self, manifold, prob, queries, n_walks, seed, **optkw):
        keep = []
        Q = np.ascontiguousarray(queries, dtype=np.float64)
        req = Request()
        req.manifold = manifold.handle
        req.f = make_fn(source_fn(prob), keep)
        if has_boundary(prob):
            req.g = make_fn(prob["g"], keep)
            req.has_g = 1
        req.c = float(prob["sigma"])
        req.queries = Q.ctypes.data
        req.n_queries = Q.shape[0]
        req.n_walks = int(n_walks)
        req.eps = float(prob.get("eps", 1e-3))
        req.seed = int(seed)
        req.opt = make_options(prob, **optkw)
        u = np.zeros(Q.shape[0])
        se = np.zeros(Q.shape[0])
        req.u_out = u.ctypes.data
        req.stderr_out = se.ctypes.data
        t = ctypes.c_uint64()
        _check(lib().mpwos_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._live[t.value] = (Q, u, se, keep, req)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int32()
        res = ctypes.c_int32()
        _check(lib().mpwos_poll(self.handle, int(ticket), ctypes.byref(done), ctypes.byref(res)))
        return bool(done.value), res.value

    def wait(self, ticket, timeout_ms=-1):
        res = ctypes.c_int32()
        _check(lib().mpwos_wait(self.handle, int(ticket), int(timeout_ms), ctypes.byref(res)))
        Q, u, se, keep, req = self._live.pop(ticket)
        _check(res.value)
        return {"u": u, "stderr": se, "status": STATUS_NAMES[res.value]}

    def times(self, ticket):
        """Timeline of a request (seconds since the server was created; -1 if
        not reached): submitted, admitted, first launch, walks done, delivered."""
        t = (ctypes.c_double * 5)()
        _check(lib().mpwos_request_times(self.handle, int(ticket), t))
        return dict(zip(("submitted", "admitted", "first_launch", "walks_done", "delivered"), list(t)))

    def stats(self):
        st = ServerStats()
        _check(lib().mpwos_server_stats_get(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            _check(lib().mpwos_server_destroy(self.handle))
            self.handle = ctypes.c_void_p()


def server_create(hbm_budget_bytes, slice_walk_steps=0):
    return Server(hbm_budget_bytes, slice_walk_steps)


def predictor_fit(prob, nt, ns, n_walks, seed, ks, kt, manifold=None, **optkw):
    """mpwos_predictor_fit: coarse baseline solve at the (th, s) nodes and the
    Fourier-sine fit; returns (coef (ks, 2 kt + 1), stats)."""
    own = manifold is None
    m = Manifold(prob) if own else manifold
    keep = []
    f = make_fn(prob.get("f", {"kind": "zero"}), keep)
    g = make_fn(prob.get("g"), keep)
    o = make_options(prob, **optkw)
    coef = np.zeros(ks * (2 * kt + 1))
    st = Stats()
    rc = lib().mpwos_predictor_fit(m.handle, ctypes.byref(f), ctypes.byref(g) if g is not None else None,
                                   float(prob["sigma"]),
                                   float(prob.get("eps", 1e-3)), int(seed), ctypes.byref(o), int(nt), int(ns),
                                   int(n_walks), int(ks), int(kt), _ptr(coef), ctypes.byref(st))
    if own:
        m.close()
    _check(rc)
    return coef.reshape(ks, 2 * kt + 1), {k: getattr(st, k) for k, _ in Stats._fields_}


def debug_ts_fit(U, ks, kt):
    """The device fit alone: node values U (nt, ns - 1) to (ks, 2 kt + 1) coefficients."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    coef = np.zeros(ks * (2 * kt + 1))
    _check(lib().mpwos_debug_ts_fit(_ptr(U), U.shape[0], U.shape[1] + 1, int(ks), int(kt), _ptr(coef)))
    return coef.reshape(ks, 2 * kt + 1)
