// Device building blocks of the MPWoS walk for gfx950: the Philox4x32-10
// counter-based stream, uniform and Gaussian maps, the screening weights, the
// radial law of the Green density and its inverse, closest-point maps and the
// source / compensation families.  Everything here is templated on the walk
// precision T (float for the mixed mode, double for the plain mode); the
// screening weight W, the weights c and omega and the score S stay FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_args.h"

namespace mpwos {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): each round multiplies words 0 and 2
// by the two Philox constants (full 64-bit products), mixes the high halves
// with the other words and the round key; the key advances by the Weyl
// increments between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)c0 * 0xD2511F53ull;
    const uint64_t m1 = (uint64_t)c2 * 0xCD9E8D57ull;
    const uint32_t a = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
    const uint32_t b = (uint32_t)m1;
    const uint32_t c = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
    const uint32_t d = (uint32_t)m0;
    c0 = a; c1 = b; c2 = c; c3 = d;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

struct Stream {
  uint32_t q, w, k0, k1;
  __device__ __forceinline__ uint4 block(uint32_t step, uint32_t sub, uint32_t blk) const {
    return philox(q, w, step, (sub << 24) | blk, k0, k1);
  }
};

// 32-bit word -> uniform in (0,1).  FP64: (x + 1/2) 2^-32.  FP32: the top 23
// bits, (x>>9 + 1/2) 2^-23, exact in binary32.
__device__ __forceinline__ double u01_64(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }
__device__ __forceinline__ float u01_32(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 0x1p-23f; }

template <class T> __device__ __forceinline__ T u01(uint32_t x);
template <> __device__ __forceinline__ double u01<double>(uint32_t x) { return u01_64(x); }
template <> __device__ __forceinline__ float u01<float>(uint32_t x) { return u01_32(x); }

// Box-Muller on one word pair.
__device__ __forceinline__ void box_muller(uint32_t x0, uint32_t x1, double& g0, double& g1) {
  const double rad = sqrt(-2.0 * log(u01_64(x0)));
  const double ang = 6.283185307179586 * u01_64(x1);
  double sn, cs;
  sincos(ang, &sn, &cs);
  g0 = rad * cs;
  g1 = rad * sn;
}
__device__ __forceinline__ void box_muller(uint32_t x0, uint32_t x1, float& g0, float& g1) {
  // v_log_f32 is log2; v_sin_f32 / v_cos_f32 take their argument in turns.
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u01_32(x0)));
  const float t = u01_32(x1);
  g0 = rad * __builtin_amdgcn_cosf(t);
  g1 = rad * __builtin_amdgcn_sinf(t);
}

// ---------------------------------------------------------------------------
// precision helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double log_(double x) { return log(x); }
__device__ __forceinline__ float log_(float x) { return 0.6931471805599453f * __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double abs_(double x) { return fabs(x); }
__device__ __forceinline__ float abs_(float x) { return fabsf(x); }

template <class T> __device__ __forceinline__ T ipow(T x, int e) {
  T r = (T)1;
  while (e > 0) {
    if (e & 1) r *= x;
    x *= x;
    e >>= 1;
  }
  return r;
}

// Neumaier compensated add.
__device__ __forceinline__ void kahan_add(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// ---------------------------------------------------------------------------
// Screening factor and volume weight for a radius that varies per step
// (Lemma 3.1 series; eq. omega_explicit_formula).  s1 = sum_{j>=1}
// (sigma r^2/4)^j / (j! (nu+1)_j);  c = 1/(1+s1);  omega = s1/(sigma(1+s1)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void weights(const WalkArgs& a, double r, double& c, double& om) {
  const double q = 0.25 * a.sigma * r * r;
  double term = 1.0, s1 = 0.0;
  for (int j = 1; j < 64; ++j) {
    term = term * q / ((double)j * (a.law.nu + (double)j));
    s1 += term;
    if (term <= 1e-18 * s1) break;
  }
  c = 1.0 / (1.0 + s1);
  om = s1 / (a.sigma * (1.0 + s1));
}

// ---------------------------------------------------------------------------
// Radial law of the normalised Green density, in s = t/r, with X = sqrt(sigma) r:
//   F(s) = norm [ t1/(1+t1) + X^2 s^2 S_{nu+1}(Xs)/(2(nu+1)) D(s) ],  t1 = S_nu(Xs) - 1
//   F'(s) = norm X^2 s S_nu(Xs) D(s)
// (flux of the Green function of the ball through the sphere of radius t).
// ---------------------------------------------------------------------------
template <class T>
struct RadialEval {
  T F, pdf;
};

// Law with X folded in (constant radius).
template <class T>
__device__ __forceinline__ RadialEval<T> radial_eval_fixed(const RadialLaw& L, const RadialFixed& R, T s) {
  const T z = s * s;
  T t1 = (T)0, S1 = (T)0, D = (T)0;
  for (int j = L.js - 1; j >= 1; --j) t1 = (t1 + (T)R.A[j]) * z;
  for (int j = L.js - 1; j >= 0; --j) S1 = S1 * z + (T)R.A1[j];
  for (int j = L.jd - 1; j >= 0; --j) D = D * z + (T)R.B[j];
  const T s2nu = ipow(s, L.n - 2);
  D -= s2nu * (T)R.Q1;
  if (L.nu_int >= 0) D -= (T)R.L * s2nu * log_(s);
  RadialEval<T> e;
  const T X2 = (T)R.X2;
  e.F = (T)R.norm * (t1 / ((T)1 + t1) + X2 * z * S1 * (T)L.inv_2nu1 * D);
  e.pdf = (T)R.norm * X2 * s * ((T)1 + t1) * D;
  return e;
}

// Law for a radius that varies per step (coefficients scaled on the fly).
__device__ __forceinline__ RadialEval<double> radial_eval_var(const RadialLaw& L, double X2, double norm, double s) {
  const double z = s * s;
  double t1 = 0.0, S1 = 0.0, Dz = 0.0, Q1 = 0.0, Lg = 0.0;
  double xp = 1.0, zp = 1.0;
  const int jm = L.js > L.jd ? L.js : L.jd;
  for (int j = 0; j < jm; ++j) {
    if (j > 0) { xp *= X2; zp *= z; }
    if (j < L.js) {
      if (j > 0) t1 += L.alpha[j] * xp * zp;
      S1 += L.alpha1[j] * xp * zp;
    }
    if (j < L.jd) {
      const double b = L.bd[j] * xp;
      if (j == L.nu_int) Lg = b;
      else { Dz += b * zp; Q1 += b; }
    }
  }
  const double s2nu = ipow(s, L.n - 2);
  double D = Dz - s2nu * Q1;
  if (L.nu_int >= 0) D -= Lg * s2nu * log(s);
  RadialEval<double> e;
  e.F = norm * (t1 / (1.0 + t1) + X2 * z * S1 * L.inv_2nu1 * D);
  e.pdf = norm * X2 * s * (1.0 + t1) * D;
  return e;
}

// 1/(1-c) for a given X^2 (varying radius).
__device__ __forceinline__ double radial_norm(const RadialLaw& L, double X2) {
  double t = 0.0, xp = 1.0;
  for (int j = 1; j < L.js; ++j) { xp *= X2; t += L.alpha[j] * xp; }
  return (1.0 + t) / t;
}

// Table guess for s(u): slice of X^2 (nearest below, linear blend) and linear
// interpolation in u; also returns the u-cell bracket of the fixed-X table.
__device__ __forceinline__ double table_guess64(const InvTable& t, double u, double X2, double& lo, double& hi) {
  const double pos = u * (double)(t.mu - 1);
  int i = (int)pos;
  i = i < 0 ? 0 : (i > t.mu - 2 ? t.mu - 2 : i);
  const double fr = pos - (double)i;
  if (t.mx == 1) {
    lo = t.s64[i];
    hi = t.s64[i + 1];
    return lo + fr * (hi - lo);
  }
  const double xpos = X2 / t.x2max * (double)(t.mx - 1);
  int k = (int)xpos;
  k = k < 0 ? 0 : (k > t.mx - 2 ? t.mx - 2 : k);
  const double fx = xpos - (double)k;
  const double* a = t.s64 + (size_t)k * t.mu;
  const double* b = a + t.mu;
  const double ga = a[i] + fr * (a[i + 1] - a[i]);
  const double gb = b[i] + fr * (b[i + 1] - b[i]);
  lo = 0.0;
  hi = 1.0;
  return ga + fx * (gb - ga);
}

__device__ __forceinline__ float table_guess32(const InvTable& t, float u, float X2) {
  const float pos = u * (float)(t.mu - 1);
  int i = (int)pos;
  i = i < 0 ? 0 : (i > t.mu - 2 ? t.mu - 2 : i);
  const float fr = pos - (float)i;
  if (t.mx == 1) return t.s32[i] + fr * (t.s32[i + 1] - t.s32[i]);
  const float xpos = X2 / (float)t.x2max * (float)(t.mx - 1);
  int k = (int)xpos;
  k = k < 0 ? 0 : (k > t.mx - 2 ? t.mx - 2 : k);
  const float fx = xpos - (float)k;
  const float* a = t.s32 + (size_t)k * t.mu;
  const float* b = a + t.mu;
  const float ga = a[i] + fr * (a[i + 1] - a[i]);
  const float gb = b[i] + fr * (b[i + 1] - b[i]);
  return ga + fx * (gb - ga);
}

// Inverse of the radial CDF in FP64: safeguarded Newton (bisection when a step
// leaves the bracket) from the table guess, to a relative step of 2^-52.
__device__ __forceinline__ double radial_inv64(const WalkArgs& a, double u, double X2, double norm) {
  double lo, hi;
  double s = table_guess64(a.tab, u, X2, lo, hi);
  const bool fixed = a.const_r != 0;
  if (fixed) {
    lo = lo * (1.0 - 1e-12);
    hi = fmin(1.0, hi * (1.0 + 1e-12));
  }
  s = fmin(fmax(s, lo), hi);
  for (int it = 0; it < 40; ++it) {
    if (!(s > 0.0)) s = 0.5 * (lo + hi);
    const RadialEval<double> e = fixed ? radial_eval_fixed<double>(a.law, a.fixed, s) : radial_eval_var(a.law, X2, norm, s);
    if (e.F < u) lo = s; else hi = s;
    double sn = s - (e.F - u) / e.pdf;
    if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
    const double ds = fabs(sn - s);
    s = sn;
    if (ds <= 0x1p-52 * s || hi - lo <= 0x1p-53 * hi) break;
  }
  return s;
}

// FP32: table guess and one Newton step with the FP32 law (fixed X), or the
// blended 2-D table alone (varying X).
__device__ __forceinline__ float radial_inv32(const WalkArgs& a, float u, float X2) {
  float s = table_guess32(a.tab, u, X2);
  if (a.const_r) {
    s = fminf(fmaxf(s, 1e-20f), 1.0f);
    const RadialEval<float> e = radial_eval_fixed<float>(a.law, a.fixed, s);
    if (e.pdf > 0.0f) {
      const float sn = s - (e.F - u) / e.pdf;
      if (sn > 0.0f && sn < 1.0f) s = sn;
    }
  }
  return s;
}

// ---------------------------------------------------------------------------
// Closest-point maps (eq. cp_map)
// ---------------------------------------------------------------------------

// Implicit torus phi(x) = (|x|^2 + R^2 - a^2)^2 - 4 R^2 (x1^2 + x2^2).
template <class T>
__device__ __forceinline__ T torus_phi(T R2, T a2, const T* x, T* g, T* H) {
  const T r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  const T s = r2 + R2 - a2;
  const T phi = s * s - (T)4 * R2 * (x[0] * x[0] + x[1] * x[1]);
  g[0] = (T)4 * s * x[0] - (T)8 * R2 * x[0];
  g[1] = (T)4 * s * x[1] - (T)8 * R2 * x[1];
  g[2] = (T)4 * s * x[2];
  if (H) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H[3 * i + j] = (T)8 * x[i] * x[j] + (i == j ? (T)4 * s : (T)0);
    H[0] -= (T)8 * R2;
    H[4] -= (T)8 * R2;
  }
  return phi;
}

// Local Newton solve for the closest point on the implicit torus.  Stage 1:
// safeguarded Newton along the gradient line through x to reach the level set
// (bracketed, so it cannot jump across the core circle).  Stage 2: Newton on
// the Lagrange system y - x + mu grad phi(y) = 0, phi(y) = 0.
template <class T>
__device__ __forceinline__ void torus_cp_newton(T R, T a, const T* x, T* y, int iters) {
  const T R2 = R * R, a2 = a * a;
  T g[3], H[9];
  const T phi0 = torus_phi(R2, a2, x, g, (T*)nullptr);
  T gn = sqrt_(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  T d[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
  // move against the sign of phi along d: y(t) = x - sgn(phi0) t d, t in [0, tmax]
  const T sg = phi0 > (T)0 ? (T)1 : (T)-1;
  T lo = (T)0, hi = (T)2 * a, t = (T)0;
  for (int it = 0; it < 40; ++it) {
    T p[3] = {x[0] - sg * t * d[0], x[1] - sg * t * d[1], x[2] - sg * t * d[2]};
    T gp[3];
    const T ph = torus_phi(R2, a2, p, gp, (T*)nullptr);
    if (ph * sg > (T)0) lo = t; else hi = t;
    const T dph = -sg * (gp[0] * d[0] + gp[1] * d[1] + gp[2] * d[2]);
    T tn = t - ph / dph;
    if (!(tn > lo && tn < hi)) tn = (T)0.5 * (lo + hi);
    const T dt = abs_(tn - t);
    t = tn;
    if (dt <= (T)(sizeof(T) == 8 ? 1e-13 : 1e-6) * a) break;
  }
  for (int i = 0; i < 3; ++i) y[i] = x[i] - sg * t * d[i];
  // stage 2: Lagrange-Newton with Schur complement of the 4x4 system
  torus_phi(R2, a2, y, g, (T*)nullptr);
  const T gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  T mu = ((x[0] - y[0]) * g[0] + (x[1] - y[1]) * g[1] + (x[2] - y[2]) * g[2]) / gg;
  for (int it = 0; it < iters; ++it) {
    const T ph = torus_phi(R2, a2, y, g, H);
    T F1[3];
    for (int i = 0; i < 3; ++i) F1[i] = y[i] - x[i] + mu * g[i];
    // A = I + mu H
    T A[9];
    for (int i = 0; i < 9; ++i) A[i] = mu * H[i];
    A[0] += (T)1; A[4] += (T)1; A[8] += (T)1;
    // adjugate inverse
    T C0 = A[4] * A[8] - A[5] * A[7], C1 = A[5] * A[6] - A[3] * A[8], C2 = A[3] * A[7] - A[4] * A[6];
    T det = A[0] * C0 + A[1] * C1 + A[2] * C2;
    T inv[9] = {C0, A[2] * A[7] - A[1] * A[8], A[1] * A[5] - A[2] * A[4],
                C1, A[0] * A[8] - A[2] * A[6], A[2] * A[3] - A[0] * A[5],
                C2, A[1] * A[6] - A[0] * A[7], A[0] * A[4] - A[1] * A[3]};
    const T id = (T)1 / det;
    T Ag[3], AF[3];
    for (int i = 0; i < 3; ++i) {
      Ag[i] = id * (inv[3 * i] * g[0] + inv[3 * i + 1] * g[1] + inv[3 * i + 2] * g[2]);
      AF[i] = id * (inv[3 * i] * F1[0] + inv[3 * i + 1] * F1[1] + inv[3 * i + 2] * F1[2]);
    }
    const T gAg = g[0] * Ag[0] + g[1] * Ag[1] + g[2] * Ag[2];
    const T gAF = g[0] * AF[0] + g[1] * AF[1] + g[2] * AF[2];
    const T dmu = (ph - gAF) / gAg;
    T dy2 = (T)0;
    for (int i = 0; i < 3; ++i) {
      const T dy = -AF[i] - dmu * Ag[i];
      y[i] += dy;
      dy2 += dy * dy;
    }
    mu += dmu;
    if (dy2 <= (T)(sizeof(T) == 8 ? 1e-32 : 1e-14) * a2) break;
  }
}

// ---------------------------------------------------------------------------
// Sources: f(z) = f_Omega(cp z) (eq. cp_extension) plus the exact
// compensation m(z) = -Lap(Eu)(z) + sigma Eu(z) - f(z) (eq. mismatch_definition)
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T legendre_sum(const double* c, T t) {
  T p0 = (T)1, p1 = t;
  T s = (T)c[0] + (T)c[1] * t;
  for (int l = 1; l < 7; ++l) {
    const T p2 = ((T)(2 * l + 1) * t * p1 - (T)l * p0) / (T)(l + 1);
    s += (T)c[l + 1] * p2;
    p0 = p1;
    p1 = p2;
  }
  return s;
}

template <class T>
__device__ __forceinline__ T legendre_lap(const double* c, double R, double sigma, T t) {
  // sum_l lam_l u_l P_l(t) with u_l = c_l / (lam_l + sigma), lam_l = l(l+1)/R^2
  T p0 = (T)1, p1 = t;
  T s = (T)0;
  const double l1 = 2.0 / (R * R);
  s += (T)(l1 * c[1] / (l1 + sigma)) * t;
  for (int l = 1; l < 7; ++l) {
    const T p2 = ((T)(2 * l + 1) * t * p1 - (T)l * p0) / (T)(l + 1);
    const double lam = (double)((l + 1) * (l + 2)) / (R * R);
    s += (T)(lam * c[l + 1] / (lam + sigma)) * p2;
    p0 = p1;
    p1 = p2;
  }
  return s;
}

// sin(phi) cos(2 psi) structure on a torus of tube radius `tube` around the
// core circle of radius R; cphi.. are the angle cosines / sines.
template <class T>
__device__ __forceinline__ T torus_neg_lap(T R, T tube, T sphi, T cpsi, T spsi) {
  const T rt = R + tube * cpsi;
  const T c2 = cpsi * cpsi - spsi * spsi;
  const T s2 = (T)2 * spsi * cpsi;
  const T u = sphi * c2;
  return (T)4 * u / (tube * tube) + u / (rt * rt) - (T)2 * sphi * spsi * s2 / (tube * rt);
}

// f_Omega(y) + m(z) for a point z of the ball and y = cp(z).
template <class T>
__device__ __forceinline__ T source(const WalkArgs& a, const T* z, const T* y, int n) {
  const FnDev& f = a.f;
  const int comp = a.comp;
  switch (f.kind) {
    case kFnZero: return (T)0;
    case kFnConst: return (T)f.coef[0];
    case kFnSphPair: {
      const T R = (T)a.p[0];
      const T iR = (T)1 / R;
      const T fv = (T)f.coef[0] * (y[f.idx[0]] * iR) * (y[f.idx[1]] * iR);
      if (!comp) return fv;
      T zz = (T)0;
      for (int i = 0; i < n; ++i) zz += z[i] * z[i];
      return fv + (T)(f.lam * f.u_scale) * fv * (R * R / zz - (T)1);
    }
    case kFnCircle: {
      const T R = (T)a.p[0];
      const T iR = (T)1 / R;
      // cos(k th), sin(k th) from the unit vector by the angle-addition recurrence
      const T cx = y[0] * iR, sx = y[1] * iR;
      T ck = (T)1, sk = (T)0;
      for (int j = 0; j < f.idx[0]; ++j) {
        const T cn = ck * cx - sk * sx;
        sk = sk * cx + ck * sx;
        ck = cn;
      }
      const T fv = (T)f.coef[0] * ck + (T)f.coef[1] * sk;
      if (!comp) return fv;
      const T zz = z[0] * z[0] + z[1] * z[1];
      return fv + (T)(f.lam * f.u_scale) * fv * (R * R / zz - (T)1);
    }
    case kFnLegendre: {
      const T R = (T)a.p[0];
      const T t = y[n - 1] / R;
      const T fv = legendre_sum<T>(f.coef, t);
      if (!comp) return fv;
      T zz = (T)0;
      for (int i = 0; i < n; ++i) zz += z[i] * z[i];
      return fv + legendre_lap<T>(f.coef, a.p[0], a.sigma, t) * (R * R / zz - (T)1);
    }
    case kFnTorus: {
      const T R = (T)a.p[0], tube = (T)a.p[1];
      // angles of y on the torus (those of z are the same: cp keeps phi and psi)
      const T rho = sqrt_(y[0] * y[0] + y[1] * y[1]);
      const T sphi = y[1] / rho;
      const T dr = rho - R;
      const T dy = sqrt_(dr * dr + y[2] * y[2]);
      const T cpsi = dr / dy, spsi = y[2] / dy;
      const T u = sphi * (cpsi * cpsi - spsi * spsi);
      const T c0 = (T)f.coef[0];
      const T nl = torus_neg_lap<T>(R, tube, sphi, cpsi, spsi);
      T v = c0 * nl + (T)a.sigma * c0 * u;
      if (comp) {
        const T rz = sqrt_(z[0] * z[0] + z[1] * z[1]);
        const T dz = sqrt_((rz - R) * (rz - R) + z[2] * z[2]);
        v += c0 * (torus_neg_lap<T>(R, dz, sphi, cpsi, spsi) - nl);
      }
      return v;
    }
    case kFnTableS1: {
      const T R = (T)a.p[0];
      // theta in turns from the unit vector, then linear interpolation
      const double th = atan2((double)y[1], (double)y[0]) * 0.15915494309189535;
      double tt = th - floor(th);
      const double pos = tt * (double)f.m;
      int64_t i0 = (int64_t)floor(pos);
      const double fr = pos - (double)i0;
      i0 %= f.m;
      const int64_t i1 = (i0 + 1) % f.m;
      const double fv = (1.0 - fr) * f.values[i0] + fr * f.values[i1];
      if (!comp) return (T)fv;
      const double us = (1.0 - fr) * f.values[f.m + i0] + fr * f.values[f.m + i1];
      const T zz = z[0] * z[0] + z[1] * z[1];
      return (T)fv + (T)(fv - a.sigma * us) * (R * R / zz - (T)1);
    }
  }
  return (T)0;
}

// g_Omega at a boundary point y.
template <class T>
__device__ __forceinline__ double boundary_value(const WalkArgs& a, const T* y, int n) {
  const FnDev& g = a.g;
  switch (g.kind) {
    case kFnZero: return 0.0;
    case kFnConst: return g.coef[0];
    case kFnSphPair: {
      const double R = a.p[0];
      return g.coef[0] * ((double)y[g.idx[0]] / R) * ((double)y[g.idx[1]] / R);
    }
    case kFnLegendre: return (double)legendre_sum<T>(g.coef, (T)((double)y[n - 1] / a.p[0]));
  }
  return 0.0;
}

}  // namespace mpwos
