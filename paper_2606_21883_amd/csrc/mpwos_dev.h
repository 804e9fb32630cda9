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
// increments between rounds.  Each three-way xor is one gfx950 v_bitop3_b32
// (truth table 0x96: the parity of the three input bits), so a round costs
// two 32x32->64 multiply-adds and two bitwise operations.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3_(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)c0 * 0xD2511F53ull;
    const uint64_t m1 = (uint64_t)c2 * 0xCD9E8D57ull;
    const uint32_t a = xor3_((uint32_t)(m1 >> 32), c1, k0);
    const uint32_t b = (uint32_t)m1;
    const uint32_t c = xor3_((uint32_t)(m0 >> 32), c3, k1);
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
// FP32 form built from the bits: 1 + m 2^-23 (m = x >> 9) minus (1 - 2^-24)
// is (m + 1/2) 2^-23 exactly.  The exponent bits and the shifted word come
// from one funnel shift: ({0x7F, x} >> 9) = 0x3F800000 | (x >> 9).
__device__ __forceinline__ float u01_32(uint32_t x) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0x1.fffffep-1f;
}

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

// Uniform direction on S^{N-1}, N = 2 or 3, from the words of one Philox
// block: the angle 2 pi u0 (N = 2), or Archimedes' hat-box construction
// (N = 3): the last coordinate 1 - 2 u0 is uniform on [-1, 1], the azimuth
// 2 pi u1 is uniform and independent of it, and the radius about the axis is
// sqrt(1 - z^2) = 2 sqrt(u0 (1 - u0)).  Exact, of unit length up to rounding,
// with no normals and no normalisation.
template <int N>
__device__ __forceinline__ void lane_direction(uint32_t x0, uint32_t x1, double* z) {
  if constexpr (N == 2) {
    sincos(6.283185307179586 * u01_64(x0), &z[1], &z[0]);
  } else {
    const double u = u01_64(x0);
    double sn, cs;
    sincos(6.283185307179586 * u01_64(x1), &sn, &cs);
    const double rho = 2.0 * sqrt(u * (1.0 - u));
    z[0] = rho * cs;
    z[1] = rho * sn;
    z[2] = 1.0 - 2.0 * u;
  }
}
template <int N>
__device__ __forceinline__ void lane_direction(uint32_t x0, uint32_t x1, float* z) {
  // v_sin_f32 / v_cos_f32 take their argument in turns
  if constexpr (N == 2) {
    const float t = u01_32(x0);
    z[0] = __builtin_amdgcn_cosf(t);
    z[1] = __builtin_amdgcn_sinf(t);
  } else {
    const float u = u01_32(x0);
    const float t = u01_32(x1);
    const float rho = 2.0f * __builtin_amdgcn_sqrtf(fmaf(-u, u, u));
    z[0] = rho * __builtin_amdgcn_cosf(t);
    z[1] = rho * __builtin_amdgcn_sinf(t);
    z[2] = fmaf(-2.0f, u, 1.0f);
  }
}

// The point Y + s zeta for the direction zeta of lane_direction.  FP64: the
// direction, then the update.  FP32: the same point with the scale folded
// into the hat-box radius, (2s) sqrt(u (1 - u)), and the axis coordinate as
// (Y_3 + s) - 2s u, which saves the separate multiplies by the radius and by
// s (rounding differs from the two-stage form by an ulp or so).
template <int N>
__device__ __forceinline__ void lane_point(uint32_t x0, uint32_t x1, double s, const double* Y, double* out) {
  double zeta[N];
  lane_direction<N>(x0, x1, zeta);
  for (int i = 0; i < N; ++i) out[i] = Y[i] + s * zeta[i];
}
template <int N>
__device__ __forceinline__ void lane_point(uint32_t x0, uint32_t x1, float s, const float* Y, float* out) {
  if constexpr (N == 2) {
    const float t = u01_32(x0);
    out[0] = fmaf(s, __builtin_amdgcn_cosf(t), Y[0]);
    out[1] = fmaf(s, __builtin_amdgcn_sinf(t), Y[1]);
  } else {
    const float u = u01_32(x0);
    const float t = u01_32(x1);
    const float s2 = 2.0f * s;
    const float sr = s2 * __builtin_amdgcn_sqrtf(fmaf(-u, u, u));
    out[0] = fmaf(sr, __builtin_amdgcn_cosf(t), Y[0]);
    out[1] = fmaf(sr, __builtin_amdgcn_sinf(t), Y[1]);
    out[2] = fmaf(-s2, u, Y[2] + s);
  }
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
// a / b: IEEE division in FP64; a times the hardware reciprocal (1 ulp) in FP32
__device__ __forceinline__ double over_(double a, double b) { return a / b; }
__device__ __forceinline__ float over_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
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
// s1 = S_nu(X) - 1 by Horner in z = X^2 = sigma r^2 with the law's
// coefficients alpha_j = 1/(4^j j! (nu+1)_j), kept while alpha_j z^j can
// exceed 1e-18 over the solve's radii: one division per step.
__device__ __forceinline__ void weights(const WalkArgs& a, double r, double& c, double& om) {
  const double z = a.sigma * r * r;
  double s1 = 0.0;
  for (int j = a.law.js - 1; j >= 1; --j) s1 = (s1 + a.law.alpha[j]) * z;
  c = 1.0 / (1.0 + s1);
  om = s1 * c * a.inv_sigma;
}

// The same weights in FP32 (mixed mode): Horner in z = sigma r^2 and c from
// the hardware reciprocal (1 ulp).  All terms are positive, so the float sum
// is accurate to a few ulps at any size.  W and S stay FP64.  For the lane
// kernels' dimensions (n <= 3) the coefficients are compile-time constants
// (alpha_j = 1/(4^j j! (nu+1)_j), nu = (n-2)/2): the first kSeries32 of them
// cover every solve whose series the host cut at kSeries32 + 1 terms
// (alpha_j z^j below 1e-10), sigma r^2 up to about 5, and the first
// kSeries32Short do when the solve's radii keep the first dropped term below
// 2^-30 of the leading one (the cap: sigma r^2 up to 0.16); wider ones and
// lane groups take the solve's float coefficients.
constexpr int kSeries32 = 8;
constexpr int kSeries32Short = 4;

template <int N>
struct SeriesCoef {
  float v[kSeries32 + 1];
  constexpr SeriesCoef() : v() {
    const double nu = 0.5 * (N - 2);
    double al = 1.0;
    v[0] = 1.0f;
    for (int j = 1; j <= kSeries32; ++j) {
      al = al / (4.0 * j * (nu + j));
      v[j] = (float)al;
    }
  }
};

template <int N>
__device__ __forceinline__ void weights32(const WalkArgs& a, float r, float& c, float& om) {
  const float z = (float)a.sigma * r * r;
  float t = 0.0f;
  if (N <= 3 && a.wjs <= kSeries32 + 1) {
    constexpr SeriesCoef<N> K;
    if (a.w32n <= kSeries32Short) {
#pragma unroll
      for (int j = kSeries32Short; j >= 1; --j) t = fmaf(t, z, K.v[j]);
    } else {
#pragma unroll
      for (int j = kSeries32; j >= 1; --j) t = fmaf(t, z, K.v[j]);
    }
  } else {
    for (int j = a.wjs - 1; j >= 1; --j) t = fmaf(t, z, a.wcoef[j]);
  }
  const float s1 = t * z;
  c = __builtin_amdgcn_rcpf(1.0f + s1);
  om = s1 * c * (float)a.inv_sigma;
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

// Table guess for s(u): the half and cell from w = sqrt(min(u, 1-u)), linear
// in w, blended linearly between X^2 slices when the radius varies; for a
// fixed radius it also returns the cell's bracket of the root.
__device__ __forceinline__ double table_guess64(const InvTable& t, double u, double X2, double& lo, double& hi) {
  const bool up = u > 0.5;
  const double w = sqrt(up ? 1.0 - u : u);
  const double pos = w * ((double)(t.mu - 1) * 1.4142135623730951);
  int i = (int)pos;
  i = i < 0 ? 0 : (i > t.mu - 2 ? t.mu - 2 : i);
  const double fr = pos - (double)i;
  if (t.mx == 1) {
    const double* r = t.s64 + (up ? t.mu : 0);
    const double a = r[i], b = r[i + 1];
    lo = a < b ? a : b;
    hi = a < b ? b : a;
    return a + fr * (b - a);
  }
  const double xpos = X2 * t.x2scale;
  int k = (int)xpos;
  k = k < 0 ? 0 : (k > t.mx - 2 ? t.mx - 2 : k);
  const double fx = xpos - (double)k;
  const double* ra = t.s64 + ((size_t)k * 2 + (up ? 1 : 0)) * t.mu;
  const double* rb = ra + 2 * (size_t)t.mu;
  const double ga = ra[i] + fr * (ra[i + 1] - ra[i]);
  const double gb = rb[i] + fr * (rb[i + 1] - rb[i]);
  lo = 0.0;
  hi = 1.0;
  return ga + fx * (gb - ga);
}

__device__ __forceinline__ float table_guess32(const InvTable& t, float u, float X2) {
  const bool up = u > 0.5f;
  const float w = __builtin_amdgcn_sqrtf(up ? 1.0f - u : u);
  const float pos = w * ((float)(t.mu - 1) * 1.41421356f);
  int i = (int)pos;
  i = i < 0 ? 0 : (i > t.mu - 2 ? t.mu - 2 : i);
  const float fr = pos - (float)i;
  // at most 17 x 2 x 1025 entries: 32-bit byte offsets from the table's
  // (uniform) base, so the loads take the scalar base and a 32-bit offset
  const char* base = (const char*)t.s32;
  if (t.mx == 1) {
    const uint32_t o = (uint32_t)((up ? t.mu : 0) + i) * 4u;
    const float a0 = *(const float*)(base + o), a1 = *(const float*)(base + o + 4u);
    return a0 + fr * (a1 - a0);
  }
  const float xpos = X2 * (float)t.x2scale;
  int k = (int)xpos;
  k = k < 0 ? 0 : (k > t.mx - 2 ? t.mx - 2 : k);
  const float fx = xpos - (float)k;
  const uint32_t oa = (uint32_t)((k * 2 + (up ? 1 : 0)) * t.mu + i) * 4u;
  const uint32_t ob = oa + (uint32_t)(2 * t.mu) * 4u;
  const float a0 = *(const float*)(base + oa), a1 = *(const float*)(base + oa + 4u);
  const float b0 = *(const float*)(base + ob), b1 = *(const float*)(base + ob + 4u);
  const float ga = a0 + fr * (a1 - a0);
  const float gb = b0 + fr * (b1 - b0);
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
    hi = fmin(1.0, hi * (1.0 + 1e-12) + 1e-300);
  }
  s = fmin(fmax(s, lo), hi);
  for (int it = 0; it < 40; ++it) {
    if (!(s > 0.0)) s = 0.5 * (lo + hi);
    const RadialEval<double> e = fixed ? radial_eval_fixed<double>(a.law, a.fixed, s) : radial_eval_var(a.law, X2, norm, s);
    const double df = e.F - u;
    if (df == 0.0) break;
    if (df < 0.0) lo = s; else hi = s;
    double sn = s - df / e.pdf;
    if (!(sn >= lo && sn <= hi)) sn = 0.5 * (lo + hi);
    const double ds = fabs(sn - s);
    s = sn;
    if (ds <= 0x1p-51 * s || hi - lo <= 0x1p-52 * hi) break;
  }
  return s;
}

// Inverse of the radial CDF in FP32: the table alone (linear in w, within
// about 1e-6 of the root for every n, below the binary32 resolution of the
// walk's positions at the radii used).
__device__ __forceinline__ float radial_inv32(const WalkArgs& a, float u, float X2) {
  return table_guess32(a.tab, u, X2);
}

// ---------------------------------------------------------------------------
// Closest-point maps (eq. cp_map)
// ---------------------------------------------------------------------------

// Local Newton solve for the closest point on the implicit torus (Sec.
// 2.3.2).  The quartic phi(x) = (|x|^2 + R^2 - a^2)^2 - 4 R^2 (x1^2 + x2^2)
// factors as phi1 phi2 with phi1 = (rho - R)^2 + x3^2 - a^2 and
// phi2 = (rho + R)^2 + x3^2 - a^2 (rho = |(x1, x2)|); phi2 > 0 for a < R, so M
// is the level set {phi1 = 0}.  Newton on it along the gradient,
//   y <- y - phi1(y) grad phi1(y) / |grad phi1(y)|^2,
// in the walk's precision: phi1 is a function of the distance D to the core
// circle, so its gradient lines are the normal lines of M and the iterates
// stay on the normal line through x (each step takes D to (D + a^2/D)/2):
// the limit is cp(x).  Near M phi1 keeps its leading bits (the quartic, a
// product with a term of size 4R^2, cancels to a few bits in FP32 there).
// The iteration stops after the first step shorter than 3e-4 a (FP32) or
// 1e-8 a (FP64): Newton's next step would be below the rounding of y.  At
// walk radii up to 0.9 a it takes 4-6 steps; on the host, in FP32, the result
// lies within 7.5e-7 of the exact projection (median 5e-8).
template <class T>
__device__ __forceinline__ void torus_cp_newton(T R, T a, const T* x, T* y) {
  constexpr bool dbl = sizeof(T) == 8;
  const T a2 = a * a;
  const T tol2 = (T)(dbl ? 1e-16 : 9e-8) * a2;
  y[0] = x[0];
  y[1] = x[1];
  y[2] = x[2];
  for (int it = 0; it < 16; ++it) {
    const T rr = y[0] * y[0] + y[1] * y[1];
    const T irho = rsqrt_(rr);
    const T e = rr * irho - R;                    // rho - R
    const T q = e * e + y[2] * y[2];              // D^2, |grad phi1|^2 = 4 q
    T f = (q - a2) / ((T)4 * q);                  // phi1 / |grad phi1|^2
    const T s2 = (T)4 * f * f * q;                // step length^2 = phi1^2 / |grad phi1|^2
    // trust region a/2: from near the core circle the full step overshoots by
    // about a^2 / (2D) and would cross the x3 axis
    if (s2 > (T)0.25 * a2) f *= (T)0.5 * a * rsqrt_(s2);
    const T ge = (T)2 * e * irho;
    y[0] -= f * ge * y[0];
    y[1] -= f * ge * y[1];
    y[2] -= f * (T)2 * y[2];
    if (s2 <= tol2) break;
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
  return over_((T)4 * u, tube * tube) + over_(u, rt * rt) - over_((T)2 * sphi * spsi * s2, tube * rt);
}

// ---- Fourier-sine series over the cut torus (Example 1's family) ---------
// u(th, s) = sum_{k=1..ks} sin(k s) [c_k0 + sum_{j=1..kt} (c_kj cos j th + d_kj sin j th)],
// rows of 2 kt + 1 coefficients (c_k0, c_k1, d_k1, ...).  Evaluated from the
// unit vectors (cos th, sin th) and (cos s, sin s) by angle addition, j
// outermost: A_j = sum_k c_kj sin(k s), B_j = sum_k d_kj sin(k s) (and the
// same with -k^2 for u_ss), so no per-k array is kept.
template <class T>
struct TsVal {
  T u, ut, utt, uss;
};

template <class T>
__device__ __forceinline__ TsVal<T> ts_eval(const double* c, int ks, int kt, T ct, T st, T cs, T ss) {
  TsVal<T> v{(T)0, (T)0, (T)0, (T)0};
  const int w = 2 * kt + 1;
  T cj = (T)1, sj = (T)0;  // cos(j th), sin(j th)
  for (int j = 0; j <= kt; ++j) {
    T A = (T)0, B = (T)0, A2 = (T)0, B2 = (T)0;
    T sk = ss, ck = cs;  // sin(k s), cos(k s) from k = 1
    for (int k = 1; k <= ks; ++k) {
      const double* row = c + (size_t)(k - 1) * w;
      const T ca = (T)(j == 0 ? row[0] : row[2 * j - 1]);
      const T cb = (T)(j == 0 ? 0.0 : row[2 * j]);
      const T kk = (T)(k * k);
      A = fma(ca, sk, A);
      B = fma(cb, sk, B);
      A2 = fma(-kk * ca, sk, A2);
      B2 = fma(-kk * cb, sk, B2);
      const T sn = sk * cs + ck * ss;
      ck = ck * cs - sk * ss;
      sk = sn;
    }
    const T jj = (T)j;
    v.u += cj * A + sj * B;
    v.ut += jj * (cj * B - sj * A);
    v.utt -= jj * jj * (cj * A + sj * B);
    v.uss += cj * A2 + sj * B2;
    const T cn = cj * ct - sj * st;
    sj = sj * ct + cj * st;
    cj = cn;
  }
  return v;
}

// The same series from a float table staged in LDS by the walk kernel: entry
// (row, j) = (c_rj, d_rj, -k^2 c_rj, -k^2 d_rj) at row (kt + 1) + j, with the
// sines sin(k s), k <= ks <= kTsMaxK, computed once per evaluation and held in
// registers.  FP32 only (the FP64 mode reads the double coefficients).
constexpr int kTsMaxK = 8;
constexpr int kTsLds = 512;

__device__ __forceinline__ TsVal<float> ts_eval_tab(const float4* tab, int ks, int kt, float ct, float st, float cs,
                                                    float ss) {
  float sk[kTsMaxK];
  {
    float sv = ss, cv = cs;
#pragma unroll
    for (int k = 0; k < kTsMaxK; ++k) {
      sk[k] = sv;
      const float sn = sv * cs + cv * ss;
      cv = cv * cs - sv * ss;
      sv = sn;
    }
  }
  TsVal<float> v{0.f, 0.f, 0.f, 0.f};
  const int w = kt + 1;
  float cj = 1.f, sj = 0.f;
  for (int j = 0; j <= kt; ++j) {
    float A = 0.f, B = 0.f, A2 = 0.f, B2 = 0.f;
#pragma unroll
    for (int k = 0; k < kTsMaxK; ++k) {
      if (k < ks) {
        const float4 q = tab[k * w + j];
        A = fmaf(q.x, sk[k], A);
        B = fmaf(q.y, sk[k], B);
        A2 = fmaf(q.z, sk[k], A2);
        B2 = fmaf(q.w, sk[k], B2);
      }
    }
    const float jj = (float)j;
    v.u += cj * A + sj * B;
    v.ut += jj * (cj * B - sj * A);
    v.utt -= jj * jj * (cj * A + sj * B);
    v.uss += cj * A2 + sj * B2;
    const float cn = cj * ct - sj * st;
    sj = sj * ct + cj * st;
    cj = cn;
  }
  return v;
}

// Stages the series of u (and of the predictor, second order) into `tab`.
// Called by every thread of the workgroup; returns whether the table is used
// (uniform: FP32 mode, series family, at most kTsMaxK rows per series and
// kTsLds entries in all).
__device__ __forceinline__ bool ts_stage(const WalkArgs& a, float4* tab) {
  const FnDev& f = a.f;
  if (f.kind != kFnTorusSine) return false;
  const int ks = f.idx[0], kt = f.idx[1], kp = a.comp == kCompSecondOrder ? f.idx[2] : 0;
  const int w = kt + 1, rows = ks + kp;
  if (ks > kTsMaxK || kp > kTsMaxK || rows * w > kTsLds) return false;
  const int stride = 2 * kt + 1;
  for (int e = threadIdx.x; e < rows * w; e += blockDim.x) {
    const int row = e / w, j = e - row * w;
    const int k = row < ks ? row + 1 : row - ks + 1;
    const double* rc = f.values + (size_t)row * stride;
    const float ca = (float)(j == 0 ? rc[0] : rc[2 * j - 1]);
    const float cb = j == 0 ? 0.f : (float)rc[2 * j];
    const float kk = (float)(k * k);
    tab[e] = make_float4(ca, cb, -kk * ca, -kk * cb);
  }
  __syncthreads();
  return true;
}

// Ambient Laplacian of the closest-point extension at distance rho from the
// core circle (the extension does not depend on rho in toroidal
// coordinates); at rho = a, the torus's Laplace-Beltrami operator:
//   L(rho) = u_thth / rho^2 - sin(th) u_th / (rho q) + u_ss / q^2,  q = R + rho cos(th).
template <class T>
__device__ __forceinline__ T ct_lap(T R, T rho, T ct, T st, const TsVal<T>& v) {
  const T q = R + rho * ct;
  return over_(v.utt, rho * rho) - over_(st * v.ut, rho * q) + over_(v.uss, q * q);
}

// f_Omega(y) + m(z) for the series family on the cut torus.  The angles come
// from y (those of z are the same: cp keeps them); z contributes its
// distance rho_z from the core circle.
//   exact m: Lap_T u(y) - Lap(Eu)(z);
//   second order (predictor u_* in the rows after u's, normal step h =
//   coef[0]): with R_*(s) = -L_*(a + s) + sigma u_*(y) - f_Omega(y),
//   m1 = (R_*(h) - R_*(-h)) / (2h), m2 = (R_*(h) - 2 R_*(0) + R_*(-h)) / h^2
//   and m_* = eta m1 + eta^2 m2 / 2, eta = rho_z - a.
// The differences are taken in closed form: L is linear in (u_thth, u_th,
// u_ss) with coefficients 1/rho^2, -sin(th)/(rho q), 1/q^2, and the central
// differences of those at a +- h are rational in a, h and q0 = R + a cos(th):
//   D1[1/rho^2] = -2a / (a^2 - h^2)^2,        D2[1/rho^2] = (6a^2 - 2h^2) / (a^2 (a^2 - h^2)^2),
//   D1[1/q^2]   = -2 q0 c / (q0^2 - h^2c^2)^2, D2[1/q^2]   = (6 q0^2 - 2h^2c^2) c^2 / (q0^2 (q0^2 - h^2c^2)^2),
//   1/(rho q) = (1/rho - c/q) / R with D1[1/rho] = -1/(a^2 - h^2), D2[1/rho] = 2 / (a (a^2 - h^2)),
//   D1[1/q] = -c / (q0^2 - h^2c^2), D2[1/q] = 2c^2 / (q0 (q0^2 - h^2c^2))   (c = cos th).
// These equal the difference quotients exactly but do not cancel, so the
// walk's own precision suffices (the quotients themselves lose
// log10(1/h^2) digits to rounding).
template <class T>
__device__ __forceinline__ T torus_sine_source(const WalkArgs& a, const T* z, const T* y,
                                               const float4* tab = nullptr) {
  const FnDev& f = a.f;
  const T R = (T)a.p[0], tube = (T)a.p[1];
  const T rxy = sqrt_(y[0] * y[0] + y[1] * y[1]);
  const T dr = rxy - R;
  const T idt = rsqrt_(dr * dr + y[2] * y[2]);
  const T ct = dr * idt, st = y[2] * idt;
  const T irxy = rcp_(rxy);
  const T cp = y[0] * irxy, sp = y[1] * irxy;
  const T cc = (T)a.cut_c, sc = (T)a.cut_s;
  const T cs = cp * cc + sp * sc, ss = sp * cc - cp * sc;
  const int ks = f.idx[0], kt = f.idx[1];
  TsVal<T> v;
  if constexpr (sizeof(T) == 4) {
    if (tab) v = ts_eval_tab(tab, ks, kt, ct, st, cs, ss);
    else v = ts_eval<T>(f.values, ks, kt, ct, st, cs, ss);
  } else {
    v = ts_eval<T>(f.values, ks, kt, ct, st, cs, ss);
  }
  const T lap_t = ct_lap<T>(R, tube, ct, st, v);
  const T fv = -lap_t + (T)a.sigma * v.u;
  if (a.comp == kCompNone) return fv;
  const T rz = sqrt_(z[0] * z[0] + z[1] * z[1]);
  const T rho = sqrt_((rz - R) * (rz - R) + z[2] * z[2]);
  if (a.comp == kCompExact) return fv + (lap_t - ct_lap<T>(R, rho, ct, st, v));
  const T h = (T)f.coef[0];
  TsVal<T> w;
  if constexpr (sizeof(T) == 4) {
    if (tab) w = ts_eval_tab(tab + ks * (kt + 1), f.idx[2], kt, ct, st, cs, ss);
    else w = ts_eval<T>(f.values + (size_t)ks * (2 * kt + 1), f.idx[2], kt, ct, st, cs, ss);
  } else {
    w = ts_eval<T>(f.values + (size_t)ks * (2 * kt + 1), f.idx[2], kt, ct, st, cs, ss);
  }
  const T h2 = h * h;
  const T e = tube * tube - h2;                      // a^2 - h^2
  const T q0 = R + tube * ct;
  const T hc2 = h2 * ct * ct;
  const T g = q0 * q0 - hc2;                         // q0^2 - h^2 c^2
  const T ie = rcp_(e), ig = rcp_(g);
  const T d1_r2 = -(T)2 * tube * ie * ie;
  const T d2_r2 = ((T)6 * tube * tube - (T)2 * h2) * ie * ie * rcp_(tube * tube);
  const T d1_q2 = -(T)2 * q0 * ct * ig * ig;
  const T d2_q2 = ((T)6 * q0 * q0 - (T)2 * hc2) * ct * ct * ig * ig * rcp_(q0 * q0);
  const T iR = rcp_(R);
  const T d1_rq = (-ie + ct * ct * ig) * iR;
  const T d2_rq = ((T)2 * ie * rcp_(tube) - (T)2 * ct * ct * ct * ig * rcp_(q0)) * iR;
  const T B = -st * w.ut;
  const T m1 = -(w.utt * d1_r2 + B * d1_rq + w.uss * d1_q2);
  const T m2 = -(w.utt * d2_r2 + B * d2_rq + w.uss * d2_q2);
  const T eta = rho - tube;
  return fv + (eta * m1 + (T)0.5 * eta * eta * m2);
}

// f_Omega(y) + m(z) for a point z of the ball and y = cp(z): the families
// with more state (circle modes, Legendre sums, tabulated S^1 data).
template <class T>
__device__ T source_rich(const WalkArgs& a, const T* z, const T* y, int n) {
  const FnDev& f = a.f;
  const int comp = a.comp;
  switch (f.kind) {
    case kFnCircle: {
      const T R = (T)a.p[0];
      const T iR = (T)a.inv_R;
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
      return fv + (T)(f.lam * f.u_scale) * fv * (over_(R * R, zz) - (T)1);
    }
    case kFnLegendre: {
      const T R = (T)a.p[0];
      const T t = y[n - 1] / R;
      const T fv = legendre_sum<T>(f.coef, t);
      if (!comp) return fv;
      T zz = (T)0;
      for (int i = 0; i < n; ++i) zz += z[i] * z[i];
      return fv + legendre_lap<T>(f.coef, a.p[0], a.sigma, t) * (over_(R * R, zz) - (T)1);
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
      return (T)fv + (T)(fv - a.sigma * us) * (over_(R * R, zz) - (T)1);
    }
    case kFnTorusSine: return torus_sine_source<T>(a, z, y);
  }
  return (T)0;
}

// f_Omega(y) + m(z) for a point z of the ball and y = cp(z).  RICH = false
// compiles only the ZERO, CONST, SPH_PAIR and TORUS_MODE families (the walk
// kernels are instantiated for both sets, so the common families do not carry
// the registers of the others).
template <class T, bool RICH = true>
__device__ __forceinline__ T source(const WalkArgs& a, const T* z, const T* y, int n) {
  const FnDev& f = a.f;
  const int comp = a.comp;
  switch (f.kind) {
    case kFnZero: return (T)0;
    case kFnConst: return (T)f.coef[0];
    case kFnSphPair: {
      const T R = (T)a.p[0];
      const T iR = (T)a.inv_R;
      const T fv = (T)f.coef[0] * (y[f.idx[0]] * iR) * (y[f.idx[1]] * iR);
      if (!comp) return fv;
      T zz = (T)0;
      for (int i = 0; i < n; ++i) zz += z[i] * z[i];
      return fv + (T)(f.lam * f.u_scale) * fv * (over_(R * R, zz) - (T)1);
    }
    case kFnTorus: {
      const T R = (T)a.p[0], tube = (T)a.p[1];
      // angles of y on the torus (those of z are the same: cp keeps phi and psi)
      const T rho = sqrt_(y[0] * y[0] + y[1] * y[1]);
      const T sphi = over_(y[1], rho);
      const T dr = rho - R;
      const T dy = sqrt_(dr * dr + y[2] * y[2]);
      const T cpsi = over_(dr, dy), spsi = over_(y[2], dy);
      const T u = sphi * (cpsi * cpsi - spsi * spsi);
      const T c0 = (T)f.coef[0];
      const T nl = torus_neg_lap<T>(R, tube, sphi, cpsi, spsi);
      T v = c0 * nl + (T)a.sigma * c0 * u;
      if (comp) {
        const T rz = sqrt_(z[0] * z[0] + z[1] * z[1]);
        const T dz = sqrt_((rz - R) * (rz - R) + z[2] * z[2]);
        if (a.kind == kCloud) {
          // a reconstructed surface moves the foot point off z's normal line:
          // the correction takes z's own angles in both terms
          const T zs = over_(z[1], rz), zc = over_(rz - R, dz), zp = over_(z[2], dz);
          v += c0 * (torus_neg_lap<T>(R, dz, zs, zc, zp) - torus_neg_lap<T>(R, tube, zs, zc, zp));
        } else {
          v += c0 * (torus_neg_lap<T>(R, dz, sphi, cpsi, spsi) - nl);
        }
      }
      return v;
    }
    default:
      if constexpr (RICH) return source_rich<T>(a, z, y, n);
      return (T)0;
  }
}

// g_Omega at a boundary point y.
template <class T>
__device__ __forceinline__ double boundary_value(const WalkArgs& a, const T* y, int n) {
  const FnDev& g = a.g;
  switch (g.kind) {
    case kFnZero: return 0.0;
    case kFnConst: return g.coef[0];
    case kFnSphPair: {
      if constexpr (sizeof(T) == 4) {
        const float iR = (float)a.inv_R;
        return (double)((float)g.coef[0] * (y[g.idx[0]] * iR) * (y[g.idx[1]] * iR));
      } else {
        const double R = a.p[0];
        return g.coef[0] * ((double)y[g.idx[0]] / R) * ((double)y[g.idx[1]] / R);
      }
    }
    case kFnLegendre:
      if constexpr (sizeof(T) == 4) return (double)legendre_sum<T>(g.coef, y[n - 1] * (float)a.inv_R);
      else return (double)legendre_sum<T>(g.coef, (T)((double)y[n - 1] / a.p[0]));
  }
  return 0.0;
}

// Entry of a batched launch that holds launch walk x (x < the padded size):
// the last entry whose begin is at most x.  Uniform when x is.
__device__ __forceinline__ int batch_entry(const WalkArgs& a, int64_t x) {
  int lo = 0, hi = a.n_batch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.batch[mid].begin <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace mpwos
