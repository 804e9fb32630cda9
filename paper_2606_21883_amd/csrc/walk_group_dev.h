// One lane group per walk on S^{n-1}_R for n >= 4 (up to n = 4092): the n
// coordinates of a walk are spread over L lanes of a wavefront (L = 4 .. 64).
// Philox block b of a sub-stream (coordinates 4b .. 4b+3) belongs to lane
// b mod L, slot b / L, so every lane draws its own normals; the norms |g|,
// |Theta|, |g'| and |Z| are butterfly sums across the group (commutative, so
// every lane ends with the same bits).  W, S and the radial inverse are
// computed redundantly by all lanes of the group.
#pragma once
#include <hip/hip_runtime.h>

#include "host_internal.h"
#include "kernel_args.h"
#include "mpwos_dev.h"

namespace mpwos {

template <int L, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
  return v;
}

template <class T, int L, int MB>
struct GroupWalk {
  T Y[4 * MB];
  T A[4 * MB];         // dumbbell source: this lane's entries of the diagonal
  double W, S, C;
  uint32_t k, q, w;
  int64_t idx;
};

// n normals of one sub-stream into this lane's slots (zeros past n).  Returns
// the radius uniform word if this lane owns it.
template <class T, int L, int MB>
__device__ __forceinline__ void group_normals(const WalkArgs& a, const Stream& rs, uint32_t step, uint32_t sub,
                                              int gl, T* g, bool want_u, uint32_t& uword) {
  const int n = a.n;
  const int npairs = (n + 1) / 2;
  const int nbd = (n + 3) / 4;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int b = gl + L * m;
    T* gm = g + 4 * m;
    gm[0] = gm[1] = gm[2] = gm[3] = (T)0;
    const bool dir = b < nbd;
    const bool rad = want_u && b == a.rblk;
    if (dir || rad) {
      const uint4 x = rs.block(step, sub, (uint32_t)b);
      if (dir) {
        T g0, g1;
        if (2 * b < npairs) {
          box_muller(x.x, x.y, g0, g1);
          gm[0] = g0;
          gm[1] = (4 * b + 1 < n) ? g1 : (T)0;
        }
        if (2 * b + 1 < npairs) {
          box_muller(x.z, x.w, g0, g1);
          gm[2] = g0;
          gm[3] = (4 * b + 3 < n) ? g1 : (T)0;
        }
      }
      if (rad) {
        const uint32_t ws[4] = {x.x, x.y, x.z, x.w};
        uword = ws[a.rword];
      }
    }
  }
}

// ---- implicit dumbbell (Sec. 4, Example 2) ---------------------------------
// M = {|x_h| = R(x_n)}, x_h the first n-1 coordinates; with x_n = kc cos(phi)
// the profile is (r, z)(phi) = (sin(phi) g, kc cos(phi)), g = 1 - a + 2a
// cos^2(phi), smooth up to the poles.
__device__ __forceinline__ void sincos_(double x, double& s, double& c) { sincos(x, &s, &c); }
__device__ __forceinline__ void sincos_(float x, float& s, float& c) {
  // v_sin_f32 / v_cos_f32 take turns
  const float t = x * 0.15915494309189535f;
  s = __builtin_amdgcn_sinf(t);
  c = __builtin_amdgcn_cosf(t);
}

template <class T>
struct DbProfile {
  T r, r1, r2, z, z1, z2, g;
};

template <class T>
__device__ __forceinline__ DbProfile<T> db_profile(T a, T kc, T phi) {
  T s, c;
  sincos_(phi, s, c);
  DbProfile<T> p;
  const T g = (T)1 - a + (T)2 * a * c * c;
  const T g1 = (T)-4 * a * c * s;
  const T g2 = (T)-4 * a * (c * c - s * s);
  p.g = g;
  p.r = s * g;
  p.r1 = c * g + s * g1;
  p.r2 = -s * g + (T)2 * c * g1 + s * g2;
  p.z = kc * c;
  p.z1 = -kc * s;
  p.z2 = -kc * c;
  return p;
}

// Profile parameter of the point of M nearest to (|x_h|, x_n) = (rho, zs):
// the best of a 128-point grid over [0, pi] (the group's lanes share the
// grid; ties go to the lower index), then Newton on D'(phi) = 0 with D the
// squared planar distance, kept by bisection inside the neighbouring cells.
// Every lane of the group returns the same value.
template <class T, int L>
__device__ __forceinline__ T db_phi(T a, T kc, T rho, T zs, int gl) {
  constexpr int G = 128;
  const T pi = (T)3.141592653589793;
  const T h = pi / (T)(G - 1);
  float bd = 3.0e38f;
  int bj = G;
  for (int j = gl; j < G; j += L) {
    // the scan only places the basin: FP32 is enough
    float s, c;
    sincos_((float)j * (float)h, s, c);
    const float r = s * ((float)1 - (float)a + (float)2 * (float)a * c * c);
    const float d = ((float)rho - r) * ((float)rho - r) + ((float)zs - (float)kc * c) * ((float)zs - (float)kc * c);
    if (d < bd) {
      bd = d;
      bj = j;
    }
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) {
    const float od = __shfl_xor(bd, o, L);
    const int oj = __shfl_xor(bj, o, L);
    if (od < bd || (od == bd && oj < bj)) {
      bd = od;
      bj = oj;
    }
  }
  T lo = bj > 0 ? (T)(bj - 1) * h : (T)0;
  T hi = bj < G - 1 ? (T)(bj + 1) * h : pi;
  T phi = (T)bj * h;
  const T tol = sizeof(T) == 8 ? (T)1e-16 : (T)1e-7;
  for (int it = 0; it < 64; ++it) {
    const DbProfile<T> p = db_profile<T>(a, kc, phi);
    const T d1 = (T)-2 * ((rho - p.r) * p.r1 + (zs - p.z) * p.z1);
    const T d2 = (T)2 * (p.r1 * p.r1 + p.z1 * p.z1) - (T)2 * ((rho - p.r) * p.r2 + (zs - p.z) * p.z2);
    if (d1 > (T)0) hi = phi;
    else lo = phi;
    T nx = d2 > (T)0 ? phi - d1 / d2 : lo - (T)1;
    if (!(nx >= lo && nx <= hi)) nx = (T)0.5 * (lo + hi);
    const T step = abs_(nx - phi);
    phi = nx;
    if (step <= tol * ((T)1 + phi) || hi - lo <= tol * ((T)1 + phi)) break;
  }
  return phi;
}

// Group sums over the first n-1 coordinates (x_h) and the last one (x_n).
template <class T, int L, int MB>
__device__ __forceinline__ void db_split(const WalkArgs& a, const T* x, int gl, T& hh, T& zs) {
  T s = (T)0, z = (T)0;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * (gl + L * m) + j;
      const T v = x[4 * m + j];
      if (i == a.n - 1) z = v;
      else s += v * v;
    }
  hh = group_sum<L>(s);
  zs = group_sum<L>(z);
}

// cp onto the dumbbell, in place on the group's coordinates.
template <class T, int L, int MB>
__device__ __forceinline__ void db_project(const WalkArgs& a, T* x, int gl) {
  T hh, zs;
  db_split<T, L, MB>(a, x, gl, hh, zs);
  const T rho = sqrt_(hh);
  const T phi = db_phi<T, L>((T)a.p[0], (T)a.p[1], rho, zs, gl);
  const DbProfile<T> p = db_profile<T>((T)a.p[0], (T)a.p[1], phi);
  const T sc = rho > (T)0 ? over_(p.r, rho) : (T)0;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * (gl + L * m) + j;
      x[4 * m + j] = (i == a.n - 1) ? p.z : x[4 * m + j] * sc;
    }
}

// f_Omega(cp z) for the dumbbell polynomial family
//   u = c0 x_n + c1 x_n^2 + c2 (1.x_h)/sqrt(n-1) + c3 x_h^T diag(A) x_h,
// -Lap_M u + sigma u by the extrinsic formula Lap_M U = Lap U - nu^T Hess U nu
// - H dU/dnu (H = k1 + (n-2) k2, outward normal nu = (N_r e, N_z)).  Only the
// sums over z's coordinates are needed, not the projected point itself.
template <class T, int L, int MB>
__device__ __forceinline__ T db_source(const WalkArgs& a, const T* z, const T* A, int gl) {
  const FnDev& f = a.f;
  if (f.kind == kFnConst) return (T)f.coef[0];
  if (f.kind != kFnDumbbell) return (T)0;
  T s1 = (T)0, sa = (T)0, s2 = (T)0, zl = (T)0;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * (gl + L * m) + j;
      const T v = z[4 * m + j];
      if (i == a.n - 1) {
        zl = v;
      } else {
        s1 += v;
        s2 += v * v;
        sa += A[4 * m + j] * v * v;
      }
    }
  s1 = group_sum<L>(s1);
  s2 = group_sum<L>(s2);
  sa = group_sum<L>(sa);
  zl = group_sum<L>(zl);
  const T rho = sqrt_(s2);
  const T phi = db_phi<T, L>((T)a.p[0], (T)a.p[1], rho, zl, gl);
  // the scalar tail in the walk's precision (no cancellation: sigma U and the
  // curvature terms add with their own signs)
  const T kc = (T)a.p[1];
  const DbProfile<T> p = db_profile<T>((T)a.p[0], kc, phi);
  const T iLp = rsqrt_(p.r1 * p.r1 + p.z1 * p.z1);
  const T Nr = -p.z1 * iLp, Nz = p.r1 * iLp;
  const T k1 = (p.z1 * p.r2 - p.r1 * p.z2) * (iLp * iLp * iLp);
  const T k2 = over_(kc * iLp, p.g);
  const T ir = rho > (T)0 ? rcp_(rho) : (T)0;
  const T e1 = s1 * ir, ea = sa * ir * ir;
  const T isq = (T)(1.0 / sqrt((double)(a.n - 1)));
  const T c0 = (T)f.coef[0], c1 = (T)f.coef[1], c2 = (T)f.coef[2], c3 = (T)f.coef[3];
  const T zz = p.z, rr = p.r;
  const T U = c0 * zz + c1 * zz * zz + c2 * rr * e1 * isq + c3 * rr * rr * ea;
  const T lapU = (T)2 * c1 + (T)2 * c3 * (T)f.lam;
  const T hess = (T)2 * c1 * Nz * Nz + (T)2 * c3 * Nr * Nr * ea;
  const T dnu = Nz * (c0 + (T)2 * c1 * zz) + Nr * (c2 * e1 * isq + (T)2 * c3 * rr * ea);
  const T H = k1 + (T)(a.n - 2) * k2;
  return -(lapU - hess - H * dnu) + (T)a.sigma * U;
}

template <class T, int L, int MB>
__device__ __forceinline__ T coord_of(const T* v, int i, int gl) {
  // value of coordinate i, broadcast from its owner lane
  const int b = i >> 2;
  const int owner = b % L;
  const int slot = b / L;
  T mine = (T)0;
#pragma unroll
  for (int m = 0; m < MB; ++m)
    if (m == slot) mine = v[4 * m + (i & 3)];
  return __shfl(mine, owner, L);
}

// ---- product manifold S^1_Fourier(R) x S^2(a) in R^9 (Sec. 4, Example 3) -----
// X(phi, w) = (R C(phi), a w), C = (cos, sin, cos 2/2, sin 2/2, cos 3/3, sin 3/3)
// of phi.  |C| is constant, so the nearest curve point of x_c maximises
// g(phi) = sum_k (a_k cos k phi + b_k sin k phi)/k, a_k = x_c[2k-2], b_k =
// x_c[2k-1]; the sphere factor is normalised.
template <class T>
__device__ __forceinline__ void pr_g(const T* xc, T phi, T& g, T& g1, T& g2) {
  T s1, c1;
  sincos_(phi, s1, c1);
  const T c2 = c1 * c1 - s1 * s1, s2 = (T)2 * s1 * c1;
  const T c3 = c2 * c1 - s2 * s1, s3 = s2 * c1 + c2 * s1;
  const T e1 = xc[0] * c1 + xc[1] * s1, e2 = xc[2] * c2 + xc[3] * s2, e3 = xc[4] * c3 + xc[5] * s3;
  g = e1 + e2 / (T)2 + e3 / (T)3;
  g1 = (-xc[0] * s1 + xc[1] * c1) + (-xc[2] * s2 + xc[3] * c2) + (-xc[4] * s3 + xc[5] * c3);
  g2 = -(e1 + (T)2 * e2 + (T)3 * e3);
}

// Curve parameter of the nearest curve point: the best of a 64-point grid
// over [0, 2 pi) shared by the group's lanes (FP32; ties to the lower index),
// then Newton on g' = 0 kept inside the neighbouring cells by bisection.
template <class T, int L>
__device__ __forceinline__ T pr_phi(const T* xc, int gl) {
  constexpr int G = 64;
  const T h = (T)6.283185307179586 / (T)G;
  float xf[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) xf[i] = (float)xc[i];
  float bg = -3.0e38f;
  int bj = G;
  for (int j = gl; j < G; j += L) {
    float g, g1, g2;
    pr_g<float>(xf, (float)j * (float)h, g, g1, g2);
    if (g > bg) {
      bg = g;
      bj = j;
    }
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) {
    const float og = __shfl_xor(bg, o, L);
    const int oj = __shfl_xor(bj, o, L);
    if (og > bg || (og == bg && oj < bj)) {
      bg = og;
      bj = oj;
    }
  }
  T lo = (T)(bj - 1) * h, hi = (T)(bj + 1) * h, phi = (T)bj * h;
  const T tol = sizeof(T) == 8 ? (T)1e-16 : (T)1e-7;
  for (int it = 0; it < 64; ++it) {
    T g, g1, g2;
    pr_g<T>(xc, phi, g, g1, g2);
    if (g1 > (T)0) lo = phi;
    else hi = phi;
    T nx = g2 < (T)0 ? phi - g1 / g2 : lo - (T)1;
    if (!(nx >= lo && nx <= hi)) nx = (T)0.5 * (lo + hi);
    const T step = abs_(nx - phi);
    phi = nx;
    if (step <= tol * ((T)1 + abs_(phi)) || hi - lo <= tol * ((T)1 + abs_(phi))) break;
  }
  return phi;
}

// cp onto the product, in place on the group's coordinates.
template <class T, int L, int MB>
__device__ __forceinline__ void pr_project(const WalkArgs& a, T* x, int gl) {
  T v[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = coord_of<T, L, MB>(x, i, gl);
  const T phi = pr_phi<T, L>(v, gl);
  T s1, c1;
  sincos_(phi, s1, c1);
  const T c2 = c1 * c1 - s1 * s1, s2 = (T)2 * s1 * c1;
  const T c3 = c2 * c1 - s2 * s1, s3 = s2 * c1 + c2 * s1;
  const T R = (T)a.p[0];
  const T yc[6] = {R * c1, R * s1, R * c2 / (T)2, R * s2 / (T)2, R * c3 / (T)3, R * s3 / (T)3};
  const T sc = (T)a.p[1] * rsqrt_(v[6] * v[6] + v[7] * v[7] + v[8] * v[8]);
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * (gl + L * m) + j;
      T out = (T)0;
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (i == c) out = yc[c];
      if (i >= 6 && i < 9) out = x[4 * m + j] * sc;
      x[4 * m + j] = out;
    }
}

// f_Omega(cp z) for u = c0 cos(phi) w1 + c1 sin(2 phi) w2 + c2 cos(3 phi)
// (w1^2 - w2^2): Lap_M is the sum of the factors' operators, (1/(3 R^2))
// d^2/dphi^2 on the curve (speed R sqrt 3) and the degree-1 and degree-2
// harmonics on S^2(a) (eigenvalues 2/a^2 and 6/a^2).
template <class T, int L, int MB>
__device__ __forceinline__ T pr_source(const WalkArgs& a, const T* z, int gl) {
  const FnDev& f = a.f;
  if (f.kind == kFnConst) return (T)f.coef[0];
  if (f.kind != kFnProduct) return (T)0;
  T v[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = coord_of<T, L, MB>(z, i, gl);
  // in the walk's precision: cos phi, sin 2phi and cos 3phi from one sincos
  // by the angle-addition formulas
  const T phi = pr_phi<T, L>(v, gl);
  const T ins = rsqrt_(v[6] * v[6] + v[7] * v[7] + v[8] * v[8]);
  const T w1 = v[6] * ins, w2 = v[7] * ins;
  T sn1, cs1;
  sincos_(phi, sn1, cs1);
  const T sn2 = (T)2 * sn1 * cs1, cs2 = cs1 * cs1 - sn1 * sn1;
  const T cs3 = cs2 * cs1 - sn2 * sn1;
  const double R = a.p[0];
  const T q = (T)(1.0 / (3.0 * R * R)), sa = (T)(1.0 / (a.p[1] * a.p[1])), sg = (T)a.sigma;
  const T k0 = (T)f.coef[0], k1 = (T)f.coef[1], k2 = (T)f.coef[2];
  return k0 * (sg + q + (T)2 * sa) * cs1 * w1 + k1 * (sg + (T)4 * q + (T)2 * sa) * sn2 * w2 +
         k2 * (sg + (T)9 * q + (T)6 * sa) * cs3 * (w1 * w1 - w2 * w2);
}

template <class T, int L, int MB, int KIND>
__device__ __forceinline__ bool group_step(const WalkArgs& a, GroupWalk<T, L, MB>& st, int gl, uint64_t seed) {
  const Stream rs{st.q, st.w, (uint32_t)seed, (uint32_t)(seed >> 32)};
  const double r = a.r0;
  const T rT = (T)r;
  const T R = (T)a.p[0];
  uint32_t dummy = 0;
  // Green samples first: they read Y only, so the next point Y' need not be
  // live beside their vectors (registers)
  T Fsum = (T)0;
  for (int l = 1; l <= a.n_v; ++l) {
    T g[4 * MB];
    uint32_t uw = 0;
    group_normals<T, L, MB>(a, rs, st.k, (uint32_t)l, gl, g, true, uw);
    uw = __shfl(uw, a.rblk % L, L);
    T s;
    if constexpr (sizeof(T) == 8) s = radial_inv64(a, u01_64(uw), a.X0 * a.X0, a.fixed.norm);
    else s = radial_inv32(a, u01_32(uw), (float)(a.X0 * a.X0));
    T gg = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) gg += g[i] * g[i];
    gg = group_sum<L>(gg);
    const T ig = rsqrt_(gg);
    const T t = rT * s;
    T Z[4 * MB];
    T zz = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) {
      Z[i] = st.Y[i] + t * (g[i] * ig);
      zz += Z[i] * Z[i];
    }
    const FnDev& f = a.f;
    T v;
    if constexpr (KIND == kDumbbell) {
      v = db_source<T, L, MB>(a, Z, st.A, gl);
    } else if constexpr (KIND == kProduct) {
      v = pr_source<T, L, MB>(a, Z, gl);
    } else if (f.kind == kFnSphPair) {
      zz = group_sum<L>(zz);
      const T zi = coord_of<T, L, MB>(Z, f.idx[0], gl);
      const T zj = coord_of<T, L, MB>(Z, f.idx[1], gl);
      // cp(Z) = R Z/|Z|; f_Omega(cp Z) = coef (Z_i/|Z|)(Z_j/|Z|)
      const T fv = (T)f.coef[0] * (zi * zj / zz);
      v = fv;
      if (a.comp) v += (T)(f.lam * f.u_scale) * fv * (over_(R * R, zz) - (T)1);
    } else if (f.kind == kFnConst) {
      v = (T)f.coef[0];
    } else {
      v = (T)0;
    }
    Fsum += v;
  }
  // sphere sample and projection: Theta = Y + r g/|g|, Y' = cp(Theta) (the
  // sphere: R Theta/|Theta|; the dumbbell: Newton in the profile parameter)
  T Yn[4 * MB];
  {
    T g[4 * MB];
    group_normals<T, L, MB>(a, rs, st.k, 0, gl, g, false, dummy);
    T gg = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) gg += g[i] * g[i];
    gg = group_sum<L>(gg);
    const T ig = rsqrt_(gg);
    T tt = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) {
      Yn[i] = st.Y[i] + rT * (g[i] * ig);
      tt += Yn[i] * Yn[i];
    }
    if constexpr (KIND == kDumbbell) {
      db_project<T, L, MB>(a, Yn, gl);
    } else if constexpr (KIND == kProduct) {
      pr_project<T, L, MB>(a, Yn, gl);
    } else {
      tt = group_sum<L>(tt);
      const T f = R * rsqrt_(tt);
#pragma unroll
      for (int i = 0; i < 4 * MB; ++i) Yn[i] *= f;
    }
  }
  const double F = (double)Fsum * a.inv_nv;
  if constexpr (sizeof(T) == 8) kahan_add(st.S, st.C, (st.W * a.om0) * F);
  else st.S += (st.W * a.om0) * F;
  st.W = st.W * a.c0;
#pragma unroll
  for (int i = 0; i < 4 * MB; ++i) st.Y[i] = Yn[i];
  st.k += 1;
  if (!(st.W >= a.tau_w)) return true;  // NaN ends the walk too
  return (int64_t)st.k >= a.max_steps;
}

// This lane's entries of the dumbbell source's diagonal (zero elsewhere).
template <class T, int L, int MB, int KIND>
__device__ __forceinline__ void group_coefs(const WalkArgs& a, GroupWalk<T, L, MB>& st, int gl) {
  if constexpr (KIND != kDumbbell) return;
  const bool db = a.f.kind == kFnDumbbell;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * (gl + L * m) + j;
      st.A[4 * m + j] = (db && i < a.n - 1) ? (T)a.f.values[i] : (T)0;
    }
}

template <class T, int L, int MB>
__device__ __forceinline__ void group_init(const WalkArgs& a, const double* queries, int64_t nw, int64_t q_offset,
                                           int64_t idx, GroupWalk<T, L, MB>& st, int gl) {
  st.idx = idx;
  const int64_t ql = idx / nw;
  st.q = (uint32_t)(ql + q_offset);
  st.w = (uint32_t)(idx - ql * nw);
  const double* y0 = queries + ql * a.n;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int b = gl + L * m;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * b + j;
      st.Y[4 * m + j] = (i < a.n) ? (T)y0[i] : (T)0;
    }
  }
  st.W = 1.0;
  st.S = 0.0;
  st.C = 0.0;
  st.k = 0;
}

// State record of a time-sliced walk: W, S, C, k and a done flag (written by
// the group's lane 0), then each lane's 4 MB coordinates.
template <class T, int L, int MB>
struct GroupRecord {
  static constexpr int64_t kBytes = (32 + (int64_t)L * 4 * MB * (int64_t)sizeof(T) + 63) / 64 * 64;
};

template <class T, int L, int MB>
__device__ __forceinline__ void group_save(char* rec, const GroupWalk<T, L, MB>& st, int gl, uint32_t flag) {
  if (gl == 0) {
    double* d = (double*)rec;
    d[0] = st.W;
    d[1] = st.S;
    d[2] = st.C;
    uint32_t* u = (uint32_t*)(rec + 24);
    u[0] = st.k;
    u[1] = flag;
  }
  if (flag) return;
  T* y = (T*)(rec + 32) + gl * 4 * MB;
#pragma unroll
  for (int i = 0; i < 4 * MB; ++i) y[i] = st.Y[i];
}

template <class T, int L, int MB>
__device__ __forceinline__ void group_load(const char* rec, int64_t idx, int64_t nw, GroupWalk<T, L, MB>& st,
                                           int gl) {
  st.idx = idx;
  const int64_t ql = idx / nw;
  st.q = (uint32_t)ql;
  st.w = (uint32_t)(idx - ql * nw);
  const double* d = (const double*)rec;
  st.W = d[0];
  st.S = d[1];
  st.C = d[2];
  st.k = ((const uint32_t*)(rec + 24))[0];
  const T* y = (const T*)(rec + 32) + gl * 4 * MB;
#pragma unroll
  for (int i = 0; i < 4 * MB; ++i) st.Y[i] = y[i];
}

// plain: group id -> walk; persistent: grid-stride over walks (closed
// spheres have one deterministic walk length, so a static split is balanced).
// Batched launches (serving) take the grid-stride form; every entry begins on
// a whole wavefront of groups and the stride is a whole number of wavefronts,
// so the groups of a wavefront always share one request (its seed stays
// uniform); launch walks past an entry's count are padding.
// The FP32 hypersphere kernels with four blocks per lane (S^99, S^999) are
// held to 128 VGPRs, four waves per SIMD instead of three, and the FP32
// dumbbell kernels to 168 VGPRs, three waves instead of two: the spilled
// registers cost less than the latency the extra wave hides (S^999 runs 10%
// faster, S^99 5%, the 1001-dimensional dumbbell 28%).
template <class T, int L, int MB, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 && MB == 4 && KIND == kSphere ? 4 : (sizeof(T) == 4 && KIND == kDumbbell ? 3 : 1)))) void walk_group_kernel(WalkArgs a) {
  const int64_t total = a.count;
  const int gl = threadIdx.x % L;
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / L;
  GroupWalk<T, L, MB> st;
  for (int64_t idx = gid; idx < total; idx += (a.persistent ? ngroups : total)) {
    const double* queries = a.queries;
    int64_t nw = a.nw, q_offset = a.q_offset, widx = a.idx_base + idx;
    uint64_t seed;
    double* walk_S = a.walk_S;
    int32_t* walk_K = a.walk_K;
    char* rec = nullptr;
    bool resume = false;
    unsigned long long* pending = nullptr;
    if (a.n_batch) {
      const int64_t first = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)idx) |
                            ((int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(idx >> 32)) << 32);
      const int e = batch_entry(a, first);
      const BatchEntry& E = a.batch[e];
      if (idx >= E.begin + E.count) continue;
      queries = E.queries;
      nw = E.nw;
      q_offset = 0;
      widx = E.idx0 + (idx - E.begin);
      seed = E.seed;
      walk_S = E.walk_S;
      walk_K = E.walk_K;
      if (E.state && a.step_budget > 0) {
        rec = E.state + widx * GroupRecord<T, L, MB>::kBytes;
        resume = E.resume != 0;
        pending = const_cast<unsigned long long*>(&a.batch[e].pending);
      }
    } else {
      seed = a.seed_dev ? *a.seed_dev : a.seed;
    }
    if (resume) {
      if (((const uint32_t*)(rec + 24))[1]) continue;   // finished in an earlier launch
      group_load<T, L, MB>(rec, widx, nw, st, gl);
    } else {
      group_init<T, L, MB>(a, queries, nw, q_offset, widx, st, gl);
    }
    group_coefs<T, L, MB, KIND>(a, st, gl);
    bool done = false;
    if (rec) {
      for (int32_t j = 0; j < a.step_budget && !done; ++j) done = group_step<T, L, MB, KIND>(a, st, gl, seed);
    } else {
      while (!group_step<T, L, MB, KIND>(a, st, gl, seed)) {
      }
      done = true;
    }
    if (done) {
      if (gl == 0) {
        walk_S[st.idx] = st.S + st.C;
        walk_K[st.idx] = (int32_t)st.k;
      }
      if (rec) group_save<T, L, MB>(rec, st, gl, 1u);
    } else {
      group_save<T, L, MB>(rec, st, gl, 0u);
      if (gl == 0) atomicAdd(pending, 1ull);
    }
  }
}

// cp of m points (n >= 4), one lane group per point (inspection).
template <class T, int L, int MB, int KIND>
__global__ __launch_bounds__(256) void cp_group_kernel(WalkArgs a, const double* x, double* y, int64_t m) {
  const int gl = threadIdx.x % L;
  const int64_t pt = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  if (pt >= m) return;
  T v[4 * MB];
#pragma unroll
  for (int k = 0; k < MB; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * (gl + L * k) + j;
      v[4 * k + j] = i < a.n ? (T)x[pt * a.n + i] : (T)0;
    }
  if constexpr (KIND == kDumbbell) {
    db_project<T, L, MB>(a, v, gl);
  } else if constexpr (KIND == kProduct) {
    pr_project<T, L, MB>(a, v, gl);
  } else {
    T s = (T)0;
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) s += v[i] * v[i];
    s = group_sum<L>(s);
    const T f = (T)a.p[0] * rsqrt_(s);
#pragma unroll
    for (int i = 0; i < 4 * MB; ++i) v[i] *= f;
  }
#pragma unroll
  for (int k = 0; k < MB; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * (gl + L * k) + j;
      if (i < a.n) y[pt * a.n + i] = (double)v[4 * k + j];
    }
}

template <class T, int L, int MB, int KIND>
static hipError_t launch_cp_group_t(const WalkArgs& a, const double* x, double* y, int64_t m, hipStream_t s) {
  const int64_t grid = (m * L + 255) / 256;
  hipLaunchKernelGGL((cp_group_kernel<T, L, MB, KIND>), dim3((unsigned)grid), dim3(256), 0, s, a, x, y, m);
  return hipGetLastError();
}

template <class T, int L, int MB, int KIND>
static hipError_t launch_group_t(const WalkArgs& a, int64_t grid, int block, hipStream_t s) {
  hipLaunchKernelGGL((walk_group_kernel<T, L, MB, KIND>), dim3((unsigned)grid), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <class T, int L, int MB, int KIND>
static int group_occ_t(int block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_group_kernel<T, L, MB, KIND>, block, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

// Dispatch of the runtime group shape (L lanes, MB blocks per lane) to the
// compiled instances of one manifold kind K.
#define MPWOS_GROUP_MB(T, LL, K, FN, ...)              \
  switch (mb) {                                        \
    case 1: return FN<T, LL, 1, K>(__VA_ARGS__);       \
    case 2: return FN<T, LL, 2, K>(__VA_ARGS__);       \
    case 4: return FN<T, LL, 4, K>(__VA_ARGS__);       \
    case 8: return FN<T, LL, 8, K>(__VA_ARGS__);       \
  }
#define MPWOS_GROUP_L(T, K, FN, ...)                                    \
  switch (L) {                                                          \
    case 4: MPWOS_GROUP_MB(T, 4, K, FN, __VA_ARGS__) break;             \
    case 8: MPWOS_GROUP_MB(T, 8, K, FN, __VA_ARGS__) break;             \
    case 16: MPWOS_GROUP_MB(T, 16, K, FN, __VA_ARGS__) break;           \
    case 32: MPWOS_GROUP_MB(T, 32, K, FN, __VA_ARGS__) break;           \
    case 64:                                                            \
      if (mb == 16) return FN<T, 64, 16, K>(__VA_ARGS__);               \
      MPWOS_GROUP_MB(T, 64, K, FN, __VA_ARGS__) break;                  \
  }
// The product manifold (n = 9) always has one block per lane.
#define MPWOS_GROUP_L1(T, K, FN, ...)                                   \
  if (mb == 1) {                                                        \
    switch (L) {                                                        \
      case 4: return FN<T, 4, 1, K>(__VA_ARGS__);                       \
      case 8: return FN<T, 8, 1, K>(__VA_ARGS__);                       \
      case 16: return FN<T, 16, 1, K>(__VA_ARGS__);                     \
      case 32: return FN<T, 32, 1, K>(__VA_ARGS__);                     \
      case 64: return FN<T, 64, 1, K>(__VA_ARGS__);                     \
    }                                                                   \
  }

// Host entry points of one kind's instances (defined in walk_group_<kind>.hip).
#define MPWOS_GROUP_KIND_ENTRIES(NAME, K, DISPATCH)                                                              \
  hipError_t group_launch_##NAME(bool fp64, int L, int mb, const WalkArgs& a, int64_t grid, int block,          \
                                 hipStream_t s) {                                                               \
    if (fp64) {                                                                                                 \
      DISPATCH(double, K, launch_group_t, a, grid, block, s)                                                    \
    } else {                                                                                                    \
      DISPATCH(float, K, launch_group_t, a, grid, block, s)                                                     \
    }                                                                                                           \
    return hipErrorInvalidValue;                                                                                \
  }                                                                                                             \
  int group_occ_##NAME(bool fp64, int L, int mb, int block) {                                                   \
    if (fp64) {                                                                                                 \
      DISPATCH(double, K, group_occ_t, block)                                                                   \
    } else {                                                                                                    \
      DISPATCH(float, K, group_occ_t, block)                                                                    \
    }                                                                                                           \
    return 1;                                                                                                   \
  }                                                                                                             \
  hipError_t launch_cp_group_##NAME(bool fp64, int L, int mb, const WalkArgs& a, const double* x, double* y,    \
                                    int64_t m, hipStream_t s) {                                                 \
    if (fp64) {                                                                                                 \
      DISPATCH(double, K, launch_cp_group_t, a, x, y, m, s)                                                     \
    } else {                                                                                                    \
      DISPATCH(float, K, launch_cp_group_t, a, x, y, m, s)                                                      \
    }                                                                                                           \
    return hipErrorInvalidValue;                                                                                \
  }

}  // namespace mpwos
