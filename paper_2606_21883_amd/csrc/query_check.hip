// On-manifold check of device-resident queries for the analytic manifolds
// (sphere, cap, implicit torus, cut torus), in FP64 on the device: the same
// rule as the host check of mpwos_solve (within 1e-9 (1 + |q|) of M, and on
// the open side of the boundary), so a solve with device queries need not
// copy them back and wait before its walks start.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "host_internal.h"

namespace mpwos {

namespace {

struct QueryRule {
  int32_t kind, n;
  double p0, p1, cut_c, cut_s;
};

__device__ bool on_manifold(const QueryRule& r, const double* y) {
  double s = 0.0;
  for (int i = 0; i < r.n; ++i) s += y[i] * y[i];
  const double tol = 1e-9 * (1.0 + sqrt(s));
  switch (r.kind) {
    case MPWOS_SPHERE:
      return fabs(sqrt(s) - r.p0) <= tol;
    case MPWOS_SPHERE_CAP:
      return fabs(sqrt(s) - r.p0) <= tol && y[r.n - 1] > r.p1;
    case MPWOS_TORUS_IMPLICIT:
    case MPWOS_CUT_TORUS: {
      const double rho = hypot(y[0], y[1]);
      const double dc = hypot(rho - r.p0, y[2]);
      if (!(fabs(dc - r.p1) <= tol)) return false;
      return r.kind == MPWOS_TORUS_IMPLICIT || y[1] * r.cut_c - y[0] * r.cut_s > 0.0;
    }
  }
  return false;
}

// slot receives the largest n_q - q over the failing queries q (so the first
// failing query is n_q - slot), and stays 0 when every query passes
__global__ void __launch_bounds__(256) query_check_kernel(QueryRule r, const double* __restrict__ q, int64_t nq,
                                                          unsigned long long* slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  if (!on_manifold(r, q + i * r.n)) atomicMax(slot, (unsigned long long)(nq - i));
}

}  // namespace

bool device_query_check(int kind) {
  return kind == MPWOS_SPHERE || kind == MPWOS_SPHERE_CAP || kind == MPWOS_TORUS_IMPLICIT ||
         kind == MPWOS_CUT_TORUS;
}

hipError_t launch_query_check(const mpwos_manifold_desc& d, const double* q, int64_t nq, unsigned long long* slot,
                              hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  QueryRule r{(int32_t)d.kind, (int32_t)d.n, d.p[0], d.p[1], 0.0, 0.0};
  if (d.kind == MPWOS_CUT_TORUS) {
    r.cut_c = std::cos(d.p[2]);
    r.cut_s = std::sin(d.p[2]);
  }
  const int64_t grid = (nq + 255) / 256;
  hipLaunchKernelGGL(query_check_kernel, dim3((unsigned)grid), dim3(256), 0, s, r, q, nq, slot);
  return hipGetLastError();
}

}  // namespace mpwos
