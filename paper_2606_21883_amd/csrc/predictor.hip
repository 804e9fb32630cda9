// Coarse predictor for the second-order compensation on the cut torus (the
// subsection on approximating the compensation term): node points of a
// uniform (th, s) grid over Omega and the discrete orthogonal projection of
// node values onto a Fourier-sine series in (th, s).
//
// Nodes: th_i = 2 pi i / nt (i < nt), s_j = pi j / ns (0 < j < ns), stored
// th-major (node i (ns - 1) + j - 1); u vanishes on the cut (s = 0, pi), so
// only interior nodes carry values.  The fit is the discrete Fourier
// transform in th times the discrete sine transform in s:
//   c_k0 = 2 / (nt ns) sum_ij U_ij sin(k s_j),
//   c_kj = 4 / (nt ns) sum_ij U_ij cos(j th_i) sin(k s_j)   (d_kj with sin),
// which reproduces any series with ks < ns and 2 kt < nt exactly.
#include <hip/hip_runtime.h>

#include "kernel_args.h"

namespace mpwos {

__global__ __launch_bounds__(256) void ct_nodes_kernel(double R, double a, double cut_c, double cut_s, int nt, int ns,
                                                       double* out) {
  const int m = nt * (ns - 1);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m) return;
  const int i = idx / (ns - 1), j = idx - i * (ns - 1) + 1;
  double st, ct, ss, cs;
  sincospi(2.0 * (double)i / (double)nt, &st, &ct);
  sincospi((double)j / (double)ns, &ss, &cs);
  // phi = phi_c + s
  const double cp = cut_c * cs - cut_s * ss, sp = cut_s * cs + cut_c * ss;
  const double rt = R + a * ct;
  out[3 * idx + 0] = rt * cp;
  out[3 * idx + 1] = rt * sp;
  out[3 * idx + 2] = a * st;
}

// One workgroup per coefficient (row k - 1, column c of 2 kt + 1); the 256
// lanes stride over the nodes and a fixed-order tree reduction in LDS sums
// them, so the result does not depend on timing.
__global__ __launch_bounds__(256) void ts_fit_kernel(const double* U, int nt, int ns, int kt, double* coef) {
  __shared__ double part[256];
  const int w = 2 * kt + 1;
  const int k = blockIdx.x / w + 1, c = blockIdx.x % w;
  const int j = (c + 1) / 2;
  const int m = nt * (ns - 1);
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < m; idx += 256) {
    const int i = idx / (ns - 1), jj = idx - i * (ns - 1) + 1;
    double wth = 1.0;
    if (c > 0) {
      double sv, cv;
      sincospi(2.0 * (double)(j * i % nt) / (double)nt, &sv, &cv);
      wth = (c & 1) ? cv : sv;
    }
    const double ws = sinpi((double)(k * jj % (2 * ns)) / (double)ns);
    acc = fma(U[idx] * wth, ws, acc);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) coef[blockIdx.x] = part[0] * ((c == 0 ? 1.0 : 2.0) * 2.0 / ((double)nt * (double)ns));
}

hipError_t launch_ct_nodes(double R, double a, double cut_c, double cut_s, int nt, int ns, double* out,
                           hipStream_t s) {
  const int m = nt * (ns - 1);
  hipLaunchKernelGGL(ct_nodes_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, R, a, cut_c, cut_s, nt,
                     ns, out);
  return hipGetLastError();
}

hipError_t launch_ts_fit(const double* U, int nt, int ns, int kt, int ks, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(ts_fit_kernel, dim3((unsigned)(ks * (2 * kt + 1))), dim3(256), 0, s, U, nt, ns, kt, coef);
  return hipGetLastError();
}

}  // namespace mpwos
