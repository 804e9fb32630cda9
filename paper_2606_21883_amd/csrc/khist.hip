// Histogram of the stopping indices K^i (Algorithm 1's walk lengths) for the
// median and 99th percentile reported in mpwos_stats.
//
// Bins: K < kKHistExact one bin per value; above, 128 bins per octave (the
// leading seven bits after the top one), so a reported quantile is exact
// below 2048 steps and within 1/128 of its value above.  One pass over the
// per-walk K array of a launch: each workgroup counts into LDS (18 KiB) and
// adds its non-zero bins to the 64-bit device histogram.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_internal.h"

namespace mpwos {

namespace {

constexpr int kHistBlock = 256;

__device__ __forceinline__ int khist_bin(int32_t k) {
  if (k < kKHistExact) return k < 0 ? 0 : k;
  const int e = 31 - __clz(k);                       // 11 .. 30
  const int sub = (k >> (e - 7)) - 128;              // 0 .. 127
  return kKHistExact + (e - 11) * 128 + sub;
}

// Each lane counts a run of equal bins in registers and adds it to LDS when
// the bin changes: walk lengths are often concentrated (a constant-radius
// walk stopped by tau_W has one length), and one LDS address taking every
// lane's atomic would serialise the pass.
__global__ void __launch_bounds__(kHistBlock) khist_kernel(const int32_t* __restrict__ K, int64_t n,
                                                            unsigned long long* __restrict__ hist) {
  __shared__ uint32_t h[kKHistBins];
  for (int i = threadIdx.x; i < kKHistBins; i += kHistBlock) h[i] = 0u;
  __syncthreads();
  int bin = 0;
  uint32_t run = 0;
  auto put = [&](int32_t k) {
    const int b = khist_bin(k);
    if (b == bin) {
      ++run;
    } else {
      if (run) atomicAdd(&h[bin], run);
      bin = b;
      run = 1;
    }
  };
  const int64_t stride = (int64_t)gridDim.x * kHistBlock;
  const int64_t t0 = (int64_t)blockIdx.x * kHistBlock + threadIdx.x;
  if (((uintptr_t)K & 15) == 0) {
    // four lengths per 16-byte load, then the tail
    const int4* K4 = (const int4*)K;
    const int64_t n4 = n / 4;
    for (int64_t i = t0; i < n4; i += stride) {
      const int4 v = K4[i];
      put(v.x);
      put(v.y);
      put(v.z);
      put(v.w);
    }
    for (int64_t i = n4 * 4 + t0; i < n; i += stride) put(K[i]);
  } else {
    for (int64_t i = t0; i < n; i += stride) put(K[i]);
  }
  if (run) atomicAdd(&h[bin], run);
  __syncthreads();
  for (int i = threadIdx.x; i < kKHistBins; i += kHistBlock)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

}  // namespace

hipError_t launch_khist(const int32_t* K, int64_t n, unsigned long long* hist, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  // at most 2048 workgroups: a workgroup's 32-bit LDS counts stay below 2^32
  // for any n a device can hold
  const int64_t grid = std::min<int64_t>(2048, (n + kHistBlock - 1) / kHistBlock);
  hipLaunchKernelGGL(khist_kernel, dim3((unsigned)grid), dim3(kHistBlock), 0, s, K, n, hist);
  return hipGetLastError();
}

int32_t khist_lower(int b) {
  if (b < kKHistExact) return b;
  const int e = 11 + (b - kKHistExact) / 128, sub = (b - kKHistExact) % 128;
  return (int32_t)((128u + (uint32_t)sub) << (e - 7));
}

void khist_quantiles(const unsigned long long* h, int32_t& p50, int32_t& p99) {
  unsigned long long total = 0;
  for (int b = 0; b < kKHistBins; ++b) total += h[b];
  p50 = p99 = 0;
  if (!total) return;
  // nearest rank: the smallest K with at least ceil(q N) walks at or below it
  const unsigned long long r50 = (total + 1) / 2, r99 = (total * 99 + 99) / 100;
  unsigned long long cum = 0;
  bool have50 = false;
  for (int b = 0; b < kKHistBins; ++b) {
    cum += h[b];
    if (!have50 && cum >= r50) {
      p50 = khist_lower(b);
      have50 = true;
    }
    if (cum >= r99) {
      p99 = khist_lower(b);
      return;
    }
  }
}

}  // namespace mpwos
