// sums.hip -- final reduction of the conserved sums (mass, momentum, total
// and kinetic energy) from the per-block partials of k_sums, shared by the
// host read-back and the device-output entry point.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ops.h"

namespace lbm {

// Partials and result of the allocation-free sums (lbm_sums_device): one
// copy of this array per GPU, held until the process ends and shared by
// every context on that GPU.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): it uses the
// address sums_scratch() obtained for the current device.
static __device__ __align__(256) double scratch[SUM_PARTIALS + SUM_Q];

hipError_t sums_scratch(double **out) {
  constexpr int MAX_DEV = 64;
  static std::mutex mu;
  static double *addr[MAX_DEV] = {};
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (double *)p;
  }
  *out = addr[dev];
  return hipSuccess;
}

struct SumCounts {
  int nb[SUM_LEVELS];
};

// one wavefront per quantity: lane j adds the partials j, j + 64, ... of
// every level in turn, then the lanes are combined by a butterfly; a fixed
// order, so every caller gets the same bits
__global__ void __launch_bounds__(64 * SUM_Q) k_sum_partials(const double *partials, SumCounts cnt, int n_levels,
                                                             double *out) {
  const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double v = 0.0;
  for (int l = 0; l < n_levels; ++l)
    for (int b = lane; b < cnt.nb[l]; b += 64) v += partials[((int64_t)l * SUM_BLOCKS + b) * SUM_Q + k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) out[k] = v;
}

void launch_sum_partials(const double *partials, const int *nb, int n_levels, double *out, hipStream_t s) {
  SumCounts cnt{};
  for (int l = 0; l < n_levels && l < SUM_LEVELS; ++l) cnt.nb[l] = nb[l];
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64 * SUM_Q), 0, s, partials, cnt, n_levels, out);
}

}  // namespace lbm
