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

// one thread per quantity adds the partials level by level, block by block:
// a fixed order, so every caller gets the same bits
__global__ void k_sum_partials(const double *partials, SumCounts cnt, int n_levels, double *out) {
  const int k = threadIdx.x;
  if (k >= SUM_Q) return;
  double v = 0.0;
  for (int l = 0; l < n_levels; ++l)
    for (int b = 0; b < cnt.nb[l]; ++b) v += partials[((int64_t)l * SUM_BLOCKS + b) * SUM_Q + k];
  out[k] = v;
}

void launch_sum_partials(const double *partials, const int *nb, int n_levels, double *out, hipStream_t s) {
  SumCounts cnt{};
  for (int l = 0; l < n_levels && l < SUM_LEVELS; ++l) cnt.nb[l] = nb[l];
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, partials, cnt, n_levels, out);
}

}  // namespace lbm
