// sums.hip -- final reduction of the conserved sums (mass, momentum, total
// and kinetic energy) from the per-block partials of k_sums, shared by the
// host read-back and the device-output entry point.
#include <hip/hip_runtime.h>

#include "ops.h"

namespace lbm {

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
