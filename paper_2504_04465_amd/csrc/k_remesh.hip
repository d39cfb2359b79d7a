// Mesh adaptation (Sec. 8): the synchronisation-point state of the old tree
// moves to the new one; every new cell's value is the weighted sum of its
// sources (one old cell with weight 1 for a copy or a uniform explosion,
// the old cells inside it with their volume shares for a coalescence).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "remesh.h"

namespace lbm {

// one thread per new cell; rows are [rows][n] FP64 arrays on both sides
__global__ void __launch_bounds__(256) k_remap(const double *__restrict__ old, int64_t n_old,
                                               double *__restrict__ out, int64_t n_new, int rows,
                                               const int64_t *__restrict__ off, const int32_t *__restrict__ src,
                                               const double *__restrict__ wt) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n_new) return;
  const int64_t b = off[j], e = off[j + 1];
  for (int r = 0; r < rows; ++r) {
    double acc = 0.0;
    for (int64_t k = b; k < e; ++k) acc += wt[k] * old[(int64_t)r * n_old + src[k]];
    out[(int64_t)r * n_new + j] = acc;
  }
}

void launch_remap(const double *old, int64_t n_old, double *out, int64_t n_new, int rows, const int64_t *off,
                  const int32_t *src, const double *wt, hipStream_t s) {
  if (n_new <= 0) return;
  hipLaunchKernelGGL(k_remap, dim3((unsigned)((n_new + 255) / 256)), dim3(256), 0, s, old, n_old, out, n_new, rows,
                     off, src, wt);
}

}  // namespace lbm
