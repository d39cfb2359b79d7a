// mlp_ops.h -- host launchers of the multiplier-surrogate kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

namespace lbm {

constexpr int MLP_PARAMS = 9176;     // packed master parameters (floats)
constexpr int MLP_TRAINABLE = 9160;  // all but the output de-normalisation

void mlp_operands(const float *w, void *P, hipStream_t st);
// gradient (written to grad[MLP_TRAINABLE]) and loss (added to *loss) of
// count samples (a multiple of 32); gpart: mlp_partials_bytes(count) of
// device scratch
void mlp_train_batch(const void *P, const float *xh, const float *th, const int32_t *perm, int64_t off,
                     int64_t count, float *gpart, float *grad, float *loss, hipStream_t st);
size_t mlp_partials_bytes(int64_t count);
void mlp_adam(float *w, float *m, float *v, float *g, void *P, float lr, int t, hipStream_t st);
void mlp_predict(const void *P, const double *x, int64_t n, double *lam, hipStream_t st);
void mlp_label(const double *x, int64_t n, double tol, int max_it, double *lam, uint8_t *ok, int *iters,
               hipStream_t st);
size_t mlp_operands_bytes();

}  // namespace lbm
