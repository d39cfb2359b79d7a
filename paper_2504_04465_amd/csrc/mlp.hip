// mlp.hip -- training and evaluation kernels of the multiplier surrogate:
// Newton-labelled samples, BF16-MFMA forward and backward with FP32
// gradient accumulation, Adam on FP32 master weights, batched prediction.
#include "kernels.cuh"
#include "mlp.cuh"
#include "mlp_ops.h"

namespace lbm {

using L21 = Lattice<LAT_D2Q21>;

// ---------------------------------------------------------------------------
// master parameter -> BF16 / FP32 operand copies
// ---------------------------------------------------------------------------
// position of input neuron k in a row of the inference copy (the inverse
// of infer_neuron): K block, lane half and slot
__device__ inline int infer_pos(int k) {
  const int q = k >> 5, rem = k & 31, a = rem >> 3, h = (rem >> 2) & 1, s = rem & 3;
  return 16 * (2 * q + (a >> 1)) + 8 * h + 4 * (a & 1) + s;
}

__device__ inline void write_operand(MlpOperands *P, int i, float v) {
  const __bf16 b = (__bf16)v;
  MlpInfer &I = P->inf;
  if (i < MB1) {
    const int n = (i - MW1) / 4, k = (i - MW1) % 4;
    P->w1[n * 16 + k] = b;
    P->w1[n * 16 + 4 + k] = b;
    I.w1[n * 16 + k] = b;
    I.w1[n * 16 + 4 + k] = b;
  } else if (i < MW2) {
    P->b1[i - MB1] = v;
    I.b1[i - MB1] = v;
  } else if (i < MB2) {
    const int n = (i - MW2) / 64, k = (i - MW2) % 64;
    P->w2[n * 64 + k] = b;
    P->w2t[k * 64 + n] = b;
    I.w2[n * 64 + infer_pos(k)] = b;
  } else if (i < MW3) {
    P->b2[i - MB2] = v;
    I.b2[i - MB2] = v;
  } else if (i < MB3) {
    const int n = (i - MW3) / 64, k = (i - MW3) % 64;
    P->w3[n * 64 + k] = b;
    P->w3t[k * 64 + n] = b;
    I.w3[n * 64 + infer_pos(k)] = b;
  } else if (i < MW4) {
    P->b3[i - MB3] = v;
    I.b3[i - MB3] = v;
  } else if (i < MB4) {
    const int n = (i - MW4) / 64, k = (i - MW4) % 64;
    P->w4[n * 64 + k] = b;
    P->w4t[k * 16 + n] = b;
    I.w4hi[n * 64 + infer_pos(k)] = b;
    I.w4lo[n * 64 + infer_pos(k)] = (__bf16)(v - (float)b);
  } else if (i < MMU) {
    P->b4[i - MB4] = v;
    I.b4[i - MB4] = v;
  } else if (i < MSIG) {
    P->mu[i - MMU] = v;
  } else if (i < MLP_NPARAM) {
    P->sig[i - MSIG] = v;
  }
}

__global__ void k_mlp_operands(const float *w, MlpOperands *P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < MLP_NPARAM) write_operand(P, i, w[i]);
}

// Adam (Kingma & Ba 2015) on the trainable entries; clears the gradient
__global__ void k_mlp_adam(float *w, float *m, float *v, float *g, MlpOperands *P, float lr,
                           float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NTRAIN) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  w[i] = wi;
  g[i] = 0.0f;
  write_operand(P, i, wi);
}

// ---------------------------------------------------------------------------
// one 32-sample tile per wavefront: forward, loss, backward.  Each block
// writes its whole gradient (every trainable entry once) and its loss to a
// slot of its own, gpart[block][MLP_NTRAIN] and lpart[block]; k_mlp_gsum
// adds the slots in block order, so that training is reproducible run to
// run (float atomics would add them in arrival order)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_mlp_train(const MlpOperands *P, const float *xh, const float *th,
                                                  const int32_t *perm, int64_t off, float inv_count,
                                                  float *gpart, float *lpart) {
  float *grad = gpart + (int64_t)blockIdx.x * MLP_NTRAIN;
  __shared__ __align__(16) __bf16 xin[32 * 16];
  __shared__ __align__(16) __bf16 h1[32 * 64];
  __shared__ __align__(16) __bf16 h2[32 * 64];
  __shared__ __align__(16) __bf16 h3[32 * 64];
  __shared__ __align__(16) __bf16 da[32 * 64];
  __shared__ __align__(16) __bf16 db[32 * 64];
  __shared__ float z[3 * 32 * 64];
  __shared__ float y[32 * 8];
  __shared__ float d4[32 * 8];
  const int l = threadIdx.x;
  const int64_t base = off + (int64_t)blockIdx.x * 32;
  if (l < 32) {
    const int64_t s = perm[base + l];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float x = xh[s * 4 + k];
      const __bf16 hi = (__bf16)x;
      xin[l * 16 + k] = hi;
      xin[l * 16 + 4 + k] = (__bf16)(x - (float)hi);
    }
#pragma unroll
    for (int k = 8; k < 16; ++k) xin[l * 16 + k] = (__bf16)0.0f;
  }
  __syncthreads();
  mlp_forward_tile(P, xin, h1, h2, h3, y, z);
  // Huber loss (delta 0.5) on the normalised outputs and its gradient
  constexpr float HD = 0.5f;
  float part = 0.0f;
  if (l < 32) {
    const int64_t s = perm[base + l];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float r = y[l * 8 + k] - th[s * 8 + k];
      const float a = fabsf(r);
      d4[l * 8 + k] = fminf(fmaxf(r, -HD), HD) * inv_count;
      part += a <= HD ? 0.5f * r * r : HD * (a - 0.5f * HD);
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) part += __shfl_xor(part, m, 64);
  if (l == 0) lpart[blockIdx.x] = part * inv_count;
  __syncthreads();
  const int kr = 8 * (l >> 5), lc = l & 31;
  // dW4 = d4^T h3 (rows: 8 outputs of 32, columns: 64 hidden), K = samples
#pragma unroll
  for (int n0 = 0; n0 < 64; n0 += 32) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 16) {
      bf16x8 a, b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int s = k0 + kr + j;
        a[j] = lc < 8 ? (__bf16)d4[s * 8 + lc] : (__bf16)0.0f;
        b[j] = h3[s * 64 + n0 + lc];
      }
      acc = mfma32(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = c_row(l, r);
      if (m < 8) grad[MW4 + m * 64 + n0 + lc] = acc[r];
    }
  }
  if (l < 8) {
    float s = 0.0f;
    for (int q = 0; q < 32; ++q) s += d4[q * 8 + l];
    grad[MB4 + l] = s;
  }
  // delta3 = (d4 W4) .* silu'(z3)
#pragma unroll
  for (int n0 = 0; n0 < 64; n0 += 32) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (kr + j) < 8 ? (__bf16)d4[lc * 8 + kr + j] : (__bf16)0.0f;
    const bf16x8 b = *(const bf16x8 *)(P->w4t + (n0 + lc) * 16 + kr);
    acc = mfma32(a, b, acc);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(l, r), col = n0 + lc;
      da[row * 64 + col] = (__bf16)(acc[r] * dsilu_f(z[4096 + row * 64 + col]));
    }
  }
  __syncthreads();
  // weight gradient of a 64 x 64 layer: dW = delta^T h (K = samples)
  auto grad_w = [&](const __bf16 *dl, const __bf16 *hp, int woff, int boff) {
#pragma unroll
    for (int m0 = 0; m0 < 64; m0 += 32)
#pragma unroll
      for (int n0 = 0; n0 < 64; n0 += 32) {
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int k0 = 0; k0 < 32; k0 += 16) {
          bf16x8 a, b;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int s = k0 + kr + j;
            a[j] = dl[s * 64 + m0 + lc];
            b[j] = hp[s * 64 + n0 + lc];
          }
          acc = mfma32(a, b, acc);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) grad[woff + (m0 + c_row(l, r)) * 64 + n0 + lc] = acc[r];
      }
    float s = 0.0f;
    for (int q = 0; q < 32; ++q) s += (float)dl[q * 64 + l];
    grad[boff + l] = s;
  };
  grad_w(da, h2, MW3, MB3);
  // delta2 = (delta3 W3) .* silu'(z2)
#pragma unroll
  for (int n0 = 0; n0 < 64; n0 += 32) {
    const f32x16 acc = gemm_aw<64>(da, 64, P->w3t, 64, n0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(l, r), col = n0 + lc;
      db[row * 64 + col] = (__bf16)(acc[r] * dsilu_f(z[2048 + row * 64 + col]));
    }
  }
  __syncthreads();
  grad_w(db, h1, MW2, MB2);
  // delta1 = (delta2 W2) .* silu'(z1)
  __syncthreads();
#pragma unroll
  for (int n0 = 0; n0 < 64; n0 += 32) {
    const f32x16 acc = gemm_aw<64>(db, 64, P->w2t, 64, n0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(l, r), col = n0 + lc;
      da[row * 64 + col] = (__bf16)(acc[r] * dsilu_f(z[row * 64 + col]));
    }
  }
  __syncthreads();
  // dW1 = delta1^T xin; the high and low input columns share the weights
#pragma unroll
  for (int m0 = 0; m0 < 64; m0 += 32) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 16) {
      bf16x8 a, b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int s = k0 + kr + j;
        a[j] = da[s * 64 + m0 + lc];
        b[j] = lc < 16 ? xin[s * 16 + lc] : (__bf16)0.0f;
      }
      acc = mfma32(a, b, acc);
    }
    // columns lc and lc + 4 (the high and low parts of input lc) share
    // the weight: their lanes (same rows) are added before the store
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v = acc[r] + __shfl_xor(acc[r], 4);
      if (lc < 4) grad[MW1 + (m0 + c_row(l, r)) * 4 + lc] = v;
    }
  }
  {
    float s = 0.0f;
    for (int q = 0; q < 32; ++q) s += (float)da[q * 64 + l];
    grad[MB1 + l] = s;
  }
}

// gradient of the batch = the blocks' slots added in block order; the
// loss is accumulated (over the batches of an epoch)
__global__ void __launch_bounds__(256) k_mlp_gsum(const float *gpart, const float *lpart, int nblk, float *grad,
                                                  float *loss) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < MLP_NTRAIN) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += gpart[(int64_t)b * MLP_NTRAIN + i];
    grad[i] = s;
  }
  if (i == 0) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += lpart[b];
    *loss += s;
  }
}

// ---------------------------------------------------------------------------
// batched prediction of the multipliers from raw states (rho, u_x, u_y, T)
// ---------------------------------------------------------------------------
// (the same inference as the collide: weights staged in LDS once per block,
// one sample per lane)
__global__ void __launch_bounds__(256) k_mlp_predict(const MlpOperands *P, const double *x, int64_t n,
                                                     double *lam) {
  __shared__ MlpInfer W;
  stage_infer(&P->inf, &W);
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool ok = s < n;
  float ux = ok ? (float)x[s * 4 + 1] : 0.0f, uy = ok ? (float)x[s * 4 + 2] : 0.0f;
  const Canon cn = canonical(ux, uy);
  float xin[4], y[8];
  mlp_normalise(ok ? (float)x[s * 4] : 1.0f, ux, uy, ok ? (float)x[s * 4 + 3] : 1.0f, xin);
  mlp_infer_wave(W, xin, y);
  if (ok) {
    double out[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = (double)P->mu[k] + (double)P->sig[k] * (double)y[k];
    uncanonical(cn, out);
#pragma unroll
    for (int k = 0; k < 8; ++k) lam[s * 8 + k] = out[k];
  }
}

// ---------------------------------------------------------------------------
// Newton labels: cold start (lambda = 0) per sample; ok = converged
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_label(const double *x, int64_t n, double tol, int max_it,
                                                   double *lam, uint8_t *ok, int *iters) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double l8[NLAM], e[L21::Q];
#pragma unroll
  for (int a = 0; a < NLAM; ++a) l8[a] = 0.0;
  const int it = newton_solve<L21>(x[s * 4 + 1], x[s * 4 + 2], x[s * 4 + 3], l8, tol, max_it, e);
  bool good = it >= 0;
#pragma unroll
  for (int a = 0; a < NLAM; ++a) {
    good = good && isfinite(l8[a]);
    lam[s * 8 + a] = l8[a];
  }
  ok[s] = good ? 1 : 0;
  iters[s] = it;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void mlp_operands(const float *w, void *P, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_operands, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, w, (MlpOperands *)P);
}

void mlp_train_batch(const void *P, const float *xh, const float *th, const int32_t *perm, int64_t off,
                     int64_t count, float *gpart, float *grad, float *loss, hipStream_t st) {
  const int nblk = (int)(count / 32);
  float *lpart = gpart + (int64_t)nblk * MLP_NTRAIN;
  hipLaunchKernelGGL(k_mlp_train, dim3((unsigned)nblk), dim3(64), 0, st, (const MlpOperands *)P, xh, th, perm, off,
                     1.0f / (float)(count * 8), gpart, lpart);
  hipLaunchKernelGGL(k_mlp_gsum, dim3((MLP_NTRAIN + 255) / 256), dim3(256), 0, st, gpart, lpart, nblk, grad, loss);
}

size_t mlp_partials_bytes(int64_t count) { return sizeof(float) * (size_t)(count / 32) * (MLP_NTRAIN + 1); }

void mlp_adam(float *w, float *m, float *v, float *g, void *P, float lr, int t, hipStream_t st) {
  const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NTRAIN + 255) / 256), dim3(256), 0, st, w, m, v, g,
                     (MlpOperands *)P, lr, c1, c2);
}

void mlp_predict(const void *P, const double *x, int64_t n, double *lam, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const MlpOperands *)P, x,
                     n, lam);
}

void mlp_label(const double *x, int64_t n, double tol, int max_it, double *lam, uint8_t *ok, int *iters,
               hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_label, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, tol, max_it, lam,
                     ok, iters);
}

size_t mlp_operands_bytes() { return sizeof(MlpOperands); }

}  // namespace lbm
