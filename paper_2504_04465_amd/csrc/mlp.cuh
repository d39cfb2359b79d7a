// mlp.cuh -- the multiplier surrogate on BF16 matrix cores (gfx950).
//
// Network 4 -> 64 -> 64 -> 64 -> 8, SiLU hidden layers, linear output, on
// normalised inputs ((rho - 2.6)/2.4, u_x/2.5, u_y/2.5, (T - 1.75)/1.25) and
// outputs (lambda = mu + sigma * y).  One wavefront evaluates a tile of 32
// samples with v_mfma_f32_32x32x16_bf16 (FP32 accumulation):
//   A operand, lane l: row l % 32, k = 8 (l / 32) + j   (8 bf16)
//   B operand, lane l: k = 8 (l / 32) + j, column l % 32 (8 bf16)
//   C, lane l, register r: row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
// Inputs enter as a high + low BF16 pair (columns 0-3 and 4-7 of a 16-wide
// K block that shares the first-layer weights), so they keep ~16 bits.
#pragma once

#include <hip/hip_runtime.h>

#include "ops.h"

namespace lbm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// packed FP32 master parameters (floats)
constexpr int MW1 = 0, MB1 = 256, MW2 = 320, MB2 = 4416, MW3 = 4480, MB3 = 8576, MW4 = 8640,
              MB4 = 9152, MMU = 9160, MSIG = 9168, MLP_NPARAM = 9176, MLP_NTRAIN = 9160;

// Inference layout (mlp_infer_wave): the layers are evaluated transposed,
// Z^T = W X^T, with the samples as the MFMA's columns.  The accumulator a
// lane holds for output block mb (rows 32 mb .. 32 mb + 31) is then, after
// the activation, the lane's B operand of the next layer for two of its
// 16-wide K blocks, without leaving the registers, provided the next
// layer's K index is permuted: K block kb, lane half h, slot j stands for
// neuron 32 (kb / 2) + 8 (2 (kb % 2) + j / 4) + 4 h + j % 4 (the row that
// accumulator register 8 (kb % 2) + j of lane half h holds).
__host__ __device__ constexpr int infer_neuron(int kb, int h, int j) {
  return 32 * (kb / 2) + 8 * (2 * (kb % 2) + j / 4) + 4 * h + j % 4;
}

struct alignas(16) MlpInfer {
  __bf16 w1[64 * 16];     // [out][16]: W1 in columns 0-3 (high input parts) and 4-7 (low parts)
  __bf16 w2[64 * 64];     // [out][permuted in]
  __bf16 w3[64 * 64];
  __bf16 w4hi[32 * 64];   // [out 32, 8 used][permuted in], high BF16 part of W4
  __bf16 w4lo[32 * 64];   // W4 - high part, rounded to BF16
  float b1[64], b2[64], b3[64], b4[8];
};

// BF16 operand copies derived from the master parameters
struct MlpOperands {
  __bf16 w1[64 * 16];   // [out][16]: W1 in columns 0-3 and again in 4-7
  __bf16 w2[64 * 64];   // [out][in]
  __bf16 w3[64 * 64];
  __bf16 w4[32 * 64];   // [out 32, 8 used][in]
  __bf16 w2t[64 * 64];  // [in][out]
  __bf16 w3t[64 * 64];
  __bf16 w4t[64 * 16];  // [in][out 16, 8 used]
  float b1[64], b2[64], b3[64], b4[32];
  float mu[8], sig[8];
  alignas(16) MlpInfer inf;  // the inference copy (transposed, permuted)
};

__device__ inline f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ inline int c_row(int l, int r) { return ((r >> 2) << 3) + ((l >> 5) << 2) + (r & 3); }

// SiLU and its derivative with the hardware exponential and reciprocal
// (about 1 ulp each; the activations are rounded to BF16 right after)
__device__ inline float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu_f(float z) { return z * sigmoid_f(z); }
__device__ inline float dsilu_f(float z) {
  const float s = sigmoid_f(z);
  return s * (1.0f + z * (1.0f - s));
}

// acc(32 x 32) = A[32 x K] (LDS row-major, lda) * B, with B[k][n] = W[n0 + n][k]
// (W row-major in global memory, ldw)
template <int K>
__device__ inline f32x16 gemm_aw(const __bf16 *A, int lda, const __bf16 *W, int ldw, int n0) {
  const int l = threadIdx.x & 63;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x8 a = *(const bf16x8 *)(A + (l & 31) * lda + k0 + 8 * (l >> 5));
    const bf16x8 b = *(const bf16x8 *)(W + (n0 + (l & 31)) * ldw + k0 + 8 * (l >> 5));
    acc = mfma32(a, b, acc);
  }
  return acc;
}

// Reflection symmetry of the multipliers: the network sees the canonical
// state u_x >= u_y >= 0; the multipliers of the actual state follow by
// swapping the x / y components back and flipping the signs of the odd ones
// (lambda order: 1, x, y, xx, xy, yy, x|xi|^2, y|xi|^2).
struct Canon {
  bool sx, sy, swap;
};

__device__ inline Canon canonical(float &ux, float &uy) {
  Canon c;
  c.sx = ux < 0.0f;
  c.sy = uy < 0.0f;
  float a = fabsf(ux), b = fabsf(uy);
  c.swap = b > a;
  ux = c.swap ? b : a;
  uy = c.swap ? a : b;
  return c;
}

__device__ inline void uncanonical(const Canon &c, double *lam) {
  if (c.swap) {
    double t = lam[1]; lam[1] = lam[2]; lam[2] = t;
    t = lam[3]; lam[3] = lam[5]; lam[5] = t;
    t = lam[6]; lam[6] = lam[7]; lam[7] = t;
  }
  if (c.sx) { lam[1] = -lam[1]; lam[4] = -lam[4]; lam[6] = -lam[6]; }
  if (c.sy) { lam[2] = -lam[2]; lam[4] = -lam[4]; lam[7] = -lam[7]; }
}

// the network's normalised inputs
__device__ inline void mlp_normalise(float rho, float ux, float uy, float T, float (&x)[4]) {
  x[0] = (rho - 2.6f) / 2.4f;
  x[1] = ux / 2.5f;
  x[2] = uy / 2.5f;
  x[3] = (T - 1.75f) / 1.25f;
}

// split one normalised input row into the high / low BF16 columns
__device__ inline void mlp_input_row(__bf16 *xin_row, float rho, float ux, float uy, float T) {
  const float x[4] = {(rho - 2.6f) / 2.4f, ux / 2.5f, uy / 2.5f, (T - 1.75f) / 1.25f};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const __bf16 hi = (__bf16)x[k];
    xin_row[k] = hi;
    xin_row[4 + k] = (__bf16)(x[k] - (float)hi);
  }
#pragma unroll
  for (int k = 8; k < 16; ++k) xin_row[k] = (__bf16)0.0f;
}

// Between the layers only the wavefront that owns a tile reads what its
// lanes wrote to LDS (every caller gives each wavefront its own tile), so
// waiting for the wavefront's own LDS writes suffices; a block barrier
// would make the block's wavefronts wait for each other.
__device__ inline void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// forward of one 32-sample tile held by one wavefront.  xin [32][16],
// ha / hb [32][64] scratch, y [32][8] output (normalised), z (optional,
// training) [3][32][64] pre-activations, h (optional) keeps h1..h3 in
// ha, hb, hc for the backward pass.
__device__ inline void mlp_forward_tile(const MlpOperands *P, const __bf16 *xin, __bf16 *h1,
                                        __bf16 *h2, __bf16 *h3, float *y, float *z) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int n0 = 0; n0 < 64; n0 += 32) {
    const f32x16 acc = gemm_aw<16>(xin, 16, P->w1, 16, n0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(l, r), col = n0 + (l & 31);
      const float v = acc[r] + P->b1[col];
      if (z) z[row * 64 + col] = v;
      h1[row * 64 + col] = (__bf16)silu_f(v);
    }
  }
  lds_wave_sync();
#pragma unroll
  for (int n0 = 0; n0 < 64; n0 += 32) {
    const f32x16 acc = gemm_aw<64>(h1, 64, P->w2, 64, n0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(l, r), col = n0 + (l & 31);
      const float v = acc[r] + P->b2[col];
      if (z) z[2048 + row * 64 + col] = v;
      h2[row * 64 + col] = (__bf16)silu_f(v);
    }
  }
  lds_wave_sync();
#pragma unroll
  for (int n0 = 0; n0 < 64; n0 += 32) {
    const f32x16 acc = gemm_aw<64>(h2, 64, P->w3, 64, n0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(l, r), col = n0 + (l & 31);
      const float v = acc[r] + P->b3[col];
      if (z) z[4096 + row * 64 + col] = v;
      h3[row * 64 + col] = (__bf16)silu_f(v);
    }
  }
  lds_wave_sync();
  {
    const f32x16 acc = gemm_aw<64>(h3, 64, P->w4, 64, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = c_row(l, r), col = l & 31;
      if (col < 8) y[row * 8 + col] = acc[r] + P->b4[col];
    }
  }
  lds_wave_sync();
}


// ---------------------------------------------------------------------------
// inference of a whole wavefront's 64 samples (two tiles of 32), weights in
// LDS (W, staged by the caller), activations in registers between layers.
// x: the lane's normalised inputs; y: its normalised outputs.
// ---------------------------------------------------------------------------
typedef short i16x8 __attribute__((ext_vector_type(8)));

__device__ inline bf16x8 lds_b128(const __bf16 *p) { return *(const bf16x8 *)p; }

// bias + SiLU of one 32-row output block, packed as the next layer's B
// operands (K blocks 2 mb and 2 mb + 1); optionally also the low parts
template <bool LO>
__device__ inline void act_pack(const f32x16 &acc, const float *bias, int mb, int h, bf16x8 *bn, bf16x8 *bl) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 32 * mb + 8 * (r >> 2) + 4 * h + (r & 3);
    const float v = silu_f(acc[r] + bias[row]);
    const __bf16 hi = (__bf16)v;
    bn[2 * mb + (r >> 3)][r & 7] = hi;
    if (LO) bl[2 * mb + (r >> 3)][r & 7] = (__bf16)(v - (float)hi);
  }
}

__device__ inline void mlp_infer_wave(const MlpInfer &W, const float (&x)[4], float (&y)[8]) {
  const int l = threadIdx.x & 63, h = l >> 5, row = l & 31;
  // the lane's inputs as high + low BF16 parts (K slots 0-3 and 4-7)
  bf16x8 xf;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const __bf16 hi = (__bf16)x[k];
    xf[k] = hi;
    xf[4 + k] = (__bf16)(x[k] - (float)hi);
  }
  // the other half's inputs (tile 1's samples sit in lanes 32-63)
  bf16x8 xo;
  {
    const i16x8 v = __builtin_bit_cast(i16x8, xf);
    i16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (short)__shfl_xor((int)v[k], 32);
    xo = __builtin_bit_cast(bf16x8, o);
  }
  bf16x8 zero;
#pragma unroll
  for (int k = 0; k < 8; ++k) zero[k] = (__bf16)0.0f;
  float out[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    // layer 1: the B operand holds the tile's inputs in lane half 0
    const bf16x8 b1 = h == 0 ? (t == 0 ? xf : xo) : zero;
    bf16x8 ba[4], bb[4], blo[4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
      acc = mfma32(lds_b128(W.w1 + (32 * mb + row) * 16 + 8 * h), b1, acc);
      act_pack<false>(acc, W.b1, mb, h, ba, blo);
    }
    // layers 2 and 3
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma32(lds_b128(W.w2 + (32 * mb + row) * 64 + 16 * kb + 8 * h), ba[kb], acc);
      act_pack<false>(acc, W.b2, mb, h, bb, blo);
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma32(lds_b128(W.w3 + (32 * mb + row) * 64 + 16 * kb + 8 * h), bb[kb], acc);
      act_pack<true>(acc, W.b3, mb, h, ba, blo);
    }
    // output layer with split operands: hi.hi + hi.lo + lo.hi
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x8 whi = lds_b128(W.w4hi + row * 64 + 16 * kb + 8 * h);
      acc = mfma32(whi, ba[kb], acc);
      acc = mfma32(whi, blo[kb], acc);
      acc = mfma32(lds_b128(W.w4lo + row * 64 + 16 * kb + 8 * h), ba[kb], acc);
    }
    // rows 0-7 are the outputs: lane half h holds outputs 4 h .. 4 h + 3
#pragma unroll
    for (int r = 0; r < 4; ++r) out[t][r] = acc[r] + W.b4[4 * h + r];
  }
  // cell of lane l: tile h, sample l % 32; outputs 0-3 from lane half 0 of
  // that tile, 4-7 from lane half 1
  float recv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) recv[r] = __shfl_xor(h == 0 ? out[1][r] : out[0][r], 32);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    y[r] = h == 0 ? out[0][r] : recv[r];
    y[4 + r] = h == 0 ? recv[r] : out[1][r];
  }
}

// copy of the inference weights into LDS by every thread of the block
__device__ inline void stage_infer(const MlpInfer *g, MlpInfer *s) {
  constexpr int N = (int)(sizeof(MlpInfer) / 16);
  const uint4 *src = (const uint4 *)g;
  uint4 *dst = (uint4 *)s;
  for (int i = threadIdx.x; i < N; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
}

}  // namespace lbm
