// kernels.cuh -- HIP kernels of the refined-grid lattice Boltzmann update for
// gfx950, templated on lattice, collision model and population storage.
//
// Data layout (HBM): populations in chunks of 4096 slots, each chunk the Q
// rows of its slots one after the other (f[pix<Q>(i, c)]), double buffered
// per level; each level's newest buffer holds post-collision populations
// (the pull of the next update streams them).  The pull source of
// population i of cell c is nbr[(i-1) * stride + c]:
//   >= vbase : a coalesced slot of a coarse ghost (unknown population),
//   >= 0     : a cell of the same level (the cell itself when the paper's
//              rule keeps the own value),
//   -1       : bounce-back on a wall or solid,
//   -2 - k   : Ladd bounce-back on the moving wall of face k.
// One thread updates one cell; a 256-thread block holds 4 wavefronts of 64
// Z-ordered cells, so a wavefront is a 8x8 (2-D) or 4x4x4 (3-D) brick.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "grid_builder.h"
#include "lattice.h"
#include "ops.h"

namespace lbm {

constexpr int BLOCK = 256;

// ---------------------------------------------------------------------------
// storage traits: FP64, FP32, FP16 holding f_i - w_i (compute in FP32).
// stn is a streaming (non-temporal) store: the collide kernel's output is not
// read again before the level's next update, so it should not displace the
// neighbour lines that other wavefronts still pull from the L2.
// ---------------------------------------------------------------------------
// pointers into global memory (address space 1): accesses through them are
// global, not flat, instructions, which take an SGPR base plus a VGPR offset
template <class T>
using gptr = __attribute__((address_space(1))) T *;

// a storage value read through a global pointer (__half by its bits: its
// class type has no constructor from that address space)
template <class S>
__device__ inline S gload(gptr<const char> p) {
  if constexpr (std::is_same<S, __half>::value) return __ushort_as_half(*(gptr<const unsigned short>)p);
  else return *(gptr<const S>)p;
}

template <class S>
struct Sto;
template <>
struct Sto<double> {
  using C = double;
  __device__ static C ld(const double *p, int64_t k, double) { return p[k]; }
  __device__ static C ldv(double v, double) { return v; }
  __device__ static C ldr(double v) { return v; }
  __device__ static void st(double *p, int64_t k, C v, double) { p[k] = v; }
  __device__ static void stn(double *p, int64_t k, C v, double) { __builtin_nontemporal_store(v, p + k); }
  __device__ static void stp(double *p, C v, double) { __builtin_nontemporal_store(v, p); }
  __device__ static void stg(gptr<double> p, C v, double) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Sto<float> {
  using C = float;
  __device__ static C ld(const float *p, int64_t k, double) { return p[k]; }
  __device__ static C ldv(float v, double) { return v; }
  __device__ static C ldr(float v) { return v; }
  __device__ static void st(float *p, int64_t k, C v, double) { p[k] = v; }
  __device__ static void stn(float *p, int64_t k, C v, double) { __builtin_nontemporal_store(v, p + k); }
  __device__ static void stp(float *p, C v, double) { __builtin_nontemporal_store(v, p); }
  __device__ static void stg(gptr<float> p, C v, double) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Sto<__half> {
  using C = float;
  __device__ static C ld(const __half *p, int64_t k, double w) {
    return __half2float(p[k]) + (float)w;
  }
  __device__ static C ldv(__half v, double w) { return __half2float(v) + (float)w; }
  // the stored value itself (f_i - w_i), for kernels that work on it
  __device__ static C ldr(__half v) { return __half2float(v); }
  // the FP32 value is rounded to FP32 before the conversion: left to
  // itself the compiler fuses the last multiply or add into a mixed-precision
  // FMA with one rounding to FP16 in some kernels and not in others, and
  // kernels that must agree bit for bit (in place vs two buffers) would not
  __device__ static __half cvt(C v, double w) {
    float t = v - (float)w;
    asm volatile("" : "+v"(t));
    return __float2half_rn(t);
  }
  __device__ static void st(__half *p, int64_t k, C v, double w) { p[k] = cvt(v, w); }
  __device__ static void stn(__half *p, int64_t k, C v, double w) {
    __builtin_nontemporal_store(__half_as_ushort(cvt(v, w)), (unsigned short *)p + k);
  }
  __device__ static void stp(__half *p, C v, double w) {
    __builtin_nontemporal_store(__half_as_ushort(cvt(v, w)), (unsigned short *)p);
  }
  __device__ static void stg(gptr<__half> p, C v, double w) {
    __builtin_nontemporal_store(__half_as_ushort(cvt(v, w)), (gptr<unsigned short>)p);
  }
};

// Newton multipliers (warm start of the numerical equilibrium) are kept in
// FP64 next to FP64 populations, so that an FP64 run restarts every solve
// from the multipliers it converged to; reduced-precision storage keeps them
// in FP32.
template <class S>
struct LamOf {
  using T = float;
};
template <>
struct LamOf<double> {
  using T = double;
};
template <class S>
using LamT = typename LamOf<S>::T;

// Blocks are dealt to the 8 XCDs round-robin; remap so that each XCD works
// on one contiguous range of Z-ordered cells and its L2 sees the neighbours.
__device__ inline int64_t xcd_map(uint32_t b, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u, x = b & 7u, loc = b >> 3;
  return (int64_t)x * q + (x < r ? x : r) + loc;
}
__device__ inline int64_t xcd_block() { return xcd_map(blockIdx.x, gridDim.x); }

template <int W, class T>
__device__ inline T group_sum(T v) {
#pragma unroll
  for (int m = 1; m < W; m <<= 1) v += __shfl_xor(v, m, W);
  return v;
}

template <class L>
__device__ constexpr int cx_(int i, int d) {
  return d == 0 ? L::S.v[i].x : d == 1 ? L::S.v[i].y : L::S.v[i].z;
}

// velocity of moving wall k projected on xi_i, selected without indexing the
// argument block dynamically
template <class L>
__device__ inline double wall_dot(const double (&uw)[6][3], int k, int i) {
  double r = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (f == k) r = cx_<L>(i, 0) * uw[f][0] + cx_<L>(i, 1) * uw[f][1] + cx_<L>(i, 2) * uw[f][2];
  return r;
}

// the cell's perturbation of the moving-wall velocity (inflow noise)
// projected on xi_i: xdu holds [Q-1][xstride] per explicit row, or is null;
// read only on a moving-wall link
__device__ inline double noise_dot(const double *xdu, int64_t xstride, int64_t row, int i) {
  return xdu ? xdu[(int64_t)(i - 1) * xstride + row] : 0.0;
}

// ---------------------------------------------------------------------------
// bricks: 64 cells (4x4x4 or 8x8) per wavefront, Z order inside the brick
// ---------------------------------------------------------------------------
template <class L>
struct Brick {
  static constexpr int SH = L::D == 3 ? 2 : 3;
  static constexpr int BS = 1 << SH;
  static constexpr int NB = L::D == 3 ? 27 : 9;
  static constexpr int NBP = L::D == 3 ? 32 : 16;
};

// element of population i of slot s (the chunked layout of the buffers)
template <int Q>
__device__ inline int64_t pix(int64_t i, int64_t s) {
  return (((s >> PCH_SH) * Q + i) << PCH_SH) + (s & (PCH - 1));
}

// offset of brick b's population-0 row in units of 64 values (32 bits for
// any buffer of fewer than 2^38 / Q slots)
template <int Q>
__device__ inline uint32_t brick_unit(int32_t b) {
  constexpr int BPC = (int)(PCH >> 6);  // bricks per chunk
  return (uint32_t)(b / BPC) * (uint32_t)(Q * BPC) + (uint32_t)(b % BPC);
}

// coordinate d of lane inside its brick
template <class L>
__device__ inline int lane_coord(int lane, int d) {
  int r = 0;
#pragma unroll
  for (int b = 0; b < Brick<L>::SH; ++b) r |= ((lane >> (L::D * b + d)) & 1) << b;
  return r;
}

// lane of local coordinate p (0 <= p < BS) along axis d
template <class L>
__device__ inline int lane_bits(int p, int d) {
  int r = 0;
#pragma unroll
  for (int b = 0; b < Brick<L>::SH; ++b) r |= ((p >> b) & 1) << (L::D * b + d);
  return r;
}

// Populations 1..Q-1 of cell c pulled through its explicit row: every
// source is loaded before any is used, so the loads overlap.
// Populations not in `want` (bit i) are neither loaded nor set.
// AA = 2: the single in-place buffer after an even step holds cell x's
// post-collision population i in row opp(i); pulls swap the rows (a wall
// returns the cell's own row i).
//
// RAW: FP16 storage only, the populations are returned as stored (f_i - w_i);
// the moving-wall term is the same in that representation.
template <class L, class S, bool PRE, bool DDF, int AA = 0, bool NZ = true, bool RAW = false>
__device__ inline void gather_row(const S *fin, const S *gin, const int32_t *xnbr, int64_t xstride, int64_t row,
                                  int64_t vbase, int64_t c, const double (&uw)[6][3], double cs2w,
                                  typename Sto<S>::C *f, typename Sto<S>::C *g, uint64_t want = ~0ull,
                                  const double *xdu = nullptr) {
  using C = typename Sto<S>::C;
  int32_t sv[L::Q];
#pragma unroll
  for (int i = 1; i < L::Q; ++i) sv[i] = ((want >> i) & 1ull) ? xnbr[(int64_t)(i - 1) * xstride + row] : 0;
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    if (!((want >> i) & 1ull)) continue;
    const int32_t s = sv[i];
    int64_t idx;
    const int ri = AA == 2 ? L::S.opp[i] : i, ro = AA == 2 ? i : L::S.opp[i];
    if (PRE) idx = pix<L::Q>(i, (int64_t)s >= vbase ? (int64_t)s : c);
    else idx = s >= 0 ? pix<L::Q>(ri, s) : pix<L::Q>(ro, c);
    // the lattice is symmetric: w of the opposite population is w_i
    f[i] = RAW ? Sto<S>::ldr(fin[idx]) : Sto<S>::ld(fin, idx, L::S.w[i]);
    if (DDF) g[i] = Sto<S>::ld(gin, idx, 0.0);
  }
  if (!PRE) {
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
      if (((want >> i) & 1ull) && sv[i] <= -2)
        f[i] += (C)(2.0 * L::S.w[i] * (wall_dot<L>(uw, -2 - sv[i], i) + (NZ ? noise_dot(xdu, xstride, row, i) : 0.0)) /
                    cs2w);
  }
}

// Gather of the Q (2Q) populations a cell pulls (f_i from x - xi_i).
//
// Bulk lanes: the source of population i sits in the brick at offset
// dir = sum_d w_d 3^d (w_d = 0, 1, 2 for a step to the lower neighbour, none,
// the upper neighbour along d) at local coordinates (lc - xi_i) mod BS.  The
// offset of every neighbour brick (brick_unit) is staged in LDS (nbs: the
// block's table, [wavefront][NBP]); per lane and axis the table K[d][xi_d]
// packs (LDS byte offset of the direction part, plus the wavefront's row in
// K[0]) << 16 | (byte offset of the local coordinate part), so a population
// costs two integer adds, a shift, an LDS read, a shift-or (a multiply-add
// for buffers over 4 GB) and a load from the population's row base.
//
// Lanes flagged in the brick's exception mask read their explicit row:
// every source is loaded before any is used, so the loads overlap.  In a
// two-buffer pull (not PRE, AA = 0) on a nearest-neighbour lattice they
// take the bulk addresses with the other lanes first and read the row only
// for the populations whose source differs (clear bits of the row's
// regular-pull mask), so the wavefront does not run a second, serial
// gather for them.  The multi-speed lattices keep the split: there the
// bulk values held across the row reads cost registers (D2Q37: 167 -> 193
// VGPRs, one wavefront per SIMD fewer) and time.
// nbs must be a staged table: gather_one reads exception rows itself.
template <class L, class S, bool PRE, bool DDF, int AA = 0, bool NZ = true, bool RAW = false, bool O32 = false>
__device__ inline void gather(const S *fin, const S *gin, const Topo &tp, const uint32_t *nbs, int64_t vbase, int64_t c, int lane, int32_t brick, uint64_t xm,
                              const double (&uw)[6][3], double cs2w, typename Sto<S>::C *f,
                              typename Sto<S>::C *g) {
  using C = typename Sto<S>::C;
  constexpr int BS = Brick<L>::BS, R = L::B, D = L::D;
  const int64_t c0 = pix<L::Q>(0, c);
  f[0] = RAW ? Sto<S>::ldr(fin[c0]) : Sto<S>::ld(fin, c0, L::S.w[0]);
  if (DDF) g[0] = Sto<S>::ld(gin, c0, 0.0);
  constexpr bool UNI = !PRE && AA == 0 && L::B == 1;
  const bool ex = (xm >> lane) & 1ull;
  if (UNI || !ex) {
    if (PRE) {
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        f[i] = RAW ? Sto<S>::ldr(fin[c0 + i * PCH]) : Sto<S>::ld(fin, c0 + i * PCH, L::S.w[i]);
        if (DDF) g[i] = Sto<S>::ld(gin, c0 + i * PCH, 0.0);
      }
      return;
    }
    // the wavefront's row of the block's table rides in K[0], so that the
    // LDS address of a population's neighbour brick is one shift of k
    const uint32_t wrow = (uint32_t)(threadIdx.x >> 6) * (uint32_t)(Brick<L>::NBP * 4);
    uint32_t K[3][2 * R + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lc = d < D ? lane_coord<L>(lane, d) : 0;
#pragma unroll
      for (int x = -R; x <= R; ++x) {
        if (d >= D) {
          K[d][x + R] = 0u;
          continue;
        }
        const int p = lc - x;
        const uint32_t w = p < 0 ? 0u : (p >= BS ? 2u : 1u);
        const uint32_t pw = d == 0 ? 1u : (d == 1 ? 3u : 9u);
        K[d][x + R] = ((w * pw * 4u + (d == 0 ? wrow : 0u)) << 16) |
                      ((uint32_t)lane_bits<L>(p & (BS - 1), d) * (uint32_t)sizeof(S));
      }
    }
    const char *fb = (const char *)fin;
    const char *gb = (const char *)gin;
    constexpr int64_t rbytes = PCH * (int64_t)sizeof(S);
    // O32: the brick's byte offset fits 32 bits (a buffer under 4 GB) and
    // is added to the uniform row base by the load itself
    using OffT = std::conditional_t<O32, uint32_t, uint64_t>;
    {
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        const uint32_t k = K[0][cx_<L>(i, 0) + R] + K[1][cx_<L>(i, 1) + R] + K[2][cx_<L>(i, 2) + R];
        const OffT off = (OffT)nbs[k >> 18] * (OffT)(64u * sizeof(S)) + (OffT)(k & 0xffffu);
        const int64_t ri = AA == 2 ? L::S.opp[i] : i;
        auto row = (gptr<const char>)(fb + ri * rbytes);
        asm("" : "+s"(row));  // the uniform row base stays in SGPRs
        const S v = gload<S>(row + off);
        f[i] = RAW ? Sto<S>::ldr(v) : Sto<S>::ldv(v, L::S.w[i]);
        if (DDF) {
          auto grow = (gptr<const char>)(gb + ri * rbytes);
          asm("" : "+s"(grow));
          g[i] = Sto<S>::ldv(gload<S>(grow + off), 0.0);
        }
      }
    }
  }
  if (ex) {
    const int64_t row = tp.xbase[brick] + __popcll(xm & ((1ull << lane) - 1ull));
    gather_row<L, S, PRE, DDF, AA, NZ, RAW>(fin, gin, tp.xnbr, tp.xstride, row, vbase, c, uw, cs2w, f, g,
                                            UNI ? ~tp.xreg[row] : ~0ull, tp.xdu);
  }
}

// In-place (AA-pattern) store after an odd step: population i of cell x goes
// to row i of x + xi_i (the cell whose pull of i reads x), or, where that is a
// wall, back to the cell's own row opp(i) with the moving-wall correction of
// population opp(i) (the bounce-back the next pull would have applied).
// RAW: f holds f_i - w_i (FP16 storage), stored as it is.
template <class L, class S, bool DDF, bool RAW = false>
__device__ inline void push_store(S *fout, S *gout, const Topo &tp, const uint32_t *nbs, int64_t c,
                                  int lane, int32_t brick, uint64_t xm, const double (&uw)[6][3], double cs2w,
                                  const typename Sto<S>::C *f, const typename Sto<S>::C *g) {
  using C = typename Sto<S>::C;
  constexpr int BS = Brick<L>::BS, R = L::B, D = L::D;
  Sto<S>::stn(fout, pix<L::Q>(0, c), f[0], RAW ? 0.0 : L::S.w[0]);
  if (DDF) Sto<S>::stn(gout, pix<L::Q>(0, c), g[0], 0.0);
  if (!((xm >> lane) & 1ull)) {
    // the wavefront's row of the block's table rides in K[0], so that the
    // LDS address of a population's neighbour brick is one shift of k
    const uint32_t wrow = (uint32_t)(threadIdx.x >> 6) * (uint32_t)(Brick<L>::NBP * 4);
    uint32_t K[3][2 * R + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lc = d < D ? lane_coord<L>(lane, d) : 0;
#pragma unroll
      for (int x = -R; x <= R; ++x) {
        if (d >= D) {
          K[d][x + R] = 0u;
          continue;
        }
        const int p = lc - x;
        const uint32_t w = p < 0 ? 0u : (p >= BS ? 2u : 1u);
        const uint32_t pw = d == 0 ? 1u : (d == 1 ? 3u : 9u);
        K[d][x + R] = ((w * pw * 4u + (d == 0 ? wrow : 0u)) << 16) |
                      ((uint32_t)lane_bits<L>(p & (BS - 1), d) * (uint32_t)sizeof(S));
      }
    }
    char *fb = (char *)fout;
    char *gb = (char *)gout;
    constexpr int64_t rbytes = PCH * (int64_t)sizeof(S);
    {
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        // x + xi_i is the pull source of the opposite population
        const int j = L::S.opp[i];
        const uint32_t k = K[0][cx_<L>(j, 0) + R] + K[1][cx_<L>(j, 1) + R] + K[2][cx_<L>(j, 2) + R];
        const uint64_t off = (uint64_t)nbs[k >> 18] * (64u * sizeof(S)) + (k & 0xffffu);
        auto row = (gptr<char>)(fb + i * rbytes);
        asm("" : "+s"(row));  // uniform row base in SGPRs
        Sto<S>::stg((gptr<S>)(row + off), f[i], RAW ? 0.0 : L::S.w[i]);
        if (DDF) {
          auto grow = (gptr<char>)(gb + i * rbytes);
          asm("" : "+s"(grow));
          Sto<S>::stg((gptr<S>)(grow + off), g[i], 0.0);
        }
      }
    }
  } else {
    const int64_t row = tp.xbase[brick] + __popcll(xm & ((1ull << lane) - 1ull));
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      const int j = L::S.opp[i];
      const int32_t s = tp.xnbr[(int64_t)(j - 1) * tp.xstride + row];
      // a population the cell pulls from itself (a fine ghost at the edge of
      // its level keeps it) is stored in its own row; nobody pulls from a
      // cell's own slot through the opposite link, so that push is dropped
      if (tp.xnbr[(int64_t)(i - 1) * tp.xstride + row] == (int32_t)c) {
        Sto<S>::stn(fout, pix<L::Q>(i, c), f[i], RAW ? 0.0 : L::S.w[i]);
        if (DDF) Sto<S>::stn(gout, pix<L::Q>(i, c), g[i], 0.0);
      }
      if (s == (int32_t)c) continue;
      if (s >= 0) {
        Sto<S>::stn(fout, pix<L::Q>(i, s), f[i], RAW ? 0.0 : L::S.w[i]);
        if (DDF) Sto<S>::stn(gout, pix<L::Q>(i, s), g[i], 0.0);
      } else {
        C v = f[i];
        if (s <= -2)
          v += (C)(2.0 * L::S.w[j] * wall_dot<L>(uw, -2 - s, j) / cs2w);  // no inflow noise in place
        Sto<S>::stn(fout, pix<L::Q>(j, c), v, RAW ? 0.0 : L::S.w[j]);
        if (DDF) Sto<S>::stn(gout, pix<L::Q>(j, c), g[i], 0.0);
      }
    }
  }
}

// Gather for one cell anywhere (no brick per wavefront): the neighbour
// brick ids come straight from the table.  Used by the sampled read-back.
template <class L, class S, bool PRE, bool DDF, int AA = 0>
__device__ inline void gather_one(const S *fin, const S *gin, const Topo &tp, int64_t vbase,
                                  int64_t c, const double (&uw)[6][3], double cs2w, typename Sto<S>::C *f,
                                  typename Sto<S>::C *g) {
  constexpr int BS = Brick<L>::BS;
  const int64_t brick = c >> 6;
  const int lane = (int)(c & 63);
  const uint64_t xm = tp.xmask[brick];
  f[0] = Sto<S>::ld(fin, pix<L::Q>(0, c), L::S.w[0]);
  if (DDF) g[0] = Sto<S>::ld(gin, pix<L::Q>(0, c), 0.0);
  if ((xm >> lane) & 1ull) {
    const int64_t row = tp.xbase[brick] + __popcll(xm & ((1ull << lane) - 1ull));
    gather_row<L, S, PRE, DDF, AA>(fin, gin, tp.xnbr, tp.xstride, row, vbase, c, uw, cs2w, f, g, ~0ull, tp.xdu);
    return;
  }
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    int64_t src = c;
    if (!PRE) {
      int dir = 0, loc = 0, pw = 1;
#pragma unroll
      for (int d = 0; d < L::D; ++d) {
        const int p = lane_coord<L>(lane, d) - cx_<L>(i, d);
        const int w = p < 0 ? 0 : (p >= BS ? 2 : 1);
        dir += w * pw;
        pw *= 3;
        loc |= lane_bits<L>(p & (BS - 1), d);
      }
      src = (int64_t)tp.nbrick[brick * Brick<L>::NBP + dir] * 64 + loc;
    }
    const int64_t ri = AA == 2 ? L::S.opp[i] : i;
    f[i] = Sto<S>::ld(fin, pix<L::Q>(ri, src), L::S.w[i]);
    if (DDF) g[i] = Sto<S>::ld(gin, pix<L::Q>(ri, src), 0.0);
  }
}

// Per-block preamble of the kernels that gather: stages the offsets
// (brick_unit) of the neighbour bricks of the block's bricks in LDS.  Every thread of
// the block must call it.  Returns the wave-uniform brick id.
template <class L, class S>
__device__ inline int32_t stage_bricks(const Topo &tp, uint32_t (*nbs)[Brick<L>::NBP], int64_t c, bool live) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t brick = __builtin_amdgcn_readfirstlane((int32_t)(c >> 6));
  if (live && lane < Brick<L>::NB) {
    const int32_t nb = tp.nbrick[(int64_t)brick * Brick<L>::NBP + lane];
    nbs[w][lane] = nb < 0 ? 0u : brick_unit<L::Q>(nb);
  }
  __syncthreads();
  return brick;
}

// ---------------------------------------------------------------------------
// product lattices (D2Q9, D3Q27): equilibrium and recursive regularisation
// on the Hermite basis {1, xi, xi^2 - cs2}^D
// ---------------------------------------------------------------------------
template <class L, class C>
__device__ inline void equilibrium_product(C rho, const C *u, C *feq) {
  constexpr C a1 = (C)(1.0 / L::cs2), a2 = (C)((1.0 - L::cs2) / (2.0 * L::cs2 * L::cs2));
  constexpr C a0 = (C)(1.0 / (2.0 * L::cs2));
  C p[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const C ud = d < L::D ? u[d] : (C)0;
    const C q = ud * ud;
    p[d][1] = (C)1 - a0 * q;
    p[d][2] = (C)1 + a1 * ud + a2 * q;
    p[d][0] = (C)1 - a1 * ud + a2 * q;
  }
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    C v = (C)L::S.w[i] * rho;
#pragma unroll
    for (int d = 0; d < L::D; ++d) v *= p[d][cx_<L>(i, d) + 1];
    feq[i] = v;
  }
}

template <class C>
__device__ inline C upow(C x, int e) {
  return e <= 0 ? (C)1 : (e == 1 ? x : x * x);
}

// f*_i = w_i sum_m H_m(xi_i) a*_m / (m! cs2^|m|), a*_m = a_eq,m + k a_neq,m,
// with a_neq,m the closed pair sum that solves the non-equilibrium
// recursion; evaluated by sum factorisation one axis at a time.
//
// SH: the shifted representation h_i = f_i - w_i on both sides.  P is then
// sum xi_a xi_b h_i (the lattice's own cs2 delta_ab left out), rho1 = rho - 1
// and rhop1 = rhop - 1 are passed as computed from the h_i, and f receives
// h*_i = f*_i - w_i: the zeroth coefficient is a*_0 - 1, every other term is
// unchanged.  No cancellation against 1 or cs2 happens in FP32.
template <class L, class C, bool SH = false>
__device__ inline void rr_product(C *f, C rho, C rhop, const C *u, C (&P)[3][3], C k,
                                  bool trace_eq, C rho1 = (C)0, C rhop1 = (C)0) {
  constexpr int D = L::D;
  constexpr C cs2 = (C)L::cs2, ics2 = (C)(1.0 / L::cs2);
  C A[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      A[a][b] = (a < D && b < D) ? P[a][b] - rho * u[a] * u[b] - (a == b ? (SH ? rho1 : rho) * cs2 : (C)0) : (C)0;
  if (trace_eq) {
    C tr = (C)0;
#pragma unroll
    for (int a = 0; a < D; ++a) tr += A[a][a];
    tr *= (C)(1.0 / D);
#pragma unroll
    for (int a = 0; a < D; ++a) A[a][a] -= tr;
  }
  C uu[3] = {u[0], u[1], D == 3 ? u[2] : (C)0};
  C b[3][3][3];
#pragma unroll
  for (int mx = 0; mx < 3; ++mx)
#pragma unroll
    for (int my = 0; my < 3; ++my)
#pragma unroll
      for (int mz = 0; mz < 3; ++mz) {
        if (D == 2 && mz > 0) { b[mx][my][mz] = (C)0; continue; }
        const int m[3] = {mx, my, mz};
        C aeq = rhop * upow(uu[0], mx) * upow(uu[1], my) * upow(uu[2], mz);
        C an = (C)0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (m[d] == 2) {
            C t = A[d][d];
#pragma unroll
            for (int e = 0; e < 3; ++e)
              if (e != d) t *= upow(uu[e], m[e]);
            an += t;
          }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int e = d + 1; e < 3; ++e) {
            if (m[d] >= 1 && m[e] >= 1) {
              C t = (C)(m[d] * m[e]) * A[d][e];
#pragma unroll
              for (int h = 0; h < 3; ++h) t *= upow(uu[h], m[h] - (h == d) - (h == e));
              an += t;
            }
          }
        C scale = (C)1;
#pragma unroll
        for (int d = 0; d < 3; ++d) scale *= (m[d] == 2 ? (C)0.5 * ics2 * ics2 : (m[d] == 1 ? ics2 : (C)1));
        b[mx][my][mz] = (aeq + k * an) * scale;
        if (SH && mx == 0 && my == 0 && mz == 0) b[0][0][0] = rhop1;
      }
  // h_0 = 1, h_1 = xi, h_2 = xi^2 - cs2 evaluated at xi in {-1, 0, 1}
  C T1[3][3][3];
#pragma unroll
  for (int mx = 0; mx < 3; ++mx)
#pragma unroll
    for (int my = 0; my < 3; ++my)
#pragma unroll
      for (int iz = 0; iz < 3; ++iz) {
        if (D == 2) { T1[mx][my][iz] = b[mx][my][0]; continue; }
        const C xi = (C)(iz - 1);
        T1[mx][my][iz] = b[mx][my][0] + xi * b[mx][my][1] + (xi * xi - cs2) * b[mx][my][2];
      }
  C T2[3][3][3];
#pragma unroll
  for (int mx = 0; mx < 3; ++mx)
#pragma unroll
    for (int iy = 0; iy < 3; ++iy)
#pragma unroll
      for (int iz = 0; iz < 3; ++iz) {
        const C xi = (C)(iy - 1);
        T2[mx][iy][iz] = T1[mx][0][iz] + xi * T1[mx][1][iz] + (xi * xi - cs2) * T1[mx][2][iz];
      }
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const int ix = cx_<L>(i, 0) + 1, iy = cx_<L>(i, 1) + 1, iz = D == 3 ? cx_<L>(i, 2) + 1 : 0;
    const C xi = (C)(ix - 1);
    const C v = T2[0][iy][iz] + xi * T2[1][iy][iz] + (xi * xi - cs2) * T2[2][iy][iz];
    f[i] = (C)L::S.w[i] * v;
  }
}

// ---------------------------------------------------------------------------
// D2Q37 fourth-order thermal equilibrium: Hermite coefficients of a
// Maxwellian of temperature T on the cs2 basis, a_m = rho prod_d A_{m_d},
// A_0..4 = 1, u, u^2+th, u^3+3 th u, u^4+6 th u^2+3 th^2, th = T - cs2
// ---------------------------------------------------------------------------
constexpr double h1c(int n, double x, double cs2) {
  return n == 0 ? 1.0
       : n == 1 ? x
       : n == 2 ? x * x - cs2
       : n == 3 ? (x * x - 3.0 * cs2) * x
                : x * x * x * x - 6.0 * cs2 * x * x + 3.0 * cs2 * cs2;
}
constexpr double fact_c(int n) { return n <= 1 ? 1.0 : n * fact_c(n - 1); }
constexpr double pow_c(double x, int n) { return n == 0 ? 1.0 : x * pow_c(x, n - 1); }

template <int Q>
struct ThermalTable {
  int mx[15], my[15];
  double hw[Q][15];
};

template <class L>
constexpr ThermalTable<L::Q> make_thermal() {
  ThermalTable<L::Q> t{};
  int k = 0;
  for (int n = 0; n <= 4; ++n)
    for (int my = 0; my <= n; ++my) {
      t.mx[k] = n - my;
      t.my[k] = my;
      ++k;
    }
  for (int i = 0; i < L::Q; ++i)
    for (int k2 = 0; k2 < 15; ++k2) {
      const int a = t.mx[k2], b = t.my[k2];
      t.hw[i][k2] = L::S.w[i] * h1c(a, L::S.v[i].x, L::cs2) * h1c(b, L::S.v[i].y, L::cs2) /
                    (fact_c(a) * fact_c(b) * pow_c(L::cs2, a + b));
    }
  return t;
}

template <class L>
struct Thermal {
  static constexpr ThermalTable<L::Q> T = make_thermal<L>();
};

template <class L, class C>
__device__ inline void equilibrium_thermal(C rho, const C *u, C T, C *feq) {
  const C th = T - (C)L::cs2;
  C A[2][5];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const C x = u[d], x2 = x * x;
    A[d][0] = (C)1;
    A[d][1] = x;
    A[d][2] = x2 + th;
    A[d][3] = x * (x2 + (C)3 * th);
    A[d][4] = x2 * x2 + (C)6 * th * x2 + (C)3 * th * th;
  }
  C a[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) a[k] = rho * A[0][Thermal<L>::T.mx[k]] * A[1][Thermal<L>::T.my[k]];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    C v = (C)0;
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      const double h = Thermal<L>::T.hw[i][k];
      if (h != 0.0) v += (C)h * a[k];
    }
    feq[i] = v;
  }
}

// ---------------------------------------------------------------------------
// third-order lattices (D2Q13, D2Q21): equilibrium and recursive
// regularisation on the full Hermite basis up to third order, the ten
// tensors (mx, my) with mx + my <= 3 and none of fourth order (App. A.2)
// ---------------------------------------------------------------------------
template <class L>
constexpr bool product_basis() {
  return L::kind == LAT_D2Q9 || L::kind == LAT_D3Q27;
}

template <int Q>
struct Hermite3Table {
  int mx[10], my[10];
  double hw[Q][10];  // w_i H_m(xi_i) / (mx! my! cs2^(mx + my))
};

template <class L>
constexpr Hermite3Table<L::Q> make_hermite3() {
  Hermite3Table<L::Q> t{};
  int k = 0;
  for (int n = 0; n <= 3; ++n)
    for (int my = 0; my <= n; ++my) {
      t.mx[k] = n - my;
      t.my[k] = my;
      ++k;
    }
  for (int i = 0; i < L::Q; ++i)
    for (int k2 = 0; k2 < 10; ++k2) {
      const int a = t.mx[k2], b = t.my[k2];
      t.hw[i][k2] = L::S.w[i] * h1c(a, L::S.v[i].x, L::cs2) * h1c(b, L::S.v[i].y, L::cs2) /
                    (fact_c(a) * fact_c(b) * pow_c(L::cs2, a + b));
    }
  return t;
}

template <class L>
struct Hermite3 {
  static constexpr Hermite3Table<L::Q> T = make_hermite3<L>();
};

// f_i = sum_m hw_im b_m
template <class L, class C>
__device__ inline void hermite3_expand(const C (&b)[10], C *f) {
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    C v = (C)0;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      const double h = Hermite3<L>::T.hw[i][k];
      if (h != 0.0) v += (C)h * b[k];
    }
    f[i] = v;
  }
}

template <class L, class C>
__device__ inline void equilibrium_hermite3(C rho, const C *u, C *feq) {
  const C px[4] = {(C)1, u[0], u[0] * u[0], u[0] * u[0] * u[0]};
  const C py[4] = {(C)1, u[1], u[1] * u[1], u[1] * u[1] * u[1]};
  C b[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) b[k] = rho * px[Hermite3<L>::T.mx[k]] * py[Hermite3<L>::T.my[k]];
  hermite3_expand<L, C>(b, feq);
}

// b_m = rhop u^m + k a_neq,m with a^(2)_neq = P - rho u u - rho cs2 I and
// the third-order a_neq from the non-equilibrium recursion (pair sums:
// xxx = 3 u_x a_xx, xxy = 2 u_x a_xy + u_y a_xx, and their mirrors)
template <class L, class C>
__device__ inline void rr_hermite3(C *f, C rho, C rhop, const C *u, const C (&P)[3][3], C k, bool trace_eq) {
  constexpr C cs2 = (C)L::cs2;
  const C ux = u[0], uy = u[1];
  C axx = P[0][0] - rho * ux * ux - rho * cs2;
  const C axy = P[0][1] - rho * ux * uy;
  C ayy = P[1][1] - rho * uy * uy - rho * cs2;
  if (trace_eq) {
    const C h = (C)0.5 * (axx + ayy);
    axx -= h;
    ayy -= h;
  }
  const C an[10] = {(C)0, (C)0, (C)0, axx, axy, ayy, (C)3 * ux * axx, (C)2 * ux * axy + uy * axx,
                    (C)2 * uy * axy + ux * ayy, (C)3 * uy * ayy};
  const C px[4] = {(C)1, ux, ux * ux, ux * ux * ux};
  const C py[4] = {(C)1, uy, uy * uy, uy * uy * uy};
  C b[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) b[m] = rhop * px[Hermite3<L>::T.mx[m]] * py[Hermite3<L>::T.my[m]] + k * an[m];
  hermite3_expand<L, C>(b, f);
}

// ---------------------------------------------------------------------------
// numerical (entropy-maximising) equilibrium, D2Q21: f_eq = rho exp(-(1 +
// lambda . m_i)) under the eight moment constraints; Newton with a Cholesky
// step and backtracking on ||G||_2, FP64
// ---------------------------------------------------------------------------
template <class L>
__device__ constexpr double mvec(int i, int a) {
  const double x = L::S.v[i].x, y = L::S.v[i].y, n2 = x * x + y * y;
  return a == 0 ? 1.0 : a == 1 ? x : a == 2 ? y : a == 3 ? x * x : a == 4 ? x * y : a == 5 ? y * y
       : a == 6 ? x * n2 : y * n2;
}

// One pass over the populations at multipliers lam (Eq. exponential):
// e_i = exp(-(1 + lam . m_i)), the constraint residuals
// G_a = sum_i e_i m_ia - M_a (Eqs. G0_8mom - G3yaa_8mom, per unit density)
// and the Newton matrix H = sum_i e_i m_i m_i^T (packed lower triangle).
// e_i is kept only in the collision precision C, for the final equilibrium,
// so that no FP64 population array stays live across the solve.
template <class L>
__device__ inline void targets(double ux, double uy, double T, double *M);

// Reflection orbits of a 2-D lattice symmetric under x -> -x and y -> -y:
// representative k is the k-th velocity with c_x >= 0 and c_y >= 0.
template <class L>
__device__ constexpr int n_reps() {
  int n = 0;
  for (int i = 0; i < L::Q; ++i) n += (L::S.v[i].x >= 0 && L::S.v[i].y >= 0);
  return n;
}
template <class L>
__device__ constexpr int rep_of(int i) {
  const int a = iabs_c(L::S.v[i].x), b = iabs_c(L::S.v[i].y);
  int k = 0;
  for (int j = 0; j < L::Q; ++j)
    if (L::S.v[j].x >= 0 && L::S.v[j].y >= 0) {
      if (L::S.v[j].x == a && L::S.v[j].y == b) return k;
      ++k;
    }
  return -1;
}
template <class L>
__device__ constexpr int rep_comp(int k, int d) {
  int n = 0;
  for (int j = 0; j < L::Q; ++j)
    if (L::S.v[j].x >= 0 && L::S.v[j].y >= 0) {
      if (n == k) return d == 0 ? L::S.v[j].x : L::S.v[j].y;
      ++n;
    }
  return 0;
}
__device__ constexpr double ipow_c(int a, int p) {
  double r = 1.0;
  for (int k = 0; k < p; ++k) r *= a;
  return r;
}
// m_a = sum of terms c x^p y^q: (1, x, y, x^2, xy, y^2, x^3 + x y^2, x^2 y + y^3)
__device__ constexpr int mterms(int a) { return a >= 6 ? 2 : 1; }
__device__ constexpr int mterm_p(int a, int t) {
  return a == 0 ? 0 : a == 1 ? 1 : a == 2 ? 0 : a == 3 ? 2 : a == 4 ? 1 : a == 5 ? 0 : a == 6 ? (t ? 1 : 3)
       : (t ? 0 : 2);
}
__device__ constexpr int mterm_q(int a, int t) {
  return a == 0 ? 0 : a == 1 ? 0 : a == 2 ? 1 : a == 3 ? 0 : a == 4 ? 1 : a == 5 ? 2 : a == 6 ? (t ? 2 : 0)
       : (t ? 3 : 1);
}

// One pass over the populations at multipliers lam (Eq. exponential):
// e_i = exp(-(1 + lam . m_i)), the constraint residuals
// G_a = sum_i e_i m_ia - M_a (Eqs. G0_8mom - G3yaa_8mom, per unit density)
// and the Newton matrix H = sum_i e_i m_i m_i^T (packed lower triangle).
// The sums go through the reflection orbits: per representative velocity
// (a, b), the four sign-weighted sums P = sum e, sum s_x e, sum s_y e,
// sum s_x s_y e over its members give every moment
// S_pq = sum_i e_i c_x^p c_y^q = sum_k a^p b^q P_k[p mod 2, q mod 2],
// and G, H are short sums of S.  e_i is kept only in the collision precision
// C, for the final equilibrium.
template <class L, class C, bool HESS = true>
__device__ inline void expo_pass(const double *lam, double ux, double uy, double T, double *G, double *H, C *e) {
  constexpr int NR = n_reps<L>();
  double P[NR][4];
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int t = 0; t < 4; ++t) P[k][t] = 0.0;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    double s = 1.0;
#pragma unroll
    for (int a = 0; a < NLAM; ++a)
      if (mvec<L>(i, a) != 0.0) s += lam[a] * mvec<L>(i, a);
    const double ei = exp(-s);
    e[i] = (C)ei;
    const int k = rep_of<L>(i);
    const bool nx = L::S.v[i].x < 0, ny = L::S.v[i].y < 0;
    P[k][0] += ei;
    if (rep_comp<L>(k, 0) != 0) P[k][1] += nx ? -ei : ei;
    if (rep_comp<L>(k, 1) != 0) P[k][2] += ny ? -ei : ei;
    if (rep_comp<L>(k, 0) != 0 && rep_comp<L>(k, 1) != 0) P[k][3] += (nx != ny) ? -ei : ei;
  }
  // S_pq for p + q <= 6
  double S[7][7];
#pragma unroll
  for (int p = 0; p <= 6; ++p)
#pragma unroll
    for (int q = 0; p + q <= 6; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const double cf = ipow_c(rep_comp<L>(k, 0), p) * ipow_c(rep_comp<L>(k, 1), q);
        if (cf != 0.0) acc += cf * P[k][(p & 1) | ((q & 1) << 1)];
      }
      S[p][q] = acc;
    }
  double M[NLAM];
  targets<L>(ux, uy, T, M);
#pragma unroll
  for (int a = 0; a < NLAM; ++a) {
    double g = 0.0;
#pragma unroll
    for (int t = 0; t < mterms(a); ++t) g += S[mterm_p(a, t)][mterm_q(a, t)];
    G[a] = g - M[a];
  }
  if (HESS)
#pragma unroll
    for (int a = 0; a < NLAM; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        double h = 0.0;
#pragma unroll
        for (int t = 0; t < mterms(a); ++t)
#pragma unroll
          for (int u = 0; u < mterms(b); ++u)
            h += S[mterm_p(a, t) + mterm_p(b, u)][mterm_q(a, t) + mterm_q(b, u)];
        H[a * (a + 1) / 2 + b] = h;
      }
}

__device__ inline double nrm2_8(const double *G) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < NLAM; ++a) s += G[a] * G[a];
  return s;
}

// largest |G_a|; a NaN propagates so that it never passes a tolerance test
__device__ inline double nrmmax_8(const double *G) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < NLAM; ++a) {
    const double v = fabs(G[a]);
    s = (v > s || v != v) ? v : s;
  }
  return s;
}

template <class L>
__device__ inline void targets(double ux, double uy, double T, double *M) {
  const double uu = ux * ux + uy * uy;
  M[0] = 1.0;
  M[1] = ux;
  M[2] = uy;
  M[3] = ux * ux + T;
  M[4] = ux * uy;
  M[5] = uy * uy + T;
  M[6] = ux * (uu + 4.0 * T);
  M[7] = uy * (uu + 4.0 * T);
}

// d = H^-1 G by an in-place Cholesky factorisation of the packed H (the
// diagonal holds the reciprocals 1 / L_jj, so the solves multiply); false
// when H is not numerically positive definite
__device__ inline bool cholesky_solve(double *H, const double *G, double *d) {
#pragma unroll
  for (int j = 0; j < NLAM; ++j) {
    double t = H[j * (j + 1) / 2 + j];
#pragma unroll
    for (int k = 0; k < j; ++k) t -= H[j * (j + 1) / 2 + k] * H[j * (j + 1) / 2 + k];
    if (!(t > 0.0)) return false;
    const double inv = rsqrt(t);
    H[j * (j + 1) / 2 + j] = inv;
#pragma unroll
    for (int i = j + 1; i < NLAM; ++i) {
      double s = H[i * (i + 1) / 2 + j];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= H[i * (i + 1) / 2 + k] * H[j * (j + 1) / 2 + k];
      H[i * (i + 1) / 2 + j] = s * inv;
    }
  }
#pragma unroll
  for (int i = 0; i < NLAM; ++i) {
    double s = G[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= H[i * (i + 1) / 2 + k] * d[k];
    d[i] = s * H[i * (i + 1) / 2 + i];
  }
#pragma unroll
  for (int i = NLAM - 1; i >= 0; --i) {
    double s = d[i];
#pragma unroll
    for (int k = i + 1; k < NLAM; ++k) s -= H[k * (k + 1) / 2 + i] * d[k];
    d[i] = s * H[i * (i + 1) / 2 + i];
  }
  return true;
}

// Newton-Raphson on the eight constraints from the multipliers in lam, with
// backtracking on the 2-norm of the residual (at most 30 halvings).  The
// stopping test max_a |G_a| <= tol is applied before every step; the first
// min_steps steps are always taken, and after exactly min_steps steps the
// looser tolerance tol_first applies (the surrogate's single correction).
// Returns the number of steps, or -1 (not converged within max_it, or H not
// positive definite).  e receives exp(-(1 + lam . m_i)) at the final lam.
template <class L, class C>
__device__ inline int newton_lean(double ux, double uy, double T, double *lam, double tol, int max_it,
                                  int min_steps, double tol_first, C *e) {
  double G[NLAM], H[NLAM * (NLAM + 1) / 2], d[NLAM], base[NLAM];
  // one evaluation site: each pass either checks a new iterate or tests a
  // trial point of the line search
  int it = 0, h = 0;
  bool trial = false;
  double n0 = 0.0, alpha = 1.0;
  for (;;) {
    expo_pass<L, C>(lam, ux, uy, T, G, H, e);
    if (trial) {
      if (!(nrm2_8(G) < n0) && h < 30) {
        ++h;
        alpha *= 0.5;
#pragma unroll
        for (int a = 0; a < NLAM; ++a) lam[a] = base[a] + alpha * d[a];
        continue;
      }
      trial = false;
      ++it;
    }
    if (it >= min_steps && nrmmax_8(G) <= (it == min_steps && min_steps > 0 ? tol_first : tol)) return it;
    if (it == max_it) return -1;
    if (!cholesky_solve(H, G, d)) return -1;
    n0 = nrm2_8(G);
    alpha = 1.0;
    h = 0;
#pragma unroll
    for (int a = 0; a < NLAM; ++a) {
      base[a] = lam[a];
      lam[a] = base[a] + alpha * d[a];
    }
    trial = true;
  }
}

// cold-or-warm Newton solve to tol (the paper's solver); FP64 equilibrium out
template <class L>
__device__ inline int newton_solve(double ux, double uy, double T, double *lam, double tol, int max_it,
                                   double *e) {
  return newton_lean<L, double>(ux, uy, T, lam, tol, max_it, 0, tol, e);
}

// ---------------------------------------------------------------------------
// kinetic sensor, Eqs. DeltaAvg and shock_function
// ---------------------------------------------------------------------------
template <class L, class C>
__device__ inline C sensor_alpha(const C *f, const C *feq, C tau, C A) {
  constexpr C tiny = sizeof(C) == 8 ? (C)1e-300 : (C)1e-30;
  C eps = (C)0;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) eps += fabs(f[i] - feq[i]) / fmax(fabs(feq[i]), tiny);
  eps *= (C)(1.0 / L::Q);
  return eps < (C)0.01 ? (C)1 : eps < (C)0.1 ? (C)1.05 : eps < (C)1 ? A : (C)1 / tau;
}

// ---------------------------------------------------------------------------
// macroscopic moments of a cell
// ---------------------------------------------------------------------------
template <class L, class C, bool DDF>
__device__ inline void cell_moments(const C *f, const C *g, C Cv, C &rho, C (&u)[3], C &T) {
  rho = (C)0;
  C j[3] = {(C)0, (C)0, (C)0};
  C e2 = (C)0, gs = (C)0;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    rho += f[i];
#pragma unroll
    for (int d = 0; d < L::D; ++d)
      if (cx_<L>(i, d) != 0) j[d] += (C)cx_<L>(i, d) * f[i];
    if (DDF) {
      const int n2 = cx_<L>(i, 0) * cx_<L>(i, 0) + cx_<L>(i, 1) * cx_<L>(i, 1) + cx_<L>(i, 2) * cx_<L>(i, 2);
      if (n2 != 0) e2 += (C)n2 * f[i];
      gs += g[i];
    }
  }
  const C inv = (C)1 / rho;
  C uu = (C)0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[d] = d < L::D ? j[d] * inv : (C)0;
    uu += u[d] * u[d];
  }
  T = DDF ? (e2 + gs - rho * uu) / ((C)2 * rho * Cv) : (C)0;
}

// index of the population with velocity (x, y, z) (z = 0 in 2-D)
template <class L>
__device__ constexpr int vel_index(int x, int y, int z) {
  for (int i = 0; i < L::Q; ++i)
    if (L::S.v[i].x == x && L::S.v[i].y == y && (L::D == 2 || L::S.v[i].z == z)) return i;
  return -1;
}

// Moments up to second order of a product lattice (velocities {-1, 0, 1}^D)
// of whatever f holds, by sums along one axis at a time: along x each line
// of three populations gives f(-1) + f(0) + f(1), f(1) - f(-1) and
// f(1) + f(-1); along y and then z only the combinations that the zeroth
// (m0), first (j) and second (P) moments need are formed.  66 additions for
// D3Q27 instead of the 170 of one running sum per moment.
template <class L, class C>
__device__ inline void moments_product(const C *f, C &m0, C (&j)[3], C (&P)[3][3]) {
  constexpr int NZ = L::D == 3 ? 3 : 1;
  C s0[3][NZ], s1[3][NZ], s2[3][NZ];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < NZ; ++c) {
      const int z = L::D == 3 ? c - 1 : 0;
      const C lo = f[vel_index<L>(-1, b - 1, z)], mid = f[vel_index<L>(0, b - 1, z)], hi = f[vel_index<L>(1, b - 1, z)];
      s2[b][c] = hi + lo;
      s1[b][c] = hi - lo;
      s0[b][c] = s2[b][c] + mid;
    }
  // along y: t_ab[c] = sum over y of xi_x^a xi_y^b (per z line)
  C t00[NZ], t01[NZ], t02[NZ], t10[NZ], t11[NZ], t20[NZ];
#pragma unroll
  for (int c = 0; c < NZ; ++c) {
    t02[c] = s0[2][c] + s0[0][c];
    t00[c] = t02[c] + s0[1][c];
    t01[c] = s0[2][c] - s0[0][c];
    t10[c] = (s1[2][c] + s1[0][c]) + s1[1][c];
    t11[c] = s1[2][c] - s1[0][c];
    t20[c] = (s2[2][c] + s2[0][c]) + s2[1][c];
  }
  C m001 = (C)0, m002 = (C)0, m011 = (C)0, m101 = (C)0;
  C m000, m010, m020, m100, m110, m200;
  if constexpr (L::D == 3) {
    m002 = t00[2] + t00[0];
    m000 = m002 + t00[1];
    m001 = t00[2] - t00[0];
    m010 = (t01[2] + t01[0]) + t01[1];
    m011 = t01[2] - t01[0];
    m020 = (t02[2] + t02[0]) + t02[1];
    m100 = (t10[2] + t10[0]) + t10[1];
    m101 = t10[2] - t10[0];
    m110 = (t11[2] + t11[0]) + t11[1];
    m200 = (t20[2] + t20[0]) + t20[1];
  } else {
    m000 = t00[0];
    m010 = t01[0];
    m020 = t02[0];
    m100 = t10[0];
    m110 = t11[0];
    m200 = t20[0];
  }
  m0 = m000;
  j[0] = m100;
  j[1] = m010;
  j[2] = m001;
  P[0][0] = m200;
  P[1][1] = m020;
  P[2][2] = m002;
  P[0][1] = P[1][0] = m110;
  P[0][2] = P[2][0] = m101;
  P[1][2] = P[2][1] = m011;
}

// the same from h_i = f_i - w_i (single distribution): rho1 = sum h_i is
// rho - 1 without rounding against 1; sum w_i xi_i = 0 leaves j unchanged
template <class L, class C>
__device__ inline void cell_moments_shifted(const C *h, C &rho1, C &rho, C (&u)[3]) {
  rho1 = (C)0;
  C j[3] = {(C)0, (C)0, (C)0};
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    rho1 += h[i];
#pragma unroll
    for (int d = 0; d < L::D; ++d)
      if (cx_<L>(i, d) != 0) j[d] += (C)cx_<L>(i, d) * h[i];
  }
  rho = (C)1 + rho1;
  const C inv = (C)1 / rho;
#pragma unroll
  for (int d = 0; d < 3; ++d) u[d] = d < L::D ? j[d] * inv : (C)0;
}

// equilibrium of any model at a macroscopic state; Newton family updates lam
template <class L, int COLL, class C>
__device__ inline int equilibrium_any(C rho, const C *u, C T, const PhysArgs &ph, double *lam,
                                      bool warm, C *feq, C *geq) {
  int it = 0;
  if constexpr (COLL == COLL_BGK || COLL == COLL_RR) {
    if constexpr (product_basis<L>()) equilibrium_product<L, C>(rho, u, feq);
    else equilibrium_hermite3<L, C>(rho, u, feq);
  } else if constexpr (COLL == COLL_DDF_POLY) {
    equilibrium_thermal<L, C>(rho, u, T, feq);
  } else {
    if (!warm)
#pragma unroll
      for (int a = 0; a < NLAM; ++a) lam[a] = 0.0;
    C e[L::Q];
    it = newton_lean<L, C>((double)u[0], (double)u[1], (double)T, lam, ph.newton_tol, ph.newton_max_it, 0,
                           ph.newton_tol, e);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) feq[i] = rho * e[i];
  }
  if constexpr (COLL >= COLL_DDF_POLY) {
    const C k = ((C)2 * (C)ph.Cv - (C)L::D) * T;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) geq[i] = k * feq[i];
  }
  return it;
}

__device__ inline void count_add(unsigned long long *ctr, int which, unsigned long long v) {
  if (v) atomicAdd(ctr + CNT_COUNT * (blockIdx.x & (CNT_COPIES - 1u)) + which, v);
}

// Histogram of the Newton steps per solve (the per-cell iteration counts
// the paper keeps to monitor stability, Sec. 4.4): bin k < NHIST - 1 counts
// solves of k steps, the last bin longer solves and failures (it < 0).  The
// active lanes of a wavefront add one atomic per distinct bin.
__device__ inline void count_hist(unsigned long long *ctr, int it) {
  const int bin = (it < 0 || it >= NHIST - 1) ? NHIST - 1 : it;
  unsigned long long *base = ctr + CNT_COUNT * (blockIdx.x & (CNT_COPIES - 1u)) + CNT_HIST0;
  uint64_t todo = __ballot(1);
  while (todo) {
    const int lead = __ffsll((unsigned long long)todo) - 1;
    const int b = __shfl(bin, lead);
    const uint64_t same = __ballot(bin == b) & todo;
    if ((int)(threadIdx.x & 63) == lead) atomicAdd(base + b, (unsigned long long)__popcll(same));
    todo &= ~same;
  }
}

// ---------------------------------------------------------------------------
// collide and stream (pull) for the cells [begin, begin + count) of a level
// ---------------------------------------------------------------------------
// Occupancy floor of the collide kernel: the single-population product
// lattices are bound by memory latency and run best with at least six
// wavefronts per SIMD (at most 85 VGPRs; four, 128 VGPRs, for FP64, which
// would otherwise spill); the compute-heavy DDF models keep the compiler's
// choice, the Newton kernels two wavefronts per SIMD (for D2Q37 that spills
// part of the Newton state, which is still 1.8x faster than one wavefront).
template <class L, int COLL, class S>
struct MinWaves {
  static constexpr int value = COLL < COLL_DDF_POLY ? (sizeof(S) == 8 ? 4 : 6) : (COLL >= COLL_DDF_NEWTON ? 2 : 1);
};

// Block size of the collide kernel: four bricks (256 threads) on every
// lattice.  With the chunked population layout this beats the 2 x 2 x 2
// cube of bricks that is consecutive in Z order (512 threads; sphere FP16
// +7.6 %, FP32 +0.9 %) and two or one bricks per block (-2 to -4 %; in 2-D
// two bricks cost 1-3 %); the cube was 1 % ahead while each population had
// a row of the whole buffer.
template <class L, int COLL>
struct CollideBlock {
  static constexpr int value = BLOCK;
};

// AA selects in-place streaming on one buffer (a.fin == a.fout): 1 = even
// step (read the cell's own rows, write population i to its row opp(i)),
// 2 = odd step (pull from the swapped rows, push to the neighbours).
//
// With a.multi.n > 0 one launch updates every level active at a substep
// (the paper's remedy for small levels that leave most of the GPU idle,
// Sec. 4.5): the grid is the concatenation of the levels' blocks, each
// level's range starting at a multiple of 8 blocks so that the round-robin
// XCD dispatch keeps its per-XCD contiguous order inside the level; a block
// takes its level's buffers, cell range and relaxation time from the table
// and runs the same update as a per-level launch.
template <class L, int COLL, class S, bool PRE, int AA = 0, bool NZ = false, bool O32 = false>
__global__ void __launch_bounds__((CollideBlock<L, COLL>::value))
    __attribute__((amdgpu_waves_per_eu(MinWaves<L, COLL, S>::value))) k_collide(const KArgs a) {
  using C = typename Sto<S>::C;
  constexpr bool DDF = COLL >= COLL_DDF_POLY;
  constexpr int Q = L::Q;
  constexpr int CB = CollideBlock<L, COLL>::value;
  __shared__ uint32_t nbs[CB / 64][Brick<L>::NBP];
  int64_t blk, begin = a.begin, count = a.count;
  const void *fin_p = a.fin, *gin_p = a.gin;
  void *fout_p = a.fout, *gout_p = a.gout;
  double tau = a.ph.tau, omega = a.ph.omega, krr = a.ph.krr;
  bool multi = false;
  if constexpr (!PRE && AA == 0 && COLL < COLL_DDF_NEWTON) multi = a.multi.n > 0;
  if (multi) {
    const int64_t b = blockIdx.x;
    int k = 0;
#pragma unroll
    for (int j = 1; j < MAX_LEVELS; ++j)
      if (j < a.multi.n && b >= a.multi.block0[j]) k = j;
    blk = xcd_map((uint32_t)(b - a.multi.block0[k]), (uint32_t)(a.multi.block0[k + 1] - a.multi.block0[k]));
    begin = a.multi.begin[k];
    count = a.multi.count[k];
    tau = a.multi.tau[k];
    omega = a.multi.omega[k];
    krr = a.multi.krr[k];
    const int p = a.multi.parity[k];
    fin_p = a.multi.f[p];
    fout_p = (void *)a.multi.f[1 - p];
    gin_p = a.multi.g[p];
    gout_p = (void *)a.multi.g[1 - p];
    if (blk * CB >= count) return;  // padding blocks of the level
  } else {
    blk = xcd_block();
  }
  const int64_t t = blk * CB + threadIdx.x;
  const bool live = t < count;  // whole wavefronts
  const int64_t c = begin + (live ? t : 0);
  // the cell's flags and its brick's exception mask do not depend on the
  // staged table: issued before the barrier, their latency overlaps the
  // table's instead of adding two round trips after it
  const uint8_t fl = a.flags[c];
  // (a vector load of the wavefront's one mask: a scalar load would be
  // sunk past the barrier to its first use)
  const uint64_t xm = a.topo.xmask[c >> 6];
  const int32_t brick = stage_bricks<L, S>(a.topo, nbs, c, live);
  if (!live) return;
  if (fl & F_HOLE) return;
  const S *fin = (const S *)fin_p;
  const S *gin = (const S *)gin_p;
  C f[Q];
  C g[DDF ? Q : 1];
  // FP16 storage with recursive regularisation on a product lattice works on
  // the stored h_i = f_i - w_i throughout: no shift on the way in or out,
  // and the moments and the regularised populations are formed from the
  // small deviations instead of from f_i ~ w_i
  constexpr bool SH = std::is_same<S, __half>::value && COLL == COLL_RR && product_basis<L>();
  gather<L, S, PRE || AA == 1, DDF, AA == 2 ? 2 : 0, NZ, SH, O32>(fin, gin, a.topo, nbs[0], a.vbase, c, threadIdx.x & 63, brick, xm,
                                                       a.ph.uw, a.ph.cs2w, f, g);
  if (!(fl & (F_FINE_GHOST | F_BC_NEUMANN | F_BC_EQ))) {
    C rho, u[3], T = (C)0, rho1 = (C)0;
    // recursive regularisation on a product lattice takes its moments, the
    // second-order ones included, from moments_product
    constexpr bool PM = COLL == COLL_RR && product_basis<L>();
    C P[3][3];
    if constexpr (PM) {
      C m0, j[3];
      moments_product<L, C>(f, m0, j, P);
      if constexpr (SH) {
        rho1 = m0;
        rho = (C)1 + rho1;
      } else {
        rho = m0;
      }
      const C inv = (C)1 / rho;
#pragma unroll
      for (int d = 0; d < 3; ++d) u[d] = d < L::D ? j[d] * inv : (C)0;
    } else if constexpr (SH) {
      cell_moments_shifted<L, C>(f, rho1, rho, u);
    } else {
      cell_moments<L, C, DDF>(f, g, (C)a.ph.Cv, rho, u, T);
    }
    C rhop = rho, rhop1 = rho1;
    if (fl & F_SPONGE) {
      const C s = (C)a.sigma[c];
      rhop = rho * ((C)1 - s) + s * (C)a.rho_inf[c];
      if constexpr (SH) rhop1 = rho1 * ((C)1 - s) + s * ((C)a.rho_inf[c] - (C)1);
    }
    if (!(rho > (C)0) || !isfinite(rho)) count_add(a.counters, CNT_NONFINITE, 1);
    if constexpr (COLL == COLL_BGK) {
      C feq[Q];
      if constexpr (product_basis<L>()) equilibrium_product<L, C>(rhop, u, feq);
      else equilibrium_hermite3<L, C>(rhop, u, feq);
      const C om = (C)omega;
#pragma unroll
      for (int i = 0; i < Q; ++i) f[i] = f[i] - om * (f[i] - feq[i]);
    } else if constexpr (COLL == COLL_RR) {
      if constexpr (!PM) {
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
          for (int y = 0; y < 3; ++y) P[x][y] = (C)0;
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
          for (int x = 0; x < L::D; ++x)
#pragma unroll
            for (int y = x; y < L::D; ++y) {
              const int cc = cx_<L>(i, x) * cx_<L>(i, y);
              if (cc != 0) P[x][y] += (C)cc * f[i];
            }
#pragma unroll
        for (int x = 0; x < L::D; ++x)
#pragma unroll
          for (int y = 0; y < x; ++y) P[x][y] = P[y][x];
      }
      if constexpr (product_basis<L>())
        rr_product<L, C, SH>(f, rho, rhop, u, P, (C)krr, a.ph.trace_eq != 0, rho1, rhop1);
      else
        rr_hermite3<L, C>(f, rho, rhop, u, P, (C)krr, a.ph.trace_eq != 0);
    } else {
      C feq[Q], geq[Q];
      double lam[NLAM];
      if constexpr (COLL >= COLL_DDF_NEWTON) {
#pragma unroll
        for (int k = 0; k < NLAM; ++k) lam[k] = (double)((const LamT<S> *)a.lam)[(int64_t)k * a.stride + c];
      }
      int it;
      if constexpr (COLL >= COLL_DDF_NEWTON) {
        // park f and g in LDS while the Newton solve needs the registers
        // (the memory clobbers keep the compiler from holding them anyway)
        __shared__ C park[BLOCK / 64][2 * Q][64];
        const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          park[wv][i][ln] = f[i];
          park[wv][Q + i][ln] = g[i];
        }
        asm volatile("" ::: "memory");
        it = equilibrium_any<L, COLL, C>(rhop, u, T, a.ph, lam, a.ph.warm != 0, feq, geq);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          f[i] = park[wv][i][ln];
          g[i] = park[wv][Q + i][ln];
        }
      } else {
        it = equilibrium_any<L, COLL, C>(rhop, u, T, a.ph, lam, a.ph.warm != 0, feq, geq);
      }
      if constexpr (COLL >= COLL_DDF_NEWTON) {
        count_add(a.counters, CNT_NEWTON_CALLS, 1);
        if (it < 0) count_add(a.counters, CNT_NEWTON_FAIL, 1);
        else count_add(a.counters, CNT_NEWTON_ITERS, (unsigned long long)it);
        count_hist(a.counters, it);
#pragma unroll
        for (int k = 0; k < NLAM; ++k) ((LamT<S> *)a.lam)[(int64_t)k * a.stride + c] = (LamT<S>)lam[k];
      }
      C te = (C)tau;
      if (a.ph.sensor_on) te *= sensor_alpha<L, C>(f, feq, te, (C)a.ph.sensor_A);
      const C om = (C)1 / te;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        f[i] = f[i] - om * (f[i] - feq[i]);
        g[i] = g[i] - om * (g[i] - geq[i]);
      }
    }
  }
  S *fout = (S *)fout_p;
  S *gout = (S *)gout_p;
  if constexpr (AA != 0) {
    // in place on a refined grid, a coarse ghost also leaves its
    // post-collision populations in its coalesced slot, row i, for the
    // explosion (pushed to the neighbours they are scattered)
    if (a.gslot) {
      const int32_t vs = a.gslot[c];
      if (vs >= 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          Sto<S>::stn(fout, pix<Q>(i, vs), f[i], SH ? 0.0 : L::S.w[i]);
          if (DDF) Sto<S>::stn(gout, pix<Q>(i, vs), g[i], 0.0);
        }
      }
    }
  }
  if constexpr (AA == 2) {
    push_store<L, S, DDF, SH>(fout, gout, a.topo, nbs[0], c, threadIdx.x & 63, brick,
                          xm, a.ph.uw, a.ph.cs2w, f, g);
  } else {
    // row base (uniform: a wavefront's brick lies in one chunk) + the
    // cell's 32-bit byte offset in the chunk: the address needs no per-lane
    // 64-bit arithmetic
    const int64_t ck = __builtin_amdgcn_readfirstlane((int32_t)(c >> PCH_SH));
    constexpr int64_t rbytes = PCH * (int64_t)sizeof(S);
    char *ob = (char *)fout + ck * Q * rbytes;
    char *gb = DDF ? (char *)gout + ck * Q * rbytes : nullptr;
    const uint32_t co = (uint32_t)(c & (PCH - 1)) * (uint32_t)sizeof(S);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int64_t r = AA == 1 ? L::S.opp[i] : i;
      // the row base stays uniform (SGPRs) and the store adds the offset
      auto row = (gptr<char>)(ob + r * rbytes);
      asm("" : "+s"(row));
      Sto<S>::stg((gptr<S>)(row + co), f[i], SH ? 0.0 : L::S.w[i]);
      if (DDF) {
        auto grow = (gptr<char>)(gb + r * rbytes);
        asm("" : "+s"(grow));
        Sto<S>::stg((gptr<S>)(grow + co), g[i], 0.0);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// coalescence (Eq. coalescence): 2^D lanes per coarse ghost, one per child;
// each lane pulls the child's population as the fine level's next update
// would, the lanes of a ghost are summed with wavefront shuffles
// ---------------------------------------------------------------------------
// In place (AAF = 2: the fine level at an odd phase, its rows swapped) the
// children are read as that level's swapped pull; SW: the coarse level is at
// an odd phase and reads population i of its coalesced slot from row opp(i).
template <class L, class S, bool PRE, bool DDF, bool LAM, int AAF = 0, bool SW = false>
__global__ void __launch_bounds__(BLOCK) k_coalesce(const CArgs a) {
  using C = typename Sto<S>::C;
  constexpr int NCH = 1 << L::D;
  const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  // lanes (ghost, group, child): group k of ngrp takes the populations
  // i = k mod ngrp, so that a small interface still spreads over many
  // compute units
  const int64_t q = t / NCH;
  const int64_t gl = q / a.ngrp;
  const int grp = (int)(q % a.ngrp);
  const bool valid = gl < a.count;
  const int64_t gk = a.g0 + gl;
  const int32_t ch = valid ? a.child[gk * NCH + (t % NCH)] : -1;
  const int32_t crow = ch >= 0 ? a.crow[gk * NCH + (t % NCH)] : 0;
  uint64_t mask = valid ? a.unknown[gk] : 0ull;
  if (a.ngrp > 1) {
    uint64_t sel = 0ull;
    for (int i = grp; i < L::Q; i += a.ngrp) sel |= 1ull << i;
    mask &= sel;
  }
  const bool lead = valid && (t % NCH) == 0;
  const C nf = group_sum<NCH, C>(ch >= 0 ? (C)1 : (C)0);
  const S *fin = (const S *)a.fin_child;
  const S *gin = (const S *)a.gin_child;
  S *fout = (S *)a.fout_coarse;
  S *gout = (S *)a.gout_coarse;
  const int64_t slot = a.vbase + gk;
  if (a.ngrp > 1) {
    // a small interface: the lane's own populations one at a time.  The
    // unrolled path below is tens of KB of code for the wide lattices, and
    // its cold instruction fetch dominates a launch of a few workgroups.
    // The NCH lanes of a group share grp and so the trip count.
    for (int i = grp == 0 ? a.ngrp : grp; i < L::Q; i += a.ngrp) {
      const bool need = (mask >> i) & 1ull;
      C v = (C)0, vg = (C)0;
      if (need && ch >= 0) {
        const int32_t sv = a.xnbr[(int64_t)(i - 1) * a.xstride + crow];
        int64_t idx;
        const int64_t ri = AAF == 2 ? L::S.opp[i] : i, ro = AAF == 2 ? i : L::S.opp[i];
        if (PRE) idx = pix<L::Q>(i, (int64_t)sv >= a.vbase ? (int64_t)sv : (int64_t)ch);
        else idx = sv >= 0 ? pix<L::Q>(ri, sv) : pix<L::Q>(ro, ch);
        v = Sto<S>::ld(fin, idx, L::S.w[i]);
        if (DDF) vg = Sto<S>::ld(gin, idx, 0.0);
        if (!PRE && sv <= -2)
          v += (C)(2.0 * L::S.w[i] * (wall_dot<L>(a.uw, -2 - sv, i) + noise_dot(a.xdu, a.xstride, crow, i)) /
                   a.cs2w);
      }
      v = group_sum<NCH, C>(v);
      if (DDF) vg = group_sum<NCH, C>(vg);
      if (lead && need) {
        const int64_t r = SW ? L::S.opp[i] : i;
        Sto<S>::st(fout, pix<L::Q>(r, slot), v / nf, L::S.w[i]);
        if (DDF) Sto<S>::st(gout, pix<L::Q>(r, slot), vg / nf, 0.0);
      }
    }
  } else {
    // the child's populations as the fine level's next update pulls them
    // (every child of a coarse ghost has an explicit row), all loads first
    C f[L::Q], g[DDF ? L::Q : 1];
    if (ch >= 0)
      gather_row<L, S, PRE, DDF, AAF>(fin, gin, a.xnbr, a.xstride, crow, a.vbase, ch, a.uw, a.cs2w, f, g,
                                      mask, a.xdu);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      const bool need = (mask >> i) & 1ull;
      C v = (need && ch >= 0) ? f[i] : (C)0;
      C vg = (DDF && need && ch >= 0) ? g[i] : (C)0;
      v = group_sum<NCH, C>(v);
      if (DDF) vg = group_sum<NCH, C>(vg);
      if (lead && need) {
        const int64_t r = SW ? L::S.opp[i] : i;
        Sto<S>::st(fout, pix<L::Q>(r, slot), v / nf, L::S.w[i]);
        if (DDF) Sto<S>::st(gout, pix<L::Q>(r, slot), vg / nf, 0.0);
      }
    }
  }
  if (LAM) {
    // the multipliers go with group 0 (a group's NCH lanes agree on it)
    const bool mine = grp == 0;
    const int64_t G = valid && mine ? a.ghost_cell[gk] : 0;
#pragma unroll
    for (int k = 0; k < NLAM; ++k) {
      double v = ch >= 0 && mine ? (double)((const LamT<S> *)a.lam)[(int64_t)k * a.stride + ch] : 0.0;
      v = group_sum<NCH, double>(v);
      if (lead && mine) ((LamT<S> *)a.lam)[(int64_t)k * a.stride + G] = (LamT<S>)(v / (double)nf);
    }
  }
}

// uniform explosion (Eq. explosion_uniform): children take every
// post-collision population of their coarse ghost (raw copy of storage).
// MODE 0: two buffers, from the ghost's slot into the child's rows.  In
// place the ghost's populations are read from its coalesced slot, where its
// collide left them; MODE 1 (fine level at an odd phase): child row opp(i)
// takes population i; MODE 2 (even phase): population i goes to row i of
// the cell that pulls it from the child, as the child's own push would have
// sent it (a wall returns it to the child's row opp(i) with the moving-wall
// term; a population the child pulls from itself stays in its row i).
template <class L, class S, bool DDF, bool LAM, int MODE = 0>
__global__ void __launch_bounds__(BLOCK) k_explode(const EArgs a) {
  using C = typename Sto<S>::C;
  constexpr int NCH = 1 << L::D;
  const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t gl = t / NCH;
  if (gl >= a.count) return;
  const int64_t gk = a.g0 + gl;
  const int32_t ch = a.child[gk * NCH + (t % NCH)];
  if (ch < 0) return;
  const int64_t G = a.ghost_cell[gk];
  const int64_t src = MODE == 0 ? G : a.vbase + gk;
  const S *fin = (const S *)a.fin_coarse;
  S *fout = (S *)a.fout_fine;
  S v[L::Q], vg[DDF ? L::Q : 1];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) v[i] = fin[pix<L::Q>(i, src)];
  if (DDF)
#pragma unroll
    for (int i = 0; i < L::Q; ++i) vg[i] = ((const S *)a.gin_coarse)[pix<L::Q>(i, src)];
  S *gout = (S *)a.gout_fine;
  if constexpr (MODE == 2) {
    const int64_t crow = a.crow[gk * NCH + (t % NCH)];
    fout[pix<L::Q>(0, ch)] = v[0];
    if (DDF) gout[pix<L::Q>(0, ch)] = vg[0];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      const int j = L::S.opp[i];
      if (a.xnbr[(int64_t)(i - 1) * a.xstride + crow] == ch) {
        fout[pix<L::Q>(i, ch)] = v[i];
        if (DDF) gout[pix<L::Q>(i, ch)] = vg[i];
      }
      const int32_t s = a.xnbr[(int64_t)(j - 1) * a.xstride + crow];
      if (s == ch) continue;
      if (s >= 0) {
        fout[pix<L::Q>(i, s)] = v[i];
        if (DDF) gout[pix<L::Q>(i, s)] = vg[i];
      } else {
        C w = Sto<S>::ldv(v[i], L::S.w[i]);
        if (s <= -2) w += (C)(2.0 * L::S.w[j] * wall_dot<L>(a.uw, -2 - s, j) / a.cs2w);
        Sto<S>::st(fout, pix<L::Q>(j, ch), w, L::S.w[j]);
        if (DDF) gout[pix<L::Q>(j, ch)] = vg[i];
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) fout[pix<L::Q>(MODE == 1 ? L::S.opp[i] : i, ch)] = v[i];
    if (DDF)
#pragma unroll
      for (int i = 0; i < L::Q; ++i) gout[pix<L::Q>(MODE == 1 ? L::S.opp[i] : i, ch)] = vg[i];
  }
  if (LAM)
#pragma unroll
    for (int k = 0; k < NLAM; ++k) ((LamT<S> *)a.lam)[(int64_t)k * a.stride + ch] = ((LamT<S> *)a.lam)[(int64_t)k * a.stride + G];
}

// ---------------------------------------------------------------------------
// boundary layers: Neumann copy of the source cell's post-collision state;
// equilibrium Dirichlet with imposed (or extrapolated) density
// ---------------------------------------------------------------------------
template <class T6>
__device__ inline T6 pick6(const T6 (&v)[6], int k) {
  T6 r = v[0];
#pragma unroll
  for (int f = 1; f < 6; ++f)
    if (f == k) r = v[f];
  return r;
}

// store of a cell's post-collision value v of population i in place at an
// even phase (MODE 2 of the fills): to row i of the cell that pulls it
// (through the cell's exception row), back into the cell's row opp(i) with
// the moving-wall term at a wall, into its own row i when it pulls that
// population from itself.  RAW copies storage values unchanged where no
// arithmetic applies.  G: the second distribution (stored without the
// weight shift, bounced back without the moving-wall term).
template <class L, class S, bool G = false>
__device__ inline void push_value(S *f, int64_t c, const int32_t *xnbr, int64_t xstride, int64_t row,
                                  int i, typename Sto<S>::C v, S raw, bool use_raw, const double (&uw)[6][3],
                                  double cs2w) {
  using C = typename Sto<S>::C;
  const int j = L::S.opp[i];
  const double wi = G ? 0.0 : L::S.w[i];
  if (xnbr[(int64_t)(i - 1) * xstride + row] == (int32_t)c) {
    if (use_raw) f[pix<L::Q>(i, c)] = raw;
    else Sto<S>::st(f, pix<L::Q>(i, c), v, wi);
  }
  const int32_t s = xnbr[(int64_t)(j - 1) * xstride + row];
  if (s == (int32_t)c) return;
  if (s >= 0) {
    if (use_raw) f[pix<L::Q>(i, s)] = raw;
    else Sto<S>::st(f, pix<L::Q>(i, s), v, wi);
  } else if (G) {
    if (use_raw) f[pix<L::Q>(j, c)] = raw;
    else Sto<S>::st(f, pix<L::Q>(j, c), v, 0.0);
  } else {
    C w = use_raw ? Sto<S>::ldv(raw, L::S.w[i]) : v;
    if (s <= -2) w += (C)(2.0 * L::S.w[j] * wall_dot<L>(uw, -2 - s, j) / cs2w);
    Sto<S>::st(f, pix<L::Q>(j, c), w, L::S.w[j]);
  }
}

// MODE 0: two buffers; 1, 2: in place, the level at an odd / even phase
// after its step (see BArgs)
template <class L, int COLL, class S, int MODE = 0>
__global__ void __launch_bounds__(BLOCK) k_bcfill(const BArgs a) {
  using C = typename Sto<S>::C;
  constexpr bool DDF = COLL >= COLL_DDF_POLY;
  constexpr bool LAM = COLL >= COLL_DDF_NEWTON;
  const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (t >= a.count) return;
  const int64_t k = a.b0 + t;
  const int64_t c = a.bc_cell[k], src = a.bc_src[k];
  const int face = a.bc_face[k];
  S *f = (S *)a.f;
  S *g = (S *)a.g;
  // where population i of the source and of the cell live
  const int64_t sbase = MODE == 2 ? (int64_t)a.stage[src] : src;
  auto srow = [&](int i) -> int64_t { return MODE == 1 ? L::S.opp[i] : i; };
  const int64_t row = MODE == 2 ? (int64_t)a.bc_row[k] : 0;
  int kind = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if (q == face) kind = a.fv.extrap[q];
  const double frho = pick6(a.fv.rho, face), fT = pick6(a.fv.T, face);
  double fu[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if (q == face) { fu[0] = a.fv.u[q][0]; fu[1] = a.fv.u[q][1]; fu[2] = a.fv.u[q][2]; }
  if (kind < 0) {  // Neumann: all loads, then all stores
    S v[L::Q], vg[DDF ? L::Q : 1];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) v[i] = f[pix<L::Q>(srow(i), sbase)];
    if (DDF)
#pragma unroll
      for (int i = 0; i < L::Q; ++i) vg[i] = g[pix<L::Q>(srow(i), sbase)];
    if constexpr (MODE == 2) {
      f[pix<L::Q>(0, c)] = v[0];
      if (DDF) g[pix<L::Q>(0, c)] = vg[0];
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        push_value<L, S>(f, c, a.xnbr, a.xstride, row, i, (C)0, v[i], true, a.ph.uw, a.ph.cs2w);
        if (DDF) push_value<L, S, true>(g, c, a.xnbr, a.xstride, row, i, (C)0, vg[i], true, a.ph.uw, 1.0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < L::Q; ++i) f[pix<L::Q>(srow(i), c)] = v[i];
      if (DDF)
#pragma unroll
        for (int i = 0; i < L::Q; ++i) g[pix<L::Q>(srow(i), c)] = vg[i];
    }
    if (LAM)
#pragma unroll
      for (int q = 0; q < NLAM; ++q) ((LamT<S> *)a.lam)[(int64_t)q * a.stride + c] = ((LamT<S> *)a.lam)[(int64_t)q * a.stride + src];
    return;
  }
  C rho = (C)frho;
  if (kind == 1) {
    rho = (C)0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) rho += Sto<S>::ld(f, pix<L::Q>(srow(i), sbase), L::S.w[i]);
  }
  C u[3] = {(C)fu[0], (C)fu[1], (C)fu[2]};
  C feq[L::Q], geq[DDF ? L::Q : 1];
  double lam[NLAM];
  if (LAM)
#pragma unroll
    for (int q = 0; q < NLAM; ++q) lam[q] = (double)((const LamT<S> *)a.lam)[(int64_t)q * a.stride + c];
  const int it = equilibrium_any<L, COLL, C>(rho, u, (C)fT, a.ph, lam, a.ph.warm != 0, feq, geq);
  if (LAM) {
    if (it < 0) count_add(a.counters, CNT_NEWTON_FAIL, 1);
#pragma unroll
    for (int q = 0; q < NLAM; ++q) ((LamT<S> *)a.lam)[(int64_t)q * a.stride + c] = (LamT<S>)lam[q];
  }
  if constexpr (MODE == 2) {
    Sto<S>::st(f, pix<L::Q>(0, c), feq[0], L::S.w[0]);
    if (DDF) Sto<S>::st(g, pix<L::Q>(0, c), geq[0], 0.0);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      push_value<L, S>(f, c, a.xnbr, a.xstride, row, i, feq[i], S(), false, a.ph.uw, a.ph.cs2w);
      if (DDF) push_value<L, S, true>(g, c, a.xnbr, a.xstride, row, i, geq[i], S(), false, a.ph.uw, 1.0);
    }
  } else {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      Sto<S>::st(f, pix<L::Q>(srow(i), c), feq[i], L::S.w[i]);
      if (DDF) Sto<S>::st(g, pix<L::Q>(srow(i), c), geq[i], 0.0);
    }
  }
}

// ---------------------------------------------------------------------------
// gathers of the synchronisation-point state (pre-collision populations;
// coarse ghosts read their coalesced slots)
// ---------------------------------------------------------------------------
template <class L, class S, bool PRE, bool DDF, int AA = 0>
__global__ void __launch_bounds__(BLOCK) k_gather(const MArgs a) {
  using C = typename Sto<S>::C;
  constexpr int Q = L::Q;
  __shared__ uint32_t nbs[BLOCK / 64][Brick<L>::NBP];
  const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (a.mode == 3) {
    // populations (and multipliers) of the listed cells of this level
    if (t >= a.count) return;
    const int64_t k = a.list_begin + t;
    const int32_t cell = a.cells_list[k];
    const int64_t c = a.slot_of[cell];
    C f[Q];
    C g[DDF ? Q : 1];
    gather_one<L, S, PRE, DDF, AA>((const S *)a.fin, (const S *)a.gin, a.topo, a.vbase, c, a.uw, a.cs2w,
                                   f, g);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      a.out[(int64_t)i * a.n + k] = (double)f[i];
      if (DDF) a.out[(int64_t)(Q + i) * a.n + k] = (double)g[i];
    }
    if (a.lam_out)
      for (int q = 0; q < NLAM; ++q) a.lam_out[(int64_t)q * a.n + k] = (double)((const LamT<S> *)a.lam)[(int64_t)q * a.stride + c];
    return;
  }
  const bool live = t < a.count;  // whole wavefronts
  const int64_t c = a.begin + (live ? t : 0);
  const int32_t brick = stage_bricks<L, S>(a.topo, nbs, c, live);
  const int32_t cell = live ? a.cell_of[c] : -1;
  const bool valid = cell >= 0;
  C f[Q];
  C g[DDF ? Q : 1];
  const bool fine_ghost = valid && (a.flags[c] & F_FINE_GHOST);
  if (valid)
    gather<L, S, PRE, DDF, AA>((const S *)a.fin, (const S *)a.gin, a.topo, nbs[0],
                               a.vbase, c, threadIdx.x & 63, brick, a.topo.xmask[brick], a.uw, a.cs2w, f, g);
  if (a.mode == 0) {
    if (!valid) return;
    const int nm = 1 + L::D + (DDF ? 1 : 0);
    if (fine_ghost) {
      for (int k = 0; k < nm; ++k) a.out[(int64_t)k * a.n + cell] = __longlong_as_double(0x7ff8000000000000ll);
      return;
    }
    C rho, u[3], T;
    cell_moments<L, C, DDF>(f, g, (C)a.Cv, rho, u, T);
    a.out[cell] = (double)rho;
    for (int d = 0; d < L::D; ++d) a.out[(int64_t)(1 + d) * a.n + cell] = (double)u[d];
    if (DDF) a.out[(int64_t)(1 + L::D) * a.n + cell] = (double)T;
    return;
  }
  if (a.mode == 1) {
    if (!valid) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      a.out[(int64_t)i * a.n + cell] = (double)f[i];
      if (DDF) a.out[(int64_t)(Q + i) * a.n + cell] = (double)g[i];
    }
    if (a.lam_out)
      for (int k = 0; k < NLAM; ++k)
        a.lam_out[(int64_t)k * a.n + cell] = (double)((const LamT<S> *)a.lam)[(int64_t)k * a.stride + c];
    return;
  }
}

// ---------------------------------------------------------------------------
// conserved sums at the synchronisation point (Sec. 4.1's reductions): mass,
// momentum, total energy (|xi|^2 f / 2 + g / 2) and kinetic energy
// (rho |u|^2 / 2) of the cells that are not fine ghosts, volume-weighted,
// in FP64.  Each block strides over the level's 256-slot tiles (tile b,
// b + gridDim.x, ...) and writes one partial per quantity, so the partials
// take gridDim.x x 6 doubles whatever the size of the level; every thread
// accumulates its tiles in a fixed order and the block reduction has a fixed
// shape, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
template <class L, class S, bool PRE, bool DDF, int AA = 0>
__global__ void __launch_bounds__(BLOCK) k_sums(const MArgs a) {
  using C = typename Sto<S>::C;
  constexpr int Q = L::Q;
  __shared__ uint32_t nbs[BLOCK / 64][Brick<L>::NBP];
  __shared__ double red[BLOCK / 64][6];
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t tiles = (a.count + BLOCK - 1) / BLOCK;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t t = tile * BLOCK + threadIdx.x;
    const bool live = t < a.count;  // whole wavefronts
    const int64_t c = a.begin + (live ? t : 0);
    const int32_t brick = stage_bricks<L, S>(a.topo, nbs, c, live);
    const int32_t cell = live ? a.cell_of[c] : -1;
    if (cell >= 0 && !(a.flags[c] & F_FINE_GHOST)) {
      C f[Q];
      C g[DDF ? Q : 1];
      gather<L, S, PRE, DDF, AA>((const S *)a.fin, (const S *)a.gin, a.topo, nbs[0],
                                 a.vbase, c, threadIdx.x & 63, brick, a.topo.xmask[brick], a.uw, a.cs2w, f, g);
      double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double fi = (double)f[i];
        q[0] += fi;
#pragma unroll
        for (int d = 0; d < L::D; ++d) q[1 + d] += fi * cx_<L>(i, d);
        const int n2 = cx_<L>(i, 0) * cx_<L>(i, 0) + cx_<L>(i, 1) * cx_<L>(i, 1) + cx_<L>(i, 2) * cx_<L>(i, 2);
        q[4] += 0.5 * (n2 * fi + (DDF ? (double)g[i] : 0.0));
      }
      // kinetic energy rho |u|^2 / 2 = |j|^2 / (2 rho) of the cell
      q[5] = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
#pragma unroll
      for (int k = 0; k < 6; ++k) s[k] += q[k] * a.vol;
    }
    __syncthreads();  // the next tile restages the brick table
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double v = s[k];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    s[k] = v;
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) red[wid][k] = s[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) {
      double v = 0.0;
      for (int w = 0; w < BLOCK / 64; ++w) v += red[w][k];
      a.partials[(int64_t)blockIdx.x * 6 + k] = v;
    }
}

// ---------------------------------------------------------------------------
// initialisation at equilibrium (App. A.3) or restore of raw populations
// ---------------------------------------------------------------------------
template <class L, int COLL, class S>
__global__ void __launch_bounds__(BLOCK) k_init(const IArgs a) {
  using C = typename Sto<S>::C;
  constexpr bool DDF = COLL >= COLL_DDF_POLY;
  constexpr bool LAM = COLL >= COLL_DDF_NEWTON;
  const int64_t k0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;  // canonical cell
  if (k0 >= a.n) return;
  const int64_t c = a.slot_of[k0];
  S *f = (S *)a.f;
  S *g = (S *)a.g;
  if (a.mode == 1) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      Sto<S>::st(f, pix<L::Q>(i, c), (C)a.src[(int64_t)i * a.n + k0], L::S.w[i]);
      if (DDF) Sto<S>::st(g, pix<L::Q>(i, c), (C)a.src_g[(int64_t)i * a.n + k0], 0.0);
    }
    if (LAM && a.src_lam)
      for (int k = 0; k < NLAM; ++k) ((LamT<S> *)a.lam)[(int64_t)k * a.stride + c] = (LamT<S>)a.src_lam[(int64_t)k * a.n + k0];
    return;
  }
  const C rho = (C)a.src[k0];
  C u[3] = {(C)0, (C)0, (C)0};
  for (int d = 0; d < L::D; ++d) u[d] = (C)a.src[(int64_t)(1 + d) * a.n + k0];
  const C T = DDF ? (C)a.src[(int64_t)(1 + L::D) * a.n + k0] : (C)0;
  C feq[L::Q], geq[DDF ? L::Q : 1];
  double lam[NLAM];
  const int it = equilibrium_any<L, COLL, C>(rho, u, T, a.ph, lam, false, feq, geq);
  if (LAM) {
    if (it < 0) count_add(a.counters, CNT_NEWTON_FAIL, 1);
    for (int k = 0; k < NLAM; ++k) ((LamT<S> *)a.lam)[(int64_t)k * a.stride + c] = (LamT<S>)lam[k];
  }
  if (!(rho > (C)0) || !isfinite(rho)) count_add(a.counters, CNT_NONFINITE, 1);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    Sto<S>::st(f, pix<L::Q>(i, c), feq[i], L::S.w[i]);
    if (DDF) Sto<S>::st(g, pix<L::Q>(i, c), geq[i], 0.0);
  }
}

// ---------------------------------------------------------------------------
// kinetic sensor of every cell at the synchronisation point (Eq. DeltaAvg):
// the mean over i of |f_i - f_eq,i| / |f_eq,i|, f_eq of the collision model
// at the cell's own moments (Newton warm-started from the stored
// multipliers, which stay untouched); NaN for fine ghosts.  It is the
// refinement criterion of mesh adaptation.
// ---------------------------------------------------------------------------
template <class L, int COLL, class S, bool PRE, int AA = 0>
__global__ void __launch_bounds__(BLOCK) k_sensor(const MArgs a, const PhysArgs ph) {
  using C = typename Sto<S>::C;
  constexpr int Q = L::Q;
  constexpr bool DDF = COLL >= COLL_DDF_POLY;
  __shared__ uint32_t nbs[BLOCK / 64][Brick<L>::NBP];
  const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool live = t < a.count;  // whole wavefronts
  const int64_t c = a.begin + (live ? t : 0);
  const int32_t brick = stage_bricks<L, S>(a.topo, nbs, c, live);
  const int32_t cell = live ? a.cell_of[c] : -1;
  if (cell < 0) return;
  if (a.flags[c] & F_FINE_GHOST) {
    a.out[cell] = __longlong_as_double(0x7ff8000000000000ll);
    return;
  }
  C f[Q];
  C g[DDF ? Q : 1];
  gather<L, S, PRE, DDF, AA>((const S *)a.fin, (const S *)a.gin, a.topo, nbs[0], a.vbase,
                             c, threadIdx.x & 63, brick, a.topo.xmask[brick], a.uw, a.cs2w, f, g);
  C rho, u[3], T;
  cell_moments<L, C, DDF>(f, g, (C)a.Cv, rho, u, T);
  double lam[NLAM];
#pragma unroll
  for (int k = 0; k < NLAM; ++k) lam[k] = COLL >= COLL_DDF_NEWTON ? (double)((const LamT<S> *)a.lam)[(int64_t)k * a.stride + c] : 0.0;
  C feq[Q], geq[Q];
  equilibrium_any<L, COLL, C>(rho, u, T, ph, lam, true, feq, geq);
  constexpr C tiny = sizeof(C) == 8 ? (C)1e-300 : (C)1e-30;
  C eps = (C)0;
#pragma unroll
  for (int i = 0; i < Q; ++i) eps += fabs(f[i] - feq[i]) / fmax(fabs(feq[i]), tiny);
  a.out[cell] = (double)(eps * (C)(1.0 / Q));
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
inline unsigned nblocks(int64_t work) { return (unsigned)((work + BLOCK - 1) / BLOCK); }

template <class L, int COLL, class S>
struct Launch {
  static constexpr bool DDF = COLL >= COLL_DDF_POLY;
  static constexpr bool LAM = COLL >= COLL_DDF_NEWTON;
  static void collide(const KArgs &a, bool pre, hipStream_t s) {
    if (a.count <= 0) return;
    constexpr int CB = CollideBlock<L, COLL>::value;
    const unsigned nb = (unsigned)((a.count + CB - 1) / CB);
    if (a.aa == 1) hipLaunchKernelGGL((k_collide<L, COLL, S, false, 1>), dim3(nb), dim3(CB), 0, s, a);
    else if (a.aa == 2) hipLaunchKernelGGL((k_collide<L, COLL, S, false, 2>), dim3(nb), dim3(CB), 0, s, a);
    else if (noisy(a)) {
      // inflow noise on the moving-wall links: separate instantiations, so
      // that the others keep their registers
      if constexpr (COLL < COLL_DDF_NEWTON) {
        if (pre) hipLaunchKernelGGL((k_collide<L, COLL, S, true, 0, true>), dim3(nb), dim3(CB), 0, s, a);
        else if (a.topo.off32) hipLaunchKernelGGL((k_collide<L, COLL, S, false, 0, true, true>), dim3(nb), dim3(CB), 0, s, a);
        else hipLaunchKernelGGL((k_collide<L, COLL, S, false, 0, true>), dim3(nb), dim3(CB), 0, s, a);
      }
    } else if (pre) hipLaunchKernelGGL((k_collide<L, COLL, S, true>), dim3(nb), dim3(CB), 0, s, a);
    else if (a.topo.off32) hipLaunchKernelGGL((k_collide<L, COLL, S, false, 0, false, true>), dim3(nb), dim3(CB), 0, s, a);
    else hipLaunchKernelGGL((k_collide<L, COLL, S, false>), dim3(nb), dim3(CB), 0, s, a);
  }
  static bool noisy(const KArgs &a) { return a.topo.xdu != nullptr; }
  static void collide_multi(const KArgs &a, hipStream_t s) {
    if constexpr (COLL < COLL_DDF_NEWTON) {
      constexpr int CB = CollideBlock<L, COLL>::value;
      const dim3 grid((unsigned)a.multi.block0[a.multi.n]);
      if (a.multi.n > 0 && a.multi.block0[a.multi.n] > 0) {
        if (noisy(a) && a.topo.off32) hipLaunchKernelGGL((k_collide<L, COLL, S, false, 0, true, true>), grid, dim3(CB), 0, s, a);
        else if (noisy(a)) hipLaunchKernelGGL((k_collide<L, COLL, S, false, 0, true>), grid, dim3(CB), 0, s, a);
        else if (a.topo.off32) hipLaunchKernelGGL((k_collide<L, COLL, S, false, 0, false, true>), grid, dim3(CB), 0, s, a);
        else hipLaunchKernelGGL((k_collide<L, COLL, S, false>), grid, dim3(CB), 0, s, a);
      }
    }
  }
  static void coalesce(const CArgs &a0, bool pre, hipStream_t s) {
    if (a0.count <= 0) return;
    // split the populations of a child over up to 8 lanes while the
    // interface is too small to give every compute unit a workgroup
    CArgs a = a0;
    const int64_t lanes = a.count << L::D;
    a.ngrp = (int)std::min<int64_t>(8, std::max<int64_t>(1, (256 * BLOCK) / lanes));
    const int64_t work = lanes * a.ngrp;
    const dim3 nb(nblocks(work));
    if (a.swap) {
      // in place, coarse level at an odd phase
      if (a.aa == 2) hipLaunchKernelGGL((k_coalesce<L, S, false, DDF, LAM, 2, true>), nb, dim3(BLOCK), 0, s, a);
      else if (pre) hipLaunchKernelGGL((k_coalesce<L, S, true, DDF, LAM, 0, true>), nb, dim3(BLOCK), 0, s, a);
      else hipLaunchKernelGGL((k_coalesce<L, S, false, DDF, LAM, 0, true>), nb, dim3(BLOCK), 0, s, a);
    } else if (a.aa == 2) {
      hipLaunchKernelGGL((k_coalesce<L, S, false, DDF, LAM, 2>), nb, dim3(BLOCK), 0, s, a);
    } else if (pre) {
      hipLaunchKernelGGL((k_coalesce<L, S, true, DDF, LAM>), nb, dim3(BLOCK), 0, s, a);
    } else {
      hipLaunchKernelGGL((k_coalesce<L, S, false, DDF, LAM>), nb, dim3(BLOCK), 0, s, a);
    }
  }
  static void explode(const EArgs &a, hipStream_t s) {
    if (a.count <= 0) return;
    const dim3 nb(nblocks(a.count << L::D));
    if (a.mode == 1) hipLaunchKernelGGL((k_explode<L, S, DDF, LAM, 1>), nb, dim3(BLOCK), 0, s, a);
    else if (a.mode == 2) hipLaunchKernelGGL((k_explode<L, S, DDF, LAM, 2>), nb, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_explode<L, S, DDF, LAM>), nb, dim3(BLOCK), 0, s, a);
  }
  static void bcfill(const BArgs &a, hipStream_t s) {
    if (a.count <= 0) return;
    const dim3 nb(nblocks(a.count));
    if (a.mode == 1) hipLaunchKernelGGL((k_bcfill<L, COLL, S, 1>), nb, dim3(BLOCK), 0, s, a);
    else if (a.mode == 2) hipLaunchKernelGGL((k_bcfill<L, COLL, S, 2>), nb, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_bcfill<L, COLL, S>), nb, dim3(BLOCK), 0, s, a);
  }
  static void gather(const MArgs &a, bool pre, hipStream_t s) {
    if (a.count <= 0) return;
    if (a.aa == 2) hipLaunchKernelGGL((k_gather<L, S, false, DDF, 2>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a);
    else if (pre) hipLaunchKernelGGL((k_gather<L, S, true, DDF>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_gather<L, S, false, DDF>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a);
  }
  static void sums(const MArgs &a, bool pre, hipStream_t s) {
    if (a.count <= 0) return;
    const dim3 nb((unsigned)sum_blocks(a.count));
    if (a.aa == 2) hipLaunchKernelGGL((k_sums<L, S, false, DDF, 2>), nb, dim3(BLOCK), 0, s, a);
    else if (pre) hipLaunchKernelGGL((k_sums<L, S, true, DDF>), nb, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_sums<L, S, false, DDF>), nb, dim3(BLOCK), 0, s, a);
  }
  static void init(const IArgs &a, hipStream_t s) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL((k_init<L, COLL, S>), dim3(nblocks(a.n)), dim3(BLOCK), 0, s, a);
  }
  static void sensor(const MArgs &a, const PhysArgs &ph, bool pre, hipStream_t s) {
    if (a.count <= 0) return;
    if (a.aa == 2)
      hipLaunchKernelGGL((k_sensor<L, COLL, S, false, 2>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a, ph);
    else if (pre) hipLaunchKernelGGL((k_sensor<L, COLL, S, true>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a, ph);
    else hipLaunchKernelGGL((k_sensor<L, COLL, S, false>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a, ph);
  }
  static Ops ops() {
    Ops o;
    o.sensor = &sensor;
    o.collide = &collide;
    o.collide_multi = COLL < COLL_DDF_NEWTON ? &collide_multi : nullptr;
    o.collide_block = CollideBlock<L, COLL>::value;
    o.coalesce = &coalesce;
    o.explode = &explode;
    o.bcfill = &bcfill;
    o.gather = &gather;
    o.sums = &sums;
    o.init = &init;
    o.sizeof_storage = (int)sizeof(S);
    return o;
  }
};

}  // namespace lbm
