// Kernel instantiations for D2Q21: double distribution with the numerical
// (entropy-maximising) equilibrium solved by Newton, or predicted by the
// multiplier surrogate (alone, or with one Newton correction and a Newton
// fallback), FP64 / FP32 storage; BGK and recursive regularisation on the
// full third-order Hermite basis, FP64 / FP32 / FP16 storage.
#include "kernels.cuh"
#include "mlp.cuh"

namespace lbm {
using L21 = Lattice<LAT_D2Q21>;

// Collide-and-stream with the surrogate: the block stages the network's
// weights in LDS once, every wavefront evaluates the MLP for its 64 cells
// (two 32-cell tiles on the matrix cores, activations kept in registers
// between the layers), then each cell
// takes the predicted multipliers (DDF_MLP), or one Newton correction from
// them with a full Newton fallback above fallback_tol (DDF_MLP_NEWTON).
// The populations are pulled twice: for the moments, and again (from the
// caches) for the collision, so that they are not live across the MLP and
// the Newton solve; holding them needs 284 registers, one wavefront per SIMD
// instead of two.
template <int COLL, class S, bool PRE>
__global__ void __launch_bounds__(BLOCK) k_collide_mlp(const KArgs a) {
  using L = L21;
  using C = typename Sto<S>::C;
  constexpr int Q = L::Q;
  __shared__ MlpInfer W;
  __shared__ uint32_t nbs[BLOCK / 64][Brick<L>::NBP];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t t = xcd_block() * BLOCK + threadIdx.x;
  const bool live = t < a.count;  // whole wavefronts
  const int64_t c = a.begin + (live ? t : 0);
  const int32_t brick = stage_bricks<L, S>(a.topo, nbs, c, live);
  const uint8_t fl = live ? a.flags[c] : (uint8_t)F_HOLE;
  const bool valid = !(fl & F_HOLE);
  C rho = (C)1, u[3] = {(C)0, (C)0, (C)0}, T = (C)1;
  if (valid) {
    C f[Q], g[Q];
    gather<L, S, PRE, true, 0, false>((const S *)a.fin, (const S *)a.gin, a.topo, nbs[0], a.vbase, c, l, brick,
                            a.topo.xmask[brick], a.ph.uw, a.ph.cs2w, f, g);
    cell_moments<L, C, true>(f, g, (C)a.ph.Cv, rho, u, T);
  }
  // the populations again, after the equilibrium (no code motion across)
  auto pull = [&](C *f, C *g) {
    asm volatile("" ::: "memory");
    gather<L, S, PRE, true, 0, false>((const S *)a.fin, (const S *)a.gin, a.topo, nbs[0], a.vbase, c, l, brick,
                            a.topo.xmask[brick], a.ph.uw, a.ph.cs2w, f, g);
  };
  const bool collide = valid && !(fl & (F_FINE_GHOST | F_BC_NEUMANN | F_BC_EQ));
  // the multipliers depend on (u, T) only; non-colliding lanes feed a benign state
  float cux = collide ? (float)u[0] : 0.0f, cuy = collide ? (float)u[1] : 0.0f;
  const Canon cn = canonical(cux, cuy);
  const MlpOperands *P = (const MlpOperands *)a.ph.mlp;
  stage_infer(&P->inf, &W);
  float xin[4], y[8];
  mlp_normalise(collide ? (float)rho : 1.0f, cux, cuy, collide ? (float)T : 1.0f, xin);
  mlp_infer_wave(W, xin, y);
  if (collide) {
    double lam[NLAM];
#pragma unroll
    for (int k = 0; k < NLAM; ++k) lam[k] = (double)P->mu[k] + (double)P->sig[k] * (double)y[k];
    uncanonical(cn, lam);
    C rhop = rho;
    if (fl & F_SPONGE) {
      const C s = (C)a.sigma[c];
      rhop = rho * ((C)1 - s) + s * (C)a.rho_inf[c];
    }
    if (!(rho > (C)0) || !isfinite(rho)) count_add(a.counters, CNT_NONFINITE, 1);
    C e[Q];
    if constexpr (COLL == COLL_DDF_MLP_NEWTON) {
      // one Newton correction from the network's multipliers; where the
      // residual then exceeds fallback_tol, Newton continues from the
      // corrected multipliers to newton_tol (from zero if the correction
      // itself failed)
      count_add(a.counters, CNT_NEWTON_CALLS, 1);
      // one call site for both attempts (a second inlined solver would
      // raise the kernel's register need)
      int it = -1;
      for (int attempt = 0; attempt < 2; ++attempt) {
        if (attempt == 1)
#pragma unroll
          for (int k = 0; k < NLAM; ++k) lam[k] = 0.0;
        it = newton_lean<L, C>((double)u[0], (double)u[1], (double)T, lam, a.ph.newton_tol, a.ph.newton_max_it,
                               attempt == 0 ? 1 : 0, attempt == 0 ? a.ph.fallback_tol : a.ph.newton_tol, e);
        if (attempt == 0 && it != 1) count_add(a.counters, CNT_MLP_FALLBACK, 1);
        if (it >= 0) break;
      }
      if (it < 0) count_add(a.counters, CNT_NEWTON_FAIL, 1);
      else count_add(a.counters, CNT_NEWTON_ITERS, (unsigned long long)it);
      count_hist(a.counters, it);
    } else {
      // the network's multipliers as they are
      double G[NLAM];
      expo_pass<L, C, false>(lam, (double)u[0], (double)u[1], (double)T, G, nullptr, e);
    }
    C feq[Q], geq[Q];
    const C kg = ((C)2 * (C)a.ph.Cv - (C)L::D) * T;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      feq[i] = rhop * e[i];
      geq[i] = kg * feq[i];
    }
    C f[Q], g[Q];
    pull(f, g);
    C te = (C)a.ph.tau;
    if (a.ph.sensor_on) te *= sensor_alpha<L, C>(f, feq, te, (C)a.ph.sensor_A);
    const C om = (C)1 / te;
    S *fout = (S *)a.fout;
    S *gout = (S *)a.gout;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      Sto<S>::stn(fout, pix<Q>(i, c), f[i] - om * (f[i] - feq[i]), L::S.w[i]);
      Sto<S>::stn(gout, pix<Q>(i, c), g[i] - om * (g[i] - geq[i]), 0.0);
    }
  } else if (valid) {
    // fine ghosts and boundary layers: streamed, not collided
    C f[Q], g[Q];
    pull(f, g);
    S *fout = (S *)a.fout;
    S *gout = (S *)a.gout;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      Sto<S>::stn(fout, pix<Q>(i, c), f[i], L::S.w[i]);
      Sto<S>::stn(gout, pix<Q>(i, c), g[i], 0.0);
    }
  }
}

template <int COLL, class S>
struct LaunchMlp {
  static void collide(const KArgs &a, bool pre, hipStream_t s) {
    if (a.count <= 0) return;
    if (pre) hipLaunchKernelGGL((k_collide_mlp<COLL, S, true>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_collide_mlp<COLL, S, false>), dim3(nblocks(a.count)), dim3(BLOCK), 0, s, a);
  }
  static Ops ops() {
    Ops o = Launch<L21, COLL_DDF_NEWTON, S>::ops();
    o.collide = &collide;
    return o;
  }
};

bool get_ops_d2q21(int coll, int storage, Ops *out) {
  // weakly compressible: BGK / recursive regularisation on the full
  // third-order Hermite basis
  if (coll == COLL_BGK || coll == COLL_RR) {
    const bool rr = coll == COLL_RR;
    if (storage == STO_FP64) { *out = rr ? Launch<L21, COLL_RR, double>::ops() : Launch<L21, COLL_BGK, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = rr ? Launch<L21, COLL_RR, float>::ops() : Launch<L21, COLL_BGK, float>::ops(); return true; }
    if (storage == STO_FP16) { *out = rr ? Launch<L21, COLL_RR, __half>::ops() : Launch<L21, COLL_BGK, __half>::ops(); return true; }
    return false;
  }
  if (storage != STO_FP64 && storage != STO_FP32) return false;
  const bool f64 = storage == STO_FP64;
  switch (coll) {
    case COLL_DDF_NEWTON:
      *out = f64 ? Launch<L21, COLL_DDF_NEWTON, double>::ops() : Launch<L21, COLL_DDF_NEWTON, float>::ops();
      return true;
    case COLL_DDF_MLP:
      *out = f64 ? LaunchMlp<COLL_DDF_MLP, double>::ops() : LaunchMlp<COLL_DDF_MLP, float>::ops();
      return true;
    case COLL_DDF_MLP_NEWTON:
      *out = f64 ? LaunchMlp<COLL_DDF_MLP_NEWTON, double>::ops() : LaunchMlp<COLL_DDF_MLP_NEWTON, float>::ops();
      return true;
    default:
      return false;
  }
}
}  // namespace lbm
