// Kernel instantiations for D2Q37: double distribution with the fourth-order
// thermal polynomial equilibrium here; the numerical equilibrium solved by
// Newton on the eight constraints (the paper's choice for its supersonic and
// shock-tube runs) is instantiated in k_d2q37_newton64.hip and
// k_d2q37_newton32.hip, one storage precision per translation unit, so that
// the two large Newton kernels compile in parallel.
#include "kernels.cuh"

namespace lbm {
using L37 = Lattice<LAT_D2Q37>;

Ops ops_d2q37_newton_fp64();
Ops ops_d2q37_newton_fp32();

bool get_ops_d2q37(int coll, int storage, Ops *out) {
  if (coll == COLL_DDF_POLY) {
    if (storage == STO_FP64) { *out = Launch<L37, COLL_DDF_POLY, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L37, COLL_DDF_POLY, float>::ops(); return true; }
  }
  if (coll == COLL_DDF_NEWTON) {
    if (storage == STO_FP64) { *out = ops_d2q37_newton_fp64(); return true; }
    if (storage == STO_FP32) { *out = ops_d2q37_newton_fp32(); return true; }
  }
  return false;
}
}  // namespace lbm
