// Kernel instantiations for D2Q37: double distribution with the fourth-order
// thermal polynomial equilibrium, or with the numerical equilibrium solved by
// Newton on the eight constraints (the paper's choice for its supersonic and
// shock-tube runs), FP64 / FP32 storage.
#include "kernels.cuh"

namespace lbm {
using L37 = Lattice<LAT_D2Q37>;

bool get_ops_d2q37(int coll, int storage, Ops *out) {
  if (coll == COLL_DDF_POLY) {
    if (storage == STO_FP64) { *out = Launch<L37, COLL_DDF_POLY, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L37, COLL_DDF_POLY, float>::ops(); return true; }
  }
  if (coll == COLL_DDF_NEWTON) {
    if (storage == STO_FP64) { *out = Launch<L37, COLL_DDF_NEWTON, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L37, COLL_DDF_NEWTON, float>::ops(); return true; }
  }
  return false;
}
}  // namespace lbm
