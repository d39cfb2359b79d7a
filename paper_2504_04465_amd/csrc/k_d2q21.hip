// Kernel instantiations for D2Q21: double distribution with the numerical
// (entropy-maximising) equilibrium solved by Newton, FP64 / FP32 storage.
#include "kernels.cuh"

namespace lbm {
using L21 = Lattice<LAT_D2Q21>;

bool get_ops_d2q21(int coll, int storage, Ops *out) {
  if (coll != COLL_DDF_NEWTON) return false;
  if (storage == STO_FP64) { *out = Launch<L21, COLL_DDF_NEWTON, double>::ops(); return true; }
  if (storage == STO_FP32) { *out = Launch<L21, COLL_DDF_NEWTON, float>::ops(); return true; }
  return false;
}
}  // namespace lbm
