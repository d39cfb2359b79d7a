// Kernel instantiations for D2Q13: double distribution with the numerical
// (entropy-maximising) equilibrium solved by Newton on the eight constraints
// (App. A.2), FP64 / FP32 storage.  The paper takes this lattice for the
// transonic runs (Mach up to about one).
#include "kernels.cuh"

namespace lbm {
using L13 = Lattice<LAT_D2Q13>;

bool get_ops_d2q13(int coll, int storage, Ops *out) {
  if (coll != COLL_DDF_NEWTON) return false;
  if (storage == STO_FP64) { *out = Launch<L13, COLL_DDF_NEWTON, double>::ops(); return true; }
  if (storage == STO_FP32) { *out = Launch<L13, COLL_DDF_NEWTON, float>::ops(); return true; }
  return false;
}
}  // namespace lbm
