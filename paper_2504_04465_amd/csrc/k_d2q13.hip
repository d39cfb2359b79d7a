// Kernel instantiations for D2Q13: BGK and recursive regularisation on the
// full third-order Hermite basis (FP64 / FP32 / FP16 storage), and the
// double distribution with the numerical (entropy-maximising) equilibrium
// solved by Newton on the eight constraints (App. A.2, FP64 / FP32).  The
// paper runs this lattice weakly compressible with RR and, with the
// numerical equilibrium, at Mach numbers up to about one.
#include "kernels.cuh"

namespace lbm {
using L13 = Lattice<LAT_D2Q13>;

bool get_ops_d2q13(int coll, int storage, Ops *out) {
  if (coll == COLL_BGK) {
    if (storage == STO_FP64) { *out = Launch<L13, COLL_BGK, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L13, COLL_BGK, float>::ops(); return true; }
    if (storage == STO_FP16) { *out = Launch<L13, COLL_BGK, __half>::ops(); return true; }
  }
  if (coll == COLL_RR) {
    if (storage == STO_FP64) { *out = Launch<L13, COLL_RR, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L13, COLL_RR, float>::ops(); return true; }
    if (storage == STO_FP16) { *out = Launch<L13, COLL_RR, __half>::ops(); return true; }
  }
  if (coll == COLL_DDF_NEWTON) {
    if (storage == STO_FP64) { *out = Launch<L13, COLL_DDF_NEWTON, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L13, COLL_DDF_NEWTON, float>::ops(); return true; }
  }
  return false;
}
}  // namespace lbm
