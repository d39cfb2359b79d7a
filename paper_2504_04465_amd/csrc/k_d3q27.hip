// Kernel instantiations for D3Q27: BGK and recursive regularisation, FP64 /
// FP32 / FP16 (f - w) storage.
#include "kernels.cuh"

namespace lbm {
using L27 = Lattice<LAT_D3Q27>;

bool get_ops_d3q27(int coll, int storage, Ops *out) {
  if (coll == COLL_BGK) {
    if (storage == STO_FP64) { *out = Launch<L27, COLL_BGK, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L27, COLL_BGK, float>::ops(); return true; }
    if (storage == STO_FP16) { *out = Launch<L27, COLL_BGK, __half>::ops(); return true; }
  }
  if (coll == COLL_RR) {
    if (storage == STO_FP64) { *out = Launch<L27, COLL_RR, double>::ops(); return true; }
    if (storage == STO_FP32) { *out = Launch<L27, COLL_RR, float>::ops(); return true; }
    if (storage == STO_FP16) { *out = Launch<L27, COLL_RR, __half>::ops(); return true; }
  }
  return false;
}
}  // namespace lbm
