// Kernel instantiation for D2Q37 with the Newton numerical equilibrium, FP32
// population storage (dispatched from k_d2q37.hip).
#include "kernels.cuh"

namespace lbm {
Ops ops_d2q37_newton_fp32() { return Launch<Lattice<LAT_D2Q37>, COLL_DDF_NEWTON, float>::ops(); }
}  // namespace lbm
