// dg_trilinear.hip -- SWIPDG apply on trilinear elements (placeholder launchers).
#include "dg_internal.hpp"
#include "dg_kernels.hpp"

namespace dg {

hipError_t launch_apply_trilinear(int, int, int, int, const MeshArgs<double>&, const MeshArgs<float>&,
                                  const void*, void*, double*, unsigned*, double*, const int*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_diag_trilinear(int, const MeshArgs<double>&, double*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace dg
