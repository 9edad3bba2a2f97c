// Instantiation of the matrix-free apply for double complex vectors.
#include "apply_impl.h"

namespace hub {

hipError_t launch_apply_c128(const ApplyLaunch& L, int grid, size_t lds, int* pgrid) {
  return dev::apply_nv<double>(L, grid, lds, pgrid);
}

}  // namespace hub
