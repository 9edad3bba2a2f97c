// Instantiation of the block two-pass apply for double complex vectors.
#include "block_impl.h"

namespace hub {

hipError_t launch_block_c128(const ApplyLaunch& L, int* pgrid) { return dev::block_nv<double>(L, pgrid); }

}  // namespace hub
