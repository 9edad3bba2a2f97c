// Instantiation of the block two-pass apply for float complex vectors.
#include "block_impl.h"

namespace hub {

hipError_t launch_block_c64(const ApplyLaunch& L, int* pgrid) { return dev::block_nv<float>(L, pgrid); }

}  // namespace hub
