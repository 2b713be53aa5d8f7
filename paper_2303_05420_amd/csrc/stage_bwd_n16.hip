// Adjoint stage kernels, tile side 16.
#include "stage_bwd.h"

namespace nk {

int launch_stage_bwd_16(const StageBwdArgs& a, bool seed, hipStream_t s) {
  return seed ? launch_bwd_seed<16>(a, s) : launch_bwd_inner<16>(a, s);
}

}  // namespace nk
