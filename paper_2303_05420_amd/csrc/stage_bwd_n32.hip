// Adjoint stage kernels, tile side 32 (the first stage of 32 x 32 images).
#include "stage_bwd.h"

namespace nk {

int launch_stage_bwd_32(const StageBwdArgs& a, bool seed, hipStream_t s) {
  if (!seed) return -2;  // a 32 x 32 tile is only ever the first stage (images are at most 32 x 32)
  return launch_bwd_seed<32>(a, s);
}

}  // namespace nk
