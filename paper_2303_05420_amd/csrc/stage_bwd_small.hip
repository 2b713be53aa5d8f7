// Adjoint stage kernels, tile sides 2, 4 and 8.
#include "stage_bwd.h"

namespace nk {

int launch_stage_bwd_small(int N, const StageBwdArgs& a, bool seed, hipStream_t s) {
  switch (N) {
    case 2: return seed ? launch_bwd_seed<2>(a, s) : launch_bwd_inner<2>(a, s);
    case 4: return seed ? launch_bwd_seed<4>(a, s) : launch_bwd_inner<4>(a, s);
    case 8: return seed ? launch_bwd_seed<8>(a, s) : launch_bwd_inner<8>(a, s);
  }
  return -2;
}

}  // namespace nk
