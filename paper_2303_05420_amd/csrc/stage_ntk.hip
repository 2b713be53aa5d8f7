// Tangent-kernel (NTK) instantiations of the fused stage kernel
// (stage_kernel.h): the stage carries the NNGP tile and the tangent tile.
#include "stage_kernel.h"

namespace nk {

size_t stage_ntk_lds_bytes(int N, int D, bool pool, bool seed) {
  switch (N) {
    case 2: return KCfg<2, true>::PPWG * slot_lds_bytes<2>(D, pool, seed, true);
    case 4: return KCfg<4, true>::PPWG * slot_lds_bytes<4>(D, pool, seed, true);
    case 8: return KCfg<8, true>::PPWG * slot_lds_bytes<8>(D, pool, seed, true);
    case 16: return KCfg<16, true>::PPWG * slot_lds_bytes<16>(D, pool, seed, true);
    case 32: return KCfg<32, true>::PPWG * slot_lds_bytes<32>(D, pool, seed, true);
  }
  return 0;
}

int launch_stage_ntk(int N, const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s) {
  switch (N) {
    case 2: return launch_n<2, true>(a, seed, pool, bias, s);
    case 4: return launch_n<4, true>(a, seed, pool, bias, s);
    case 8: return launch_n<8, true>(a, seed, pool, bias, s);
    case 16: return launch_n<16, true>(a, seed, pool, bias, s);
    case 32: return launch_n<32, true>(a, seed, pool, bias, s);
  }
  return -2;
}

}  // namespace nk
