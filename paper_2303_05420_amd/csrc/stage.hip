// NNGP instantiations of the fused stage kernel (stage_kernel.h) and the
// host-side launch helpers shared by the one-block and batched passes.
#include "stage_kernel.h"

namespace nk {

// Resident workgroups per CU of a stage kernel (and sets its LDS attribute,
// so that a later launch makes no attribute call, e.g. under graph capture).
// ppm: pairs-per-workgroup multiplier of tiles of at most 16 x 16 (1 or 2;
// ignored above).
int stage_occupancy(int N, int D, bool seed, bool pool, bool bias, int C, int ppm) {
  if (N == 32 && pool) return stage32_occupancy(D, seed, bias, C);
  if (ppm == 2) {
    switch (N) {
      case 2: return occ_n<2, false, 2>(D, seed, pool, bias);
      case 4: return occ_n<4, false, 2>(D, seed, pool, bias);
      case 8: return occ_n<8, false, 2>(D, seed, pool, bias);
      case 16: return occ_n<16, false, 2>(D, seed, pool, bias);
    }
  }
  switch (N) {
    case 2: return occ_n<2, false>(D, seed, pool, bias);
    case 4: return occ_n<4, false>(D, seed, pool, bias);
    case 8: return occ_n<8, false>(D, seed, pool, bias);
    case 16: return occ_n<16, false>(D, seed, pool, bias);
    case 32: return occ_n<32, false>(D, seed, pool, bias);
  }
  return -2;
}

int prime_stage(int N, int D, bool seed, bool pool, bool bias, int C, int ppm) {
  const int r = stage_occupancy(N, D, seed, pool, bias, C, ppm);
  return r < 0 ? r : 0;
}

int stage_pairs_per_wg(int N, bool pool, int ppm) {
  if (N == 32 && pool) return 1;
  const int lpp = N * N;
  return (lpp >= 256 ? 1 : 256 / lpp) * (N <= 16 && ppm == 2 ? 2 : 1);
}

// Tile table of a batched pass -> device memory through kernel arguments
// (32 descriptors per launch): the arguments are copied at launch, so the
// host array may go away at once, and the launches can be captured.
struct TileBatch {
  int n, pad;
  TileDesc d[32];
};

__global__ void put_tiles_kernel(const TileBatch b, TileDesc* __restrict__ dst) {
  if ((int)threadIdx.x < b.n) dst[threadIdx.x] = b.d[threadIdx.x];
}

int launch_put_tiles(const TileDesc* host, int n, TileDesc* dst, hipStream_t stream) {
  for (int i = 0; i < n; i += 32) {
    TileBatch b;
    b.n = n - i < 32 ? n - i : 32;
    b.pad = 0;
    for (int k = 0; k < b.n; ++k) b.d[k] = host[i + k];
    hipLaunchKernelGGL(put_tiles_kernel, dim3(1), dim3(32), 0, stream, b, dst + i);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  return 0;
}

size_t stage_lds_bytes(int N, int D, bool pool, bool seed) {
  if (N == 32 && pool) return stage32_lds_bytes(D, seed);
  switch (N) {
    case 2: return KCfg<2>::PPWG * slot_lds_bytes<2>(D, pool, seed);
    case 4: return KCfg<4>::PPWG * slot_lds_bytes<4>(D, pool, seed);
    case 8: return KCfg<8>::PPWG * slot_lds_bytes<8>(D, pool, seed);
    case 16: return KCfg<16>::PPWG * slot_lds_bytes<16>(D, pool, seed);
    case 32: return KCfg<32>::PPWG * slot_lds_bytes<32>(D, pool, seed);
  }
  return 0;
}

int launch_stage(int N, const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s, int ppm) {
  // 32x32 pooling stages: two tile columns per lane (stage32.hip)
  if (N == 32 && pool) return launch_stage32(a, seed, bias, s);
  if (ppm == 2) {
    switch (N) {
      case 2: return launch_n<2, false, 2>(a, seed, pool, bias, s);
      case 4: return launch_n<4, false, 2>(a, seed, pool, bias, s);
      case 8: return launch_n<8, false, 2>(a, seed, pool, bias, s);
      case 16: return launch_n<16, false, 2>(a, seed, pool, bias, s);
    }
  }
  switch (N) {
    case 2: return launch_n<2, false>(a, seed, pool, bias, s);
    case 4: return launch_n<4, false>(a, seed, pool, bias, s);
    case 8: return launch_n<8, false>(a, seed, pool, bias, s);
    case 16: return launch_n<16, false>(a, seed, pool, bias, s);
    case 32: return launch_n<32, false>(a, seed, pool, bias, s);
  }
  return -2;
}

}  // namespace nk
