// Device building blocks shared by the forward and adjoint stage kernels:
// the sheared N x N tile of displacement classes (see stage.hip) with one
// segment of N lanes per tile, lane = column, register = row.
#pragma once
#include "nk_kernels.h"

namespace nk {

template <int N>
struct KCfg {
  static constexpr int THREADS = (N * N > 256) ? N * N : 256;
  static constexpr int PPWG = THREADS / (N * N);
};

// LDS per pair: [tables x1: D N^2 float2][tables x2, rows twice: 2 D N^2 float2]
// [pooling row / readout partials][images as float4 (seeding stage only):
// x1, then x2 with its rows twice]
template <int N>
__host__ __device__ inline size_t slot_lds_bytes(int D, bool pool, bool seed) {
  size_t t = (size_t)D * N * N * 8 + (size_t)D * 2 * N * N * 8 + (seed ? (size_t)3 * N * N * 16 : 0);
  size_t r = pool ? (size_t)N * N * N / 8 * 4 : (size_t)N * N * 8;
  if (r < 16) r = 16;
  return (t + r + 15) & ~(size_t)15;
}

// Masked 3-tap sum along the lanes of a segment,
//   x + x(lane - 1) mL + x(lane + 1) mR   (0 past the ends of the wave),
// with each lane shift fused into its FMA as a DPP source operand (the
// compiler keeps DPP moves separate from FMAs).  The s_nop gives the two
// wait states a DPP source needs after a VALU write to it.
__device__ __forceinline__ float hsum3(float x, float mL, float mR) {
  float h;
  asm("v_mov_b32 %0, %1\n\t"
      "s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %0, %1, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=&v"(h)
      : "v"(x), "v"(mL), "v"(mR));
  return h;
}

// wave-uniform 0/1 factor (kept in a scalar register)
__device__ __forceinline__ float uniform_mask(bool zero) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, zero ? 0.f : 1.f)));
}

// One [3x3 conv, ReLU] layer on a tile held as A[r] (row r, this lane's column).
template <int N, bool SIGNED, bool BIAS>
__device__ __forceinline__ void tile_layer(float (&A)[N], const float2* __restrict__ c1,
                                           const float2* __restrict__ c2, int seam, float mL, float mR,
                                           float sb2) {
  float hm = 0.f;
  float h0 = hsum3(A[0], mL, mR);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    float hp = 0.f;
    if (r + 1 < N) hp = hsum3(A[r + 1], mL, mR);
    float v = h0;
    if (r > 0) v = __builtin_fmaf(uniform_mask(r == seam), hm, v);
    if (r + 1 < N) v = __builtin_fmaf(uniform_mask(r + 1 == seam), hp, v);
    if (BIAS) v += sb2;
    const float2 a = c1[r * N];
    const float2 b = c2[r * N];
    const float rr = a.x * b.x;
    const float J = SIGNED ? j1_signed_vr(v, rr) : j1_nonneg(v * rr);
    A[r] = (a.y * b.y) * J;
    hm = h0;
    h0 = hp;
  }
}

// In-place masked 3x3 box sum of a tile (the conv's linear part; it is its
// own adjoint, the masks being symmetric).
template <int N>
__device__ __forceinline__ void tile_box(float (&G)[N], int seam, float mL, float mR) {
  float hm = 0.f;
  float h0 = hsum3(G[0], mL, mR);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    float hp = 0.f;
    if (r + 1 < N) hp = hsum3(G[r + 1], mL, mR);
    float v = h0;
    if (r > 0) v = __builtin_fmaf(uniform_mask(r == seam), hm, v);
    if (r + 1 < N) v = __builtin_fmaf(uniform_mask(r + 1 == seam), hp, v);
    G[r] = v;
    hm = h0;
    h0 = hp;
  }
}

}  // namespace nk
