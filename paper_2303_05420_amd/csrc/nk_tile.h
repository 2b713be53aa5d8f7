// Device building blocks shared by the forward and adjoint stage kernels:
// the sheared N x N tile of displacement classes (see stage.hip) with one
// segment of N lanes per tile, lane = column, register = row.
#pragma once
#include "nk_kernels.h"

namespace nk {

// Workgroup shape of the forward stage kernel.  A segment of N lanes owns
// CPS tile columns; the 32x32 tangent kernel (two tiles per column plus
// their pooling rows) takes two columns per segment on half the lanes, so
// that each wave has twice the registers.  PPM multiplies the pairs of one
// workgroup (tiles of at most 16 x 16: 256 or 512 threads); the arithmetic
// of a pair does not depend on it.
template <int N, bool NTK = false, int PPM = 1>
struct KCfg {
  static_assert(PPM == 1 || (PPM == 2 && N <= 16), "pairs multiplier 2 only for tiles of at most 16 x 16");
  static constexpr int CPS = (NTK && N == 32) ? 2 : 1;  // tile columns per segment
  static constexpr int LPP = N * N / CPS;                // lanes per pair
  static constexpr int THREADS = (LPP > 256 ? LPP : 256) * PPM;
  static constexpr int PPWG = THREADS / LPP;
};

// LDS bytes of one carried quantity's pooling row (or readout partials).
template <int N>
__host__ __device__ constexpr size_t red_bytes_q(bool pool) {
  return pool ? (size_t)N * N * N / 8 * 4 : (size_t)N * N * 8;
}

// LDS per pair: [tables x1: D N^2 float2][tables x2, rows twice: 2 D N^2 float2]
// [pooling row / readout partials, per carried quantity][images as float4
// (seeding stage only): x1, then x2 with its rows twice]
template <int N>
__host__ __device__ inline size_t slot_lds_bytes(int D, bool pool, bool seed, bool ntk = false) {
  size_t t = (size_t)D * N * N * 8 + (size_t)D * 2 * N * N * 8 + (seed ? (size_t)3 * N * N * 16 : 0);
  size_t r = red_bytes_q<N>(pool) * (ntk ? 2 : 1);
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

// Settles the candidates (same == 2) of the PPWG slots: a pair of two
// arrays holding the same image element for element counts as identical
// (same = 1), because then its displacement-0 correlation is 1 exactly at
// every layer, as on the diagonal of a symmetric block.  Every thread of the
// workgroup calls this (the loop condition is uniform).
template <int PPWG, int THREADS>
__device__ inline void identical_pairs(int* same, const float* const* x1, const float* const* x2,
                                       int64_t nfl) {
  for (int s = 0; s < PPWG; ++s) {
    if (same[s] != 2) continue;
    int eq = 1;
    for (int64_t e = threadIdx.x; e < nfl; e += THREADS) eq &= (x1[s][e] == x2[s][e]) ? 1 : 0;
    eq = __syncthreads_and(eq);
    if (threadIdx.x == 0) same[s] = eq ? 1 : 0;
  }
  __syncthreads();
}

// wave-uniform 0/1 factor (kept in a scalar register)
__device__ __forceinline__ float uniform_mask(bool zero) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, zero ? 0.f : 1.f)));
}

// One [3x3 conv, ReLU] layer on a tile held as A[r] (row r, this lane's
// column), forward NNGP (the map with the degree-3 fit).
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
    const float J = SIGNED ? j1_signed_vr3(v, rr) : j1_nonneg3(v * rr);
    A[r] = (a.y * b.y) * J;
    hm = h0;
    h0 = hp;
  }
}

// One layer of the tangent kernel on the tile pair (A, C): A as tile_layer
// (kappa F), C = kappa (F + Fdot T) with T = box(C) + sigma_b2, or T = S on
// the network's first layer (SIGNED), whose C input is not read.
// kh = kappa / 2 of this layer; kappa Fdot = kh (1 - acos(rho) / pi), and
// kh acos(|rho|) / pi for rho < 0.  acos has an infinite slope at rho = 1, so
// the rounding of rho (about 1e-7) would move Fdot by about 1e-4 where rho
// is 1 exactly: on the displacement-0 tile of a pair of identical images
// (i = j) the caller passes umax = 0, which pins u = 1 - rho to 0 there
// (umax = 1 elsewhere: the plain clamp).  J1 uses the degree-3 fit of H (as
// the NNGP stages) and acos the degree-4 fit of G (absolute error 1.5e-6 of
// acos(rho) / pi); the adjoint, which differentiates the map, keeps the
// degree-4 fit of H and a degree-5 fit of G.
template <int N, bool SIGNED, bool BIAS>
__device__ __forceinline__ void tile_layer_ntk(float (&A)[N], float (&C)[N], const float2* __restrict__ c1,
                                               const float2* __restrict__ c2, int seam, float mL, float mR,
                                               float sb2, float kh, float umax) {
  float hm = 0.f;
  float h0 = hsum3(A[0], mL, mR);
  float gm = 0.f;
  float g0 = SIGNED ? 0.f : hsum3(C[0], mL, mR);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    float hp = 0.f, gp = 0.f;
    if (r + 1 < N) {
      hp = hsum3(A[r + 1], mL, mR);
      if (!SIGNED) gp = hsum3(C[r + 1], mL, mR);
    }
    const float mu = uniform_mask(r == seam), md = uniform_mask(r + 1 == seam);
    float v = h0;
    if (r > 0) v = __builtin_fmaf(mu, hm, v);
    if (r + 1 < N) v = __builtin_fmaf(md, hp, v);
    if (BIAS) v += sb2;
    float vt = v;
    if (!SIGNED) {
      vt = g0;
      if (r > 0) vt = __builtin_fmaf(mu, gm, vt);
      if (r + 1 < N) vt = __builtin_fmaf(md, gp, vt);
      if (BIAS) vt += sb2;
    }
    const float2 a = c1[r * N];
    const float2 b = c2[r * N];
    const float rr = a.x * b.x;
    float J, th;
    if (SIGNED) {
      const float u = __builtin_amdgcn_fmed3f(__builtin_fmaf(-__builtin_fabsf(v), rr, 1.0f), 0.0f, umax);
      const float cc = __builtin_amdgcn_fmed3f(__builtin_fmaf(v, rr, 1.0f), 0.0f, 1.0f);
      const float sq = __builtin_amdgcn_sqrtf(u);
      J = __builtin_fmaf(-u, __builtin_fmaf(-sq, relu_poly3(u), 1.0f), cc);
      th = sq * acos_g_pi4(u);
    } else {
      const float u = __builtin_amdgcn_fmed3f(__builtin_fmaf(-v, rr, 1.0f), 0.0f, umax);
      const float sq = __builtin_amdgcn_sqrtf(u);
      J = __builtin_fmaf(-u, __builtin_fmaf(-sq, relu_poly3(u), 1.0f), 1.0f);
      th = sq * acos_g_pi4(u);
    }
    const float kfd = (SIGNED && v < 0.f) ? kh * th : __builtin_fmaf(-th, kh, kh);
    const float an = (a.y * b.y) * J;
    A[r] = an;
    C[r] = __builtin_fmaf(kfd, vt, an);
    hm = h0;
    h0 = hp;
    gm = g0;
    g0 = gp;
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
