// Shared device/host definitions of libnk (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// ReLU arc-cosine map, normalised: J1(rho) = (sin t + (pi - t) rho) / pi with
// cos t = rho, written as J1 = rho + u^{3/2} H(u), u = 1 - rho.  H is our own
// degree-4 weighted-minimax polynomial fit on [0, 1] (gen_relu_poly.py; max
// relative error of J1 1.3e-7 in exact arithmetic, about two float32
// roundings).  Then
//   E[relu(a) relu(b)] = sqrt(q q') / 2 * J1(s / sqrt(q q'))
// for (a, b) ~ N(0, [[q, s], [s, q']]).
#define NK_J1_C0 0.30011793971061707f
#define NK_J1_C1 0.014882231131196022f
#define NK_J1_C2 0.0028328807093203068f
#define NK_J1_C3 -7.56633744458668e-05f
#define NK_J1_C4 0.0005524527514353395f

// The same form with a degree-3 fit of H (gen_relu_poly.py; max relative
// error of J1 1.3e-6 in exact arithmetic), one FMA less per entry-layer.
// Used by the forward NNGP kernels only: over the 9 ReLU layers of Myrtle-10
// it keeps the normalised kernel error near 2e-6, but the adjoint and the
// tangent kernel differentiate the map, which amplifies the fit error, so
// they keep the degree-4 fit.
#define NK_J1D3_C0 0.3000355064868927f
#define NK_J1D3_C1 0.015479165129363537f
#define NK_J1D3_C2 0.0013594607589766383f
#define NK_J1D3_C3 0.001435322454199195f

// acos(1 - u) = sqrt(u) G(u) with G analytic on [0, 1]; G is our own fit
// (gen_relu_poly.py).  Degree 5 (absolute error of sqrt(u) G(u) / pi
// 2.0e-7): the adjoint.
#define NK_ACOSD5_C0 1.414205551147461f
#define NK_ACOSD5_C1 0.11805802583694458f
#define NK_ACOSD5_C2 0.024997970089316368f
#define NK_ACOSD5_C3 0.012558783404529095f
#define NK_ACOSD5_C4 -0.003935873042792082f
#define NK_ACOSD5_C5 0.00491119921207428f
// degree-4 fit of G (absolute error of sqrt(u) G(u) / pi 1.5e-6): the
// tangent kernel's forward pass
#define NK_ACOSD4_C0 1.4142640829086304f
#define NK_ACOSD4_C1 0.11692662537097931f
#define NK_ACOSD4_C2 0.031181575730443f
#define NK_ACOSD4_C3 -0.0013137111673131585f
#define NK_ACOSD4_C4 0.009732994250953197f

#define NK_MAX_STAGES 4
#define NK_MAX_DEPTH 4
#define NK_MAX_C 16

namespace nk {

// Network as the kernels see it (square images, 3x3 filters).
struct NetDesc {
  int hw;                    // input resolution (H == W)
  int C;                     // input channels
  int S;                     // stages
  int depth[NK_MAX_STAGES];  // conv+ReLU blocks per stage
  float sw2, sb2;
};

__host__ __device__ inline int stage_res(const NetDesc& n, int s) { return n.hw >> s; }

// float2 (alpha, beta) entries per image in the variance tables.
__host__ __device__ inline int table_len(const NetDesc& n) {
  int t = 0;
  for (int s = 0; s < n.S; ++s) t += n.depth[s] * stage_res(n, s) * stage_res(n, s);
  return t;
}
__host__ __device__ inline int table_off(const NetDesc& n, int stage) {
  int t = 0;
  for (int s = 0; s < stage; ++s) t += n.depth[s] * stage_res(n, s) * stage_res(n, s);
  return t;
}

// Pair index -> (a, b) for a block of n1 x n2 (or the upper triangle of
// n x n when sym), enumerated in T x T image tiles so that consecutive pairs
// share images.  Tile rows in order, tiles left to right, row-major inside.
__host__ __device__ inline void pair_of(int64_t p, int64_t n1, int64_t n2, int sym, int T, int64_t* a,
                                        int64_t* b) {
  if (!sym) {
    int64_t ta = p / ((int64_t)T * n2);
    int64_t rem = p - ta * (int64_t)T * n2;
    int64_t h = n1 - ta * T;
    if (h > T) h = T;
    int64_t tb = rem / (h * T);
    int64_t rem2 = rem - tb * h * T;
    int64_t w = n2 - tb * T;
    if (w > T) w = T;
    *a = ta * T + rem2 / w;
    *b = tb * T + rem2 % w;
    return;
  }
  int64_t n = n1;
  int64_t NT = (n + T - 1) / T;
  // C(t): pairs before tile row t (all earlier rows are full): t T(T+1)/2 + T (t n - T t (t+1)/2)
  int64_t lo = 0, hi = NT - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    int64_t c = mid * (int64_t)T * (T + 1) / 2 + (int64_t)T * (mid * n - (int64_t)T * mid * (mid + 1) / 2);
    if (c <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  int64_t ta = lo;
  int64_t rem = p - (ta * (int64_t)T * (T + 1) / 2 + (int64_t)T * (ta * n - (int64_t)T * ta * (ta + 1) / 2));
  int64_t r = n - ta * T;
  if (r > T) r = T;
  int64_t ndiag = r * (r + 1) / 2;
  if (rem < ndiag) {
    // upper triangle of the diagonal tile, row-major
    int64_t al = 0;
    while (rem >= r - al) {
      rem -= r - al;
      ++al;
    }
    *a = ta * T + al;
    *b = ta * T + al + rem;
    return;
  }
  rem -= ndiag;
  int64_t tb = ta + 1 + rem / (r * T);
  int64_t rem3 = rem - (tb - ta - 1) * r * T;
  int64_t w = n - tb * T;
  if (w > T) w = T;
  *a = ta * T + rem3 / w;
  *b = tb * T + rem3 % w;
}

__host__ __device__ inline int64_t pair_count(int64_t n1, int64_t n2, int sym) {
  return sym ? n1 * (n1 + 1) / 2 : n1 * n2;
}

// Value of lane - 1 / lane + 1 across the whole wave (0 past the ends).
__device__ __forceinline__ float lane_prev(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, true));
}

// A zero the compiler cannot see through: added to an LDS index inside a
// loop it keeps loads of loop-invariant addresses inside the loop (otherwise
// they are hoisted and pin one register per value for the whole loop).
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

__device__ __forceinline__ float relu_poly(float u) {
  float p = NK_J1_C4;
  p = __builtin_fmaf(p, u, NK_J1_C3);
  p = __builtin_fmaf(p, u, NK_J1_C2);
  p = __builtin_fmaf(p, u, NK_J1_C1);
  p = __builtin_fmaf(p, u, NK_J1_C0);
  return p;
}

__device__ __forceinline__ float relu_poly3(float u) {
  float p = NK_J1D3_C3;
  p = __builtin_fmaf(p, u, NK_J1D3_C2);
  p = __builtin_fmaf(p, u, NK_J1D3_C1);
  p = __builtin_fmaf(p, u, NK_J1D3_C0);
  return p;
}

// j1_nonneg and j1_signed_vr (below) with the degree-3 fit (forward NNGP).
__device__ __forceinline__ float j1_nonneg3(float rho) {
  float u = __builtin_amdgcn_fmed3f(1.0f - rho, 0.0f, 1.0f);
  float sq = __builtin_amdgcn_sqrtf(u);
  return __builtin_fmaf(-u, __builtin_fmaf(-sq, relu_poly3(u), 1.0f), 1.0f);
}
__device__ __forceinline__ float j1_signed_vr3(float v, float rr) {
  const float u = __builtin_amdgcn_fmed3f(__builtin_fmaf(-__builtin_fabsf(v), rr, 1.0f), 0.0f, 1.0f);
  const float c = __builtin_amdgcn_fmed3f(__builtin_fmaf(v, rr, 1.0f), 0.0f, 1.0f);
  const float sq = __builtin_amdgcn_sqrtf(u);
  return __builtin_fmaf(-u, __builtin_fmaf(-sq, relu_poly3(u), 1.0f), c);
}

// J1 for rho >= 0 (every ReLU after the first: inputs are sums of
// non-negative terms), as 1 - u (1 - sqrt(u) H(u)) with u = 1 - rho clamped to
// [0, 1] (two FMAs after the polynomial; rho > 1 from rounding gives J1(1) = 1).
__device__ __forceinline__ float j1_nonneg(float rho) {
  float u = __builtin_amdgcn_fmed3f(1.0f - rho, 0.0f, 1.0f);
  float sq = __builtin_amdgcn_sqrtf(u);
  return __builtin_fmaf(-u, __builtin_fmaf(-sq, relu_poly(u), 1.0f), 1.0f);
}

// J1 of rho = v rr for rho in [-1, 1] (rr > 0): J1(rho) = J1(|rho|) - |rho|
// for rho < 0, i.e. 1 - u (1 - sqrt(u) H(u)) + min(rho, 0) with u = 1 - |rho|;
// both u and 1 + min(rho, 0) = clamp(1 + rho) come out of one clamped FMA each.
__device__ __forceinline__ float j1_signed_vr(float v, float rr) {
  const float u = __builtin_amdgcn_fmed3f(__builtin_fmaf(-__builtin_fabsf(v), rr, 1.0f), 0.0f, 1.0f);
  const float c = __builtin_amdgcn_fmed3f(__builtin_fmaf(v, rr, 1.0f), 0.0f, 1.0f);
  const float sq = __builtin_amdgcn_sqrtf(u);
  return __builtin_fmaf(-u, __builtin_fmaf(-sq, relu_poly(u), 1.0f), c);
}

// J1 for rho in [-1, 1]: J1(rho) = J1(|rho|) - |rho| for rho < 0.
__device__ __forceinline__ float j1_signed(float rho) {
  float u = __builtin_amdgcn_fmed3f(1.0f - __builtin_fabsf(rho), 0.0f, 1.0f);
  float sq = __builtin_amdgcn_sqrtf(u);
  return __builtin_fmaf(u * sq, relu_poly(u), __builtin_fmaxf(rho, 0.0f));
}

// acos(1 - u) / pi = sqrt(u) G(u) / pi with the degree-5 fit of G (the
// adjoint), 1/pi folded into its coefficients.
__device__ __forceinline__ float acos_g_pi5(float u) {
  constexpr float ip = 0.31830988618379067f;
  float p = NK_ACOSD5_C5 * ip;
  p = __builtin_fmaf(p, u, NK_ACOSD5_C4 * ip);
  p = __builtin_fmaf(p, u, NK_ACOSD5_C3 * ip);
  p = __builtin_fmaf(p, u, NK_ACOSD5_C2 * ip);
  p = __builtin_fmaf(p, u, NK_ACOSD5_C1 * ip);
  p = __builtin_fmaf(p, u, NK_ACOSD5_C0 * ip);
  return p;
}

// The same with the degree-4 fit (the tangent kernel's forward pass).
__device__ __forceinline__ float acos_g_pi4(float u) {
  constexpr float ip = 0.31830988618379067f;
  float p = NK_ACOSD4_C4 * ip;
  p = __builtin_fmaf(p, u, NK_ACOSD4_C3 * ip);
  p = __builtin_fmaf(p, u, NK_ACOSD4_C2 * ip);
  p = __builtin_fmaf(p, u, NK_ACOSD4_C1 * ip);
  p = __builtin_fmaf(p, u, NK_ACOSD4_C0 * ip);
  return p;
}

// Logical workgroup index with consecutive indices on the same XCD: the
// dispatcher deals workgroups round-robin over the 8 XCDs, so remap so that
// each XCD walks one contiguous range of the pair order (shared images stay
// in that XCD's L2).
__device__ __forceinline__ int64_t xcd_logical_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t x = b & 7, q = nb >> 3, r = nb & 7;
  const int64_t start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return start + (b >> 3);
}

}  // namespace nk
