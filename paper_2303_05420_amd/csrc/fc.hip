// FC NNGP block (App. A, FC listing: Flatten, depth x [Dense, ReLU], Dense).
//
//   K_1(x, x') = sigma_w2 x.x' / d + sigma_b2
//   K_{l+1}    = sigma_w2 F(K_l, K_l(x, x), K_l(x', x')) + sigma_b2
//   F(s, q, q') = sqrt(q q') / 2 J1(s / sqrt(q q'))
//
// The first layer's dot products are a dense (n1 x d) (d x n2) contraction:
// they run on the fp32 matrix cores (v_mfma_f32_16x16x4_f32), and the ReLU
// recursion is applied in the epilogue of the same kernel.  The diagonals
// follow K_{l+1}(x, x) = sigma_w2 K_l(x, x) / 2 + sigma_b2 (F(q, q, q) = q/2).
#include "nk_kernels.h"

namespace nk {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// first-layer diagonal sigma_w2 |x|^2 / d + sigma_b2, one wave per row
__global__ __launch_bounds__(256) void fc_diag_kernel(const float* __restrict__ x, int64_t n, int d, float sw2,
                                                      float sb2, float* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const float* p = x + row * (int64_t)d;
  double s = 0.0;
  for (int k = lane; k < d; k += 64) s += (double)p[k] * (double)p[k];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[row] = (float)((double)sw2 * s / d + (double)sb2);
}

__device__ __forceinline__ float4 load4_guard(const float* __restrict__ p, int64_t row, int64_t nrows, int d,
                                               int k, bool vec) {
  if (row >= nrows) return make_float4(0.f, 0.f, 0.f, 0.f);
  const float* q = p + row * (int64_t)d + k;
  if (vec && k + 3 < d) return *reinterpret_cast<const float4*>(q);
  float v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = (k + t < d) ? q[t] : 0.f;
  return make_float4(v[0], v[1], v[2], v[3]);
}

// 64 x 64 output tile per workgroup; each wave a 32 x 32 quadrant as 2 x 2
// blocks of 16 x 16 MFMA.  Lane l feeds A[i = l % 16][k-slot l / 16] and
// B[k-slot l / 16][j = l % 16]; each lane loads 4 consecutive k per k-slot
// (a float4) and issues 4 MFMAs, so one iteration covers 16 k.
__global__ __launch_bounds__(256) void fc_kernel(const FcArgs a) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.y * 64 + 32 * (w >> 1);
  const int64_t col0 = (int64_t)blockIdx.x * 64 + 32 * (w & 1);
  const int li = lane & 15, ks = lane >> 4;
  const bool vec = (a.d & 3) == 0;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < a.d; k0 += 16) {
    float4 av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i] = load4_guard(a.x1, row0 + 16 * i + li, a.n1, a.d, k0 + 4 * ks, vec);
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = load4_guard(a.x2, col0 + 16 * j + li, a.n2, a.d, k0 + 4 * ks, vec);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].x, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].y, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].z, bv[j].z, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].w, bv[j].w, acc[i][j], 0, 0, 0);
      }
  }
  const float inv_d = 1.0f / (float)a.d;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + 16 * i + 4 * ks + v;
        const int64_t c = col0 + 16 * j + li;
        if (r >= a.n1 || c >= a.n2) continue;
        float k = a.sw2 * acc[i][j][v] * inv_d + a.sb2;
        float q1 = a.d1[r], q2 = a.d2[c];
        for (int l = 0; l < a.depth; ++l) {
          const float qq = q1 * q2;
          float f = 0.f;
          if (qq > 0.f) {
            const float rs = __builtin_amdgcn_rsqf(qq);
            const float rho = k * rs;
            f = 0.5f * (qq * rs) * (l == 0 ? j1_signed(rho) : j1_nonneg(rho));
          }
          k = a.sw2 * f + a.sb2;
          q1 = 0.5f * a.sw2 * q1 + a.sb2;
          q2 = 0.5f * a.sw2 * q2 + a.sb2;
        }
        a.K[r * a.ldk + c] = k;
      }
}

int launch_fc(const FcArgs& a, float* d1, float* d2, hipStream_t stream) {
  hipLaunchKernelGGL(fc_diag_kernel, dim3((unsigned)((a.n1 + 3) / 4)), dim3(256), 0, stream, a.x1, a.n1, a.d, a.sw2,
                     a.sb2, d1);
  hipLaunchKernelGGL(fc_diag_kernel, dim3((unsigned)((a.n2 + 3) / 4)), dim3(256), 0, stream, a.x2, a.n2, a.d, a.sw2,
                     a.sb2, d2);
  FcArgs b = a;
  b.d1 = d1;
  b.d2 = d2;
  hipLaunchKernelGGL(fc_kernel, dim3((unsigned)((a.n2 + 63) / 64), (unsigned)((a.n1 + 63) / 64)), dim3(256), 0,
                     stream, b);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace nk
