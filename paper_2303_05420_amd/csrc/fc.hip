// FC NNGP block (App. A, FC listing: Flatten, depth x [Dense, ReLU], Dense).
//
//   K_1(x, x') = sigma_w2 x.x' / d + sigma_b2
//   K_{l+1}    = sigma_w2 F(K_l, K_l(x, x), K_l(x', x')) + sigma_b2
//   F(s, q, q') = sqrt(q q') / 2 J1(s / sqrt(q q'))
//
// The first layer's dot products are a dense (n1 x d) (d x n2) contraction:
// they run on the fp32 matrix cores (v_mfma_f32_16x16x4f32) from LDS tiles,
// and the ReLU recursion is applied in the epilogue of the same kernel.  The diagonals
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

// Tiling of the first-layer contraction.  A workgroup (4 waves) owns a
// 128 x 128 output tile, each wave a 64 x 64 quadrant as 4 x 4 blocks of
// 16 x 16 v_mfma_f32_16x16x4f32 accumulators (64 registers).  The k range
// runs in tiles of FC_BK = 32: the 128 rows of x1 and of x2 for the tile sit
// in LDS as [row][k] (row padded by 4 floats: 16-byte aligned rows, and the
// 16 rows a block reads start on different banks); the next tile is loaded
// into registers (4 + 4 float4 per thread) while the current one feeds the
// MFMAs, and written to LDS between two barriers.  For a block, lane l feeds
// A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16] of each 4-wide k step.
constexpr int FC_BM = 128, FC_BK = 32, FC_LDR = FC_BK + 4;
// Tile order.  Workgroups go to the 8 XCDs round-robin in launch order and
// each XCD has its own L2, so the launch index is first mapped to one
// contiguous range of tiles per XCD; each range walks the output in groups
// of FC_GROUP tile rows, column by column, so that the tiles an XCD runs at
// the same time share few x1 row tiles and x2 column tiles.  A symmetric
// block (x2 the same images as x1) runs only the tiles on and above the
// diagonal, in the pair order of the Myrtle stages over tile indices
// (groups of FC_GROUP), and each off-diagonal tile also writes its mirror.
constexpr int FC_GROUP = 8;

__global__ __launch_bounds__(256) void fc_kernel(const FcArgs a) {
  __shared__ __attribute__((aligned(16))) float As[FC_BM * FC_LDR];
  __shared__ __attribute__((aligned(16))) float Bs[FC_BM * FC_LDR];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int64_t r0, c0;
  bool mirror = false;
  {
    const int64_t gx = gridDim.x, gy = gridDim.y, nb = gx * gy;
    const int64_t lin = (int64_t)blockIdx.y * gx + blockIdx.x;
    const int64_t xcd = lin & 7, q = nb >> 3, rem = nb & 7;
    const int64_t id = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + (lin >> 3);
    if (a.sym) {
      const int64_t nt = (a.n1 + FC_BM - 1) / FC_BM;
      int64_t ti, tj;
      pair_of(id, nt, nt, 1, FC_GROUP, &ti, &tj);
      r0 = ti * FC_BM;
      c0 = tj * FC_BM;
      mirror = ti != tj;
    } else {
      const int64_t grp = id / (FC_GROUP * gx), first = grp * FC_GROUP;
      const int64_t rows = gy - first < FC_GROUP ? gy - first : FC_GROUP;
      const int64_t in = id - first * gx;
      r0 = (first + in % rows) * FC_BM;
      c0 = (in / rows) * FC_BM;
    }
  }
  const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
  const int li = lane & 15, ks = lane >> 4;
  const bool vec = (a.d & 3) == 0;
  float4 pa[4], pb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int q = tid + 256 * m, row = q >> 3, kq = 4 * (q & 7);
      pa[m] = load4_guard(a.x1, r0 + row, a.n1, a.d, k0 + kq, vec);
      pb[m] = load4_guard(a.x2, c0 + row, a.n2, a.d, k0 + kq, vec);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int q = tid + 256 * m, row = q >> 3, kq = 4 * (q & 7);
      *reinterpret_cast<float4*>(&As[row * FC_LDR + kq]) = pa[m];
      *reinterpret_cast<float4*>(&Bs[row * FC_LDR + kq]) = pb[m];
    }
  };
  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  fetch(0);
  store();
  __syncthreads();
  for (int k0 = 0; k0 < a.d; k0 += FC_BK) {
    // (the last tile re-requests its own k range: in bounds, never stored)
    fetch(k0 + FC_BK < a.d ? k0 + FC_BK : k0);
#pragma unroll
    for (int kk = 0; kk < FC_BK; kk += 4) {
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[(wr + 16 * i + li) * FC_LDR + kk + ks];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[(wc + 16 * j + li) * FC_LDR + kk + ks];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (k0 + FC_BK < a.d) {
      __syncthreads();
      store();
      __syncthreads();
    }
  }
  const float inv_d = 1.0f / (float)a.d;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t rb = r0 + wr + 16 * i + 4 * ks;  // rows rb .. rb + 3 of this lane
      const int64_t c = c0 + wc + 16 * j + li;
      if (c >= a.n2) continue;
      float kv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = rb + v;
        if (r >= a.n1) {
          kv[v] = 0.f;
          continue;
        }
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
        kv[v] = k;
        a.K[r * a.ldk + c] = k;
      }
      if (mirror) {
        // row c of the block, columns rb .. rb + 3 (one 16-byte store when
        // they are in range and aligned)
        float* m = a.K + c * a.ldk + rb;
        if (rb + 3 < a.n1 && (reinterpret_cast<uintptr_t>(m) & 15) == 0) {
          *reinterpret_cast<float4*>(m) = make_float4(kv[0], kv[1], kv[2], kv[3]);
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (rb + v < a.n1) m[v] = kv[v];
        }
      }
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
  const int64_t t1 = (a.n1 + FC_BM - 1) / FC_BM, t2 = (a.n2 + FC_BM - 1) / FC_BM;
  if (a.sym) {
    // (the x2 diagonals equal the x1 ones; both are computed, as for any block)
    hipLaunchKernelGGL(fc_kernel, dim3((unsigned)(t1 * (t1 + 1) / 2)), dim3(256), 0, stream, b);
  } else {
    hipLaunchKernelGGL(fc_kernel, dim3((unsigned)t2, (unsigned)t1), dim3(256), 0, stream, b);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace nk
