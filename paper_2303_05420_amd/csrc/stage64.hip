// First stage of the Myrtle NNGP at 64x64 inputs: seed, D <= 2 [3x3 conv,
// ReLU] layers at 64x64 and the 2x2 average pool (App. A), writing the
// pooled 32x32 covariance of each pair for the next stage.
//
// The sheared tile layout and the per-tile arithmetic are those of the
// smaller stages (lane = column ix, register = row, one tile per column kx
// and displacement row ky), but a pair no longer fits one workgroup's lanes
// and registers: 64 tile columns of 64 lanes, each lane holding 64 rows of
// the tile plus 2 x 32 pooling accumulators.  So one workgroup of 8 waves
// owns one pair and sweeps its tile columns in 8 groups of 8 (wave w takes
// kx = 8 g + w), each group sweeping all 64 displacement rows ky.
//
// LDS holds the pair's variance tables (both images, D layers, 64 KiB per
// layer) -- the second image's rows are not stored twice as in the smaller
// stages, its row index wraps instead -- and one coarse row of 4 pooled
// tiles for the x part of the pool.  The images are read from global memory
// (L1/L2) once per tile.
//
// Pooling.  The y part runs in registers along the ky sweep as in the
// smaller stages, except that coarse row 0 (its first part comes at ky = 1,
// the rest at the end of the sweep, ky = 0) is emitted twice and summed in
// the output, as in the tangent-kernel stages: that keeps 32 registers free.
// The x part: coarse column Kx takes both lanes of each
// pair (2J, 2J+1) of fine column 2Kx, lane 2J of column 2Kx + 1 and lane
// 2J + 1 of column 2Kx - 1.  Group g covers fine columns 8g .. 8g + 7, i.e.
// coarse columns 4g .. 4g + 3 apart from one contribution at each end: the
// odd lanes of column 8g + 7 belong to coarse column 4g + 4 (4g + 4 mod 32).
// Those are stored straight into the output when group g emits, and group
// g + 1 adds its own part to them; for the last group the target is coarse
// column 0, which group 0 wrote earlier, so they are added.  All sums have a
// fixed order, so results are bitwise reproducible.
#include "nk_tile.h"

namespace nk {

constexpr int S64_THREADS = 512;  // 8 waves, one tile column each

// Rows of the first image kept in LDS (channel-major per row, lane-contiguous
// reads) for the first batch of seed rows: what fits beside the tables and
// the pooling row at depth 2 (12 KiB at 3 channels); none at 4 channels.
__host__ __device__ constexpr int s64_x1_rows(int C) { return C <= 3 ? 16 : 0; }

// [3x3 conv, ReLU] on one 64-row tile; as tile_layer, with the second
// image's table rows wrapping: row r of tile (ky, kx) reads pixel row
// (r + ky) mod 64 of x2.  The map is the forward NNGP's degree-3 fit, and
// each row's tables are requested two rows before its map (at two waves per
// SIMD the LDS latency is not hidden by other waves alone; the compiler
// barrier keeps each request ahead of the row it runs before).
template <bool SIGNED, bool BIAS>
__device__ __forceinline__ void s64_layer(float (&A)[64], const float2* __restrict__ c1,
                                          const float2* __restrict__ t2l, int ky, int jx, int seam, float mL,
                                          float mR, float sb2) {
  float2 ta[64], tb[64];  // (registers: three rows live at a time)
  auto fetch = [&](int r) {
    ta[r] = c1[r * 64];
    tb[r] = t2l[((r + ky) & 63) * 64 + jx];
  };
  fetch(0);
  fetch(1);
  float hm = 0.f;
  float h0 = hsum3(A[0], mL, mR);
#pragma unroll
  for (int r = 0; r < 64; ++r) {
    if (r + 2 < 64) fetch(r + 2);
    asm volatile("" ::: "memory");
    float hp = 0.f;
    if (r + 1 < 64) hp = hsum3(A[r + 1], mL, mR);
    float v = h0;
    if (r > 0) v = __builtin_fmaf(uniform_mask(r == seam), hm, v);
    if (r + 1 < 64) v = __builtin_fmaf(uniform_mask(r + 1 == seam), hp, v);
    if (BIAS) v += sb2;
    const float2 a = ta[r];
    const float2 b = tb[r];
    const float rr = a.x * b.x;
    const float J = SIGNED ? j1_signed_vr3(v, rr) : j1_nonneg3(v * rr);
    A[r] = (a.y * b.y) * J;
    hm = h0;
    h0 = hp;
  }
}

template <int C, bool BIAS>
__global__ __launch_bounds__(S64_THREADS) void stage64_kernel(const StageArgs args) {
  constexpr int N = 64, H = 32, NN = N * N, H2 = H * H, H3 = H * H * H;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int D = args.D;
  float2* t1 = reinterpret_cast<float2*>(smem);
  float2* t2 = t1 + D * NN;
  float* red = reinterpret_cast<float*>(t2 + D * NN);  // [4][H][H]: one coarse row of the group's 4 columns
  constexpr int XR = s64_x1_rows(C);
  float* x1l = red + 4 * H2;  // [XR][C][N]: the first XR rows of the first image
  const int tid = threadIdx.x, w = tid >> 6, ix = tid & 63;

  const int64_t pl = xcd_logical_block();
  if (pl >= args.np) return;  // whole workgroup, before any barrier
  int64_t ia, ib;
  pair_of(args.p0 + pl, args.n1, args.n2, args.sym, args.T, &ia, &ib);
  for (int e = tid; e < D * NN; e += S64_THREADS) {
    t1[e] = args.tab1[ia * args.tablen + args.taboff + e];
    t2[e] = args.tab2[ib * args.tablen + args.taboff + e];
  }
  for (int e = tid; e < XR * N * C; e += S64_THREADS) {
    const int row = e / (N * C), col = (e / C) % N, c = e % C;  // e = (row N + col) C + c
    x1l[(row * C + c) * N + col] = args.x1[ia * NN * C + e];
  }
  __syncthreads();
  const float* x1p = args.x1 + (ia * NN + ix) * C;
  const float* x2p = args.x2 + ib * NN * C;
  float* out = args.out + pl * (int64_t)H * H3;
  const float ss = args.seed_scale;

#pragma unroll 1
  for (int g = 0; g < 8; ++g) {
    const int kx = 8 * g + w;
    const float mL = (ix >= 1 && ix != N - kx) ? 1.f : 0.f;
    const float mR = (ix + 1 < N && ix + 1 != N - kx) ? 1.f : 0.f;
    const int jx = (ix + kx) & (N - 1);
    const float* x2c = x2p + jx * C;
    float acc[H];
#pragma unroll
    for (int I = 0; I < H; ++I) acc[I] = 0.f;
#pragma unroll 1
    for (int step = 0; step < N; ++step) {
      const int ky = (step + 1) & (N - 1);
      const int seam = ky == 0 ? -1 : N - ky;
      // coarse row completed (or, at ky = 1, begun) at this step: ky = 1
      // and ky = 0 emit coarse row 0 in two parts, every odd ky > 1 ends row
      // (ky - 1) / 2
      const bool emit = ky == 0 || (ky & 1);
      const int Ky = ky == 0 ? 0 : (ky - 1) >> 1;
      // the second part of coarse row 0 and the carried boundary columns add
      // to what the output already holds
      const bool add_all = ky == 0;
      float A[N];
      constexpr int SR = 16;  // seed rows whose pixels are requested together
      // (an opaque offset keeps the 64 row addresses of each image from being
      // hoisted out of the sweep: they would pin 256 registers)
      const int z = opaque_zero();
      const float* x1s = x1p + z;
      const float* x2s = x2c + z;
#pragma unroll
      for (int r0 = 0; r0 < N; r0 += SR) {
        float u[SR][C], v[SR][C];
#pragma unroll
        for (int k = 0; k < SR; ++k) {
          const float* p1 = x1s + (r0 + k) * N * C;
          const float* p2 = x2s + ((r0 + k + ky) & (N - 1)) * N * C;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            u[k][c] = r0 + k < XR ? x1l[((r0 + k) * C + c) * N + ix] : p1[c];
            v[k][c] = p2[c];
          }
        }
#pragma unroll
        for (int k = 0; k < SR; ++k) {
          float sd = 0.f;
#pragma unroll
          for (int c = 0; c < C; ++c) sd = __builtin_fmaf(u[k][c], v[k][c], sd);
          A[r0 + k] = sd * ss;
        }
      }
      const float2* c1 = t1 + ix;
      s64_layer<true, BIAS>(A, c1, t2, ky, jx, seam, mL, mR, args.sb2);
      if (D > 1) s64_layer<false, BIAS>(A, c1 + NN, t2 + NN, ky, jx, seam, mL, mR, args.sb2);

      // y part of the pool
      if (ky == 1) {
#pragma unroll
        for (int I = 0; I < H; ++I) acc[I] = A[2 * I];
      } else if ((ky & 1) == 0) {
#pragma unroll
        for (int I = 0; I < H; ++I) acc[I] = acc[I] + (A[2 * I] + A[2 * I + 1]);
      } else {
#pragma unroll
        for (int I = 0; I < H; ++I) acc[I] = acc[I] + A[2 * I];
      }
      if (emit) {
        // x part: red[m] is coarse column 4g + m of coarse row Ky
        const int m = w >> 1;
        const bool lead = !(kx & 1) && !(ix & 1);
#pragma unroll
        for (int I = 0; I < H; ++I) {
          // (the lane shift runs on all lanes; only the store is predicated)
          const float t = acc[I] + lane_next(acc[I]);
          if (lead) red[(m * H + I) * H + (ix >> 1)] = t;
        }
        __syncthreads();
        if ((kx & 1) && !(ix & 1)) {
#pragma unroll
          for (int I = 0; I < H; ++I) red[(m * H + I) * H + (ix >> 1)] += acc[I];
        }
        __syncthreads();
        if ((kx & 1) && (ix & 1)) {
          if (m < 3) {
#pragma unroll
            for (int I = 0; I < H; ++I) red[((m + 1) * H + I) * H + (ix >> 1)] += acc[I];
          } else {
            // odd lanes of column 8g + 7: coarse column 4g + 4 of the next
            // group (stored, the next group adds to it; added at the second
            // part of row 0) or, for the last group, coarse column 0 (which
            // group 0 wrote: added)
            float* o = out + (int64_t)Ky * H3 + (int64_t)(((4 * g + 4) & (H - 1)) * H) * H + (ix >> 1);
            const bool add = g == 7 || add_all;
#pragma unroll
            for (int I = 0; I < H; ++I) o[I * H] = add ? o[I * H] + acc[I] : acc[I];
          }
        }
        __syncthreads();
        {
          float* o = out + (int64_t)Ky * H3 + (int64_t)(4 * g) * H2;
          for (int e = tid; e < 4 * H2; e += S64_THREADS)
            o[e] = (add_all || (g > 0 && e < H2)) ? o[e] + red[e] : red[e];
        }
        __syncthreads();
        if (ky != 0) {
#pragma unroll
          for (int I = 0; I < H; ++I) acc[I] = A[2 * I + 1];
        }
      }
    }
  }
}

size_t stage64_lds_bytes(int D, int C) {
  return (size_t)2 * D * 64 * 64 * sizeof(float2) + (size_t)4 * 32 * 32 * sizeof(float) +
         (size_t)s64_x1_rows(C) * C * 64 * sizeof(float);
}

template <int C, bool BIAS>
static int launch_s64_t(const StageArgs& a, hipStream_t s) {
  auto fn = stage64_kernel<C, BIAS>;
  const size_t lds = stage64_lds_bytes(a.D, C);
  static std::atomic<size_t> seen[kMaxDevices];  // per instantiation
  if (allow_dyn_lds((const void*)fn, lds, seen)) return -3;
  hipLaunchKernelGGL(fn, dim3((unsigned)a.np), dim3(S64_THREADS), lds, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int C>
static int launch_s64_c(const StageArgs& a, bool bias, hipStream_t s) {
  return bias ? launch_s64_t<C, true>(a, s) : launch_s64_t<C, false>(a, s);
}

int launch_stage64(const StageArgs& a, bool bias, hipStream_t s) {
  if (a.np <= 0) return 0;
  if (a.D < 1 || a.D > 2 || !a.out || a.tiles) return -1;
  switch (a.C) {
    case 1: return launch_s64_c<1>(a, bias, s);
    case 2: return launch_s64_c<2>(a, bias, s);
    case 3: return launch_s64_c<3>(a, bias, s);
    case 4: return launch_s64_c<4>(a, bias, s);
  }
  return -1;
}

}  // namespace nk
