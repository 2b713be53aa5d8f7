// Fused stage kernel of the Myrtle NNGP forward pass.
//
// One Myrtle stage at resolution N x N (App. A: depth blocks of [3x3 SAME
// conv, ReLU], then a 2x2 average pool or, after the last stage, global
// average pooling and the Dense readout) for a chunk of image pairs.
//
// Layout.  A pair carries the covariance S(i, j) over pixel pairs, N^4
// entries.  A 3x3 conv maps (i, j) -> (i + d, j + d), so it keeps the
// displacement j - i; we index entries by k = (j - i) mod N per axis and call
// the N x N entries with one k = (ky, kx) a tile: entry (iy, ix) of tile k is
// i = (iy, ix), j = ((iy + ky) mod N, (ix + kx) mod N).  Inside a tile the
// conv is a 3x3 box filter, except across the seam where j wraps (there the
// two sides are different displacements, k and k - N) and at the tile edge;
// those neighbour terms are masked to zero, which is exactly the zero padding
// of the SAME convolution.  Every tile has N^2 entries, so the work is
// perfectly regular.
//
// Mapping.  A tile lives in one N-lane segment of a wave: lane = ix, register
// r = iy.  Horizontal neighbours come from DPP lane shifts (masked by two
// per-lane 0/1 factors fixed for the segment's kx), vertical ones from the
// neighbouring register (masked by a wave-uniform 0/1 factor at the seam
// row N - ky).  Each segment owns one kx and sweeps ky = 1, 2, ..., N-1, 0.
//
// ReLU.  With the per-image tables (alpha, beta) of prepare.hip:
//   rho = (box + sigma_b2) alpha(i) alpha'(j),   out = beta(i) beta'(j) J1(rho),
// which is kappa times the ReLU output, kappa the scale of the next linear
// step; so the next layer's pre-activation is simply box(out) + sigma_b2.
//
// Pooling (2x2, stride 2).  Coarse tile K = ((k + a) >> 1) mod N/2 and row
// I = i >> 1 for fine row i = 2I + a: even ky rows pool in pairs into K = ky/2,
// odd ky send even rows to (ky - 1)/2 and odd rows to (ky + 1)/2.  The y part
// is accumulated in registers along the sweep; the x part (neighbouring kx
// segments) is combined through LDS in a fixed order, and each finished
// coarse row of tiles is written once to the next stage's input.  All sums
// have a fixed order, so results are bitwise reproducible.
#include "nk_tile.h"

namespace nk {



// Pair p of the pass -> table rows of both images, their pixels (first
// stage) and where its kernel value goes (and its mirror in a symmetric
// block).  One block: the block order of pair_of.  Batched pass: the tile
// holding p (binary search over the tiles' first pairs), then its block order.
__device__ inline void resolve_pair(const StageArgs& a, int64_t p, int64_t img_floats, int64_t* t1, int64_t* t2,
                                    const float** x1, const float** x2, float** k, float** km) {
  int64_t ia, ib;
  if (a.tiles == nullptr) {
    pair_of(p, a.n1, a.n2, a.sym, a.T, &ia, &ib);
    *t1 = ia;
    *t2 = ib;
    *x1 = a.x1 + ia * img_floats;
    *x2 = a.x2 + ib * img_floats;
    *k = a.K ? a.K + ia * a.ldk + ib : nullptr;
    *km = (a.K && a.sym && ia != ib) ? a.K + ib * a.ldk + ia : nullptr;
    return;
  }
  int lo = 0, hi = a.ntiles - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.tiles[mid].p_begin <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  const TileDesc& t = a.tiles[lo];
  pair_of(p - t.p_begin, t.n1, t.n2, t.sym, a.T, &ia, &ib);
  *t1 = t.t1 + ia;
  *t2 = t.t2 + ib;
  *x1 = t.x1 + ia * img_floats;
  *x2 = t.x2 + ib * img_floats;
  *k = t.K + ia * t.ldk + ib;
  *km = (t.sym && ia != ib) ? t.K + ib * t.ldk + ia : nullptr;
}

// Work units (groups of PPWG consecutive pairs of the chunk) of this
// workgroup.  Plain grid: one unit per workgroup, XCD-remapped.  Persistent
// grid (a multiple of 8 workgroups, all resident): the dispatcher deals
// workgroups round-robin over the 8 XCDs, so the workgroups of XCD x split
// one contiguous eighth of the units between them and advance together: the
// pairs in flight on an XCD at any time are neighbours in the pair order and
// share images in that XCD's L2.
__device__ inline void unit_range(int64_t nunits, int persist, int64_t* first, int64_t* step, int64_t* end) {
  if (persist <= 0) {
    *first = xcd_logical_block();
    *step = nunits;
    *end = *first + 1;
    return;
  }
  const int64_t b = blockIdx.x, x = b & 7, s = b >> 3, per_xcd = gridDim.x >> 3;
  const int64_t R = (nunits + 7) >> 3;
  *first = x * R + s;
  *step = per_xcd;
  *end = (x + 1) * R < nunits ? (x + 1) * R : nunits;
}

template <int N, bool SEED, bool POOL, bool BIAS>
__global__ __launch_bounds__(KCfg<N>::THREADS) void stage_kernel(const StageArgs args) {
  constexpr int THREADS = KCfg<N>::THREADS, PPWG = KCfg<N>::PPWG;
  constexpr int H = N / 2;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ int64_t s_t1[PPWG], s_t2[PPWG];
  __shared__ const float* s_x1[PPWG];
  __shared__ const float* s_x2[PPWG];
  __shared__ float* s_k[PPWG];
  __shared__ float* s_km[PPWG];

  const int tid = threadIdx.x;
  const int slot = tid / (N * N);
  const int within = tid - slot * N * N;
  const int kx = within / N, ix = within - kx * N;
  const int D = args.D;
  const size_t slot_bytes = slot_lds_bytes<N>(D, POOL, SEED);
  const int TL = D * N * N;

  const int64_t nunits = (args.np + PPWG - 1) / PPWG;
  int64_t unit, ustep, uend;
  unit_range(nunits, args.persist, &unit, &ustep, &uend);
  for (; unit < uend; unit += ustep) {
  if (tid < PPWG) {
    int64_t pl = unit * PPWG + tid;
    if (pl >= args.np) pl = args.np - 1;
    resolve_pair(args, args.p0 + pl, (int64_t)N * N * args.C, &s_t1[tid], &s_t2[tid], &s_x1[tid], &s_x2[tid],
                 &s_k[tid], &s_km[tid]);
  }
  __syncthreads();
  // this stage's (alpha, beta) tables of both images -> LDS; x2's rows twice
  for (int e = tid; e < PPWG * TL; e += THREADS) {
    const int s = e / TL, r = e - s * TL;
    float2* d1 = reinterpret_cast<float2*>(smem + s * slot_bytes);
    d1[r] = args.tab1[s_t1[s] * args.tablen + args.taboff + r];
    const float2 v = args.tab2[s_t2[s] * args.tablen + args.taboff + r];
    const int l = r / (N * N), rr = r - l * N * N;
    float2* d2 = d1 + TL + l * 2 * N * N;
    d2[rr] = v;
    d2[rr + N * N] = v;
  }
  if (SEED) {
    // images as float4 per pixel (channels zero padded to 4)
    const size_t rb = POOL ? (size_t)N * N * N / 8 * 4 : (size_t)N * N * 8;
    for (int e = tid; e < PPWG * N * N; e += THREADS) {
      const int s = e / (N * N), px = e - s * (N * N);
      float4* d = reinterpret_cast<float4*>(smem + s * slot_bytes + (size_t)TL * 24 + (rb < 16 ? 16 : rb));
      const float* p1 = s_x1[s] + px * args.C;
      const float* p2 = s_x2[s] + px * args.C;
      float u[4] = {0.f, 0.f, 0.f, 0.f}, w[4] = {0.f, 0.f, 0.f, 0.f};
      for (int c = 0; c < args.C && c < 4; ++c) {
        u[c] = p1[c];
        w[c] = p2[c];
      }
      // the seed scale sigma_w2 / (9 C) rides on the second image
      const float sc = args.seed_scale;
      // (the second image twice, so that its rows are read without wrapping)
      d[px] = make_float4(u[0], u[1], u[2], u[3]);
      const float4 ws = make_float4(sc * w[0], sc * w[1], sc * w[2], sc * w[3]);
      d[N * N + px] = ws;
      d[2 * N * N + px] = ws;
    }
  }
  __syncthreads();

  const int64_t pl = unit * PPWG + slot;
  const bool valid = pl < args.np;
  const float2* t1 = reinterpret_cast<const float2*>(smem + slot * slot_bytes);
  const float2* t2 = t1 + TL;
  float* red = reinterpret_cast<float*>(smem + slot * slot_bytes + (size_t)TL * 24);
  const size_t red_bytes = POOL ? (size_t)N * N * N / 8 * 4 : (size_t)N * N * 8;
  const float4* img1 = reinterpret_cast<const float4*>(smem + slot * slot_bytes + (size_t)TL * 24 +
                                                       (red_bytes < 16 ? 16 : red_bytes));
  const float4* img2 = img1 + N * N;

  const float mL = (ix >= 1 && ix != N - kx) ? 1.f : 0.f;
  const float mR = (ix + 1 < N && ix + 1 != N - kx) ? 1.f : 0.f;
  const int jx = (ix + kx) & (N - 1);

  float acc[H], wrap[H];
#pragma unroll
  for (int I = 0; I < H; ++I) acc[I] = wrap[I] = 0.f;
  double gsum = 0.0;

  const float* inp = nullptr;
  if (!SEED) inp = args.in + (pl < args.np ? pl : args.np - 1) * (int64_t)N * N * N * N;

  for (int step = 0; step < N; ++step) {
    const int ky = (step + 1) & (N - 1);
    const int seam = ky == 0 ? -1 : N - ky;
    float A[N];
    if (SEED) {
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const float4 u = img1[r * N + ix];
        const float4 w = img2[(r + ky) * N + jx];
        A[r] = __builtin_fmaf(u.w, w.w, __builtin_fmaf(u.z, w.z, __builtin_fmaf(u.y, w.y, u.x * w.x)));
      }
    } else {
      const float* p = inp + ((int64_t)ky * N + kx) * N * N + ix;
#pragma unroll
      for (int r = 0; r < N; ++r) A[r] = p[r * N];
    }
    const float2* c1 = t1 + ix;
    const float2* c2 = t2 + ky * N + jx;
    int l = 0;
    if (SEED) {
      tile_layer<N, true, BIAS>(A, c1, c2, seam, mL, mR, args.sb2);
      c1 += N * N;
      c2 += 2 * N * N;
      l = 1;
    }
    for (; l < D; ++l) {
      tile_layer<N, false, BIAS>(A, c1, c2, seam, mL, mR, args.sb2);
      c1 += N * N;
      c2 += 2 * N * N;
    }

    if (POOL) {
      bool emit = false;
      int Ky = 0;
      if (ky == 1) {
#pragma unroll
        for (int I = 0; I < H; ++I) {
          wrap[I] = A[2 * I];
          acc[I] = A[2 * I + 1];
        }
        if (N == 2) {
          // one coarse row only: it completes at ky = 0
        }
      } else if (ky == 0) {
#pragma unroll
        for (int I = 0; I < H; ++I) acc[I] = acc[I] + (A[2 * I] + A[2 * I + 1]) + wrap[I];
        emit = true;
        Ky = 0;
      } else if ((ky & 1) == 0) {
#pragma unroll
        for (int I = 0; I < H; ++I) acc[I] = acc[I] + (A[2 * I] + A[2 * I + 1]);
      } else {
#pragma unroll
        for (int I = 0; I < H; ++I) acc[I] = acc[I] + A[2 * I];
        emit = true;
        Ky = (ky - 1) >> 1;
      }
      if (emit) {
        // x combine: coarse Kx gets lanes (2I, 2I+1) of kx = 2Kx, lane 2I of
        // kx = 2Kx + 1 and lane 2I + 1 of kx = 2Kx - 1
        float s[H];
#pragma unroll
        for (int I = 0; I < H; ++I) s[I] = acc[I] + lane_next(acc[I]);
        if (!(kx & 1) && !(ix & 1)) {
#pragma unroll
          for (int I = 0; I < H; ++I) red[((kx >> 1) * H + I) * H + (ix >> 1)] = s[I];
        }
        __syncthreads();
        if ((kx & 1) && !(ix & 1)) {
#pragma unroll
          for (int I = 0; I < H; ++I) red[((kx >> 1) * H + I) * H + (ix >> 1)] += acc[I];
        }
        __syncthreads();
        if ((kx & 1) && (ix & 1)) {
          const int Kx = ((kx + 1) >> 1) & (H - 1);
#pragma unroll
          for (int I = 0; I < H; ++I) red[(Kx * H + I) * H + (ix >> 1)] += acc[I];
        }
        __syncthreads();
        if (valid) {
          float* o = args.out + pl * (int64_t)H * H * H * H + (int64_t)Ky * H * H * H;
          for (int e = within; e < H * H * H; e += N * N) o[e] = red[e];
        }
        __syncthreads();
        if (ky != 0) {
#pragma unroll
          for (int I = 0; I < H; ++I) acc[I] = A[2 * I + 1];
        }
      }
    } else {
      float ts[N];
#pragma unroll
      for (int r = 0; r < N; ++r) ts[r] = A[r];
#pragma unroll
      for (int w = N / 2; w >= 1; w >>= 1) {
#pragma unroll
        for (int r = 0; r < w; ++r) ts[r] = ts[r] + ts[r + w];
      }
      gsum += (double)ts[0];
    }
  }

  if (!POOL) {
    double* part = reinterpret_cast<double*>(red);
    part[within] = gsum;
    __syncthreads();
    if (within == 0 && valid) {
      double t = 0.0;
      for (int e = 0; e < N * N; ++e) t += part[e];
      const float kv = (float)(t + (double)args.sb2);
      *s_k[slot] = kv;
      if (s_km[slot]) *s_km[slot] = kv;
    }
  }
  __syncthreads();  // LDS and the slot table are reused by the next unit
  }  // units of this workgroup
}

template <int N, bool SEED, bool POOL, bool BIAS>
static int set_attr(size_t lds) {
  auto fn = stage_kernel<N, SEED, POOL, BIAS>;
  if (lds > 64 * 1024) {
    static size_t attr_bytes = 0;  // per instantiation
    if (attr_bytes < lds) {
      if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return -3;
      attr_bytes = lds;
    }
  }
  return 0;
}

template <int N, bool SEED, bool POOL, bool BIAS>
static int launch_t(const StageArgs& a, hipStream_t stream) {
  const int64_t nwg = (a.np + KCfg<N>::PPWG - 1) / KCfg<N>::PPWG;
  const size_t lds = (size_t)KCfg<N>::PPWG * slot_lds_bytes<N>(a.D, POOL, SEED);
  if (set_attr<N, SEED, POOL, BIAS>(lds)) return -3;
  const int64_t grid = a.persist > 0 ? a.persist : nwg;
  hipLaunchKernelGGL((stage_kernel<N, SEED, POOL, BIAS>), dim3((unsigned)grid), dim3(KCfg<N>::THREADS), lds, stream,
                     a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int N, bool SEED, bool POOL, bool BIAS>
static int occ_t(int D) {
  const size_t lds = (size_t)KCfg<N>::PPWG * slot_lds_bytes<N>(D, POOL, SEED);
  if (set_attr<N, SEED, POOL, BIAS>(lds)) return -3;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage_kernel<N, SEED, POOL, BIAS>, KCfg<N>::THREADS, lds) !=
      hipSuccess)
    return -3;
  return nb;
}

template <int N>
static int occ_n(int D, bool seed, bool pool, bool bias) {
  if (seed) {
    if (pool) return bias ? occ_t<N, true, true, true>(D) : occ_t<N, true, true, false>(D);
    return bias ? occ_t<N, true, false, true>(D) : occ_t<N, true, false, false>(D);
  }
  if (pool) return bias ? occ_t<N, false, true, true>(D) : occ_t<N, false, true, false>(D);
  return bias ? occ_t<N, false, false, true>(D) : occ_t<N, false, false, false>(D);
}

// Resident workgroups per CU of a stage kernel (and sets its LDS attribute,
// so that a later launch makes no attribute call, e.g. under graph capture).
int stage_occupancy(int N, int D, bool seed, bool pool, bool bias) {
  switch (N) {
    case 2: return occ_n<2>(D, seed, pool, bias);
    case 4: return occ_n<4>(D, seed, pool, bias);
    case 8: return occ_n<8>(D, seed, pool, bias);
    case 16: return occ_n<16>(D, seed, pool, bias);
    case 32: return occ_n<32>(D, seed, pool, bias);
  }
  return -2;
}

int prime_stage(int N, int D, bool seed, bool pool, bool bias) {
  const int r = stage_occupancy(N, D, seed, pool, bias);
  return r < 0 ? r : 0;
}

template <int N>
static int launch_n(const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s) {
  if (seed) {
    if (pool) return bias ? launch_t<N, true, true, true>(a, s) : launch_t<N, true, true, false>(a, s);
    return bias ? launch_t<N, true, false, true>(a, s) : launch_t<N, true, false, false>(a, s);
  }
  if (pool) return bias ? launch_t<N, false, true, true>(a, s) : launch_t<N, false, true, false>(a, s);
  return bias ? launch_t<N, false, false, true>(a, s) : launch_t<N, false, false, false>(a, s);
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
  switch (N) {
    case 2: return KCfg<2>::PPWG * slot_lds_bytes<2>(D, pool, seed);
    case 4: return KCfg<4>::PPWG * slot_lds_bytes<4>(D, pool, seed);
    case 8: return KCfg<8>::PPWG * slot_lds_bytes<8>(D, pool, seed);
    case 16: return KCfg<16>::PPWG * slot_lds_bytes<16>(D, pool, seed);
    case 32: return KCfg<32>::PPWG * slot_lds_bytes<32>(D, pool, seed);
  }
  return 0;
}

int launch_stage(int N, const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s) {
  switch (N) {
    case 2: return launch_n<2>(a, seed, pool, bias, s);
    case 4: return launch_n<4>(a, seed, pool, bias, s);
    case 8: return launch_n<8>(a, seed, pool, bias, s);
    case 16: return launch_n<16>(a, seed, pool, bias, s);
    case 32: return launch_n<32>(a, seed, pool, bias, s);
  }
  return -2;
}

}  // namespace nk
