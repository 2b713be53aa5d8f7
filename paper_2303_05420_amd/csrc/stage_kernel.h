// Fused stage kernel of the Myrtle NNGP and NTK forward pass.
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
// row N - ky).  Each segment owns CPS tile columns kx (one, except the 32x32
// tangent kernel, which carries two tiles per column and runs on half the
// lanes) and sweeps ky = 1, 2, ..., N-1, 0.
//
// ReLU.  With the per-image tables (alpha, beta) of prepare.hip:
//   rho = (box + sigma_b2) alpha(i) alpha'(j),   out = beta(i) beta'(j) J1(rho),
// which is kappa times the ReLU output, kappa the scale of the next linear
// step; so the next layer's pre-activation is simply box(out) + sigma_b2.
//
// Tangent kernel (NTK).  Beside A = kappa F the kernel carries
// C = kappa (F + Fdot T), T the pre-activation tangent kernel and
// Fdot = (pi - t) / (2 pi) = E[relu' relu'].  The conv then gives
// T' = S' + kappa box(Fdot T) = box(C) + sigma_b2, and on the first layer
// T = S (the inputs carry no parameters).  Pools and the readout are linear,
// so C is pooled like A and the NTK is sum(C) + sigma_b2 where the NNGP is
// sum(A) + sigma_b2.
//
// Pooling (2x2, stride 2).  Coarse tile K = ((k + a) >> 1) mod N/2 and row
// I = i >> 1 for fine row i = 2I + a: even ky rows pool in pairs into K = ky/2,
// odd ky send even rows to (ky - 1)/2 and odd rows to (ky + 1)/2.  The y part
// is accumulated in registers along the sweep; the x part (neighbouring kx
// segments) is combined through LDS in a fixed order, and each finished
// coarse row of tiles is written once to the next stage's input.  All sums
// have a fixed order, so results are bitwise reproducible.
#pragma once
#include "nk_tile.h"

namespace nk {

// Pair p of the pass -> table rows of both images, their pixels (first
// stage), the element offsets of its kernel value (and of its mirror in a
// symmetric block, -1 if none) in its output, and whether both images are
// the same image (the diagonal of a symmetric block; with `detect`, 2 marks
// a pair of distinct images whose first elements agree, a candidate for
// identical_pairs below).  One block: the block order of pair_of.  Batched
// pass: the tile holding p (binary search over the tiles' first pairs), then
// its block order.
__device__ inline void resolve_pair(const StageArgs& a, int64_t p, int64_t img_floats, int64_t* t1, int64_t* t2,
                                    const float** x1, const float** x2, float** kbase, int64_t* off,
                                    int64_t* offm, int* same, bool detect) {
  int64_t ia, ib;
  if (a.tiles == nullptr) {
    pair_of(p, a.n1, a.n2, a.sym, a.T, &ia, &ib);
    *same = a.sym && ia == ib;
    *t1 = ia;
    *t2 = ib;
    *x1 = a.x1 + ia * img_floats;
    *x2 = a.x2 + ib * img_floats;
    *kbase = a.K;
    *off = ia * a.ldk + ib;
    *offm = (a.sym && ia != ib) ? ib * a.ldk + ia : -1;
    if (detect && !*same && (*x1)[0] == (*x2)[0]) *same = 2;
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
  *same = t.sym && ia == ib;
  *t1 = t.t1 + ia;
  *t2 = t.t2 + ib;
  *x1 = t.x1 + ia * img_floats;
  *x2 = t.x2 + ib * img_floats;
  *kbase = t.K;
  *off = ia * t.ldk + ib;
  *offm = (t.sym && ia != ib) ? ib * t.ldk + ia : -1;
  if (detect && !*same && (*x1)[0] == (*x2)[0]) *same = 2;
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

template <int N, bool SEED, bool POOL, bool BIAS, bool NTK, int PPM = 1>
__global__ __launch_bounds__((KCfg<N, NTK, PPM>::THREADS)) void stage_kernel(const StageArgs args) {
  using Cfg = KCfg<N, NTK, PPM>;
  constexpr int THREADS = Cfg::THREADS, PPWG = Cfg::PPWG, CPS = Cfg::CPS, LPP = Cfg::LPP;
  constexpr int H = N / 2;
  constexpr int HC = NTK ? H : 1, NC = NTK ? N : 1;  // sizes of the tangent-kernel arrays
  constexpr size_t RQ = red_bytes_q<N>(POOL);          // LDS bytes of one quantity's pooling row
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ int64_t s_t1[PPWG], s_t2[PPWG], s_off[PPWG], s_offm[PPWG];
  __shared__ const float* s_x1[PPWG];
  __shared__ const float* s_x2[PPWG];
  __shared__ float* s_k[PPWG];
  __shared__ int s_same[PPWG];

  const int tid = threadIdx.x;
  const int slot = tid / LPP;
  const int within = tid - slot * LPP;
  const int seg = within / N, ix = within - seg * N;
  const int D = args.D;
  const size_t slot_bytes = slot_lds_bytes<N>(D, POOL, SEED, NTK);
  const int TL = D * N * N;
  const size_t red_region = (NTK ? 2 : 1) * RQ < 16 ? 16 : (NTK ? 2 : 1) * RQ;

  const int64_t nunits = (args.np + PPWG - 1) / PPWG;
  int64_t unit, ustep, uend;
  unit_range(nunits, args.persist, &unit, &ustep, &uend);
  for (; unit < uend; unit += ustep) {
  if (tid < PPWG) {
    int64_t pl = unit * PPWG + tid;
    if (pl >= args.np) pl = args.np - 1;
    resolve_pair(args, args.p0 + pl, args.img_floats, &s_t1[tid], &s_t2[tid], &s_x1[tid], &s_x2[tid],
                 &s_k[tid], &s_off[tid], &s_offm[tid], &s_same[tid], NTK);
  }
  __syncthreads();
  if constexpr (NTK) identical_pairs<PPWG, THREADS>(s_same, s_x1, s_x2, args.img_floats);
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
    for (int e = tid; e < PPWG * N * N; e += THREADS) {
      const int s = e / (N * N), px = e - s * (N * N);
      float4* d = reinterpret_cast<float4*>(smem + s * slot_bytes + (size_t)TL * 24 + red_region);
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
  const int64_t plc = valid ? pl : args.np - 1;
  const float2* t1 = reinterpret_cast<const float2*>(smem + slot * slot_bytes);
  const float2* t2 = t1 + TL;
  float* red = reinterpret_cast<float*>(smem + slot * slot_bytes + (size_t)TL * 24);
  float* redC = red + RQ / 4;
  const float4* img1 = reinterpret_cast<const float4*>(smem + slot * slot_bytes + (size_t)TL * 24 + red_region);
  const float4* img2 = img1 + N * N;

  // y-pool accumulators; the NNGP keeps coarse row 0's first part (ky = 1,
  // even rows) in `wrap` until the sweep ends, the NTK (short of registers)
  // emits it at once and adds the rest to it in memory at the end
  constexpr int HW = NTK ? 1 : H;
  float acc[CPS][H], wrap[CPS][HW], accC[CPS][HC];
#pragma unroll
  for (int c = 0; c < CPS; ++c) {
#pragma unroll
    for (int I = 0; I < H; ++I) acc[c][I] = 0.f;
#pragma unroll
    for (int I = 0; I < HW; ++I) wrap[c][I] = 0.f;
#pragma unroll
    for (int I = 0; I < (NTK ? HC : 0); ++I) accC[c][I] = 0.f;
  }
  double gsum = 0.0, gsumC = 0.0;

  const float* inp = nullptr;
  const float* inpC = nullptr;
  if (!SEED) {
    inp = args.in + plc * (int64_t)N * N * N * N;
    if (NTK) inpC = args.in2 + plc * (int64_t)N * N * N * N;
  }

  for (int step = 0; step < N; ++step) {
    const int ky = (step + 1) & (N - 1);
    const int seam = ky == 0 ? -1 : N - ky;
    // coarse row completed at this step: ky = 0 ends coarse row 0, every odd
    // ky > 1 ends row (ky - 1) / 2
    const bool emit = POOL && (NTK || ky != 1) && (ky == 0 || (ky & 1));
    const int Ky = ky == 0 ? 0 : (ky - 1) >> 1;
    if (CPS > 1 && emit) {
      // several column passes add into the pooling rows: clear them first
      for (int e = within; e < H * H * H; e += LPP) {
        red[e] = 0.f;
        if (NTK) redC[e] = 0.f;
      }
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < CPS; ++c) {
      const int kx = seg + c * (N / CPS);
      const float mL = (ix >= 1 && ix != N - kx) ? 1.f : 0.f;
      const float mR = (ix + 1 < N && ix + 1 != N - kx) ? 1.f : 0.f;
      const int jx = (ix + kx) & (N - 1);
      float A[N], Cq[NC];
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
        if (NTK) {
          const float* pc = inpC + ((int64_t)ky * N + kx) * N * N + ix;
#pragma unroll
          for (int r = 0; r < NC; ++r) Cq[r] = pc[r * N];
        }
      }
      const float2* c1 = t1 + ix;
      const float2* c2 = t2 + ky * N + jx;
      // displacement-0 tile of a pair of identical images: rho = 1 exactly
      const float umax = (NTK && s_same[slot] && ky == 0 && kx == 0) ? 0.f : 1.f;
      int l = 0;
      if (SEED) {
        if constexpr (NTK)
          tile_layer_ntk<N, true, BIAS>(A, Cq, c1, c2, seam, mL, mR, args.sb2, args.kh[0], umax);
        else
          tile_layer<N, true, BIAS>(A, c1, c2, seam, mL, mR, args.sb2);
        c1 += N * N;
        c2 += 2 * N * N;
        l = 1;
      }
      for (; l < D; ++l) {
        if constexpr (NTK)
          tile_layer_ntk<N, false, BIAS>(A, Cq, c1, c2, seam, mL, mR, args.sb2, args.kh[l], umax);
        else
          tile_layer<N, false, BIAS>(A, c1, c2, seam, mL, mR, args.sb2);
        c1 += N * N;
        c2 += 2 * N * N;
      }

      if (POOL) {
        // y part of the pool
        if (ky == 1) {
          if constexpr (NTK) {
            // coarse row 0, first part: emitted now (odd rows start row 1 after it)
#pragma unroll
            for (int I = 0; I < H; ++I) acc[c][I] = A[2 * I];
#pragma unroll
            for (int I = 0; I < (NTK ? HC : 0); ++I) accC[c][I] = Cq[2 * I];
          } else {
#pragma unroll
            for (int I = 0; I < H; ++I) {
              wrap[c][I] = A[2 * I];
              acc[c][I] = A[2 * I + 1];
            }
          }
        } else if (ky == 0) {
          if constexpr (NTK) {
#pragma unroll
            for (int I = 0; I < H; ++I) acc[c][I] = acc[c][I] + (A[2 * I] + A[2 * I + 1]);
#pragma unroll
            for (int I = 0; I < (NTK ? HC : 0); ++I) accC[c][I] = accC[c][I] + (Cq[2 * I] + Cq[2 * I + 1]);
          } else {
#pragma unroll
            for (int I = 0; I < H; ++I) acc[c][I] = acc[c][I] + (A[2 * I] + A[2 * I + 1]) + wrap[c][I % HW];
          }
        } else if ((ky & 1) == 0) {
#pragma unroll
          for (int I = 0; I < H; ++I) acc[c][I] = acc[c][I] + (A[2 * I] + A[2 * I + 1]);
#pragma unroll
          for (int I = 0; I < (NTK ? HC : 0); ++I) accC[c][I] = accC[c][I] + (Cq[2 * I] + Cq[2 * I + 1]);
        } else {
#pragma unroll
          for (int I = 0; I < H; ++I) acc[c][I] = acc[c][I] + A[2 * I];
#pragma unroll
          for (int I = 0; I < (NTK ? HC : 0); ++I) accC[c][I] = accC[c][I] + Cq[2 * I];
        }
        if (emit) {
          // x combine: coarse Kx gets lanes (2I, 2I+1) of kx = 2Kx, lane 2I of
          // kx = 2Kx + 1 and lane 2I + 1 of kx = 2Kx - 1
          float s[H], sC[HC];
#pragma unroll
          for (int I = 0; I < H; ++I) s[I] = acc[c][I] + lane_next(acc[c][I]);
#pragma unroll
          for (int I = 0; I < (NTK ? HC : 0); ++I) sC[I] = accC[c][I] + lane_next(accC[c][I]);
          if (!(kx & 1) && !(ix & 1)) {
#pragma unroll
            for (int I = 0; I < H; ++I) {
              float* d = &red[((kx >> 1) * H + I) * H + (ix >> 1)];
              *d = CPS > 1 ? *d + s[I] : s[I];
            }
#pragma unroll
            for (int I = 0; I < (NTK ? HC : 0); ++I) {
              float* d = &redC[((kx >> 1) * H + I) * H + (ix >> 1)];
              *d = CPS > 1 ? *d + sC[I] : sC[I];
            }
          }
          __syncthreads();
          if ((kx & 1) && !(ix & 1)) {
#pragma unroll
            for (int I = 0; I < H; ++I) red[((kx >> 1) * H + I) * H + (ix >> 1)] += acc[c][I];
#pragma unroll
            for (int I = 0; I < (NTK ? HC : 0); ++I) redC[((kx >> 1) * H + I) * H + (ix >> 1)] += accC[c][I];
          }
          __syncthreads();
          if ((kx & 1) && (ix & 1)) {
            const int Kx = ((kx + 1) >> 1) & (H - 1);
#pragma unroll
            for (int I = 0; I < H; ++I) red[(Kx * H + I) * H + (ix >> 1)] += acc[c][I];
#pragma unroll
            for (int I = 0; I < (NTK ? HC : 0); ++I) redC[(Kx * H + I) * H + (ix >> 1)] += accC[c][I];
          }
          __syncthreads();
          if (ky != 0) {
#pragma unroll
            for (int I = 0; I < H; ++I) acc[c][I] = A[2 * I + 1];
#pragma unroll
            for (int I = 0; I < (NTK ? HC : 0); ++I) accC[c][I] = Cq[2 * I + 1];
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
        if (NTK) {
          float tc[NC];
#pragma unroll
          for (int r = 0; r < NC; ++r) tc[r] = Cq[r];
#pragma unroll
          for (int w = NC / 2; w >= 1; w >>= 1) {
#pragma unroll
            for (int r = 0; r < w; ++r) tc[r] = tc[r] + tc[r + w];
          }
          gsumC += (double)tc[0];
        }
      }
    }  // tile columns of this segment
    if (emit) {
      if (valid) {
        float* o = args.out + pl * (int64_t)H * H * H * H + (int64_t)Ky * H * H * H;
        if (NTK && ky == 0) {
          // the rest of coarse row 0 (this thread stored its first part at ky = 1)
          float* o2 = args.out2 + pl * (int64_t)H * H * H * H;
          for (int e = within; e < H * H * H; e += LPP) {
            o[e] += red[e];
            o2[e] += redC[e];
          }
        } else {
          for (int e = within; e < H * H * H; e += LPP) o[e] = red[e];
          if (NTK) {
            float* o2 = args.out2 + pl * (int64_t)H * H * H * H + (int64_t)Ky * H * H * H;
            for (int e = within; e < H * H * H; e += LPP) o2[e] = redC[e];
          }
        }
      }
      __syncthreads();
    }
  }

  if (!POOL) {
    double* part = reinterpret_cast<double*>(red);
    double* partC = reinterpret_cast<double*>(redC);
    part[within] = gsum;
    if (NTK) partC[within] = gsumC;
    __syncthreads();
    if (within == 0 && valid) {
      double t = 0.0;
      for (int e = 0; e < LPP; ++e) t += part[e];
      const float kv = (float)(t + (double)args.sb2);
      if (s_k[slot]) {
        s_k[slot][s_off[slot]] = kv;
        if (s_offm[slot] >= 0) s_k[slot][s_offm[slot]] = kv;
      }
      if (NTK) {
        double tc = 0.0;
        for (int e = 0; e < LPP; ++e) tc += partC[e];
        const float kt = (float)(tc + (double)args.sb2);
        args.K2[s_off[slot]] = kt;
        if (s_offm[slot] >= 0) args.K2[s_offm[slot]] = kt;
      }
    }
  }
  __syncthreads();  // LDS and the slot table are reused by the next unit
  }  // units of this workgroup
}

// Allows one instantiation its dynamic LDS on the current device.
template <int N, bool SEED, bool POOL, bool BIAS, bool NTK, int PPM>
int set_attr(size_t lds) {
  static std::atomic<size_t> seen[kMaxDevices];  // per instantiation
  return allow_dyn_lds((const void*)stage_kernel<N, SEED, POOL, BIAS, NTK, PPM>, lds, seen);
}

template <int N, bool SEED, bool POOL, bool BIAS, bool NTK, int PPM>
int launch_t(const StageArgs& a, hipStream_t stream) {
  using Cfg = KCfg<N, NTK, PPM>;
  const int64_t nwg = (a.np + Cfg::PPWG - 1) / Cfg::PPWG;
  const size_t lds = (size_t)Cfg::PPWG * slot_lds_bytes<N>(a.D, POOL, SEED, NTK);
  if (set_attr<N, SEED, POOL, BIAS, NTK, PPM>(lds)) return -3;
  const int64_t grid = a.persist > 0 ? a.persist : nwg;
  hipLaunchKernelGGL((stage_kernel<N, SEED, POOL, BIAS, NTK, PPM>), dim3((unsigned)grid), dim3(Cfg::THREADS), lds,
                     stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int N, bool SEED, bool POOL, bool BIAS, bool NTK, int PPM>
int occ_t(int D) {
  using Cfg = KCfg<N, NTK, PPM>;
  const size_t lds = (size_t)Cfg::PPWG * slot_lds_bytes<N>(D, POOL, SEED, NTK);
  if (set_attr<N, SEED, POOL, BIAS, NTK, PPM>(lds)) return -3;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage_kernel<N, SEED, POOL, BIAS, NTK, PPM>, Cfg::THREADS,
                                                   lds) != hipSuccess)
    return -3;
  return nb;
}

template <int N, bool NTK, int PPM = 1>
int launch_n(const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s) {
  if (seed) {
    if (pool)
      return bias ? launch_t<N, true, true, true, NTK, PPM>(a, s) : launch_t<N, true, true, false, NTK, PPM>(a, s);
    return bias ? launch_t<N, true, false, true, NTK, PPM>(a, s) : launch_t<N, true, false, false, NTK, PPM>(a, s);
  }
  if (pool)
    return bias ? launch_t<N, false, true, true, NTK, PPM>(a, s) : launch_t<N, false, true, false, NTK, PPM>(a, s);
  return bias ? launch_t<N, false, false, true, NTK, PPM>(a, s) : launch_t<N, false, false, false, NTK, PPM>(a, s);
}

template <int N, bool NTK, int PPM = 1>
int occ_n(int D, bool seed, bool pool, bool bias) {
  if (seed) {
    if (pool) return bias ? occ_t<N, true, true, true, NTK, PPM>(D) : occ_t<N, true, true, false, NTK, PPM>(D);
    return bias ? occ_t<N, true, false, true, NTK, PPM>(D) : occ_t<N, true, false, false, NTK, PPM>(D);
  }
  if (pool) return bias ? occ_t<N, false, true, true, NTK, PPM>(D) : occ_t<N, false, true, false, NTK, PPM>(D);
  return bias ? occ_t<N, false, false, true, NTK, PPM>(D) : occ_t<N, false, false, false, NTK, PPM>(D);
}

}  // namespace nk
