// The 32x32 pooling stage of the Myrtle NNGP forward pass (App. A, Myrtle
// listing: [3x3 SAME conv, ReLU] blocks at 32x32, then a 2x2 average pool),
// the stage that carries almost all of the work at 32x32x3 inputs.
//
// Same sheared tile layout and pooling order as stage_kernel.h (see there):
// tile k = (ky, kx) holds entry (iy, ix) = pixel i of x against pixel
// j = ((iy + ky) mod 32, (ix + kx) mod 32) of x', one layer of a stage is a
// masked 3x3 box on a tile, and ky is swept 1, 2, ..., 31, 0 with the y part
// of the pool in registers and the x part in LDS.  What differs is the lane
// map: a segment is a 16-lane DPP row that owns tile column kx, and lane l
// of it holds the two tile columns ix0 = 2l and ix1 = 2l + 1 (all 32 rows of
// each in registers).  So
//  - the horizontal 3-tap sum of a row costs 2 VALU instructions per entry
//    instead of 3: the link between ix0 and ix1 is inside the lane, and each
//    column has one lane-shifted neighbour (a DPP operand of an FMA, the
//    row's ends reading 0);
//  - the vertical 3-tap sum shares the middle pair: rows are taken in pairs
//    (r, r + 1) with p = h(r) + h(r + 1), out(r) = p + h(r - 1) and
//    out(r + 1) = p + h(r + 2), 1.5 instructions per entry instead of 2.  A
//    pair must not straddle the seam row 32 - ky, so odd ky pair rows (1, 2),
//    (3, 4), ... and even ky pair rows (0, 1), (2, 3), ...; the sweep runs
//    two ky per iteration, one of each parity, each with its own unrolled
//    code;
//  - the x part of the pool adds the two columns of a lane in registers.
// The map is the forward NNGP's (degree-3 fit) and the seed skips the
// padding channel for inputs of at most 3 channels.  512 threads per pair
// (8 waves, two per SIMD), up to 256 registers per lane; with only two waves
// per SIMD the LDS latency is hidden by requesting each row's tables two rows
// ahead of its map.
//
// LDS per pair: x1 tables [D][32][32] float2; x2 tables [D][64][33] float2
// (rows twice so that rows r + ky are read without wrapping; each row split
// into its even columns 0, 2, ..., 32 -- column 32 repeating column 0 -- and
// its odd columns 1, ..., 31, so that the 16 lanes of a segment read 16
// consecutive words whichever parity their column jx starts at); the x-pool
// exchange [2][2][8][16 x 16] float (s32_emit); first stage only: x1 pixels
// [32][32] float4 (each row split into even and odd columns) and x2 pixels
// [64][33] float4 (as the x2 tables).  The x part of the pool needs no
// workgroup barrier: a coarse column is summed inside one wave but for one
// term from the wave before, passed through LDS under per-wave flags (one
// barrier per coarse row, even a single one, cost 5 % here: the waves'
// drift over two ky steps).  Plain row-major rows would put the lanes of a segment 16 or
// 32 bytes apart and cost LDS bank conflicts.
#include "stage_kernel.h"

namespace nk {

namespace {

constexpr int kN = 32, kH = 16, kThreads = 512, kP = 33;  // kP: padded row of the x2 arrays

__host__ __device__ constexpr size_t s32_t1_bytes(int D) { return (size_t)D * kN * kN * 8; }
__host__ __device__ constexpr size_t s32_t2_bytes(int D) { return (size_t)D * 2 * kN * kP * 8; }
// x-pool exchange (emit without a workgroup barrier): per buffer (two, by
// parity of the emit), per wave, a 16 x 16 block [I][lane] of the coarse row
// for `part` (one coarse column less its cross-wave third) and one for
// `carry` (that third, for the next wave); then per wave a [8][16] staging
// block through which 16-lane rows of results leave as float4 stores of
// whole waves.
constexpr int kWaves = kThreads / 64;
constexpr int kStage = 8 * kH;  // floats of one wave's staging block
__host__ __device__ constexpr size_t s32_xfer_bytes() {
  return (size_t)2 * 2 * kWaves * kH * kH * 4 + (size_t)kWaves * kStage * 4;
}
__host__ __device__ constexpr size_t s32_lds_bytes(int D, bool seed) {
  return s32_t1_bytes(D) + s32_t2_bytes(D) + s32_xfer_bytes() +
         (seed ? (size_t)kN * kN * 16 + (size_t)2 * kN * kP * 16 : 0);
}

// Horizontal masked 3-sums of one row of the lane's two columns,
//   h0 = x0 + x1 mM + x1(lane - 1) mL,   h1 = x1 + x0 mM + x0(lane + 1) mR,
// the lane shifts inside the segment's 16-lane DPP row (0 at its ends).  The
// two plain FMAs come first: they are the two wait states a DPP source needs
// after a VALU write to it.
__device__ __forceinline__ void hsum2(float x0, float x1, float mL, float mM, float mR, float& h0, float& h1) {
  asm("v_fma_f32 %0, %3, %4, %2\n\t"
      "v_fma_f32 %1, %2, %4, %3\n\t"
      "v_fmac_f32_dpp %0, %3, %5 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %2, %6 row_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=&v"(h0), "=&v"(h1)
      : "v"(x0), "v"(x1), "v"(mM), "v"(mL), "v"(mR));
}

// Position of column col of a split row: even columns first (col / 2), then
// the odd ones (17 + col / 2).
__host__ __device__ constexpr int split_col(int col) { return (col & 1) ? kH + 1 + (col >> 1) : (col >> 1); }

// The ReLU map of the two entries of row r (tables: a = (alpha, beta) of
// pixels ix0, ix1 of x; b0, b1 = those of pixels jx, jx + 1 of x').
template <bool SIGNED, bool BIAS>
__device__ __forceinline__ void map2(float v0, float v1, float4 a, float2 b0, float2 b1, float sb2, float& o0,
                                     float& o1) {
  if (BIAS) {
    v0 += sb2;
    v1 += sb2;
  }
  const float rr0 = a.x * b0.x, rr1 = a.z * b1.x;
  const float J0 = SIGNED ? j1_signed_vr3(v0, rr0) : j1_nonneg3(v0 * rr0);
  const float J1 = SIGNED ? j1_signed_vr3(v1, rr1) : j1_nonneg3(v1 * rr1);
  o0 = (a.y * b0.y) * J0;
  o1 = (a.w * b1.y) * J1;
}

// One [3x3 conv, ReLU] layer on the lane's two columns, in place.  PAR is the
// parity of the seam row (the row pairs start at PAR); seam < 0: no seam.
// c2 and c2b point at columns jx and jx + 1 of row ky of the split x2 tables.
template <int PAR, bool SIGNED, bool BIAS>
__device__ __forceinline__ void layer2(float (&A0)[kN], float (&A1)[kN], const float4* __restrict__ c1,
                                       const float2* __restrict__ c2, const float2* __restrict__ c2b, int seam,
                                       float mL, float mM, float mR, float sb2) {
  float h0[kN], h1[kN];  // (registers: each row's h is consumed two rows later)
  // The tables of row r + 2 are requested before row r is computed: at two
  // waves per SIMD the LDS latency is not hidden by other waves alone.
  float4 ta[kN];
  float2 tb0[kN], tb1[kN];
  auto load_row = [&](int r) {
    ta[r] = c1[r * (kN / 2)];
    tb0[r] = c2[r * kP];
    tb1[r] = c2b[r * kP];
  };
  load_row(0);
  load_row(1);
  auto out_row = [&](int r, float v0, float v1) {
    if (r + 2 < kN) load_row(r + 2);
    asm volatile("" ::: "memory");
    map2<SIGNED, BIAS>(v0, v1, ta[r], tb0[r], tb1[r], sb2, A0[r], A1[r]);
  };
  hsum2(A0[0], A1[0], mL, mM, mR, h0[0], h1[0]);
  hsum2(A0[1], A1[1], mL, mM, mR, h0[1], h1[1]);
  if constexpr (PAR == 1) {
    // row 0 alone: its upper neighbour is off the image
    {
      const float md = uniform_mask(seam == 1);
      out_row(0, __builtin_fmaf(md, h0[1], h0[0]), __builtin_fmaf(md, h1[1], h1[0]));
    }
#pragma unroll
    for (int r = 1; r + 1 < kN; r += 2) {
      hsum2(A0[r + 1], A1[r + 1], mL, mM, mR, h0[r + 1], h1[r + 1]);
      if (r + 2 < kN) hsum2(A0[r + 2], A1[r + 2], mL, mM, mR, h0[r + 2], h1[r + 2]);
      const float p0 = h0[r] + h0[r + 1], p1 = h1[r] + h1[r + 1];
      const float mu = uniform_mask(seam == r), md = uniform_mask(seam == r + 2);
      out_row(r, __builtin_fmaf(mu, h0[r - 1], p0), __builtin_fmaf(mu, h1[r - 1], p1));
      if (r + 2 < kN)
        out_row(r + 1, __builtin_fmaf(md, h0[r + 2], p0), __builtin_fmaf(md, h1[r + 2], p1));
      else
        out_row(r + 1, p0, p1);
    }
    {
      // row 31 alone: its lower neighbour is off the image
      const float mu = uniform_mask(seam == kN - 1);
      out_row(kN - 1, __builtin_fmaf(mu, h0[kN - 2], h0[kN - 1]), __builtin_fmaf(mu, h1[kN - 2], h1[kN - 1]));
    }
  } else {
#pragma unroll
    for (int r = 0; r < kN; r += 2) {
      if (r + 2 < kN) hsum2(A0[r + 2], A1[r + 2], mL, mM, mR, h0[r + 2], h1[r + 2]);
      if (r + 3 < kN) hsum2(A0[r + 3], A1[r + 3], mL, mM, mR, h0[r + 3], h1[r + 3]);
      const float p0 = h0[r] + h0[r + 1], p1 = h1[r] + h1[r + 1];
      if (r > 0) {
        const float mu = uniform_mask(seam == r);
        out_row(r, __builtin_fmaf(mu, h0[r - 1], p0), __builtin_fmaf(mu, h1[r - 1], p1));
      } else {
        out_row(r, p0, p1);
      }
      if (r + 2 < kN) {
        const float md = uniform_mask(seam == r + 2);
        out_row(r + 1, __builtin_fmaf(md, h0[r + 2], p0), __builtin_fmaf(md, h1[r + 2], p1));
      } else {
        out_row(r + 1, p0, p1);
      }
    }
  }
}

struct S32Ctx {
  const float2* t1;   // x1 tables
  const float2* t2;   // x2 tables (padded rows, twice)
  float* xfer;        // x-pool exchange: [part, carry][buffer][wave][16 x 16], then [wave][8 x 16] staging
  int* fprod;         // per wave: last emit whose part and carry it has written
  int* fcons;         // per wave: last emit whose carry (of the wave before) it has taken
  int* abort;         // a wait ran out (set only by a broken protocol): outputs become NaN
  const float4* img1;
  const float4* img2;
  int D, l16, seg, ix0;
  float mL, mM, mR;
  int jx0, sj0, sj1;  // x2 column jx0 and its split-row positions of columns jx0, jx0 + 1
  const float* inp;   // stage input of this pair (non-seed stages)
};

// Waits until *f >= v.  The loop is wave-uniform (one LDS word); a wait that
// runs out (only a broken protocol could make one) sets *abort, after which
// no wait blocks and the workgroup's outputs are NaN.
__device__ __forceinline__ void s32_wait(const int* f, int v, int* abort) {
  int n = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < v) {
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
    __builtin_amdgcn_s_sleep(1);
    if (++n == (1 << 20)) {
      __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      break;
    }
  }
  asm volatile("" ::: "memory");
}

// Makes this wave's earlier LDS writes (or reads) complete, then sets *f = v.
__device__ __forceinline__ void s32_publish(int* f, int v) {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The x part of the pool for coarse row Ky, without a workgroup barrier.
// Wave w holds tile columns kx = 4w + q in its four 16-lane rows q; coarse
// column Kx takes both columns of kx = 2 Kx, column ix0 (acc0) of 2 Kx + 1 and
// column ix1 (acc1) of 2 Kx - 1.  So coarse column 2w + 1 lies inside the wave
// (rows 2, 3 and the acc1 of row 1) and is summed in row 3 with two lane
// swaps and written at once; coarse column 2w lacks the acc1 of row 3 of
// wave w - 1: row 1 leaves its sum (`part`) in LDS, row 3 leaves its acc1
// (`carry`) for wave w + 1, and the column is completed one emit later
// (s32_consume).  The sums are formed in the order of a plain
// ((both + acc0) + acc1).  Buffers alternate by emit parity; before reusing
// one, a wave waits until wave w + 1 has taken its carry from two emits ago.
__device__ __forceinline__ void s32_emit(const StageArgs& args, const S32Ctx& c, const float (&acc0)[kH],
                                         const float (&acc1)[kH], const float (&dead0)[kN], const float (&dead1)[kN],
                                         int Ky, int E, bool valid, int64_t pl) {
  const int w = threadIdx.x >> 6, q = (threadIdx.x >> 4) & 3, lane = threadIdx.x & 63;
  const int b = E & 1;
  float* part = c.xfer + ((0 * 2 + b) * kWaves + w) * (kH * kH);
  float* carry = c.xfer + ((1 * 2 + b) * kWaves + w) * (kH * kH);
  float* stage = c.xfer + 2 * 2 * kWaves * (kH * kH) + w * kStage;
  if (E > 2) s32_wait(&c.fcons[(w + 1) & (kWaves - 1)], E - 2, c.abort);
  // the carry (acc1 of row 3) goes first: the swaps below clobber acc1
  if (q == 3) {
#pragma unroll
    for (int I = 0; I < kH; ++I) carry[I * kH + c.l16] = acc1[I];
  }
  float res[kH];
  const float m3 = q == 3 ? 1.f : 0.f;
  // Each swap moves the half it is asked for into the rows that need it; its
  // other operand is an even fine row of the tile, already pooled and dead
  // here, and only its first result is used, so no copies are made.
#pragma unroll
  for (int I = 0; I < kH; ++I) {
    const float u = acc0[I] + acc1[I];
    // rows 1 and 3 receive u of rows 0 and 2
    const auto pu = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, dead0[2 * I]),
                                                     __builtin_bit_cast(unsigned, u), false, false);
    // rows 2 and 3 receive acc1 of rows 0 and 1
    const auto pa = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, dead1[2 * I]),
                                                     __builtin_bit_cast(unsigned, acc1[I]), false, false);
    res[I] = __builtin_fmaf(m3, __builtin_bit_cast(float, pa[0]), __builtin_bit_cast(float, pu[0]) + acc0[I]);
  }
  if (q == 1) {
#pragma unroll
    for (int I = 0; I < kH; ++I) part[I * kH + c.l16] = res[I];
  }
  s32_publish(&c.fprod[w], E);
  // coarse column 2w + 1 (row 3) out through the staging block, half a row
  // of 16 I values at a time, as float4 stores of 32 lanes
  const bool bad = __hip_atomic_load(c.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
  float* o = args.out + pl * (int64_t)kH * kH * kH * kH + ((int64_t)Ky * kH + 2 * w + 1) * kH * kH;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (q == 3) {
#pragma unroll
      for (int I = 0; I < kH / 2; ++I) stage[I * kH + c.l16] = res[h * (kH / 2) + I];
    }
    asm volatile("" ::: "memory");
    if (lane < 32) {
      float4 v = reinterpret_cast<const float4*>(stage)[lane];
      if (bad) v = make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""));
      if (valid) reinterpret_cast<float4*>(o + h * (kH / 2) * kH)[lane] = v;
    }
    asm volatile("" ::: "memory");
  }
}

// Completes coarse column 2w of coarse row Ky (emit E): this wave's part
// plus the carry of wave w - 1 (one float4 per lane), then frees the carry
// buffer.
__device__ __forceinline__ void s32_consume(const StageArgs& args, const S32Ctx& c, int Ky, int E, bool valid,
                                            int64_t pl) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wp = (w + kWaves - 1) & (kWaves - 1);
  const int b = E & 1;
  const float4* part = reinterpret_cast<const float4*>(c.xfer + ((0 * 2 + b) * kWaves + w) * (kH * kH));
  const float4* carry = reinterpret_cast<const float4*>(c.xfer + ((1 * 2 + b) * kWaves + wp) * (kH * kH));
  s32_wait(&c.fprod[wp], E, c.abort);
  const float4 p = part[lane], r = carry[lane];
  s32_publish(&c.fcons[w], E);
  float4 v = make_float4(p.x + r.x, p.y + r.y, p.z + r.z, p.w + r.w);
  if (__hip_atomic_load(c.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
    v = make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""));
  float* o = args.out + pl * (int64_t)kH * kH * kH * kH + ((int64_t)Ky * kH + 2 * w) * kH * kH;
  if (valid) reinterpret_cast<float4*>(o)[lane] = v;
}

// One ky step: the tile's layers, the y part of the pool, and on the steps
// that complete a coarse row (E: that emit's number, counted over the
// workgroup's life from 1) the x part and the write of that row.
template <int PAR, bool SEED, bool BIAS, bool C4>
__device__ __forceinline__ void s32_step(const StageArgs& args, const S32Ctx& c, int ky, int E, float (&acc0)[kH],
                                         float (&acc1)[kH], float (&wrap0)[kH], float (&wrap1)[kH], bool valid,
                                         int64_t pl) {
  const int seam = ky == 0 ? -1 : kN - ky;
  const int kx = c.seg;
  float A0[kN], A1[kN];
  if constexpr (SEED) {
    const float4* i1 = c.img1 + c.l16;  // x1 rows split into 16 even and 16 odd columns
    const float4* i2a = c.img2 + ky * kP + c.sj0;
    const float4* i2b = c.img2 + ky * kP + c.sj1;
#pragma unroll
    for (int r = 0; r < kN; ++r) {
      const float4 u0 = i1[r * kN], u1 = i1[r * kN + kH];
      const float4 w0 = i2a[r * kP], w1 = i2b[r * kP];
      float s0 = __builtin_fmaf(u0.z, w0.z, __builtin_fmaf(u0.y, w0.y, u0.x * w0.x));
      float s1 = __builtin_fmaf(u1.z, w1.z, __builtin_fmaf(u1.y, w1.y, u1.x * w1.x));
      if (C4) {
        s0 = __builtin_fmaf(u0.w, w0.w, s0);
        s1 = __builtin_fmaf(u1.w, w1.w, s1);
      }
      else {
        // keep the padding channel live: the pixels are then read as one
        // 16-byte load each (a 12-byte load is slower here)
        asm volatile("" ::"v"(u0.w), "v"(u1.w), "v"(w0.w), "v"(w1.w));
      }
      A0[r] = s0;
      A1[r] = s1;
    }
  } else {
    const float2* p = reinterpret_cast<const float2*>(c.inp + ((int64_t)ky * kN + kx) * kN * kN + c.ix0);
#pragma unroll
    for (int r = 0; r < kN; ++r) {
      const float2 v = p[r * (kN / 2)];
      A0[r] = v.x;
      A1[r] = v.y;
    }
  }
  const float4* c1 = reinterpret_cast<const float4*>(c.t1 + c.ix0);
  const float2* c2 = c.t2 + ky * kP + c.sj0;
  const float2* c2b = c.t2 + ky * kP + c.sj1;
  int l = 0;
  if (SEED) {
    layer2<PAR, true, BIAS>(A0, A1, c1, c2, c2b, seam, c.mL, c.mM, c.mR, args.sb2);
    c1 += kN * kN / 2;
    c2 += 2 * kN * kP;
    c2b += 2 * kN * kP;
    l = 1;
  }
  for (; l < c.D; ++l) {
    layer2<PAR, false, BIAS>(A0, A1, c1, c2, c2b, seam, c.mL, c.mM, c.mR, args.sb2);
    c1 += kN * kN / 2;
    c2 += 2 * kN * kP;
    c2b += 2 * kN * kP;
  }

  // y part of the pool (coarse row I gets fine rows 2I, 2I + 1 of the tiles
  // ky = 2K and the even rows of ky = 2K + 1, odd rows of ky = 2K - 1)
  const bool emit = ky != 1 && (ky == 0 || (ky & 1));
  if (ky == 1) {
#pragma unroll
    for (int I = 0; I < kH; ++I) {
      wrap0[I] = A0[2 * I];
      wrap1[I] = A1[2 * I];
      acc0[I] = A0[2 * I + 1];
      acc1[I] = A1[2 * I + 1];
    }
  } else if (ky == 0) {
#pragma unroll
    for (int I = 0; I < kH; ++I) {
      acc0[I] = acc0[I] + (A0[2 * I] + A0[2 * I + 1]) + wrap0[I];
      acc1[I] = acc1[I] + (A1[2 * I] + A1[2 * I + 1]) + wrap1[I];
    }
  } else if ((ky & 1) == 0) {
#pragma unroll
    for (int I = 0; I < kH; ++I) {
      acc0[I] = acc0[I] + (A0[2 * I] + A0[2 * I + 1]);
      acc1[I] = acc1[I] + (A1[2 * I] + A1[2 * I + 1]);
    }
  } else {
#pragma unroll
    for (int I = 0; I < kH; ++I) {
      acc0[I] = acc0[I] + A0[2 * I];
      acc1[I] = acc1[I] + A1[2 * I];
    }
  }
  if (!emit) return;
  s32_emit(args, c, acc0, acc1, A0, A1, ky == 0 ? 0 : (ky - 1) >> 1, E, valid, pl);
  if (ky != 0) {
#pragma unroll
    for (int I = 0; I < kH; ++I) {
      acc0[I] = A0[2 * I + 1];
      acc1[I] = A1[2 * I + 1];
    }
  }
}

template <bool SEED, bool BIAS, bool C4>
__global__ __launch_bounds__(kThreads) void stage32_kernel(const StageArgs args) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ int64_t s_t1, s_t2, s_off, s_offm;
  __shared__ const float* s_x1;
  __shared__ const float* s_x2;
  __shared__ float* s_k;
  __shared__ int s_same;
  __shared__ int s_fprod[kWaves], s_fcons[kWaves], s_abort;

  const int tid = threadIdx.x;
  S32Ctx c;
  c.D = args.D;
  c.seg = tid >> 4;
  c.l16 = tid & 15;
  c.ix0 = 2 * c.l16;
  const int kx = c.seg, ix1 = c.ix0 + 1;
  c.mL = (c.ix0 >= 1 && c.ix0 != kN - kx) ? 1.f : 0.f;
  c.mM = (ix1 != kN - kx) ? 1.f : 0.f;
  c.mR = (ix1 + 1 < kN && ix1 + 1 != kN - kx) ? 1.f : 0.f;
  c.jx0 = (c.ix0 + kx) & (kN - 1);
  c.sj0 = split_col(c.jx0);
  c.sj1 = split_col(c.jx0 + 1);
  const int TL = c.D * kN * kN;
  char* base = smem;
  c.t1 = reinterpret_cast<const float2*>(base);
  c.t2 = reinterpret_cast<const float2*>(base + s32_t1_bytes(c.D));
  c.xfer = reinterpret_cast<float*>(base + s32_t1_bytes(c.D) + s32_t2_bytes(c.D));
  c.fprod = s_fprod;
  c.fcons = s_fcons;
  c.abort = &s_abort;
  if (tid < kWaves) {
    s_fprod[tid] = 0;
    s_fcons[tid] = 0;
    if (tid == 0) s_abort = 0;
  }
  c.img1 = reinterpret_cast<const float4*>(base + s32_t1_bytes(c.D) + s32_t2_bytes(c.D) + s32_xfer_bytes());
  c.img2 = c.img1 + kN * kN;
  float2* t1w = reinterpret_cast<float2*>(base);
  float2* t2w = reinterpret_cast<float2*>(base + s32_t1_bytes(c.D));
  float4* i1w = const_cast<float4*>(c.img1);
  float4* i2w = const_cast<float4*>(c.img2);

  const int64_t nunits = args.np;
  int E0 = 0;  // emits of the units before this one
  int64_t unit, ustep, uend;
  unit_range(nunits, args.persist, &unit, &ustep, &uend);
  for (; unit < uend; unit += ustep) {
    if (tid == 0) {
      int64_t pl = unit < args.np ? unit : args.np - 1;
      resolve_pair(args, args.p0 + pl, args.img_floats, &s_t1, &s_t2, &s_x1, &s_x2, &s_k, &s_off, &s_offm, &s_same,
                   false);
    }
    __syncthreads();
    // tables -> LDS: x2's rows twice and its column 0 again at column 32
    {
      const float2* g1 = args.tab1 + s_t1 * args.tablen + args.taboff;
      const float2* g2 = args.tab2 + s_t2 * args.tablen + args.taboff;
      for (int e = tid; e < TL; e += kThreads) {
        t1w[e] = g1[e];
        const float2 v = g2[e];
        const int l = e >> 10, r = (e >> 5) & (kN - 1), col = e & (kN - 1);
        float2* d = t2w + l * 2 * kN * kP + r * kP;
        d[split_col(col)] = v;
        d[kN * kP + split_col(col)] = v;
        if (col == 0) {
          d[split_col(kN)] = v;
          d[kN * kP + split_col(kN)] = v;
        }
      }
    }
    if (SEED) {
      // pixels as float4 (channels zero padded); the seed scale rides on x2
      const float sc = args.seed_scale;
      for (int px = tid; px < kN * kN; px += kThreads) {
        const float* p1 = s_x1 + px * args.C;
        const float* p2 = s_x2 + px * args.C;
        float u[4] = {0.f, 0.f, 0.f, 0.f}, w[4] = {0.f, 0.f, 0.f, 0.f};
        for (int ch = 0; ch < args.C && ch < 4; ++ch) {
          u[ch] = p1[ch];
          w[ch] = sc * p2[ch];
        }
        const int r = px >> 5, col = px & (kN - 1);
        i1w[r * kN + (col & 1) * kH + (col >> 1)] = make_float4(u[0], u[1], u[2], u[3]);
        const float4 ws = make_float4(w[0], w[1], w[2], w[3]);
        float4* d = i2w + r * kP;
        d[split_col(col)] = ws;
        d[kN * kP + split_col(col)] = ws;
        if (col == 0) {
          d[split_col(kN)] = ws;
          d[kN * kP + split_col(kN)] = ws;
        }
      }
    }
    __syncthreads();

    const int64_t pl = unit;
    const bool valid = pl < args.np;
    const int64_t plc = valid ? pl : args.np - 1;
    c.inp = SEED ? nullptr : args.in + plc * (int64_t)kN * kN * kN * kN;
    float acc0[kH], acc1[kH], wrap0[kH], wrap1[kH];
#pragma unroll
    for (int I = 0; I < kH; ++I) acc0[I] = acc1[I] = wrap0[I] = wrap1[I] = 0.f;
    // ky = 1, 2, ..., 31, 0 in pairs (odd ky: seam row 32 - ky odd; even ky:
    // even or none).  Emits: ky = 2t + 1 (t >= 1) is emit E0 + t of coarse
    // row t, ky = 0 emit E0 + 16 of coarse row 0; each is completed after
    // the next one.
#pragma unroll 1
    for (int t = 0; t < kN / 2; ++t) {
      s32_step<1, SEED, BIAS, C4>(args, c, 2 * t + 1, E0 + t, acc0, acc1, wrap0, wrap1, valid, pl);
      if (t >= 2) s32_consume(args, c, t - 1, E0 + t - 1, valid, pl);
      s32_step<0, SEED, BIAS, C4>(args, c, (2 * t + 2) & (kN - 1), E0 + kH, acc0, acc1, wrap0, wrap1, valid, pl);
    }
    s32_consume(args, c, kH - 1, E0 + kH - 1, valid, pl);
    s32_consume(args, c, 0, E0 + kH, valid, pl);
    E0 += kH;
    __syncthreads();  // LDS is reused by the next unit
  }
}

template <bool SEED, bool BIAS, bool C4>
int s32_attr(size_t lds) {
  static std::atomic<size_t> seen[kMaxDevices];
  return allow_dyn_lds((const void*)stage32_kernel<SEED, BIAS, C4>, lds, seen);
}

template <bool SEED, bool BIAS, bool C4>
int s32_launch(const StageArgs& a, hipStream_t stream) {
  const size_t lds = s32_lds_bytes(a.D, SEED);
  if (s32_attr<SEED, BIAS, C4>(lds)) return -3;
  const int64_t grid = a.persist > 0 ? a.persist : a.np;
  hipLaunchKernelGGL((stage32_kernel<SEED, BIAS, C4>), dim3((unsigned)grid), dim3(kThreads), lds, stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <bool SEED, bool BIAS, bool C4>
int s32_occ(int D) {
  const size_t lds = s32_lds_bytes(D, SEED);
  if (s32_attr<SEED, BIAS, C4>(lds)) return -3;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stage32_kernel<SEED, BIAS, C4>, kThreads, lds) != hipSuccess)
    return -3;
  return nb;
}

}  // namespace

size_t stage32_lds_bytes(int D, bool seed) { return s32_lds_bytes(D, seed); }

int launch_stage32(const StageArgs& a, bool seed, bool bias, hipStream_t s) {
  const bool c4 = a.C > 3;
  if (seed) {
    if (bias) return c4 ? s32_launch<true, true, true>(a, s) : s32_launch<true, true, false>(a, s);
    return c4 ? s32_launch<true, false, true>(a, s) : s32_launch<true, false, false>(a, s);
  }
  return bias ? s32_launch<false, true, false>(a, s) : s32_launch<false, false, false>(a, s);
}

int stage32_occupancy(int D, bool seed, bool bias, int C) {
  const bool c4 = C > 3;
  if (seed) {
    if (bias) return c4 ? s32_occ<true, true, true>(D) : s32_occ<true, true, false>(D);
    return c4 ? s32_occ<true, false, true>(D) : s32_occ<true, false, false>(D);
  }
  return bias ? s32_occ<false, true, false>(D) : s32_occ<false, false, false>(D);
}

}  // namespace nk
