// Adjoint stage kernel of the Myrtle NNGP for cross pairs: reverse mode of
// one stage of stage.hip, templated on the tile side N, the number of
// [conv, ReLU] layers D of the stage and (first stage only) the number of
// image channels CC.
//
// The forward state is not stored: each tile re-runs the stage from its
// input (the seed, or the pooled input that the forward stage kernels write
// into the chunk buffers), layer by layer.  On the kernel's own variables
//   rho = (v + sigma_b2) alpha(i) alpha'(j),  out = beta(i) beta'(j) J1(rho),
// with output adjoint g the reverse step is
//   rho_bar = g beta beta' J1'(rho),  v_bar = rho_bar alpha alpha',
//   input_bar = box(v_bar)                       (the box is self-adjoint),
// and the table adjoints reduce to one number per entry,
//   w = g out - rho_bar rho,
// summed over j onto pixel i of x and over i onto pixel j of x' (since
// alpha = q^{-1/2} and beta = (q kappa / 2)^{1/2}, the variance map then
// receives q_bar = sum w / (2 q)).  The seed adjoint gives the image
// gradients, x_bar(i) = s sum_j G(i, j) x'(j) and x'_bar(j) = s sum_i G(i, j) x(i).
//
// Accumulation.  A segment of lanes owns one tile column kx at a time and
// sweeps ky; a lane owns the rows [row0, row0 + RPL) of its column ix.  In
// the sheared layout entry (r, ix) of tile (ky, kx) is pixel i = (r, ix) of x
// and pixel j = (r + ky, ix + kx) mod N of x'.  So the i-sums stay in fixed
// registers, and the j-sums are kept in registers of a frame that follows the
// sweep: after each ky step the j-accumulators move up one row, after each
// column one lane left.  No atomics are issued per entry (LDS float atomics
// are slow on this chip); the per-lane partial sums of the segments of one
// pair are combined once at the end, in registers inside a wave and in LDS
// across waves, and added to the float64 per-image sums in global memory.
#pragma once
#include "nk_tile.h"

namespace nk {

// Workgroup shape of the adjoint.  At N = 32 a tile column is split over two
// 32-lane halves of a wave (16 rows each); otherwise a segment of N lanes
// holds whole columns.  WIDE (N = 32 only): eight segments of four columns
// per pair instead of four of eight, so that the one pair's workgroup has two
// waves on each SIMD (for kernels whose registers fit in 256 per lane).
template <int N, bool WIDE = false>
struct BCfg {
  static_assert(!WIDE || N == 32, "the wide shape is for 32 x 32 tiles");
  static constexpr int RS = (N == 32) ? 2 : 1;   // lane groups a column's rows are split over
  static constexpr int RPL = N / RS;             // rows per lane
  static constexpr int LPS = N * RS;             // lanes per segment
  static constexpr int SPP = (N == 32) ? (WIDE ? 8 : 4) : N;  // segments per pair
  static constexpr int CPS = N / SPP;            // tile columns per segment
  static constexpr int TPP = SPP * LPS;          // threads per pair
  static constexpr int THREADS = TPP > 256 ? TPP : 256;
  static constexpr int PPWG = THREADS / TPP;     // pairs per workgroup
  static constexpr int SPAN = TPP < 64 ? TPP : 64;  // lanes of one pair inside a wave
  static constexpr int WPP = TPP > 64 ? TPP / 64 : 1;  // waves per pair
};

// LDS per pair: tables x1 [D N^2 float2], tables x2 with rows twice
// [2 D N^2 float2], images as float4 (first stage: x1, then x2 with its rows
// twice, so that its rows are read without wrapping).  After the sweep the
// same bytes hold the combined sums [w1: D N^2][w2: D N^2][xbar1: N^2 C][xbar2: N^2 C].
template <int N>
__host__ __device__ constexpr size_t bwd_slot_lds_bytes(int D, bool seed) {
  return (((size_t)D * N * N * 24 + (seed ? (size_t)N * N * 48 : 0)) + 16 + 15) & ~(size_t)15;
}

// Exchange between the two 32-lane halves of a wave (one VALU instruction,
// v_permlane32_swap, instead of a round trip through the LDS crossbar).  The
// instruction swaps the upper 32 lanes of its first operand with the lower
// 32 lanes of its second, so lane l < 32 gets x(l + 32) and lane l >= 32
// gets y(l - 32).
__device__ __forceinline__ float halves_swap(float x, float y, int part) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                  false, false);
  return __builtin_bit_cast(float, part ? r[0] : r[1]);
}

// h-values of the rows just outside this lane's rows (the row above the first
// and the one below the last), from the other half of the column.
template <int N, int RS>
__device__ __forceinline__ void edge_rows(float hfirst, float hlast, int part, float& hup, float& hdn) {
  if constexpr (RS == 1) {
    hup = 0.f;
    hdn = 0.f;
  } else {
    static_assert(N == 32, "the two row halves of a column are the two halves of a wave");
    // upper half: the lower half's last row; lower half: the upper half's first row
    const float recv = halves_swap(hfirst, hlast, part);
    hup = part ? recv : 0.f;
    hdn = part ? 0.f : recv;
  }
}

// 0/1 factor of the vertical link between local rows rr - 1 and rr; the link
// is cut at local row `cut` (the seam of the sheared tile).
template <int RS>
__device__ __forceinline__ float link(int rr, int cut) {
  if constexpr (RS == 1) return uniform_mask(rr == cut);
  return rr == cut ? 0.f : 1.f;
}

// Vertical 3-sum of the masked horizontal 3-sums of this lane's rows; calls
// f(rr, v) for each row in order (f may overwrite row rr of X).
template <int N, int RS, int RPL, class F>
__device__ __forceinline__ void box_rows(const float (&X)[RPL], int cut, int part, float mL, float mR, F&& f) {
  const float hf = hsum3(X[0], mL, mR);
  const float hl = hsum3(X[RPL - 1], mL, mR);
  float hup, hdn;
  edge_rows<N, RS>(hf, hl, part, hup, hdn);
  float hm = hup;
  float h0 = hf;
#pragma unroll
  for (int rr = 0; rr < RPL; ++rr) {
    float hp;
    if (rr + 1 == RPL)
      hp = hdn;
    else if (rr + 2 == RPL)
      hp = hl;
    else
      hp = hsum3(X[rr + 1], mL, mR);
    float v = h0;
    if (RS > 1 || rr > 0) v = __builtin_fmaf(link<RS>(rr, cut), hm, v);
    if (RS > 1 || rr + 1 < RPL) v = __builtin_fmaf(link<RS>(rr + 1, cut), hp, v);
    f(rr, v);
    hm = h0;
    h0 = hp;
  }
}

// The tables of this lane's rows, each requested two rows before its use:
// at one or two waves per SIMD little else hides the LDS latency.  (The compiler
// barrier keeps each request ahead of the row it runs before.)
template <int N, int RPL>
struct RowTables {
  float2 a[RPL], b[RPL];
  const float2* c1;
  const float2* c2;
  __device__ __forceinline__ RowTables(const float2* p1, const float2* p2) : c1(p1), c2(p2) {
    fetch(0);
    if (RPL > 1) fetch(1);
  }
  __device__ __forceinline__ void fetch(int rr) {
    a[rr] = c1[rr * N];
    b[rr] = c2[rr * N];
  }
  // before row rr is computed
  __device__ __forceinline__ void advance(int rr) {
    if (rr + 2 < RPL) fetch(rr + 2);
    asm volatile("" ::: "memory");
  }
};

// Forward [3x3 conv, ReLU] layer on this lane's rows (recompute); BIAS:
// sigma_b2 != 0 (else its add is left out).
template <int N, int RS, int RPL, bool SGN, bool BIAS>
__device__ __forceinline__ void bwd_layer_fwd(float (&A)[RPL], const float2* __restrict__ c1,
                                              const float2* __restrict__ c2, int cut, int part, float mL, float mR,
                                              float sb2) {
  RowTables<N, RPL> t(c1, c2);
  box_rows<N, RS, RPL>(A, cut, part, mL, mR, [&](int rr, float v) {
    t.advance(rr);
    const float2 a = t.a[rr];
    const float2 b = t.b[rr];
    const float rho = (BIAS ? v + sb2 : v) * (a.x * b.x);
    A[rr] = (a.y * b.y) * (SGN ? j1_signed(rho) : j1_nonneg(rho));
  });
}

// Reverse of one layer: A holds the layer input, G the adjoint of the layer
// output on entry and v_bar on return; w is added to the i- and j-sums.
// J1'(rho) = 1 - acos(rho) / pi has an infinite slope at rho = 1, so a
// float32 rho rounded by 1e-7 would move it by about 1e-4 where rho is 1
// exactly: on the displacement-0 tile of a pair of identical images the
// caller passes umax = 0, which pins u = 1 - rho to 0 there (umax = 1
// elsewhere: the plain clamp).
template <int N, int RS, int RPL, bool SGN, bool BIAS>
__device__ __forceinline__ void bwd_layer_rev(const float (&A)[RPL], float (&G)[RPL], const float2* __restrict__ c1,
                                              const float2* __restrict__ c2, int cut, int part, float mL, float mR,
                                              float sb2, float umax, float (&Wi)[RPL], float (&Wj)[RPL], float& sw,
                                              float& sb) {
  RowTables<N, RPL> t(c1, c2);
  box_rows<N, RS, RPL>(A, cut, part, mL, mR, [&](int rr, float v) {
    t.advance(rr);
    const float2 a = t.a[rr];
    const float2 b = t.b[rr];
    const float rr_ = a.x * b.x, ss = a.y * b.y;
    const float rho = (BIAS ? v + sb2 : v) * rr_;
    const float arho = SGN ? __builtin_fabsf(rho) : rho;
    const float u = __builtin_amdgcn_fmed3f(1.0f - arho, 0.0f, umax);
    const float sq = __builtin_amdgcn_sqrtf(u);
    const float J = __builtin_fmaf(u * sq, relu_poly(u), SGN ? __builtin_fmaxf(rho, 0.0f) : rho);
    const float th = sq * acos_g_pi5(u);  // acos(|rho|) / pi
    const float Jp = (SGN && rho < 0.f) ? th : 1.0f - th;
    // with gs = g beta beta': g out = gs J, rho_bar = gs J', w = gs (J - J' rho)
    const float gs = G[rr] * ss;
    const float rhob = gs * Jp;
    const float vb = rhob * rr_;
    const float w = gs * __builtin_fmaf(-Jp, rho, J);
    Wi[rr] += w;
    Wj[rr] += w;
    sw = __builtin_fmaf(gs, J, sw);
    sb += vb;
    G[rr] = vb;
  });
}

// In-place box of the adjoint (the conv's linear part is self-adjoint).
// (in place: box_rows has read rows rr - 1 .. rr + 1 before f(rr) writes row rr)
template <int N, int RS, int RPL>
__device__ __forceinline__ void bwd_box(float (&G)[RPL], int cut, int part, float mL, float mR) {
  box_rows<N, RS, RPL>(G, cut, part, mL, mR, [&](int rr, float v) { G[rr] = v; });
}

// j-frame accumulators one row up (after a ky step): row rr takes row rr + 1,
// the last row takes the first row of the next lane group (cyclically).
template <int N, int RS, int RPL>
__device__ __forceinline__ void rot_rows(float (&A)[RPL], int part) {
  const float first = RS == 1 ? A[0] : halves_swap(A[0], A[0], part);
#pragma unroll
  for (int rr = 0; rr + 1 < RPL; ++rr) A[rr] = A[rr + 1];
  A[RPL - 1] = first;
}

template <int RPL>
__device__ __forceinline__ void take_lane(float (&A)[RPL], int src) {
#pragma unroll
  for (int rr = 0; rr < RPL; ++rr) A[rr] = __shfl(A[rr], src);
}

// Sum over the segments of one pair inside a wave (they share the frame).
template <int N, int RPL>
__device__ __forceinline__ void seg_reduce(float (&A)[RPL]) {
  constexpr int LPS = BCfg<N>::LPS, SPAN = BCfg<N>::SPAN;
#pragma unroll
  for (int off = LPS; off < SPAN; off <<= 1)
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) A[rr] += __shfl_xor(A[rr], off);
}

// Waves per SIMD to compile for: the live registers of a lane are about
// RPL (2 + 2 D + 2 CC) (tile, adjoint and the four kinds of sums) plus ~80
// of addresses and temporaries.  Without this bound the compiler would take
// a 256-thread workgroup as licence to use all 512 registers for one wave.
// At N = 32 a kernel whose registers fit in 256 (RPL (3 + 2 D + CC + CJ), the
// above with the kept stage input and only the j-side seed sums it keeps, at
// most 160) takes the wide shape and two waves per SIMD.
template <int N, int D, int CC, bool XJ>
struct BOcc {
  static constexpr int CJ = XJ ? CC : 0;
  static constexpr bool WIDE = N == 32 && BCfg<N>::RPL * (3 + 2 * D + CC + CJ) <= 160;
  static constexpr int est = BCfg<N>::RPL * (2 + 2 * D + 2 * CC) + 80;
  static constexpr int W = WIDE ? 2 : (512 / est < 1 ? 1 : (512 / est > 8 ? 8 : 512 / est));
  static constexpr int THREADS = BCfg<N, WIDE>::THREADS;
};

// XJ: accumulate the second image's seed gradients (the j-side sums, which
// follow the sweep in a rotating frame); without them (args.xj = 0, callers
// that need no gradient for x2) the lane keeps 48 fewer registers at C = 3.
// BIAS: sigma_b2 != 0.
template <int N, int D, int CC, bool XJ, bool BIAS>
__global__ __launch_bounds__((BOcc<N, D, CC, XJ>::THREADS))
__attribute__((amdgpu_waves_per_eu(BOcc<N, D, CC, XJ>::W)))
void stage_bwd_kernel(const StageBwdArgs args) {
  using B = BCfg<N, BOcc<N, D, CC, XJ>::WIDE>;
  constexpr bool SEED = CC > 0;
  constexpr int RS = B::RS, RPL = B::RPL, LPS = B::LPS, CPS = B::CPS, TPP = B::TPP, PPWG = B::PPWG;
  constexpr int THREADS = B::THREADS, SPAN = B::SPAN, WPP = B::WPP;
  constexpr int NN = N * N, TL = D * NN, H = N / 2;
  constexpr int DA = D > 0 ? D : 1, CA = CC > 0 ? CC : 1;
  constexpr int CJ = XJ ? CC : 0, CJA = CJ > 0 ? CJ : 1;  // j-side seed sums kept
  constexpr size_t SLOT = bwd_slot_lds_bytes<N>(D, SEED);
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ int64_t s_pa[PPWG], s_pb[PPWG];
  __shared__ double s_sum[PPWG][2];
  __shared__ int s_same[PPWG];
  __shared__ const float* s_x1[PPWG];
  __shared__ const float* s_x2[PPWG];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int slot = tid / TPP;
  const int within = tid - slot * TPP;
  const int seg = within / LPS, lis = within - seg * LPS;
  const int part = lis / N, ix = lis - part * N;
  const int row0 = part * RPL;

  const int64_t wg = xcd_logical_block();
  if (tid < PPWG) {
    int64_t pl = wg * PPWG + tid;
    if (pl >= args.np) pl = args.np - 1;
    int64_t a, b;
    pair_of(args.p0 + pl, args.n1, args.n2, args.sym, args.T, &a, &b);
    s_pa[tid] = a;
    s_pb[tid] = b;
    s_sum[tid][0] = 0.0;
    s_sum[tid][1] = 0.0;
    s_x1[tid] = args.x1 + a * args.img_floats;
    s_x2[tid] = args.x2 + b * args.img_floats;
    s_same[tid] = (args.sym && a == b) ? 1 : (s_x1[tid][0] == s_x2[tid][0] ? 2 : 0);
  }
  __syncthreads();
  identical_pairs<PPWG, THREADS>(s_same, s_x1, s_x2, args.img_floats);
  char* sbase = smem + slot * SLOT;
  float2* t1 = reinterpret_cast<float2*>(sbase);
  float2* t2 = t1 + TL;
  float4* img1 = reinterpret_cast<float4*>(t2 + 2 * TL);
  float4* img2 = img1 + NN;

  for (int e = tid; e < PPWG * TL; e += THREADS) {
    const int s = e / TL, r = e - s * TL;
    float2* d1 = reinterpret_cast<float2*>(smem + s * SLOT);
    d1[r] = args.tab1[s_pa[s] * args.tablen + args.taboff + r];
    const float2 v = args.tab2[s_pb[s] * args.tablen + args.taboff + r];
    const int l = r / NN, rr = r - l * NN;
    float2* d2 = d1 + TL + l * 2 * NN;
    d2[rr] = v;
    d2[rr + NN] = v;
  }
  if constexpr (SEED) {
    for (int e = tid; e < PPWG * NN; e += THREADS) {
      const int s = e / NN, px = e - s * NN;
      float4* i1 = reinterpret_cast<float4*>(reinterpret_cast<float2*>(smem + s * SLOT) + 3 * TL);
      const float* p1 = args.x1 + (s_pa[s] * (int64_t)NN + px) * CC;
      const float* p2 = args.x2 + (s_pb[s] * (int64_t)NN + px) * CC;
      float u[4] = {0.f, 0.f, 0.f, 0.f}, w[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        u[c] = p1[c];
        w[c] = p2[c];
      }
      i1[px] = make_float4(u[0], u[1], u[2], u[3]);
      i1[NN + px] = make_float4(w[0], w[1], w[2], w[3]);
      i1[2 * NN + px] = make_float4(w[0], w[1], w[2], w[3]);
    }
  }
  __syncthreads();

  const int64_t pl = wg * PPWG + slot;
  const bool valid = pl < args.np;
  const int64_t pa = s_pa[slot], pb = s_pb[slot];
  const int64_t plc = valid ? pl : args.np - 1;
  const bool last = args.last != 0;

  // A slot past the chunk end re-runs the last pair of the chunk (pa, pb
  // and plc are clamped) with the same cotangent, so whatever it writes to
  // the chunk buffers equals what the owning slot writes; its sums are dropped.
  float gpair = 0.f;
  if (last) {
    // (dk_t: the block's cotangent is stored transposed, [x2 row][x1 row])
    gpair = args.dk_t ? args.dK[pb * args.lddk + pa] : args.dK[pa * args.lddk + pb];
    if (args.sym && pa != pb) gpair += args.dK[pb * args.lddk + pa];
  }

  float Wi[DA][RPL], Wj[DA][RPL], Xi[CA][RPL], Xj[CJA][RPL];
#pragma unroll
  for (int rr = 0; rr < RPL; ++rr) {
#pragma unroll
    for (int l = 0; l < DA; ++l) Wi[l][rr] = Wj[l][rr] = 0.f;
#pragma unroll
    for (int c = 0; c < CA; ++c) Xi[c][rr] = 0.f;
#pragma unroll
    for (int c = 0; c < CJA; ++c) Xj[c][rr] = 0.f;
  }
  const float sb2 = args.sb2, ssd = args.seed_scale;
  double swd = 0.0, sbd = 0.0;
#pragma unroll 1
  for (int cc = 0; cc < CPS; ++cc) {
    const int kx = seg * CPS + cc;
    if (cc > 0) {
      // next column: lane ix takes the j-sums of lane ix + 1
      const int src = (lane & ~(N - 1)) | ((ix + 1) & (N - 1));
#pragma unroll
      for (int l = 0; l < D; ++l) take_lane<RPL>(Wj[l], src);
#pragma unroll
      for (int c = 0; c < CJ; ++c) take_lane<RPL>(Xj[c], src);
    }
    const float mL = (ix >= 1 && ix != N - kx) ? 1.f : 0.f;
    const float mR = (ix + 1 < N && ix + 1 != N - kx) ? 1.f : 0.f;
    const int jx = (ix + kx) & (N - 1);
    const float* inp = SEED ? nullptr : args.in + plc * (int64_t)NN * NN + (int64_t)kx * NN + row0 * N + ix;
#pragma unroll 1
    for (int ky = 0; ky < N; ++ky) {
      const int cut = (ky == 0 ? -N : N - ky) - row0;
      // displacement-0 tile of a pair of identical images: rho = 1 exactly
      const float umax = (s_same[slot] == 1 && ky == 0 && kx == 0) ? 0.f : 1.f;
      float A[RPL], G[RPL];
      // Every read of the LDS images and tables below goes through an
      // opaque offset, so that repeated reads of one address in the layer
      // loop are re-issued rather than kept live in registers across it.
      auto load_input = [&](float (&X)[RPL]) {
        if constexpr (SEED) {
          // (row bases formed once: the rows are then constant offsets)
          const int z = opaque_zero();
          const float4* im1 = img1 + z + row0 * N + ix;
          const float4* im2 = img2 + z + (row0 + ky) * N + jx;
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr) {
            const float4 u = im1[rr * N];
            const float4 w = im2[rr * N];
            X[rr] = ssd * __builtin_fmaf(u.w, w.w, __builtin_fmaf(u.z, w.z, __builtin_fmaf(u.y, w.y, u.x * w.x)));
          }
        } else {
          const float* q = inp + (int64_t)ky * N * NN;
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr) X[rr] = q[rr * N];
        }
      };
      if (last) {
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) G[rr] = gpair;
      } else {
        // pooling adjoint: fine entry (r, ix) of tile (ky, kx) reads coarse
        // tile (((ky + (r & 1)) >> 1) mod H, ((kx + (ix & 1)) >> 1) mod H), entry (r >> 1, ix >> 1)
        const float* q = args.gin + plc * (int64_t)H * H * H * H;
        const int Kx = ((kx + (ix & 1)) >> 1) & (H - 1);
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
          const int r = row0 + rr;
          const int Ky = ((ky + (r & 1)) >> 1) & (H - 1);
          G[rr] = q[(((int64_t)Ky * H + Kx) * H + (r >> 1)) * H + (ix >> 1)];
        }
      }
      float sw = 0.f, sb = 0.f;
      // the stage input, loaded once per tile and kept for the later passes
      float S[RPL];
#pragma unroll
      for (int l = D - 1; l >= 0; --l) {
        if (l == D - 1) {
          load_input(A);
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr) S[rr] = A[rr];
        } else {
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr) A[rr] = S[rr];
        }
#pragma unroll
        for (int m = 0; m < l; ++m) {
          const int z = opaque_zero();
          const float2* c1 = t1 + z + m * NN + row0 * N + ix;
          const float2* c2 = t2 + z + m * 2 * NN + (ky + row0) * N + jx;
          if (SEED && m == 0)
            bwd_layer_fwd<N, RS, RPL, true, BIAS>(A, c1, c2, cut, part, mL, mR, sb2);
          else
            bwd_layer_fwd<N, RS, RPL, false, BIAS>(A, c1, c2, cut, part, mL, mR, sb2);
        }
        const int z = opaque_zero();
        const float2* c1 = t1 + z + l * NN + row0 * N + ix;
        const float2* c2 = t2 + z + l * 2 * NN + (ky + row0) * N + jx;
        if (SEED && l == 0)
          bwd_layer_rev<N, RS, RPL, true, BIAS>(A, G, c1, c2, cut, part, mL, mR, sb2, umax, Wi[l], Wj[l], sw, sb);
        else
          bwd_layer_rev<N, RS, RPL, false, BIAS>(A, G, c1, c2, cut, part, mL, mR, sb2, umax, Wi[l], Wj[l], sw, sb);
        bwd_box<N, RS, RPL>(G, cut, part, mL, mR);
      }
      // G = adjoint of the stage input.  The seed sums are kept without the
      // seed scale s (applied once after the sweep), and the seed layer's
      // share of the sigma_w2 sum, sum over tiles of G a0 with
      // a0 = s <x(i), x'(j)>, is formed after the sweep as well:
      // s sum_c x_c(i) Xi_c(i), since pixel i of a lane row is fixed.
      if constexpr (SEED) {
        const int z = opaque_zero();
        const float4* im1 = img1 + z + row0 * N + ix;
        const float4* im2 = img2 + z + (row0 + ky) * N + jx;
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
          const float4 w = im2[rr * N];
          const float wc[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int c = 0; c < CC; ++c) Xi[c][rr] = __builtin_fmaf(G[rr], wc[c], Xi[c][rr]);
          if constexpr (XJ) {
            const float4 u = im1[rr * N];
            const float uc[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int c = 0; c < CC; ++c) Xj[c][rr] = __builtin_fmaf(G[rr], uc[c], Xj[c][rr]);
          }
        }
      } else {
        float* q = args.gout + plc * (int64_t)NN * NN + ((int64_t)ky * N + kx) * NN + row0 * N + ix;
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) q[rr * N] = G[rr];
      }
      swd += sw;
      sbd += sb;
      // j-frame follows the sweep to ky + 1
#pragma unroll
      for (int l = 0; l < D; ++l) rot_rows<N, RS, RPL>(Wj[l], part);
#pragma unroll
      for (int c = 0; c < CJ; ++c) rot_rows<N, RS, RPL>(Xj[c], part);
    }
  }
  if constexpr (SEED) {
    // the seed layer's sigma_w2 share and the seed scale of the seed sums
    const float4* im1 = img1 + row0 * N + ix;
    float t = 0.f;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
      const float4 u = im1[rr * N];
      const float uc[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int c = 0; c < CC; ++c) t = __builtin_fmaf(uc[c], Xi[c][rr], t);
    }
    swd += (double)(ssd * t);
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
#pragma unroll
      for (int c = 0; c < CC; ++c) Xi[c][rr] *= ssd;
#pragma unroll
      for (int c = 0; c < CJ; ++c) Xj[c][rr] *= ssd;
    }
  }
  // j-sums back to lane ix <-> pixel column ix (the frame is at the last column)
  {
    const int src = (lane & ~(N - 1)) | ((ix - (seg * CPS + CPS - 1)) & (N - 1));
#pragma unroll
    for (int l = 0; l < D; ++l) take_lane<RPL>(Wj[l], src);
#pragma unroll
    for (int c = 0; c < CJ; ++c) take_lane<RPL>(Xj[c], src);
  }
#pragma unroll
  for (int l = 0; l < D; ++l) {
    seg_reduce<N, RPL>(Wi[l]);
    seg_reduce<N, RPL>(Wj[l]);
  }
#pragma unroll
  for (int c = 0; c < CC; ++c) seg_reduce<N, RPL>(Xi[c]);
#pragma unroll
  for (int c = 0; c < CJ; ++c) seg_reduce<N, RPL>(Xj[c]);
  // scalars: wave sums (a slot past the chunk end re-ran a clamped pair and
  // adds nothing; such slots are the last ones of the workgroup)
  if (!valid) {
    swd = 0.0;
    sbd = 0.0;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    swd += __shfl_xor(swd, off);
    sbd += __shfl_xor(sbd, off);
  }
  __syncthreads();  // tables and images are dead from here: their bytes take the sums
  if (lane == 0) {
    atomicAdd(&s_sum[slot][0], swd);
    atomicAdd(&s_sum[slot][1], sbd);
  }
  float* aw1 = reinterpret_cast<float*>(sbase);
  float* aw2 = aw1 + TL;
  float* ax1 = aw2 + TL;
  float* ax2 = ax1 + NN * CC;
  const bool lead = (within % SPAN) < LPS;  // first segment of this pair in this wave
  const int wip = within / 64;              // wave index inside the pair (WPP > 1)
#pragma unroll
  for (int w = 0; w < WPP; ++w) {
    if (lead && (WPP == 1 || wip == w)) {
#pragma unroll
      for (int rr = 0; rr < RPL; ++rr) {
        const int px = (row0 + rr) * N + ix;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          aw1[l * NN + px] = (w == 0 ? 0.f : aw1[l * NN + px]) + Wi[l][rr];
          aw2[l * NN + px] = (w == 0 ? 0.f : aw2[l * NN + px]) + Wj[l][rr];
        }
#pragma unroll
        for (int c = 0; c < CC; ++c) ax1[px * CC + c] = (w == 0 ? 0.f : ax1[px * CC + c]) + Xi[c][rr];
#pragma unroll
        for (int c = 0; c < CJ; ++c) ax2[px * CC + c] = (w == 0 ? 0.f : ax2[px * CC + c]) + Xj[c][rr];
      }
    }
    __syncthreads();
  }
  if (!valid) return;
  for (int e = within; e < TL; e += TPP) {
    atomicAdd(&args.W1[pa * args.tablen + args.taboff + e], (double)aw1[e]);
    atomicAdd(&args.W2[pb * args.tablen + args.taboff + e], (double)aw2[e]);
  }
  if constexpr (SEED) {
    for (int e = within; e < NN * CC; e += TPP) {
      atomicAdd(&args.xbar1[pa * (int64_t)NN * CC + e], (double)ax1[e]);
      if constexpr (XJ) atomicAdd(&args.xbar2[pb * (int64_t)NN * CC + e], (double)ax2[e]);
    }
  }
  if (within == 0) {
    atomicAdd(&args.sums[0], s_sum[slot][0]);
    atomicAdd(&args.sums[1], s_sum[slot][1] + (last ? (double)gpair : 0.0));
  }
}

template <int N, int D, int CC, bool XJ, bool BIAS>
int launch_bwd_xb(const StageBwdArgs& a, hipStream_t stream) {
  using B = BCfg<N, BOcc<N, D, CC, XJ>::WIDE>;
  static_assert(B::PPWG == BCfg<N>::PPWG, "the LDS size is computed for the narrow shape");
  const int64_t nwg = (a.np + B::PPWG - 1) / B::PPWG;
  const size_t lds = (size_t)B::PPWG * bwd_slot_lds_bytes<N>(D, CC > 0);
  auto fn = stage_bwd_kernel<N, D, CC, XJ, BIAS>;
  static std::atomic<size_t> seen[kMaxDevices];  // per instantiation
  if (allow_dyn_lds((const void*)fn, lds, seen)) return -3;
  hipLaunchKernelGGL(fn, dim3((unsigned)nwg), dim3(B::THREADS), lds, stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int N, int D, int CC, bool XJ>
int launch_bwd_x(const StageBwdArgs& a, hipStream_t stream) {
  return a.sb2 != 0.f ? launch_bwd_xb<N, D, CC, XJ, true>(a, stream) : launch_bwd_xb<N, D, CC, XJ, false>(a, stream);
}

// The seed-stage kernel without the second image's seed gradients exists for
// 32x32 tiles (the adjoint's dominant case); elsewhere they are always
// accumulated, so xbar2 must then be given.
template <int N, int D, int CC>
int launch_bwd_t(const StageBwdArgs& a, hipStream_t stream) {
  if constexpr (N == 32 && CC > 0) {
    if (!a.xj) return launch_bwd_x<N, D, CC, false>(a, stream);
  } else {
    if (CC > 0 && !a.xj && !a.xbar2) return -2;
  }
  return launch_bwd_x<N, D, CC, true>(a, stream);
}

template <int N, int D>
int launch_bwd_seed_c(const StageBwdArgs& a, hipStream_t s) {
  switch (a.C) {
    case 1: return launch_bwd_t<N, D, 1>(a, s);
    case 2: return launch_bwd_t<N, D, 2>(a, s);
    case 3: return launch_bwd_t<N, D, 3>(a, s);
    case 4: return launch_bwd_t<N, D, 4>(a, s);
  }
  return -2;
}

// Seed-stage adjoints of tile side N (D = 1..4 layers, C = 1..4 channels).
template <int N>
int launch_bwd_seed(const StageBwdArgs& a, hipStream_t s) {
  switch (a.D) {
    case 1: return launch_bwd_seed_c<N, 1>(a, s);
    case 2: return launch_bwd_seed_c<N, 2>(a, s);
    case 3: return launch_bwd_seed_c<N, 3>(a, s);
    case 4: return launch_bwd_seed_c<N, 4>(a, s);
  }
  return -2;
}

// Adjoints of later stages of tile side N (D = 0..4 layers).
template <int N>
int launch_bwd_inner(const StageBwdArgs& a, hipStream_t s) {
  switch (a.D) {
    case 0: return launch_bwd_t<N, 0, 0>(a, s);
    case 1: return launch_bwd_t<N, 1, 0>(a, s);
    case 2: return launch_bwd_t<N, 2, 0>(a, s);
    case 3: return launch_bwd_t<N, 3, 0>(a, s);
    case 4: return launch_bwd_t<N, 4, 0>(a, s);
  }
  return -2;
}

}  // namespace nk
