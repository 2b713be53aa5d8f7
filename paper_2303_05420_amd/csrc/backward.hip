// Adjoint of the Myrtle NNGP (gradients with respect to the input images and
// both sigmas), hand-written reverse mode of the forward in stage.hip and
// prepare.hip.
//
// Cross pairs (stage_bwd_kernel).  The forward state is not stored: each
// stage is re-run from its input (the seed, or the pooled input the forward
// stage kernels rewrite into the chunk buffers), layer by layer from that
// checkpoint.  On the kernel's own variables
//   rho = (v + sigma_b2) alpha(i) alpha'(j),  out = beta(i) beta'(j) J1(rho),
// with output adjoint g the reverse step is
//   rho_bar = g beta beta' J1'(rho),  v_bar = rho_bar alpha alpha',
//   input_bar = box(v_bar)                       (the box is self-adjoint),
// and the table adjoints reduce to one number per entry,
//   w = g out - rho_bar rho,
// accumulated onto pixel i of x and pixel j of x': since alpha = q^{-1/2} and
// beta = (q kappa / 2)^{1/2}, the variance map receives q_bar = sum w / (2 q).
// Every scale that is proportional to sigma_w2 (conv and readout factors
// kappa, the seed scale) contributes g out / sigma_w2 to d/dsigma_w2, every
// bias term contributes v_bar to d/dsigma_b2.  J1' = 1 - acos(rho) / pi uses
// the acos fit of nk_common.h; nothing differentiates sqrt or acos at rho = 1.
//
// Self recursions (prepare_bwd_kernel, float64).  The variance maps are the
// output of the reduced self recursion of prepare.hip; it is re-run with its
// intermediate pre-activations kept, and reversed: ReLU partials
//   dF/ds = (pi - t)/(2 pi),  dF/dq = sin t sqrt(q'/q) / (4 pi)
// on the slices, the box chains of the diagonal, the pools and the seed.
#include "nk_tile.h"

namespace nk {

// Workgroup shape of the adjoint: at N = 32 a pair gets 512 threads and each
// N-lane segment reverses two tile columns in turn (the adjoint keeps three
// tile-sized arrays live and needs the larger register budget of 8 waves).
template <int N>
struct BCfg {
  static constexpr int TPP = (N == 32) ? 512 : N * N;  // threads per pair
  static constexpr int CPS = N * N / TPP;              // tile columns per segment
  static constexpr int THREADS = TPP > 256 ? TPP : 256;
  static constexpr int PPWG = THREADS / TPP;
};

// LDS per pair in the adjoint: tables as in the forward (x2 rows twice),
// images (seed stage), per-layer w accumulators for both images, seed
// gradients for both images, 2 scalars.
template <int N>
__host__ __device__ inline size_t bwd_slot_lds_bytes(int D, bool seed, int C) {
  size_t t = (size_t)D * N * N * 8 + (size_t)D * 2 * N * N * 8;
  if (seed) t += (size_t)2 * N * N * 16 + (size_t)2 * N * N * C * 4;
  t += (size_t)2 * D * N * N * 4 + 16;
  return (t + 15) & ~(size_t)15;
}

// Sum of v over the segments of this wave that belong to the same pair: the
// segments share their first-image pixel (row, lane) mapping, so their
// contributions to that pixel can be combined before one LDS atomic (atomic
// adds that hit one address from several lanes of an instruction serialise).
template <int N>
__device__ __forceinline__ float seg_sum(float v) {
  constexpr int TPP = BCfg<N>::TPP;
  constexpr int span = TPP < 64 ? TPP : 64;  // lanes of one pair inside a wave
#pragma unroll
  for (int off = N; off < span; off <<= 1) v += __shfl_xor(v, off);
  return v;
}

// reverse of one [3x3 conv, ReLU] layer; Aw holds the layer input, G the
// adjoint of the layer output on entry and of the layer input on return
// forward layer with the first-ReLU (signed) handling chosen at run time
template <int N, bool BIAS>
__device__ __forceinline__ void tile_layer_rt(float (&A)[N], const float2* __restrict__ c1,
                                              const float2* __restrict__ c2, int seam, float mL, float mR, float sb2,
                                              bool sgn) {
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
    const float rho = v * (a.x * b.x);
    const float arho = sgn ? __builtin_fabsf(rho) : rho;
    const float u = __builtin_amdgcn_fmed3f(1.0f - arho, 0.0f, 1.0f);
    const float sq = __builtin_amdgcn_sqrtf(u);
    const float J = __builtin_fmaf(u * sq, relu_poly(u), sgn ? __builtin_fmaxf(rho, 0.0f) : rho);
    A[r] = (a.y * b.y) * J;
    hm = h0;
    h0 = hp;
  }
}

template <int N, bool BIAS>
__device__ __forceinline__ void tile_layer_bwd(const float (&Aw)[N], float (&G)[N], const float2* __restrict__ c1,
                                               const float2* __restrict__ c2, int seam, float mL, float mR,
                                               float sb2, float* __restrict__ w1, float* __restrict__ w2, int ix,
                                               int jx, int ky, float& sw, float& sb, bool sgn, bool lead) {
  float hm = 0.f;
  float h0 = hsum3(Aw[0], mL, mR);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    float hp = 0.f;
    if (r + 1 < N) hp = hsum3(Aw[r + 1], mL, mR);
    float v = h0;
    if (r > 0) v = __builtin_fmaf(uniform_mask(r == seam), hm, v);
    if (r + 1 < N) v = __builtin_fmaf(uniform_mask(r + 1 == seam), hp, v);
    if (BIAS) v += sb2;
    const float2 a = c1[r * N];
    const float2 b = c2[r * N];
    const float rr = a.x * b.x, ss = a.y * b.y;
    const float rho = v * rr;
    float J, Jp;
    {
      const float arho = sgn ? __builtin_fabsf(rho) : rho;
      const float u = __builtin_amdgcn_fmed3f(1.0f - arho, 0.0f, 1.0f);
      const float sq = __builtin_amdgcn_sqrtf(u);
      const float base = sgn ? __builtin_fmaxf(rho, 0.0f) : rho;
      J = __builtin_fmaf(u * sq, relu_poly(u), base);
      const float th = sq * acos_g(u) * 0.31830988618379067f;  // acos(|rho|) / pi
      Jp = (sgn && rho < 0.f) ? th : 1.0f - th;
    }
    const float out = ss * J;
    const float gb = G[r];
    const float rhob = gb * ss * Jp;
    const float vb = rhob * rr;
    const float w = gb * out - rhob * rho;
    const float wsum = seg_sum<N>(w);
    if (lead) atomicAdd(&w1[r * N + ix], wsum);
    atomicAdd(&w2[((r + ky) & (N - 1)) * N + jx], w);
    sw = __builtin_fmaf(gb, out, sw);
    sb += vb;
    G[r] = vb;
    hm = h0;
    h0 = hp;
  }
}

template <int N, bool SEED, bool LAST, bool BIAS>
__global__ __launch_bounds__(BCfg<N>::THREADS) void stage_bwd_kernel(const StageBwdArgs args) {
  constexpr int THREADS = BCfg<N>::THREADS, PPWG = BCfg<N>::PPWG, TPP = BCfg<N>::TPP, CPS = BCfg<N>::CPS;
  constexpr int H = N / 2;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ int64_t s_pa[PPWG], s_pb[PPWG];

  const int tid = threadIdx.x;
  const int slot = tid / TPP;
  const int within = tid - slot * TPP;
  const int seg = within / N, ix = within - seg * N;
  const int D = args.D, C = args.C;
  const size_t slot_bytes = bwd_slot_lds_bytes<N>(D, SEED, C);
  const int TL = D * N * N;

  const int64_t wg = xcd_logical_block();
  if (tid < PPWG) {
    int64_t pl = wg * PPWG + tid;
    if (pl >= args.np) pl = args.np - 1;
    int64_t a, b;
    pair_of(args.p0 + pl, args.n1, args.n2, args.sym, args.T, &a, &b);
    s_pa[tid] = a;
    s_pb[tid] = b;
  }
  __syncthreads();
  char* sbase = smem + slot * slot_bytes;
  float2* t1 = reinterpret_cast<float2*>(sbase);
  float2* t2 = t1 + TL;
  char* p = reinterpret_cast<char*>(t2 + 2 * TL);
  float4* img1 = nullptr;
  float4* img2 = nullptr;
  float* xb1 = nullptr;
  float* xb2 = nullptr;
  if (SEED) {
    img1 = reinterpret_cast<float4*>(p);
    img2 = img1 + N * N;
    xb1 = reinterpret_cast<float*>(img2 + N * N);
    xb2 = xb1 + N * N * C;
    p = reinterpret_cast<char*>(xb2 + N * N * C);
  }
  float* w1 = reinterpret_cast<float*>(p);
  float* w2 = w1 + TL;
  float* scal = w2 + TL;

  for (int e = tid; e < PPWG * TL; e += THREADS) {
    const int s = e / TL, r = e - s * TL;
    char* sb = smem + s * slot_bytes;
    float2* d1 = reinterpret_cast<float2*>(sb);
    d1[r] = args.tab1[s_pa[s] * args.tablen + args.taboff + r];
    const float2 v = args.tab2[s_pb[s] * args.tablen + args.taboff + r];
    const int l = r / (N * N), rr = r - l * N * N;
    float2* d2 = d1 + TL + l * 2 * N * N;
    d2[rr] = v;
    d2[rr + N * N] = v;
  }
  // zero accumulators, load images
  for (int e = tid; e < PPWG * N * N; e += THREADS) {
    const int s = e / (N * N), px = e - s * (N * N);  // pair slot, pixel
    char* sb = smem + s * slot_bytes;
    char* q = reinterpret_cast<char*>(reinterpret_cast<float2*>(sb) + 3 * TL);
    if (SEED) {
      float4* i1 = reinterpret_cast<float4*>(q);
      float4* i2 = i1 + N * N;
      const float* p1 = args.x1 + (s_pa[s] * (int64_t)N * N + px) * C;
      const float* p2 = args.x2 + (s_pb[s] * (int64_t)N * N + px) * C;
      float u[4] = {0.f, 0.f, 0.f, 0.f}, w[4] = {0.f, 0.f, 0.f, 0.f};
      for (int c = 0; c < C && c < 4; ++c) {
        u[c] = p1[c];
        w[c] = p2[c];
      }
      i1[px] = make_float4(u[0], u[1], u[2], u[3]);
      i2[px] = make_float4(w[0], w[1], w[2], w[3]);
      float* x1b = reinterpret_cast<float*>(i2 + N * N);
      for (int c = 0; c < C; ++c) {
        x1b[px * C + c] = 0.f;
        x1b[N * N * C + px * C + c] = 0.f;
      }
      q = reinterpret_cast<char*>(x1b + 2 * N * N * C);
    }
    float* ww = reinterpret_cast<float*>(q);
    for (int l = 0; l < D; ++l) {
      ww[l * N * N + px] = 0.f;
      ww[TL + l * N * N + px] = 0.f;
    }
    if (px < 2) ww[2 * TL + px] = 0.f;
  }
  __syncthreads();

  const int64_t pl = wg * PPWG + slot;
  const bool valid = pl < args.np;
  const int64_t pa = s_pa[slot], pb = s_pb[slot];
  const int64_t plc = valid ? pl : args.np - 1;

  float gpair = 0.f;
  if (LAST && valid) {
    gpair = args.dK[pa * args.lddk + pb];
    if (args.sym && pa != pb) gpair += args.dK[pb * args.lddk + pa];
  }

  // the lowest segment of this pair inside this wave does the combined
  // first-image atomics
  const bool lead = ((tid & 63) % (TPP < 64 ? TPP : 64)) < N;
  double swd = 0.0, sbd = 0.0;
  for (int cc = 0; cc < CPS; ++cc) {
  const int kx = seg + cc * (TPP / N);
  const float mL = (ix >= 1 && ix != N - kx) ? 1.f : 0.f;
  const float mR = (ix + 1 < N && ix + 1 != N - kx) ? 1.f : 0.f;
  const int jx = (ix + kx) & (N - 1);
  const float* inp = SEED ? nullptr : args.in + plc * (int64_t)N * N * N * N + (int64_t)kx * N * N + ix;
  for (int ky = 0; ky < N; ++ky) {
    const int seam = ky == 0 ? -1 : N - ky;
    const float4* im1 = img1 + opaque_zero();
    float Aw[N], G[N];
    // stage input of this tile (recomputed / reloaded instead of kept)
    auto load_input = [&](float (&A)[N]) {
      if (SEED) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const int jy = (r + ky) & (N - 1);
          const float4 u = im1[r * N + ix];
          const float4 w = img2[jy * N + jx];
          A[r] = args.seed_scale *
                 __builtin_fmaf(u.w, w.w, __builtin_fmaf(u.z, w.z, __builtin_fmaf(u.y, w.y, u.x * w.x)));
          if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);  // bound the loads in flight
        }
      } else {
        const float* q = inp + (int64_t)ky * N * N * N;
#pragma unroll
        for (int r = 0; r < N; ++r) A[r] = q[r * N];
      }
    };
    if (LAST) {
#pragma unroll
      for (int r = 0; r < N; ++r) G[r] = gpair;
    } else {
      // pooling adjoint: fine entry (r, ix) of tile (ky, kx) -> coarse tile
      // (((ky + (r & 1)) >> 1) mod H, ((kx + (ix & 1)) >> 1) mod H), entry (r >> 1, ix >> 1)
      const float* q = args.gin + plc * (int64_t)H * H * H * H;
      const int Kx = ((kx + (ix & 1)) >> 1) & (H - 1);
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const int Ky = ((ky + (r & 1)) >> 1) & (H - 1);
        G[r] = q[(((int64_t)Ky * H + Kx) * H + (r >> 1)) * H + (ix >> 1)];
      }
    }
    float sw = 0.f, sb = 0.f;
    for (int l = D - 1; l >= 0; --l) {
      // input of layer l, re-run from the stage input
      load_input(Aw);
      for (int m = 0; m < l; ++m) {
        const float2* c1 = t1 + m * N * N + ix;
        const float2* c2 = t2 + m * 2 * N * N + ky * N + jx;
        tile_layer_rt<N, BIAS>(Aw, c1, c2, seam, mL, mR, args.sb2, SEED && m == 0);
      }
      const float2* c1 = t1 + l * N * N + ix;
      const float2* c2 = t2 + l * 2 * N * N + ky * N + jx;
      tile_layer_bwd<N, BIAS>(Aw, G, c1, c2, seam, mL, mR, args.sb2, w1 + l * N * N, w2 + l * N * N, ix, jx, ky, sw,
                              sb, SEED && l == 0, lead);
      tile_box<N>(G, seam, mL, mR);
    }
    // G = adjoint of the stage input
    if (SEED) {
      const float ssd = args.seed_scale;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const int jy = (r + ky) & (N - 1);
        const float4 u = im1[r * N + ix];
        const float4 w = img2[jy * N + jx];
        const float gb = G[r] * ssd;
        const float a0 = args.seed_scale *
                         __builtin_fmaf(u.w, w.w, __builtin_fmaf(u.z, w.z, __builtin_fmaf(u.y, w.y, u.x * w.x)));
        sw = __builtin_fmaf(G[r], a0, sw);
        float* d1 = &xb1[(r * N + ix) * C];
        float* d2 = &xb2[(jy * N + jx) * C];
        const int c1 = C > 1 ? 1 : 0, c2 = C > 2 ? 2 : 0, c3 = C > 3 ? 3 : 0;
        const float s0 = seg_sum<N>(gb * w.x);
        const float s1 = seg_sum<N>(C > 1 ? gb * w.y : 0.f);
        const float s2 = seg_sum<N>(C > 2 ? gb * w.z : 0.f);
        const float s3 = seg_sum<N>(C > 3 ? gb * w.w : 0.f);
        if (lead) {
          atomicAdd(d1, s0);
          atomicAdd(d1 + c1, s1);
          atomicAdd(d1 + c2, s2);
          atomicAdd(d1 + c3, s3);
        }
        atomicAdd(d2, gb * u.x);
        atomicAdd(d2 + c1, C > 1 ? gb * u.y : 0.f);
        atomicAdd(d2 + c2, C > 2 ? gb * u.z : 0.f);
        atomicAdd(d2 + c3, C > 3 ? gb * u.w : 0.f);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    } else if (valid) {
      float* q = args.gout + pl * (int64_t)N * N * N * N + ((int64_t)ky * N + kx) * N * N + ix;
#pragma unroll
      for (int r = 0; r < N; ++r) q[r * N] = G[r];
    }
    swd += sw;
    sbd += sb;
  }
  }  // tile columns of this segment
  // scalars: wave sums, then per pair (a wave may hold several pair slots;
  // slots past the chunk end re-ran a clamped pair and must add nothing)
  if (!valid) {
    swd = 0.0;
    sbd = 0.0;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    swd += __shfl_xor(swd, off);
    sbd += __shfl_xor(sbd, off);
  }
  __syncthreads();
  if ((tid & 63) == 0) {
    atomicAdd(&scal[0], (float)swd);
    atomicAdd(&scal[1], (float)sbd);
  }
  __syncthreads();
  if (!valid) return;
  for (int e = within; e < TL; e += TPP) {
    atomicAdd(&args.W1[pa * args.tablen + args.taboff + e], (double)w1[e]);
    atomicAdd(&args.W2[pb * args.tablen + args.taboff + e], (double)w2[e]);
  }
  if (SEED) {
    for (int e = within; e < N * N * C; e += TPP) {
      atomicAdd(&args.xbar1[pa * (int64_t)N * N * C + e], (double)xb1[e]);
      atomicAdd(&args.xbar2[pb * (int64_t)N * N * C + e], (double)xb2[e]);
    }
  }
  if (within == 0) {
    atomicAdd(&args.sums[0], (double)scal[0]);
    atomicAdd(&args.sums[1], (double)scal[1] + (LAST ? (double)gpair : 0.0));
  }
}

// ---------------------------------------------------------------------------
// Self recursions, float64, one workgroup per image.
// ---------------------------------------------------------------------------

__device__ inline double relu_map64b(double s, double q1, double q2, double* ds, double* dq1, double* dq2) {
  const double qq = q1 * q2;
  if (!(qq > 0.0)) {
    *ds = *dq1 = *dq2 = 0.0;
    return 0.0;
  }
  const double nrm = sqrt(qq);
  double rho = s / nrm;
  rho = rho > 1.0 ? 1.0 : (rho < -1.0 ? -1.0 : rho);
  const double th = acos(rho);
  const double sn = sqrt(fmax(1.0 - rho * rho, 0.0));
  *ds = (M_PI - th) * (0.5 / M_PI);
  *dq1 = sn * sqrt(q2 / q1) * (0.25 / M_PI);
  *dq2 = sn * sqrt(q1 / q2) * (0.25 / M_PI);
  return nrm * (sn + (M_PI - th) * rho) * (0.5 / M_PI);
}

__device__ inline double box9b(const double* m, int n, int y, int x) {
  double s = 0.0;
  for (int dy = -1; dy <= 1; ++dy) {
    const int yy = y + dy;
    if (yy < 0 || yy >= n) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = x + dx;
      if (xx < 0 || xx >= n) continue;
      s += m[yy * n + xx];
    }
  }
  return s;
}

__device__ inline int prep_R2(const NetDesc& net, int s) { return (1 << (net.S - 1 - s)) - 1; }

// Doubles of scratch per workgroup for prepare_bwd_kernel.
int64_t prep_bwd_scratch_doubles(const NetDesc& net) {
  int64_t t = 0;
  for (int s = 0; s < net.S; ++s) {
    const int n = stage_res(net, s), R = (1 << (net.S - 1 - s)) - 1, side = 2 * R + 1;
    const int64_t n2 = (int64_t)n * n;
    t += net.depth[s] * n2 * 2;              // q maps, q bar
    t += n2;                                 // base
    if (s + 1 < net.S) t += (int64_t)side * side * net.depth[s] * n2;  // tape of pre-activations
    t += (int64_t)side * side * n2 * 2;      // input slices and their adjoints
  }
  t += 4LL * net.hw * net.hw;  // work buffers
  return (t + 31) & ~31LL;
}

__global__ __launch_bounds__(256) void prepare_bwd_kernel(const PrepBwdArgs args) {
  const int64_t img = blockIdx.x;
  if (img >= args.n) return;
  const NetDesc& net = args.net;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int C = net.C;
  const float* x = args.x + img * (int64_t)net.hw * net.hw * C;
  const double c = (double)net.sw2 / 9.0, b = (double)net.sb2;
  const double* W = args.W + img * (int64_t)args.tablen;
  double* xbar = args.xbar + img * (int64_t)net.hw * net.hw * C;

  // scratch layout (per stage: q, qbar, base, tape, slices in, slices in adjoint)
  double* sc = args.scratch + (int64_t)blockIdx.x * args.scratch_per_img;
  double* q_[NK_MAX_STAGES];
  double* qb_[NK_MAX_STAGES];
  double* base_[NK_MAX_STAGES];
  double* tape_[NK_MAX_STAGES];
  double* sin_[NK_MAX_STAGES];
  double* sinb_[NK_MAX_STAGES];
  {
    double* p = sc;
    for (int s = 0; s < net.S; ++s) {
      const int n = stage_res(net, s), R = prep_R2(net, s), side = 2 * R + 1;
      const int64_t n2 = (int64_t)n * n;
      q_[s] = p;
      p += net.depth[s] * n2;
      qb_[s] = p;
      p += net.depth[s] * n2;
      base_[s] = p;
      p += n2;
      tape_[s] = p;
      if (s + 1 < net.S) p += (int64_t)side * side * net.depth[s] * n2;
      sin_[s] = p;
      p += (int64_t)side * side * n2;
      sinb_[s] = p;
      p += (int64_t)side * side * n2;
    }
    (void)p;
  }
  double* wA = sc + args.scratch_per_img - 4LL * net.hw * net.hw;
  double* wB = wA + (int64_t)net.hw * net.hw;
  double* wC = wB + (int64_t)net.hw * net.hw;
  double* wD = wC + (int64_t)net.hw * net.hw;

  double accw = 0.0, accb = 0.0;  // d/dsigma_w2 (times sigma_w2), d/dsigma_b2

  // ---------------- forward with tape ----------------
  for (int s = 0; s < net.S; ++s) {
    const int n = stage_res(net, s), D = net.depth[s], R = prep_R2(net, s), side = 2 * R + 1;
    const int64_t n2 = (int64_t)n * n;
    for (int i = tid; i < n2; i += nt) {
      double v;
      if (s == 0) {
        v = 0.0;
        for (int k = 0; k < C; ++k) v += (double)x[i * C + k] * (double)x[i * C + k];
        v /= C;
      } else {
        v = sin_[s][(int64_t)(R * side + R) * n2 + i];
      }
      base_[s][i] = v;
    }
    __syncthreads();
    for (int l = 0; l < D; ++l) {
      const double* src = l == 0 ? base_[s] : q_[s] + (l - 1) * n2;
      const double f = l == 0 ? 1.0 : 0.5;
      for (int i = tid; i < n2; i += nt) q_[s][l * n2 + i] = c * f * box9b(src, n, i / n, i % n) + b;
      __syncthreads();
    }
    if (s + 1 == net.S) break;
    const int Rn = prep_R2(net, s + 1), nn = n / 2, side_n = 2 * Rn + 1;
    double* nxt = sin_[s + 1];
    for (int i = tid; i < side_n * side_n * nn * nn; i += nt) nxt[i] = 0.0;
    __syncthreads();
    for (int dyi = -R; dyi <= R; ++dyi)
      for (int dxi = -R; dxi <= R; ++dxi) {
        const int sl = (dyi + R) * side + (dxi + R);
        for (int i = tid; i < n2; i += nt) {
          const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
          double v = 0.0;
          if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) {
            if (s == 0) {
              for (int k = 0; k < C; ++k) v += (double)x[i * C + k] * (double)x[(y2 * n + x2) * C + k];
              v /= C;
            } else {
              v = sin_[s][(int64_t)sl * n2 + i];
            }
          }
          wA[i] = v;
        }
        __syncthreads();
        for (int l = 0; l < D; ++l) {
          const double* q = q_[s] + l * n2;
          double* tp = tape_[s] + ((int64_t)sl * D + l) * n2;
          for (int i = tid; i < n2; i += nt) {
            const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
            double v = 0.0, sg = 0.0;
            if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) {
              sg = c * box9b(wA, n, y, xx) + b;
              double d0, d1, d2;
              v = relu_map64b(sg, q[i], q[y2 * n + x2], &d0, &d1, &d2);
            }
            tp[i] = sg;
            wB[i] = v;
          }
          __syncthreads();
          for (int i = tid; i < n2; i += nt) wA[i] = wB[i];
          __syncthreads();
        }
        for (int e = tid; e < side_n * side_n * nn * nn; e += nt) {
          const int Ii = e % (nn * nn), sl2 = e / (nn * nn);
          const int DY = sl2 / side_n - Rn, DX = sl2 % side_n - Rn;
          const int IY = Ii / nn, IX = Ii % nn;
          double acc = 0.0;
          for (int ay = 0; ay < 2; ++ay) {
            const int fy = 2 * IY + ay, gy = fy + dyi;
            if (gy < 0 || gy >= n || (gy >> 1) != IY + DY) continue;
            for (int ax = 0; ax < 2; ++ax) {
              const int fx = 2 * IX + ax, gx = fx + dxi;
              if (gx < 0 || gx >= n || (gx >> 1) != IX + DX) continue;
              acc += wA[fy * n + fx];
            }
          }
          nxt[e] += acc / 16.0;
        }
        __syncthreads();
      }
  }

  // ---------------- reverse ----------------
  for (int s = 0; s < net.S; ++s) {
    const int n = stage_res(net, s), D = net.depth[s];
    const int64_t n2 = (int64_t)n * n;
    const int64_t toff = table_off(net, s);
    for (int l = 0; l < D; ++l)
      for (int i = tid; i < n2; i += nt) {
        const double qv = q_[s][l * n2 + i];
        qb_[s][l * n2 + i] = qv > 0.0 ? W[toff + l * n2 + i] / (2.0 * qv) : 0.0;
      }
    const int R = prep_R2(net, s), side = 2 * R + 1;
    for (int i = tid; i < side * side * n2; i += nt) sinb_[s][i] = 0.0;
  }
  __syncthreads();

  for (int s = net.S - 1; s >= 0; --s) {
    const int n = stage_res(net, s), D = net.depth[s], R = prep_R2(net, s), side = 2 * R + 1;
    const int64_t n2 = (int64_t)n * n;
    if (s + 1 < net.S) {
      const int Rn = prep_R2(net, s + 1), nn = n / 2, side_n = 2 * Rn + 1;
      const double* pb = sinb_[s + 1];
      for (int dyi = -R; dyi <= R; ++dyi)
        for (int dxi = -R; dxi <= R; ++dxi) {
          const int sl = (dyi + R) * side + (dxi + R);
          // adjoint of this slice's stage output, from the pooled slices
          for (int i = tid; i < n2; i += nt) {
            const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
            double v = 0.0;
            if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) {
              const int IY = y >> 1, IX = xx >> 1, DY = (y2 >> 1) - IY, DX = (x2 >> 1) - IX;
              if (DY >= -Rn && DY <= Rn && DX >= -Rn && DX <= Rn)
                v = pb[((int64_t)(DY + Rn) * side_n + (DX + Rn)) * nn * nn + IY * nn + IX] / 16.0;
            }
            wA[i] = v;
          }
          __syncthreads();
          for (int l = D - 1; l >= 0; --l) {
            const double* q = q_[s] + l * n2;
            const double* tp = tape_[s] + ((int64_t)sl * D + l) * n2;
            double* qb = qb_[s] + l * n2;
            // pass 1: sigma bar, q bar at i
            for (int i = tid; i < n2; i += nt) {
              const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
              double sgb = 0.0, dq2 = 0.0;
              if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) {
                double d0, d1;
                relu_map64b(tp[i], q[i], q[y2 * n + x2], &d0, &d1, &dq2);
                sgb = wA[i] * d0;
                qb[i] += wA[i] * d1;
                accw += sgb * (tp[i] - b);
                accb += sgb;
              }
              wB[i] = sgb;
              wC[i] = wA[i] * dq2;
            }
            __syncthreads();
            // pass 2: q bar at i + delta (a bijection, no races)
            for (int i = tid; i < n2; i += nt) {
              const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
              if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) qb[y2 * n + x2] += wC[i];
            }
            __syncthreads();
            for (int i = tid; i < n2; i += nt) {
              const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
              wA[i] = (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) ? c * box9b(wB, n, y, xx) : 0.0;
            }
            __syncthreads();
          }
          // wA = adjoint of the stage-input slice
          if (s == 0) {
            for (int i = tid; i < n2; i += nt) {
              const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
              if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n)
                for (int k = 0; k < C; ++k) xbar[i * C + k] += wA[i] * (double)x[(y2 * n + x2) * C + k] / C;
            }
            __syncthreads();
            for (int i = tid; i < n2; i += nt) {
              const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
              if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n)
                for (int k = 0; k < C; ++k) xbar[(y2 * n + x2) * C + k] += wA[i] * (double)x[i * C + k] / C;
            }
          } else {
            for (int i = tid; i < n2; i += nt) sinb_[s][(int64_t)sl * n2 + i] += wA[i];
          }
          __syncthreads();
        }
    }
    // diagonal chain: q_1 = c box(base) + b, q_{l+1} = c box(q_l / 2) + b
    for (int l = D - 1; l >= 0; --l) {
      const double* qbl = qb_[s] + l * n2;
      const double* ql = q_[s] + l * n2;
      for (int i = tid; i < n2; i += nt) {
        accw += qbl[i] * (ql[i] - b);
        accb += qbl[i];
      }
      double* dst = l > 0 ? qb_[s] + (l - 1) * n2 : wD;
      const double f = l > 0 ? 0.5 : 1.0;
      __syncthreads();
      for (int i = tid; i < n2; i += nt) {
        const double v = c * f * box9b(qbl, n, i / n, i % n);
        if (l > 0)
          dst[i] += v;
        else
          dst[i] = v;
      }
      __syncthreads();
    }
    if (D > 0) {
      // wD = adjoint of the base map
      if (s == 0) {
        for (int i = tid; i < n2; i += nt)
          for (int k = 0; k < C; ++k) xbar[i * C + k] += 2.0 * wD[i] * (double)x[i * C + k] / C;
      } else {
        for (int i = tid; i < n2; i += nt) sinb_[s][(int64_t)(R * side + R) * n2 + i] += wD[i];
      }
    }
    __syncthreads();
  }
  // sums: accw is sum of s_bar (s - b) = sigma_w2 * d/dsigma_w2 contributions
  for (int off = 32; off >= 1; off >>= 1) {
    accw += __shfl_xor(accw, off);
    accb += __shfl_xor(accb, off);
  }
  if ((tid & 63) == 0) {
    atomicAdd(&args.sums[0], accw);
    atomicAdd(&args.sums[1], accb);
  }
}

// dx (float) = xbar (double) over n images
__global__ __launch_bounds__(256) void cast_grad_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                                        int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = (float)src[e];
}

__global__ void finish_sigma_kernel(const double* __restrict__ sums, double sw2, float* __restrict__ dsigma) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dsigma[0] = (float)(sums[0] / sw2);
    dsigma[1] = (float)sums[1];
  }
}

__global__ __launch_bounds__(256) void zero_f64_kernel(double* __restrict__ p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = 0.0;
}

template <int N, bool SEED, bool LAST, bool BIAS>
static int launch_bwd_t(const StageBwdArgs& a, hipStream_t stream) {
  const int64_t nwg = (a.np + BCfg<N>::PPWG - 1) / BCfg<N>::PPWG;
  const size_t lds = (size_t)BCfg<N>::PPWG * bwd_slot_lds_bytes<N>(a.D, SEED, a.C);
  auto fn = stage_bwd_kernel<N, SEED, LAST, BIAS>;
  if (lds > 64 * 1024) {
    static size_t attr_bytes = 0;
    if (attr_bytes < lds) {
      if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return -3;
      attr_bytes = lds;
    }
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)nwg), dim3(BCfg<N>::THREADS), lds, stream, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int N>
static int launch_bwd_n(const StageBwdArgs& a, bool seed, bool last, bool bias, hipStream_t s) {
  if (seed) {
    if (last) return bias ? launch_bwd_t<N, true, true, true>(a, s) : launch_bwd_t<N, true, true, false>(a, s);
    return bias ? launch_bwd_t<N, true, false, true>(a, s) : launch_bwd_t<N, true, false, false>(a, s);
  }
  if (last) return bias ? launch_bwd_t<N, false, true, true>(a, s) : launch_bwd_t<N, false, true, false>(a, s);
  return bias ? launch_bwd_t<N, false, false, true>(a, s) : launch_bwd_t<N, false, false, false>(a, s);
}

size_t stage_bwd_lds_bytes(int N, int D, bool seed, int C) {
  switch (N) {
    case 2: return BCfg<2>::PPWG * bwd_slot_lds_bytes<2>(D, seed, C);
    case 4: return BCfg<4>::PPWG * bwd_slot_lds_bytes<4>(D, seed, C);
    case 8: return BCfg<8>::PPWG * bwd_slot_lds_bytes<8>(D, seed, C);
    case 16: return BCfg<16>::PPWG * bwd_slot_lds_bytes<16>(D, seed, C);
    case 32: return BCfg<32>::PPWG * bwd_slot_lds_bytes<32>(D, seed, C);
  }
  return 0;
}

int launch_stage_bwd(int N, const StageBwdArgs& a, bool seed, bool last, bool bias, hipStream_t s) {
  switch (N) {
    case 2: return launch_bwd_n<2>(a, seed, last, bias, s);
    case 4: return launch_bwd_n<4>(a, seed, last, bias, s);
    case 8: return launch_bwd_n<8>(a, seed, last, bias, s);
    case 16: return launch_bwd_n<16>(a, seed, last, bias, s);
    case 32: return launch_bwd_n<32>(a, seed, last, bias, s);
  }
  return -2;
}

int launch_prepare_bwd(const float* x, int64_t n, const NetDesc& net, const double* W, int tablen, double* xbar,
                       double* sums, double* scratch, int64_t max_blocks, hipStream_t stream) {
  const int64_t per = prep_bwd_scratch_doubles(net);
  for (int64_t s = 0; s < n; s += max_blocks) {
    const int64_t cnt = n - s < max_blocks ? n - s : max_blocks;
    PrepBwdArgs a;
    a.x = x + s * (int64_t)net.hw * net.hw * net.C;
    a.n = cnt;
    a.net = net;
    a.W = W + s * (int64_t)tablen;
    a.tablen = tablen;
    a.xbar = xbar + s * (int64_t)net.hw * net.hw * net.C;
    a.sums = sums;
    a.scratch = scratch;
    a.scratch_per_img = per;
    hipLaunchKernelGGL(prepare_bwd_kernel, dim3((unsigned)cnt), dim3(256), 0, stream, a);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  return 0;
}

int launch_cast_grad(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(cast_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_finish_sigma(const double* sums, double sw2, float* dsigma, hipStream_t s) {
  hipLaunchKernelGGL(finish_sigma_kernel, dim3(1), dim3(64), 0, s, sums, sw2, dsigma);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_zero_f64(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(zero_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace nk
