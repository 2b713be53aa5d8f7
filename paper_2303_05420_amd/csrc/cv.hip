// CNN-VEC NNGP (App. "Neural Kernel Architecture", CNN-VEC listing: `depth`
// blocks of [3x3 SAME conv, ReLU] at full resolution, Flatten, Dense).
//
// The flatten readout averages the covariance of each pixel of x with the
// same pixel of x', and a conv maps entry (i, j) to (i + d, j + d): so only
// the displacement-0 entries (i, i) are ever needed, one h x w map per pair
// and layer instead of the (h w)^2 of a pooled network.  That map is the
// k = (0, 0) tile of the sheared layout of the Myrtle stage kernel (lane =
// column, register = row, no seam): every pair runs in one N-lane segment
// and carries its tile through all layers in registers.
//
// Tables (cv_prepare_kernel, float64 inside): per image, layer and pixel,
//   alpha = q^{-1/2},  beta = (kappa q / 2)^{1/2},
// q the pre-activation variance of the image at that ReLU (its own
// displacement-0 recursion, where the ReLU map of (q, q, q) is q / 2), kappa
// the scale that multiplies the layer's output downstream: sigma_w2 / 9 of
// the next conv, sigma_w2 / (h w) of the readout after the last layer.  The
// seed's sigma_w2 / (9 C) rides on the second image's pixels.
#include "nk_tile.h"

namespace nk {

// One image per workgroup, one thread per pixel (N * N threads).
__global__ void cv_prepare_kernel(const float* __restrict__ x, int N, int C, int D, double sw2, double sb2,
                                  float2* __restrict__ tab, float* __restrict__ kdiag) {
  extern __shared__ double cv_maps[];  // S then V, N * N doubles each
  double* S = cv_maps;
  double* V = cv_maps + N * N;
  const int px = threadIdx.x;
  const int iy = px / N, ix = px - iy * N;
  const int64_t img = blockIdx.x;
  const float* xi = x + (img * N * N + px) * C;
  double s = 0.0;
  for (int c = 0; c < C; ++c) s += (double)xi[c] * (double)xi[c];
  S[px] = s / C;
  __syncthreads();
  float2* t = tab + img * (int64_t)D * N * N;
  for (int l = 0; l < D; ++l) {
    double b = 0.0;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int y = iy + dy, xx = ix + dx;
        if (y >= 0 && y < N && xx >= 0 && xx < N) b += S[y * N + xx];
      }
    const double q = sw2 / 9.0 * b + sb2;
    V[px] = q;
    const double kappa = l + 1 < D ? sw2 / 9.0 : sw2 / (double)(N * N);
    t[(int64_t)l * N * N + px] = make_float2((float)(1.0 / sqrt(q)), (float)sqrt(kappa * q * 0.5));
    __syncthreads();
    S[px] = 0.5 * q;
    __syncthreads();
  }
  if (px == 0) {
    double m = 0.0;
    for (int e = 0; e < N * N; ++e) m += S[e];
    kdiag[img] = (float)(sw2 * m / (double)(N * N) + sb2);
  }
}

struct CvArgs {
  const float* x1;
  const float* x2;
  int64_t n1, n2;
  int sym, T, C, D;
  const float2* tab1;
  const float2* tab2;
  float* K;
  int64_t ldk;
  float sb2, seed_scale;
  int64_t nb1, nb2, nblocks;  // 4 x 4 pair blocks per side, and in the pass
};

// Workgroup shape.  A workgroup computes a block of 4 x 4 pairs (images
// 4 bi + 0..3 of x1 against 4 bj + 0..3 of x2), one N-lane segment per pair,
// so that the tables of 8 images serve 16 pairs.  Each layer's tables of the
// 8 images sit in LDS (8 N^2 float2: 64 KiB at N = 32); the next layer's are
// fetched into registers while the current layer is
// computed, and written to LDS between two barriers.
template <int N>
struct CvB {
  static constexpr int PAIRS = 16;
  static constexpr int THREADS = PAIRS * N < 64 ? 64 : PAIRS * N;
  static constexpr int NN = N * N;
  static constexpr size_t LDS = (size_t)8 * NN * sizeof(float2);
  static constexpr int RH = N / 2;  // row before which the next layer's tables are requested
};

// One [3x3 conv, ReLU] layer of a displacement-0 tile (no seam: the
// vertical links are all present), with the forward NNGP's degree-3 fit of
// the map.  The next layer's table float4s of this
// thread (src + m * TPS, m < NV) are requested before row RH, so that the
// registers they land in are live for the rest of the layer only.
template <int N, bool SIGNED, bool BIAS, int RH, int NV, int TPS, bool FULL>
__device__ __forceinline__ void cv_layer(float (&A)[N], const float2* __restrict__ c1,
                                         const float2* __restrict__ c2, float mL, float mR, float sb2,
                                         const float4* __restrict__ src, int sj, int half, float (&pf)[NV][4]) {
  float hm = 0.f;
  float h0 = hsum3(A[0], mL, mR);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (r == RH) {
#pragma unroll
      for (int m = 0; m < NV; ++m)
        if (FULL || sj + m * TPS < half) {
          const float4 v = src[m * TPS];
          pf[m][0] = v.x;
          pf[m][1] = v.y;
          pf[m][2] = v.z;
          pf[m][3] = v.w;
        }
    }
    float hp = 0.f;
    if (r + 1 < N) hp = hsum3(A[r + 1], mL, mR);
    float v = h0;
    if (r > 0) v += hm;
    if (r + 1 < N) v += hp;
    if (BIAS) v += sb2;
    const float2 ta = c1[r * N];
    const float2 tb = c2[r * N];
    const float rr = ta.x * tb.x;
    const float J = SIGNED ? j1_signed_vr3(v, rr) : j1_nonneg3(v * rr);
    A[r] = (ta.y * tb.y) * J;
    hm = h0;
    h0 = hp;
  }
}

template <int N, int C, bool BIAS>
__global__ __launch_bounds__(CvB<N>::THREADS) __attribute__((amdgpu_waves_per_eu(4)))
void cv_block_kernel(const CvArgs a) {
  using B = CvB<N>;
  constexpr int NN = B::NN, THREADS = B::THREADS, HALF = NN / 2;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  float2* lds = reinterpret_cast<float2*>(smem);
  float4* lds4 = reinterpret_cast<float4*>(smem);
  const int tid = threadIdx.x;
  const int q = tid / N, ix = tid - q * N;
  const int qa = (q >> 2) & 3, qb = q & 3;
  int64_t bi, bj;
  pair_of(xcd_logical_block(), a.nb1, a.nb2, a.sym, a.T, &bi, &bj);
  const int64_t ia = bi * 4 + qa, ib = bj * 4 + qb;
  // a pair outside the block (ragged edge, or below the diagonal of a
  // symmetric diagonal block) runs on clamped images and writes nothing
  const bool valid = q < B::PAIRS && ia < a.n1 && ib < a.n2 && !(a.sym && bi == bj && qa > qb);
  const int64_t iac = ia < a.n1 ? ia : a.n1 - 1, ibc = ib < a.n2 ? ib : a.n2 - 1;

  // staging: THREADS / 8 threads per table slot (slots 0..3: images 4 bi + s
  // of x1, 4..7: images 4 bj + s - 4 of x2), each moving NV float4 of it
  constexpr int TPS = THREADS / 8, NV = (HALF + TPS - 1) / TPS;
  const int sl = tid / TPS, sj = tid - sl * TPS;
  const float4* src;
  {
    int64_t img = sl < 4 ? bi * 4 + sl : bj * 4 + (sl - 4);
    const int64_t lim = sl < 4 ? a.n1 : a.n2;
    if (img >= lim) img = lim - 1;
    src = reinterpret_cast<const float4*>(sl < 4 ? a.tab1 : a.tab2) + img * (int64_t)a.D * HALF + sj;
  }
  float4* dst = lds4 + sl * HALF + sj;
  // (plain floats: an array of float4 structs is not kept in registers)
  float pf[NV][4];
#define CV_FETCH(l)                                                                          \
  _Pragma("unroll") for (int m = 0; m < NV; ++m) if (HALF % TPS == 0 || sj + m * TPS < HALF) { \
    const float4 v = src[(int64_t)(l) * HALF + m * TPS];                                     \
    pf[m][0] = v.x;                                                                          \
    pf[m][1] = v.y;                                                                          \
    pf[m][2] = v.z;                                                                          \
    pf[m][3] = v.w;                                                                          \
  }
#define CV_STORE()                                                                           \
  _Pragma("unroll") for (int m = 0; m < NV; ++m) if (HALF % TPS == 0 || sj + m * TPS < HALF) \
      dst[m * TPS] = make_float4(pf[m][0], pf[m][1], pf[m][2], pf[m][3])

  // seed: the pixels of SR rows are requested together, then combined
  constexpr int SR = N < 4 ? N : 4;
  const float* p1 = a.x1 + (iac * NN + ix) * C;
  const float* p2 = a.x2 + (ibc * NN + ix) * C;
  float A[N];
#pragma unroll
  for (int r0 = 0; r0 < N; r0 += SR) {
    float u[SR][C], w[SR][C];
#pragma unroll
    for (int k = 0; k < SR; ++k)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        u[k][c] = p1[(r0 + k) * N * C + c];
        w[k][c] = p2[(r0 + k) * N * C + c];
      }
#pragma unroll
    for (int k = 0; k < SR; ++k) {
      float sd = 0.f;
#pragma unroll
      for (int c = 0; c < C; ++c) sd = __builtin_fmaf(u[k][c], w[k][c], sd);
      A[r0 + k] = sd * a.seed_scale;
    }
  }
  CV_FETCH(0);
  CV_STORE();
  __syncthreads();

  const float mL = ix >= 1 ? 1.f : 0.f;
  const float mR = ix + 1 < N ? 1.f : 0.f;
  const float2* c1 = lds + qa * NN + ix;
  const float2* c2 = lds + (4 + qb) * NN + ix;
  constexpr bool FULL = HALF % TPS == 0;
  for (int l = 0; l < a.D; ++l) {
    // (the last layer re-reads its own tables: always in bounds, never stored;
    // a conditional fetch would keep the registers live across the layer)
    const float4* nsrc = src + (int64_t)(l + 1 < a.D ? l + 1 : l) * HALF;
    if (l == 0)
      cv_layer<N, true, BIAS, B::RH, NV, TPS, FULL>(A, c1, c2, mL, mR, a.sb2, nsrc, sj, HALF, pf);
    else
      cv_layer<N, false, BIAS, B::RH, NV, TPS, FULL>(A, c1, c2, mL, mR, a.sb2, nsrc, sj, HALF, pf);
    if (l + 1 < a.D) {
      __syncthreads();
      CV_STORE();
      __syncthreads();
    }
  }
  // readout: the tile's sum (its scale rides on the last layer's tables)
  float t[N];
#pragma unroll
  for (int r = 0; r < N; ++r) t[r] = A[r];
#pragma unroll
  for (int w = N / 2; w >= 1; w >>= 1) {
#pragma unroll
    for (int r = 0; r < w; ++r) t[r] = t[r] + t[r + w];
  }
  double sum = (double)t[0];
#pragma unroll
  for (int off = N / 2; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, N);
  if (ix == 0 && valid) {
    const float kv = (float)(sum + (double)a.sb2);
    a.K[ia * a.ldk + ib] = kv;
    if (a.sym && ia != ib) a.K[ib * a.ldk + ia] = kv;
  }
}
#undef CV_FETCH
#undef CV_STORE

size_t cv_prepare_lds_bytes(int N) { return (size_t)2 * N * N * sizeof(double); }

int launch_cv_prepare(const float* x, int64_t n, int N, int C, int D, double sw2, double sb2, float2* tab,
                      float* kdiag, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(cv_prepare_kernel, dim3((unsigned)n), dim3((unsigned)(N * N)), cv_prepare_lds_bytes(N), s, x,
                     N, C, D, sw2, sb2, tab, kdiag);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int N, int C>
int launch_cv_pairs_nc(const CvArgs& a, bool bias, hipStream_t s) {
  using B = CvB<N>;
  if (bias)
    hipLaunchKernelGGL((cv_block_kernel<N, C, true>), dim3((unsigned)a.nblocks), dim3(B::THREADS), B::LDS, s, a);
  else
    hipLaunchKernelGGL((cv_block_kernel<N, C, false>), dim3((unsigned)a.nblocks), dim3(B::THREADS), B::LDS, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int N>
int launch_cv_pairs_n(const CvArgs& a, bool bias, hipStream_t s) {
  switch (a.C) {
    case 1: return launch_cv_pairs_nc<N, 1>(a, bias, s);
    case 2: return launch_cv_pairs_nc<N, 2>(a, bias, s);
    case 3: return launch_cv_pairs_nc<N, 3>(a, bias, s);
    case 4: return launch_cv_pairs_nc<N, 4>(a, bias, s);
    default: return -1;
  }
}

int launch_cv_pairs(int N, const float* x1, const float* x2, int64_t n1, int64_t n2, int sym, int T, int C, int D,
                    const float2* tab1, const float2* tab2, float* K, int64_t ldk, float sb2, float seed_scale,
                    hipStream_t s) {
  CvArgs a;
  a.x1 = x1;
  a.x2 = x2;
  a.n1 = n1;
  a.n2 = n2;
  a.sym = sym;
  a.T = T;
  a.C = C;
  a.D = D;
  a.tab1 = tab1;
  a.tab2 = tab2;
  a.K = K;
  a.ldk = ldk;
  a.sb2 = sb2;
  a.seed_scale = seed_scale;
  a.nb1 = (n1 + 3) / 4;
  a.nb2 = (n2 + 3) / 4;
  a.nblocks = pair_count(a.nb1, a.nb2, sym);
  if (a.nblocks <= 0) return 0;
  if (a.nblocks > 0x7fffffff) return -1;
  const bool bias = sb2 != 0.f;
  switch (N) {
    case 2: return launch_cv_pairs_n<2>(a, bias, s);
    case 4: return launch_cv_pairs_n<4>(a, bias, s);
    case 8: return launch_cv_pairs_n<8>(a, bias, s);
    case 16: return launch_cv_pairs_n<16>(a, bias, s);
    case 32: return launch_cv_pairs_n<32>(a, bias, s);
    default: return -1;
  }
}

}  // namespace nk
