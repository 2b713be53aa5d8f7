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
  int64_t np;
};

// Pairs per workgroup: 256 / N segments of N lanes.
template <int N, bool BIAS>
__global__ __launch_bounds__(256) void cv_pair_kernel(const CvArgs a) {
  constexpr int SEGS = 256 / N;
  const int seg = threadIdx.x / N, ix = threadIdx.x - seg * N;
  const int64_t p = (int64_t)xcd_logical_block() * SEGS + seg;
  const bool valid = p < a.np;
  int64_t ia = 0, ib = 0;
  pair_of(valid ? p : a.np - 1, a.n1, a.n2, a.sym, a.T, &ia, &ib);
  const float* p1 = a.x1 + (ia * N * N + ix) * a.C;
  const float* p2 = a.x2 + (ib * N * N + ix) * a.C;
  float A[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    float s = 0.f;
    for (int c = 0; c < a.C; ++c) s = __builtin_fmaf(p1[r * N * a.C + c], p2[r * N * a.C + c], s);
    A[r] = s * a.seed_scale;
  }
  const float mL = ix >= 1 ? 1.f : 0.f;
  const float mR = ix + 1 < N ? 1.f : 0.f;
  const float2* c1 = a.tab1 + ia * (int64_t)a.D * N * N + ix;
  const float2* c2 = a.tab2 + ib * (int64_t)a.D * N * N + ix;
  tile_layer<N, true, BIAS>(A, c1, c2, -1, mL, mR, a.sb2);
  for (int l = 1; l < a.D; ++l) {
    c1 += N * N;
    c2 += N * N;
    tile_layer<N, false, BIAS>(A, c1, c2, -1, mL, mR, a.sb2);
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

size_t cv_prepare_lds_bytes(int N) { return (size_t)2 * N * N * sizeof(double); }

int launch_cv_prepare(const float* x, int64_t n, int N, int C, int D, double sw2, double sb2, float2* tab,
                      float* kdiag, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(cv_prepare_kernel, dim3((unsigned)n), dim3((unsigned)(N * N)), cv_prepare_lds_bytes(N), s, x,
                     N, C, D, sw2, sb2, tab, kdiag);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int N>
int launch_cv_pairs_n(const CvArgs& a, bool bias, hipStream_t s) {
  constexpr int SEGS = 256 / N;
  const int64_t nwg = (a.np + SEGS - 1) / SEGS;
  if (bias)
    hipLaunchKernelGGL((cv_pair_kernel<N, true>), dim3((unsigned)nwg), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((cv_pair_kernel<N, false>), dim3((unsigned)nwg), dim3(256), 0, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
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
  a.np = pair_count(n1, n2, sym);
  if (a.np <= 0) return 0;
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
