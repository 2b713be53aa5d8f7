// Dense float64 building blocks of the approximate kernel-regression solvers
// (Sec. 2, "Approximations to the linear system"; sequenced by the host API
// entry points nk_krr_nystrom, nk_krr_sor, nk_krr_block_diag, nk_krr_bcm): a tiled
// GEMM with float32 or float64 operands and float64 accumulation (optionally
// compensated), symmetric-matrix loads with a diagonal shift, identity
// fills, row updates and casts.
#include "nk_kernels.h"

namespace nk {

constexpr int DN_T = 32;  // output tile side; 256 threads hold 4 outputs each

// C (M x N, double, ldc) = beta C + alpha op(A) B.
//   op(A) = A (M x K, lda) or, with TA_T, A^T where A is K x M (lda);
//   B is K x N (ldb), row-major.
// COMP: each output's sum carries its rounding error (exact product errors
// by FMA, TwoSum for the additions) and is rounded once -- for sums whose
// result is later subtracted from a nearly equal quantity.
template <typename TA, typename TB, bool TA_T, bool COMP>
__global__ __launch_bounds__(256) void dn_gemm_kernel(const TA* __restrict__ A, int64_t lda,
                                                      const TB* __restrict__ B, int64_t ldb, double* __restrict__ Cm,
                                                      int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha,
                                                      double beta) {
#pragma clang fp contract(off)
  __shared__ double sA[DN_T][DN_T + 1];  // sA[row of C][k]
  __shared__ double sB[DN_T][DN_T + 1];  // sB[k][col of C]
  const int64_t r0 = (int64_t)blockIdx.y * DN_T, c0 = (int64_t)blockIdx.x * DN_T;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double hi[4] = {0.0, 0.0, 0.0, 0.0}, lo[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < K; k0 += DN_T) {
    for (int y = ty; y < DN_T; y += 8) {
      // A tile: rows r0 + y of op(A), columns k0 + tx
      const int64_t r = r0 + y, k = k0 + tx;
      double av = 0.0;
      if (r < M && k < K) av = TA_T ? (double)A[k * lda + r] : (double)A[r * lda + k];
      sA[y][tx] = av;
      const int64_t kb = k0 + y, cb = c0 + tx;
      sB[y][tx] = (kb < K && cb < N) ? (double)B[kb * ldb + cb] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < DN_T; ++k) {
      const double bv = sB[k][tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double av = sA[ty + 8 * q][k];
        if (COMP) {
          const double p = av * bv;
          const double pe = __builtin_fma(av, bv, -p);
          const double s = hi[q] + p;
          const double bb = s - hi[q];
          lo[q] += ((hi[q] - (s - bb)) + (p - bb)) + pe;
          hi[q] = s;
        } else {
          hi[q] = __builtin_fma(av, bv, hi[q]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t r = r0 + ty + 8 * q, c = c0 + tx;
    if (r < M && c < N) {
      const double v = alpha * (hi[q] + lo[q]);
      double* o = Cm + r * ldc + c;
      *o = beta == 0.0 ? v : __builtin_fma(beta, *o, v);
    }
  }
}

template <typename TA, typename TB, bool TA_T, bool COMP>
static int dn_gemm_t(const TA* A, int64_t lda, const TB* B, int64_t ldb, double* C, int64_t ldc, int64_t M,
                     int64_t N, int64_t K, double alpha, double beta, hipStream_t s) {
  if (M <= 0 || N <= 0) return 0;
  const dim3 grid((unsigned)((N + DN_T - 1) / DN_T), (unsigned)((M + DN_T - 1) / DN_T));
  hipLaunchKernelGGL((dn_gemm_kernel<TA, TB, TA_T, COMP>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K,
                     alpha, beta);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int dn_gemm_ff(const float* A, int64_t lda, bool a_t, const float* B, int64_t ldb, double* C, int64_t ldc, int64_t M,
               int64_t N, int64_t K, double alpha, double beta, bool comp, hipStream_t s) {
  if (a_t) return comp ? dn_gemm_t<float, float, true, true>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s)
                       : dn_gemm_t<float, float, true, false>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s);
  return comp ? dn_gemm_t<float, float, false, true>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s)
              : dn_gemm_t<float, float, false, false>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s);
}

int dn_gemm_fd(const float* A, int64_t lda, bool a_t, const double* B, int64_t ldb, double* C, int64_t ldc,
               int64_t M, int64_t N, int64_t K, double alpha, double beta, bool comp, hipStream_t s) {
  if (a_t) return comp ? dn_gemm_t<float, double, true, true>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s)
                       : dn_gemm_t<float, double, true, false>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s);
  return comp ? dn_gemm_t<float, double, false, true>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s)
              : dn_gemm_t<float, double, false, false>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s);
}

int dn_gemm_dd(const double* A, int64_t lda, bool a_t, const double* B, int64_t ldb, double* C, int64_t ldc,
               int64_t M, int64_t N, int64_t K, double alpha, double beta, bool comp, hipStream_t s) {
  if (a_t) return comp ? dn_gemm_t<double, double, true, true>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s)
                       : dn_gemm_t<double, double, true, false>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s);
  return comp ? dn_gemm_t<double, double, false, true>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s)
              : dn_gemm_t<double, double, false, false>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, s);
}

// D (n x n, double, dense) = S (float, lds) + shift I; clears info[0] when given.
__global__ __launch_bounds__(256) void dn_load_shift_kernel(const float* __restrict__ S, int64_t lds, int64_t n,
                                                            double shift, double* __restrict__ D,
                                                            int* __restrict__ info) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (info && e == 0) info[0] = 0;
  if (e >= n * n) return;
  const int64_t i = e / n, j = e - i * n;
  D[e] = (double)S[i * lds + j] + (i == j ? shift : 0.0);
}

int dn_load_shift(const float* S, int64_t lds, int64_t n, double shift, double* D, int* info, hipStream_t s) {
  hipLaunchKernelGGL(dn_load_shift_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, S, lds, n, shift,
                     D, info);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// D (n x n double) += shift I and (optionally) clears info[0]
__global__ __launch_bounds__(256) void dn_shift_kernel(double* __restrict__ D, int64_t n, double shift,
                                                       int* __restrict__ info) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (info && i == 0) info[0] = 0;
  if (i < n) D[i * n + i] += shift;
}

int dn_shift(double* D, int64_t n, double shift, int* info, hipStream_t s) {
  hipLaunchKernelGGL(dn_shift_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, D, n, shift, info);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// I (n x n double) = identity
__global__ __launch_bounds__(256) void dn_identity_kernel(double* __restrict__ I, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  I[e] = (e / n == e % n) ? 1.0 : 0.0;
}

int dn_identity(double* I, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(dn_identity_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, I, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// out (rows x cols double, ldo) = in (float, ldi), transposed when trans
__global__ __launch_bounds__(256) void dn_copy_f_kernel(const float* __restrict__ in, int64_t ldi, int64_t rows,
                                                        int64_t cols, bool trans, double* __restrict__ out,
                                                        int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  out[i * ldo + j] = trans ? (double)in[j * ldi + i] : (double)in[i * ldi + j];
}

int dn_copy_f(const float* in, int64_t ldi, int64_t rows, int64_t cols, bool trans, double* out, int64_t ldo,
              hipStream_t s) {
  if (rows * cols <= 0) return 0;
  hipLaunchKernelGGL(dn_copy_f_kernel, dim3((unsigned)((rows * cols + 255) / 256)), dim3(256), 0, s, in, ldi, rows,
                     cols, trans, out, ldo);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// X (n x c double) = (Yf - X) * scale, Yf float (ldy)
__global__ __launch_bounds__(256) void dn_residual_scale_kernel(const float* __restrict__ Y, int64_t ldy, int64_t n,
                                                                int64_t c, double scale, double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c, j = e - i * c;
  X[e] = ((double)Y[i * ldy + j] - X[e]) * scale;
}

int dn_residual_scale(const float* Y, int64_t ldy, int64_t n, int64_t c, double scale, double* X, hipStream_t s) {
  hipLaunchKernelGGL(dn_residual_scale_kernel, dim3((unsigned)((n * c + 255) / 256)), dim3(256), 0, s, Y, ldy, n, c,
                     scale, X);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// out (float, ldo) = in (double, rows x cols dense)
__global__ __launch_bounds__(256) void dn_cast_kernel(const double* __restrict__ in, int64_t rows, int64_t cols,
                                                      float* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  out[i * ldo + j] = (float)in[e];
}

int dn_cast(const double* in, int64_t rows, int64_t cols, float* out, int64_t ldo, hipStream_t s) {
  if (rows * cols <= 0) return 0;
  hipLaunchKernelGGL(dn_cast_kernel, dim3((unsigned)((rows * cols + 255) / 256)), dim3(256), 0, s, in, rows, cols,
                     out, ldo);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// D = alpha D + beta E elementwise over n doubles (alpha = 0: D is not read)
__global__ __launch_bounds__(256) void dn_axpby_kernel(double* __restrict__ D, const double* __restrict__ E,
                                                       int64_t n, double alpha, double beta) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  D[e] = alpha == 0.0 ? beta * E[e] : __builtin_fma(alpha, D[e], beta * E[e]);
}

int dn_axpby(double* D, const double* E, int64_t n, double alpha, double beta, hipStream_t s) {
  hipLaunchKernelGGL(dn_axpby_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, D, E, n, alpha, beta);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace nk
