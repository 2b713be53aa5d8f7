// Kernel ridge regression in float64: the linear system of Sec. 2 (the one
// the paper's preconditioned conjugate gradients solve iteratively), solved
// here directly by Cholesky factorisation, which is its exact solution.
//
//   lambda = ridge_rel mean(diag K_train),  A = K_train + lambda I = L L^T,
//   alpha = L^{-T} L^{-1} Y,  pred = K_test alpha.
//
// Blocked right-looking Cholesky (block NB): factor the diagonal block in LDS,
// solve the panel below it, update the trailing lower triangle; then copy L^T
// into the strict upper triangle.  Substitutions are blocked the same way:
// panel triangles one thread per right-hand side, the rest by float64 GEMM.
#include "nk_kernels.h"

namespace nk {

constexpr int CH_NB = 64;

__global__ __launch_bounds__(256) void krr_diag_mean_kernel(const float* __restrict__ K, int64_t n, int64_t ld,
                                                            double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)K[i * ld + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (double)n;
}

// A = K + (ridge_rel * mean) I   (lower triangle and diagonal are what matter)
__global__ __launch_bounds__(256) void krr_build_kernel(const float* __restrict__ K, int64_t n, const double* mean,
                                                        double ridge_rel, double lam_abs, double* __restrict__ A,
                                                        int* __restrict__ info) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e == 0) info[0] = 0;
  if (e >= n * n) return;
  const int64_t i = e / n, j = e - i * n;
  double v = (double)K[e];
  if (i == j) v += ridge_rel >= 0.0 ? ridge_rel * mean[0] : lam_abs;
  A[e] = v;
}

// Cholesky of the nb x nb diagonal block at (k, k), in LDS.
__global__ __launch_bounds__(256) void chol_diag_kernel(double* __restrict__ A, int64_t n, int64_t k, int nb,
                                                        int* __restrict__ info) {
  __shared__ double L[CH_NB][CH_NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    L[i][j] = A[(k + i) * n + k + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double d = L[j][j];
      if (!(d > 0.0)) {
        info[0] = 1;
        L[j][j] = 1.0;
      } else {
        L[j][j] = sqrt(d);
      }
    }
    __syncthreads();
    const double djj = L[j][j];
    for (int i = j + 1 + tid; i < nb; i += 256) L[i][j] /= djj;
    __syncthreads();
    // trailing update of the block (lower part)
    for (int e = tid; e < (nb - j - 1) * (nb - j - 1); e += 256) {
      const int i = j + 1 + e / (nb - j - 1), c = j + 1 + e % (nb - j - 1);
      if (c <= i) L[i][c] -= L[i][j] * L[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    if (j <= i) A[(k + i) * n + k + j] = L[i][j];
  }
}

// Panel: rows i >= k + nb: A[i, k:k+nb] <- A[i, k:k+nb] L_kk^{-T}; one thread per row.
__global__ __launch_bounds__(256) void chol_trsm_kernel(double* __restrict__ A, int64_t n, int64_t k, int nb) {
  __shared__ double L[CH_NB][CH_NB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    L[i][j] = j <= i ? A[(k + i) * n + k + j] : 0.0;
  }
  __syncthreads();
  const int64_t i = k + nb + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  // (loops fully unrolled so that x stays in registers)
  double x[CH_NB];
  double* row = A + i * n + k;
#pragma unroll
  for (int j = 0; j < CH_NB; ++j) x[j] = j < nb ? row[j] : 0.0;
#pragma unroll
  for (int j = 0; j < CH_NB; ++j) {
    if (j < nb) {
      double v = x[j];
#pragma unroll
      for (int t = 0; t < j; ++t) v = fma(-x[t], L[j][t], v);
      x[j] = v / L[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < CH_NB; ++j)
    if (j < nb) row[j] = x[j];
}

// Trailing update: A[i][j] -= sum_t A[i][k+t] A[j][k+t] for k+nb <= j <= i < n.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ A, int64_t n, int64_t k, int nb) {
  const int64_t base = k + nb;
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ double Pi[CH_NB][CH_NB + 1], Pj[CH_NB][CH_NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * nb; e += 256) {
    const int r = e / nb, t = e - r * nb;
    const int64_t gi = base + bi * 64 + r, gj = base + bj * 64 + r;
    Pi[r][t] = gi < n ? A[gi * n + k + t] : 0.0;
    Pj[r][t] = gj < n ? A[gj * n + k + t] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    const int64_t gi = base + bi * 64 + r, gj = base + bj * 64 + c;
    if (gi >= n || gj >= n || gj > gi) continue;
    double s = 0.0;
    for (int t = 0; t < nb; ++t) s += Pi[r][t] * Pj[c][t];
    A[gi * n + gj] -= s;
  }
}

// strict upper triangle <- L^T
__global__ __launch_bounds__(256) void chol_mirror_kernel(double* __restrict__ A, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e / n, j = e - i * n;
  if (j > i) A[i * n + j] = A[j * n + i];
}

// out (m x c, float) = K (m x n, float, leading dim ld) X (n x c, double)
__global__ __launch_bounds__(256) void krr_matmul_kernel(const float* __restrict__ K, int64_t m, int64_t n,
                                                         int64_t ld, const double* __restrict__ X, int64_t c,
                                                         float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * c) return;
  const int64_t i = e / c, j = e - i * c;
  double s = 0.0;
  const float* row = K + i * ld;
  for (int64_t t = 0; t < n; ++t) s += (double)row[t] * X[t * c + j];
  out[e] = (float)s;
}

// pred = K_ts alpha (m x c); resid = pred - Y_t; G = 2 resid / (m c); sq = resid^2
__global__ __launch_bounds__(256) void krr_resid_kernel(const float* __restrict__ Kts, int64_t m, int64_t n,
                                                        const double* __restrict__ alpha, int64_t c,
                                                        const float* __restrict__ Yt, double* __restrict__ G,
                                                        double* __restrict__ sq) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * c) return;
  const int64_t i = e / c, k = e - i * c;
  double p = 0.0;
  for (int64_t t = 0; t < n; ++t) p += (double)Kts[i * n + t] * alpha[t * c + k];
  const double r = p - (double)Yt[e];
  G[e] = 2.0 * r / (double)(m * c);
  sq[e] = r * r;
}

// loss = sum(sq) / count, fixed-order reduction in one workgroup
__global__ __launch_bounds__(256) void krr_loss_kernel(const double* __restrict__ sq, int64_t cnt,
                                                       double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += 256) s += sq[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (double)cnt;
}

// B (n x c) = K_ts^T G
__global__ __launch_bounds__(256) void krr_ktg_kernel(const float* __restrict__ Kts, int64_t m, int64_t n,
                                                      const double* __restrict__ G, int64_t c,
                                                      double* __restrict__ B) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * c) return;
  const int64_t t = e / c, k = e - t * c;
  double s = 0.0;
  for (int64_t i = 0; i < m; ++i) s += (double)Kts[i * n + t] * G[i * c + k];
  B[e] = s;
}

// out (rows x cols, float) = scale * U V^T with U (rows x c), V (cols x c) double
__global__ __launch_bounds__(256) void krr_outer_kernel(const double* __restrict__ U, int64_t rows,
                                                        const double* __restrict__ V, int64_t cols, int64_t c,
                                                        double scale, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, t = e - i * cols;
  double s = 0.0;
  for (int64_t k = 0; k < c; ++k) s += U[i * c + k] * V[t * c + k];
  out[e] = (float)(scale * s);
}

int launch_krr_mse_bwd(const float* Kts, int64_t m, int64_t n, const double* alpha, int64_t c, const float* Yt,
                       double* G, double* sq, double* loss, double* B, hipStream_t s) {
  const unsigned g1 = (unsigned)((m * c + 255) / 256), g2 = (unsigned)((n * c + 255) / 256);
  hipLaunchKernelGGL(krr_resid_kernel, dim3(g1), dim3(256), 0, s, Kts, m, n, alpha, c, Yt, G, sq);
  hipLaunchKernelGGL(krr_loss_kernel, dim3(1), dim3(256), 0, s, sq, m * c, loss);
  hipLaunchKernelGGL(krr_ktg_kernel, dim3(g2), dim3(256), 0, s, Kts, m, n, G, c, B);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_krr_outer(const double* U, int64_t rows, const double* V, int64_t cols, int64_t c, double scale,
                     float* out, hipStream_t s) {
  hipLaunchKernelGGL(krr_outer_kernel, dim3((unsigned)((rows * cols + 255) / 256)), dim3(256), 0, s, U, rows, V, cols,
                     c, scale, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_cholesky(double* A, int64_t n, int* info, hipStream_t s) {
  for (int64_t k = 0; k < n; k += CH_NB) {
    const int nb = (int)((n - k) < CH_NB ? (n - k) : CH_NB);
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, A, n, k, nb, info);
    const int64_t rest = n - k - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(chol_trsm_kernel, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, s, A, n, k, nb);
      const unsigned nbk = (unsigned)((rest + 63) / 64);
      hipLaunchKernelGGL(chol_update_kernel, dim3(nbk, nbk), dim3(256), 0, s, A, n, k, nb);
    }
  }
  hipLaunchKernelGGL(chol_mirror_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, A, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---- blocked substitution for many right-hand sides ----------------------
//
// X = A^{-1} B with A = L L^T factored in place (L in the lower triangle):
// forward L Z = B and backward L^T X = Z in panels of CH_NB rows.  Each
// panel's triangle is solved with one thread per right-hand side (the
// triangle in LDS, the panel's unknowns in registers), and the rows not yet
// solved are updated with the float64 GEMM (X_rest -= L_rest,panel X_panel).

// X (n x c double) = B (float or double, n x c)
__global__ __launch_bounds__(256) void chol_rhs_copy_kernel(const float* __restrict__ Bf,
                                                            const double* __restrict__ Bd, int64_t nc,
                                                            double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < nc) X[e] = Bf ? (double)Bf[e] : Bd[e];
}

// Triangle of panel [k, k + nb) for every column: forward (L) or backward (L^T).
template <bool BACK>
__global__ __launch_bounds__(256) void chol_panel_kernel(const double* __restrict__ A, int64_t n, int64_t k, int nb,
                                                         double* __restrict__ X, int64_t c) {
  __shared__ double T[CH_NB][CH_NB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    T[i][j] = j <= i ? A[(k + i) * n + k + j] : 0.0;  // L of the panel
  }
  __syncthreads();
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= c) return;
  double x[CH_NB];
#pragma unroll
  for (int i = 0; i < CH_NB; ++i) x[i] = i < nb ? X[(k + i) * c + col] : 0.0;
  if (!BACK) {
#pragma unroll
    for (int i = 0; i < CH_NB; ++i) {
      if (i < nb) {
        double v = x[i];
#pragma unroll
        for (int j = 0; j < i; ++j) v = fma(-T[i][j], x[j], v);
        x[i] = v / T[i][i];
      }
    }
  } else {
#pragma unroll
    for (int i = CH_NB - 1; i >= 0; --i) {
      if (i < nb) {
        double v = x[i];
#pragma unroll
        for (int j = i + 1; j < CH_NB; ++j)
          if (j < nb) v = fma(-T[j][i], x[j], v);
        x[i] = v / T[i][i];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < CH_NB; ++i)
    if (i < nb) X[(k + i) * c + col] = x[i];
}

int launch_tri_solve(const double* A, int64_t n, double* X, int64_t c, bool upper, hipStream_t s) {
  if (n <= 0 || c <= 0) return 0;
  const unsigned gc = (unsigned)((c + 255) / 256);
  if (!upper) {
    for (int64_t k = 0; k < n; k += CH_NB) {
      const int nb = (int)((n - k) < CH_NB ? (n - k) : CH_NB);
      hipLaunchKernelGGL(chol_panel_kernel<false>, dim3(gc), dim3(256), 0, s, A, n, k, nb, X, c);
      const int64_t rest = n - k - nb;
      if (rest > 0 && dn_gemm_dd(A + (k + nb) * n + k, n, false, X + k * c, c, X + (k + nb) * c, c, rest, c, nb,
                                 -1.0, 1.0, false, s))
        return -3;
    }
  } else {
    const int64_t last = ((n - 1) / CH_NB) * CH_NB;
    for (int64_t k = last; k >= 0; k -= CH_NB) {
      const int nb = (int)((n - k) < CH_NB ? (n - k) : CH_NB);
      hipLaunchKernelGGL(chol_panel_kernel<true>, dim3(gc), dim3(256), 0, s, A, n, k, nb, X, c);
      // rows [0, k): X -= (L[k:k+nb, 0:k])^T X_panel
      if (k > 0 && dn_gemm_dd(A + k * n, n, true, X + k * c, c, X, c, k, c, nb, -1.0, 1.0, false, s)) return -3;
    }
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_chol_solve(const double* A, int64_t n, const float* Bf, const double* Bd, int64_t c, double* X,
                      hipStream_t s) {
  if (n <= 0 || c <= 0) return 0;
  hipLaunchKernelGGL(chol_rhs_copy_kernel, dim3((unsigned)((n * c + 255) / 256)), dim3(256), 0, s, Bf, Bd, n * c, X);
  if (launch_tri_solve(A, n, X, c, false, s) || launch_tri_solve(A, n, X, c, true, s)) return -3;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_krr_build(const float* K, int64_t n, double ridge_rel, double lam_abs, double* mean, double* A,
                     int* info, hipStream_t s) {
  if (ridge_rel >= 0.0) hipLaunchKernelGGL(krr_diag_mean_kernel, dim3(1), dim3(256), 0, s, K, n, n, mean);
  hipLaunchKernelGGL(krr_build_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, K, n, mean,
                     ridge_rel, lam_abs, A, info);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_krr_matmul(const float* K, int64_t m, int64_t n, int64_t ld, const double* X, int64_t c, float* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(krr_matmul_kernel, dim3((unsigned)((m * c + 255) / 256)), dim3(256), 0, s, K, m, n, ld, X, c,
                     out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace nk
