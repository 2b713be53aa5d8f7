// Kernel regression by preconditioned conjugate gradients in float64
// (Sec. 2, "Iterative solvers": CG with the partial pivoted Cholesky
// preconditioner; Sec. 1, related work: the preconditioner's origin and the
// need for high precision on neural kernels).
//
// System (K + lam I) X = Y, K the float32 Gram matrix the kernel entry points
// write (n x n, leading dim ldk, row-major, symmetric), Y and X float64
// (n x c).  Every product and sum runs in float64 on the float32 values of
// K, so the system solved is exactly double(K) + lam I.
//
// Pieces:
//   * pchol_*: greedy partial pivoted Cholesky K ~ L L^T (L n x r, column
//     major), one kernel per pivot: every workgroup reduces the previous
//     step's per-workgroup maxima of the residual diagonal d (largest value,
//     lowest index on ties), then forms its rows of the new column and
//     updates d.  Picked indices hold d = -inf.
//   * The preconditioner Ph = L L^T + lam I is applied with the Woodbury
//     identity Ph^{-1} v = (v - L M^{-1} L^T v) / lam, M = lam I + L^T L.
//     With M = R R^T (Cholesky) and U = L R^{-T}, formed once in place of L
//     by a blocked forward substitution, this is (v - U (U^T v)) / lam: two
//     skinny products per application and an operator that stays symmetric
//     in floating point (an explicitly inverted M does not, and CG then
//     stalls above small tolerances).
//   * kmv_*: Q = (K + lam I) P, the product that dominates each iteration:
//     K is streamed once from HBM as float4 rows.  Because K is symmetric,
//     Q[i] = sum_j K[j][i] P[j]: lane l of a wave owns columns 4l..4l+3 of a
//     1024-wide column block and walks the rows j of its row split; P[j][:]
//     is the same for the whole wave, so it arrives through scalar loads and
//     feeds the FMAs as a scalar operand.  Row splits write partial sums,
//     reduced in a fixed order by the next kernel (which also adds lam P and
//     the per-workgroup partials of p.q).
//   * CG vector steps; every dot product is reduced in a fixed order (per
//     workgroup partials, then one pass), so results are reproducible.
//     Per-column state (gamma, beta, active flag, iteration count, relative
//     residual) lives in device memory; a column that meets the tolerance
//     is frozen (alpha = beta = 0 from then on).
#include <float.h>
#include <limits.h>

#include "nk_kernels.h"

namespace nk {

constexpr int PC_TPB = 256;
constexpr double kNegInf = -__builtin_huge_val();

__device__ __forceinline__ bool pc_better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// Deterministic (value, index) maximum over a 256-thread workgroup.
__device__ inline void pc_block_argmax(double& v, int& i) {
  __shared__ double sv[PC_TPB];
  __shared__ int si[PC_TPB];
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = i;
  __syncthreads();
  for (int w = PC_TPB / 2; w >= 1; w >>= 1) {
    if (t < w && pc_better(sv[t + w], si[t + w], sv[t], si[t])) {
      sv[t] = sv[t + w];
      si[t] = si[t + w];
    }
    __syncthreads();
  }
  v = sv[0];
  i = si[0];
  __syncthreads();
}

// Fixed-order column sums by the PC_TPB threads of a workgroup: out[c] =
// sum_b part[b][c] (b < nb, c < C), through `red` (PC_TPB x C doubles of
// LDS); every thread sees out after the call.
template <int C>
__device__ inline void pc_colsum(const double* __restrict__ part, int nb, double* red, double* out) {
  const int t = threadIdx.x;
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  for (int b = t; b < nb; b += PC_TPB) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] += part[(int64_t)b * C + c];
  }
#pragma unroll
  for (int c = 0; c < C; ++c) red[t * C + c] = acc[c];
  __syncthreads();
  for (int w = PC_TPB / 2; w >= 1; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int c = 0; c < C; ++c) red[t * C + c] += red[(t + w) * C + c];
    }
    __syncthreads();
  }
  if (t < C) out[t] = red[t];
  __syncthreads();
}

// Fixed-order workgroup sums of one value per thread and column, written to
// out[0..C) (global), through `red` (PC_TPB x C doubles of LDS).
template <int C>
__device__ inline void pc_block_sums(const double (&v)[C], double* red, double* __restrict__ out) {
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < C; ++c) red[t * C + c] = v[c];
  __syncthreads();
  for (int w = PC_TPB / 2; w >= 1; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int c = 0; c < C; ++c) red[t * C + c] += red[(t + w) * C + c];
    }
    __syncthreads();
  }
  if (t < C) out[t] = red[t];
  __syncthreads();
}

// Fixed-order block sum of one value per thread, written to out (thread 0).
__device__ inline void pc_block_sum_store(double v, double* out) {
  __shared__ double red[PC_TPB];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = PC_TPB / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
  __syncthreads();
}

// d = diag(K); per-workgroup maximum of d.
__global__ __launch_bounds__(PC_TPB) void pchol_init_kernel(const float* __restrict__ K, int64_t n, int64_t ldk,
                                                            double* __restrict__ d, double* __restrict__ pv,
                                                            int* __restrict__ pi) {
  const int64_t i = (int64_t)blockIdx.x * PC_TPB + threadIdx.x;
  double v = -DBL_MAX;
  int idx = INT_MAX;
  if (i < n) {
    v = (double)K[i * ldk + i];
    d[i] = v;
    idx = (int)i;
  }
  pc_block_argmax(v, idx);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = v;
    pi[blockIdx.x] = idx;
  }
}

// Pivot step m: column m of L (column major, leading dim n) and the update of d.
__global__ __launch_bounds__(PC_TPB) void pchol_step_kernel(const float* __restrict__ K, int64_t n, int64_t ldk,
                                                            double* __restrict__ L, int m, double* __restrict__ d,
                                                            const double* __restrict__ pv_in,
                                                            const int* __restrict__ pi_in, int nb,
                                                            double* __restrict__ pv_out, int* __restrict__ pi_out,
                                                            int* __restrict__ piv, double* __restrict__ dpiv,
                                                            double pivot_tol) {
  extern __shared__ double lp[];  // L[p][0..m)
  const int t = threadIdx.x;
  double v = -DBL_MAX;
  int idx = INT_MAX;
  for (int b = t; b < nb; b += PC_TPB) {
    if (pc_better(pv_in[b], pi_in[b], v, idx)) {
      v = pv_in[b];
      idx = pi_in[b];
    }
  }
  pc_block_argmax(v, idx);
  const double dmax = v;
  const int p = idx;
  const double dmax0 = m == 0 ? dmax : dpiv[0];
  const int64_t i = (int64_t)blockIdx.x * PC_TPB + t;
  if (!(dmax > 0.0) || dmax <= pivot_tol * dmax0 || p >= n) {
    // rank reached: zero column, and pass the same maximum on so that every
    // later step stops too
    if (i < n) L[(int64_t)m * n + i] = 0.0;
    if (t == 0) {
      pv_out[blockIdx.x] = dmax;
      pi_out[blockIdx.x] = p;
      if (blockIdx.x == 0) {
        piv[m] = -1;
        dpiv[m] = 0.0;
      }
    }
    return;
  }
  for (int k = t; k < m; k += PC_TPB) lp[k] = L[(int64_t)k * n + p];
  __syncthreads();
  const double sp = sqrt(dmax);
  double nv = -DBL_MAX;
  int nidx = INT_MAX;
  if (i < n) {
    double di = d[i];
    double l;
    if (i == p) {
      l = sp;
      di = kNegInf;
    } else if (di == kNegInf) {
      l = 0.0;
    } else {
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < m; ++k) acc = fma(L[(int64_t)k * n + i], lp[k], acc);
      l = ((double)K[(int64_t)p * ldk + i] - acc) / sp;
      di -= l * l;
    }
    L[(int64_t)m * n + i] = l;
    d[i] = di;
    nv = di;
    nidx = (int)i;
  }
  pc_block_argmax(nv, nidx);
  if (t == 0) {
    pv_out[blockIdx.x] = nv;
    pi_out[blockIdx.x] = nidx;
    if (blockIdx.x == 0) {
      piv[m] = p;
      dpiv[m] = dmax;
    }
  }
}

int launch_pchol(const float* K, int64_t n, int64_t ldk, int rank, double pivot_tol, double* L, int* piv,
                 double* d, double* pv, int* pi, double* dpiv, hipStream_t s) {
  const int nb = (int)((n + PC_TPB - 1) / PC_TPB);
  hipLaunchKernelGGL(pchol_init_kernel, dim3(nb), dim3(PC_TPB), 0, s, K, n, ldk, d, pv, pi);
  for (int m = 0; m < rank; ++m) {
    const int a = m & 1, b = a ^ 1;
    hipLaunchKernelGGL(pchol_step_kernel, dim3(nb), dim3(PC_TPB), (size_t)(m > 0 ? m : 1) * sizeof(double), s, K,
                       n, ldk, L, m, d, pv + (size_t)a * nb, pi + (size_t)a * nb, nb, pv + (size_t)b * nb,
                       pi + (size_t)b * nb, piv, dpiv, pivot_tol);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---- preconditioner set-up ----------------------------------------------

// Lr (n x r, row major) <- L (n x r, column major)
__global__ __launch_bounds__(PC_TPB) void pc_transpose_kernel(const double* __restrict__ L, int64_t n, int r,
                                                              double* __restrict__ Lr) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int a0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int a = a0 + y;
    const int64_t i = i0 + tx;
    tile[y][tx] = (a < r && i < n) ? L[(int64_t)a * n + i] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t i = i0 + y;
    const int a = a0 + tx;
    if (a < r && i < n) Lr[i * r + a] = tile[tx][y];
  }
}

// M = lam I + L^T L (r x r, row major), 32 x 32 output tiles; also clears the
// factorisation flag.  The Woodbury form subtracts L M^{-1} L^T from the
// identity, which along the leading directions of K leaves only about
// lam / sigma^2 (sigma^2 up to the largest eigenvalue of K): so M has to
// match L^T L to about one rounding of its entries, or the preconditioner
// loses definiteness there and CG stalls.  A plain running sum over n rows
// is off by up to n roundings; the sums here carry their error terms
// (exact product errors by FMA, TwoSum for the additions) and round once.
__global__ __launch_bounds__(PC_TPB) void pc_ltl_kernel(const double* __restrict__ L, int64_t n, int r, double lam,
                                                        double* __restrict__ M, int* __restrict__ info) {
#pragma clang fp contract(off)
  __shared__ double A[32][33], B[32][33];
  const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of threads, 4 outputs each
  double hi[4] = {0.0, 0.0, 0.0, 0.0}, lo[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = 0; i0 < n; i0 += 32) {
    for (int y = ty; y < 32; y += 8) {
      const int64_t i = i0 + tx;
      A[y][tx] = (a0 + y < r && i < n) ? L[(int64_t)(a0 + y) * n + i] : 0.0;
      B[y][tx] = (b0 + y < r && i < n) ? L[(int64_t)(b0 + y) * n + i] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k) {
      const double bv = B[tx][k];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double av = A[ty + 8 * q][k];
        const double p = av * bv;
        const double pe = __builtin_fma(av, bv, -p);  // av bv - p exactly
        const double s = hi[q] + p;
        const double bb = s - hi[q];
        const double se = (hi[q] - (s - bb)) + (p - bb);  // hi + p - s exactly
        hi[q] = s;
        lo[q] += se + pe;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = a0 + ty + 8 * q, b = b0 + tx;
    if (a < r && b < r) {
      double v = hi[q];
      double e = lo[q];
      if (a == b) {
        const double s = v + lam;
        const double bb = s - v;
        e += (v - (s - bb)) + (lam - bb);
        v = s;
      }
      M[(int64_t)a * r + b] = v + e;
    }
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) info[0] = 0;
}

int launch_pc_setup(double* LU, int64_t n, int r, double lam, double* Ur, double* M, int* info, hipStream_t s) {
  if (r == 0) return 0;
  const unsigned g = (unsigned)((r + 31) / 32);
  hipLaunchKernelGGL(pc_ltl_kernel, dim3(g, g), dim3(PC_TPB), 0, s, LU, n, r, lam, M, info);
  if (launch_cholesky(M, r, info, s)) return -3;
  // U = L R^{-T} in place: with L stored column major (an r x n row-major
  // array), U^T = R^{-1} L^T is a forward substitution with n right-hand
  // sides, run blocked (panel triangles and float64 GEMM updates)
  if (launch_tri_solve(M, r, LU, n, false, s)) return -3;
  hipLaunchKernelGGL(pc_transpose_kernel, dim3((unsigned)((n + 31) / 32), (unsigned)((r + 31) / 32)), dim3(PC_TPB),
                     0, s, LU, n, r, Ur);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---- Q = (K + lam I) P ----------------------------------------------------

constexpr int KMV_COLS = 1024;  // columns of K per workgroup (4 waves x 64 lanes x 4)
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Partial sums over rows [j0, j1) of K for the 1024 columns of this block:
// part[s][i][c] = sum_j K[j][i] P[j][c].
// A kernel of a conjugate-gradient iteration returns at once when its gate
// (the solver's "some column still iterates" flag) reads 0.
#define NK_PCG_GATE(g) \
  if ((g) != nullptr && *(g) == 0) return;

template <int C, bool VEC>
__global__ __launch_bounds__(PC_TPB) void kmv_partial_kernel(const float* __restrict__ K, int64_t n, int64_t ldk,
                                                             const double* __restrict__ P, int64_t rows_per_split,
                                                             double* __restrict__ part, const int* __restrict__ gate) {
  NK_PCG_GATE(gate)
  const int64_t i0 = (int64_t)blockIdx.x * KMV_COLS + 4 * threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t j1 = j0 + rows_per_split < n ? j0 + rows_per_split : n;
  double acc[4][C];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[e][c] = 0.0;
  if (i0 < n && j0 < j1) {
    if (VEC) {
      // four rows per step, all four loads issued before their FMAs; K is
      // read once per product, so its loads are non-temporal (they do not
      // evict P from the caches)
      const float* kb = K + i0;
      int64_t j = j0;
      for (; j + 4 <= j1; j += 4) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(kb + (j + u) * ldk));
          v[u] = make_float4(t.x, t.y, t.z, t.w);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float kv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
          const double* pr = P + (j + u) * C;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double kd = (double)kv[e];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[e][c] = fma(kd, pr[c], acc[e][c]);
          }
        }
      }
      for (; j < j1; ++j) {
        const float4 v = *reinterpret_cast<const float4*>(kb + j * ldk);
        const float kv[4] = {v.x, v.y, v.z, v.w};
        const double* pr = P + j * C;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double kd = (double)kv[e];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[e][c] = fma(kd, pr[c], acc[e][c]);
        }
      }
    } else {
      const float* kp = K + j0 * ldk + i0;
      for (int64_t j = j0; j < j1; ++j, kp += ldk) {
        float kv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) kv[e] = i0 + e < n ? kp[e] : 0.f;
        const double* pr = P + j * C;
        double pj[C];
#pragma unroll
        for (int c = 0; c < C; ++c) pj[c] = pr[c];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double kd = (double)kv[e];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[e][c] = fma(kd, pj[c], acc[e][c]);
        }
      }
    }
  }
  double* out = part + (int64_t)blockIdx.y * n * C;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (i0 + e < n) {
#pragma unroll
      for (int c = 0; c < C; ++c) out[(i0 + e) * C + c] = acc[e][c];
    }
  }
}

// Q[i] = sum_s part[s][i] + lam P[i]; per-workgroup partials of p.q per column.
template <int C>
__global__ __launch_bounds__(PC_TPB) void kmv_reduce_kernel(const double* __restrict__ part, int S, int64_t n,
                                                            const double* __restrict__ P, double lam,
                                                            double* __restrict__ Q, double* __restrict__ pq_part,
                                                            const int* __restrict__ gate) {
  NK_PCG_GATE(gate)
  __shared__ double red[PC_TPB * C];
  const int64_t i = (int64_t)blockIdx.x * PC_TPB + threadIdx.x;
  double q[C], d[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    q[c] = 0.0;
    d[c] = 0.0;
  }
  if (i < n) {
#pragma unroll 4
    for (int s = 0; s < S; ++s) {
      const double* ps = part + ((int64_t)s * n + i) * C;
#pragma unroll
      for (int c = 0; c < C; ++c) q[c] += ps[c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double pv = P[i * C + c];
      q[c] = fma(lam, pv, q[c]);
      Q[i * C + c] = q[c];
      d[c] = pv * q[c];
    }
  }
  pc_block_sums<C>(d, red, pq_part + (int64_t)blockIdx.x * C);
}

// Row splits of the product: about 512 workgroups (8 waves per CU, each with
// four rows in flight), at least 64 rows each.  Measured on a 32768 x 32768
// K: 16 splits stream at 6.5-6.7 TB/s, 32 at 6.0, 64 at 5.5, 8 at 4.8.
int kmv_splits(int64_t n) {
  const int64_t ncb = (n + KMV_COLS - 1) / KMV_COLS;
  int64_t S = (512 + ncb - 1) / ncb;
  const int64_t maxS = (n + 63) / 64;
  if (S > maxS) S = maxS;
  if (S > 64) S = 64;
  return (int)(S < 1 ? 1 : S);
}

template <int C>
int launch_kmv_c(const float* K, int64_t n, int64_t ldk, const double* P, double lam, double* part, double* Q,
                 double* pq_part, const int* gate, hipStream_t s, ProfHook* hook) {
  const int S = kmv_splits(n);
  const int64_t rows = (n + S - 1) / S;
  const bool vec = (ldk % 4 == 0) && ((reinterpret_cast<uintptr_t>(K) & 15) == 0);
  const dim3 grid((unsigned)((n + KMV_COLS - 1) / KMV_COLS), (unsigned)S);
  if (hook) hook->begin(s);
  if (vec)
    hipLaunchKernelGGL((kmv_partial_kernel<C, true>), grid, dim3(PC_TPB), 0, s, K, n, ldk, P, rows, part, gate);
  else
    hipLaunchKernelGGL((kmv_partial_kernel<C, false>), grid, dim3(PC_TPB), 0, s, K, n, ldk, P, rows, part, gate);
  if (hook) hook->end(s);
  hipLaunchKernelGGL((kmv_reduce_kernel<C>), dim3((unsigned)((n + PC_TPB - 1) / PC_TPB)), dim3(PC_TPB), 0, s, part,
                     S, n, P, lam, Q, pq_part, gate);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---- CG vector steps ------------------------------------------------------

// Per-column state of a CG pass.
struct PcgState {
  double* gamma;   // r.z of the current residual
  double* beta;    // last beta
  double* ynorm;   // ||y||
  double* relres;  // ||r|| / ||y|| at the column's last update
  int* active;     // 1 while the column iterates
  int* iters;      // updates taken
  int* any;        // 1 while some column iterates (the gate of every iteration kernel)
};

// st.any = OR of st.active[0..C) (after a barrier that follows the last
// write of st.active)
template <int C>
__device__ inline void pc_store_any(const PcgState& st) {
  if (threadIdx.x == 0) {
    int a = 0;
    for (int c = 0; c < C; ++c) a |= st.active[c];
    *st.any = a;
  }
}

// R = Y[:, c0:c0+C], X = 0; partials of ||y||^2.
template <int C>
__global__ __launch_bounds__(PC_TPB) void pcg_init_kernel(const double* __restrict__ Y, int64_t ldy, int64_t c0,
                                                          int64_t n, double* __restrict__ R, double* __restrict__ X,
                                                          double* __restrict__ yy_part) {
  const int64_t i = (int64_t)blockIdx.x * PC_TPB + threadIdx.x;
  double y[C];
#pragma unroll
  for (int c = 0; c < C; ++c) y[c] = 0.0;
  if (i < n) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      y[c] = Y[i * ldy + c0 + c];
      R[i * C + c] = y[c];
      X[i * C + c] = 0.0;
    }
  }
  __shared__ double red[PC_TPB * C];
  double yy[C];
#pragma unroll
  for (int c = 0; c < C; ++c) yy[c] = y[c] * y[c];
  pc_block_sums<C>(yy, red, yy_part + (int64_t)blockIdx.x * C);
}

template <int C>
__global__ __launch_bounds__(PC_TPB) void pcg_init_state_kernel(const double* __restrict__ yy_part, int nb,
                                                                PcgState st) {
  __shared__ double red[PC_TPB * C];
  __shared__ double sum[C];
  pc_colsum<C>(yy_part, nb, red, sum);
  const int c = threadIdx.x;
  if (c < C) {
    const double yn = sqrt(sum[c]);
    st.ynorm[c] = yn;
    st.active[c] = yn > 0.0 ? 1 : 0;
    st.iters[c] = 0;
    st.relres[c] = yn > 0.0 ? 1.0 : 0.0;
    st.beta[c] = 0.0;
  }
  __syncthreads();
  pc_store_any<C>(st);
}

// W partial: wpart[s][a][c] = sum_{i in split s} Ur[i][a] V[i][c].  A
// workgroup takes 64 columns a (lanes) of one row split; its four waves take
// every fourth row of the split (eight rows in flight each) and add in LDS.
template <int C>
__global__ __launch_bounds__(PC_TPB) void pc_lt_kernel(const double* __restrict__ Ur, int64_t n, int r,
                                                       const double* __restrict__ V, int64_t rows_per_split,
                                                       double* __restrict__ wpart, const int* __restrict__ gate) {
  NK_PCG_GATE(gate)
  __shared__ double red[3][64][C];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int a = blockIdx.x * 64 + lane;
  const int64_t i0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t i1 = i0 + rows_per_split < n ? i0 + rows_per_split : n;
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  if (a < r) {
#pragma unroll 8
    for (int64_t i = i0 + wv; i < i1; i += 4) {
      const double l = Ur[i * r + a];
      const double* vr = V + i * C;
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = fma(l, vr[c], acc[c]);
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int c = 0; c < C; ++c) red[wv - 1][lane][c] = acc[c];
  }
  __syncthreads();
  if (wv == 0 && a < r) {
    double* o = wpart + ((int64_t)blockIdx.y * r + a) * C;
#pragma unroll
    for (int c = 0; c < C; ++c) o[c] = ((acc[c] + red[0][lane][c]) + red[1][lane][c]) + red[2][lane][c];
  }
}

// W[a][c] = sum_s wpart[s][a][c]
template <int C>
__global__ __launch_bounds__(PC_TPB) void pc_w_reduce_kernel(const double* __restrict__ wpart, int S, int r,
                                                             double* __restrict__ W, const int* __restrict__ gate) {
  NK_PCG_GATE(gate)
  const int e = blockIdx.x * PC_TPB + threadIdx.x;
  if (e >= r * C) return;
  double s = 0.0;
#pragma unroll 8
  for (int q = 0; q < S; ++q) s += wpart[(int64_t)q * r * C + e];
  W[e] = s;
}

// Rows of the preconditioned vector per workgroup of pc_z_kernel (its four
// waves take a quarter of the rank each and add in LDS).
constexpr int PC_ZROWS = 64;

// Z[i] = (V[i] - sum_a U[a][i] W[a]) / lam; partials of v.z per column.
template <int C>
__global__ __launch_bounds__(PC_TPB) void pc_z_kernel(const double* __restrict__ U, int64_t n, int r,
                                                      const double* __restrict__ W, const double* __restrict__ V,
                                                      double lam, double* __restrict__ Z,
                                                      double* __restrict__ vz_part, const int* __restrict__ gate) {
  NK_PCG_GATE(gate)
  __shared__ double red[4][PC_ZROWS][C];  // wave partials, then the block sums (PC_TPB x C)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * PC_ZROWS + lane;
  const int a0 = (int)((int64_t)r * wv / 4), a1 = (int)((int64_t)r * (wv + 1) / 4);
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  if (i < n) {
#pragma unroll 4
    for (int a = a0; a < a1; ++a) {
      const double l = U[(int64_t)a * n + i];
      const double* w = W + (int64_t)a * C;
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = fma(l, w[c], acc[c]);
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int c = 0; c < C; ++c) red[wv - 1][lane][c] = acc[c];
  }
  __syncthreads();
  double d[C];
#pragma unroll
  for (int c = 0; c < C; ++c) d[c] = 0.0;
  if (wv == 0 && i < n) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double t = ((acc[c] + red[0][lane][c]) + red[1][lane][c]) + red[2][lane][c];
      const double v = V[i * C + c];
      const double z = (v - t) / lam;
      Z[i * C + c] = z;
      d[c] = v * z;
    }
  }
  __syncthreads();
  pc_block_sums<C>(d, &red[0][0][0], vz_part + (int64_t)blockIdx.x * C);
}

// alpha = gamma / p.q for active columns (0 otherwise); X += alpha P,
// R -= alpha Q; partials of ||r||^2.
template <int C>
__global__ __launch_bounds__(PC_TPB) void pcg_update_kernel(int64_t n, const double* __restrict__ pq_part, int nb,
                                                            PcgState st, const double* __restrict__ P,
                                                            const double* __restrict__ Q, double* __restrict__ X,
                                                            double* __restrict__ R, double* __restrict__ rr_part) {
  NK_PCG_GATE(st.any)
  __shared__ double red[PC_TPB * C];
  __shared__ double alpha[C];
  pc_colsum<C>(pq_part, nb, red, alpha);
  if (threadIdx.x < C) {
    const int c = threadIdx.x;
    alpha[c] = st.active[c] ? st.gamma[c] / alpha[c] : 0.0;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * PC_TPB + threadIdx.x;
  double rr[C];
#pragma unroll
  for (int c = 0; c < C; ++c) rr[c] = 0.0;
  if (i < n) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t e = i * C + c;
      X[e] = fma(alpha[c], P[e], X[e]);
      const double rv = fma(-alpha[c], Q[e], R[e]);
      R[e] = rv;
      rr[c] = rv * rv;
    }
  }
  pc_block_sums<C>(rr, red, rr_part + (int64_t)blockIdx.x * C);
}

// After the update of iteration `it`: residuals, stopping test, counts, and
// the gate for the rest of the pass.
template <int C>
__global__ __launch_bounds__(PC_TPB) void pcg_residual_kernel(const double* __restrict__ rr_part, int nb,
                                                              PcgState st, int it, double tol) {
  NK_PCG_GATE(st.any)
  __shared__ double red[PC_TPB * C];
  __shared__ double sum[C];
  pc_colsum<C>(rr_part, nb, red, sum);
  const int c = threadIdx.x;
  if (c < C && st.active[c]) {
    const double rel = sqrt(sum[c]) / st.ynorm[c];
    st.relres[c] = rel;
    st.iters[c] = it + 1;
    if (rel <= tol) st.active[c] = 0;
  }
  __syncthreads();
  pc_store_any<C>(st);
}

// gamma' = r.z; beta = gamma'/gamma for active columns (0 otherwise);
// gamma <- gamma' for active columns.  first: gamma <- gamma' only.
template <int C>
__global__ __launch_bounds__(PC_TPB) void pcg_beta_kernel(const double* __restrict__ rz_part, int nb, PcgState st,
                                                          int first) {
  NK_PCG_GATE(st.any)
  __shared__ double red[PC_TPB * C];
  __shared__ double sum[C];
  pc_colsum<C>(rz_part, nb, red, sum);
  const int c = threadIdx.x;
  if (c >= C) return;
  const double g = sum[c];
  if (first) {
    st.gamma[c] = g;
    st.beta[c] = 0.0;
    return;
  }
  const bool act = st.active[c] != 0;
  st.beta[c] = act ? g / st.gamma[c] : 0.0;
  if (act) st.gamma[c] = g;
}

// P = Z + beta P  (first: P = Z)
template <int C>
__global__ __launch_bounds__(PC_TPB) void pcg_direction_kernel(int64_t n, PcgState st, const double* __restrict__ Z,
                                                               double* __restrict__ P, int first) {
  NK_PCG_GATE(st.any)
  const int64_t e = (int64_t)blockIdx.x * PC_TPB + threadIdx.x;
  if (e >= n * C) return;
  const int c = (int)(e % C);
  P[e] = first ? Z[e] : fma(st.beta[c], P[e], Z[e]);
}

// X[:, c0:c0+C] of the caller's n x ldx output
template <int C>
__global__ __launch_bounds__(PC_TPB) void pcg_store_kernel(int64_t n, const double* __restrict__ Xg,
                                                           double* __restrict__ X, int64_t ldx, int64_t c0) {
  const int64_t e = (int64_t)blockIdx.x * PC_TPB + threadIdx.x;
  if (e >= n * C) return;
  const int64_t i = e / C;
  const int c = (int)(e - i * C);
  X[i * ldx + c0 + c] = Xg[e];
}

// One CG pass over a group of C <= 16 right-hand-side columns.  The host
// enqueues iterations ahead of the device and reads the gate of iteration
// it - 2 (copied to pinned host memory behind an event) before enqueueing
// iteration it, so the device never waits for the host; iterations
// enqueued after every column stopped return at once.
template <int C>
int pcg_group(const PcgArgs& a, int64_t c0, hipStream_t s) {
  const int64_t n = a.n;
  const int nb = (int)((n + PC_TPB - 1) / PC_TPB);
  const int nbz = (int)((n + PC_ZROWS - 1) / PC_ZROWS);
  const unsigned gv = (unsigned)((n * C + PC_TPB - 1) / PC_TPB);
  PcgState st{a.gamma, a.beta, a.ynorm, a.relres, a.active, a.iters, a.any};
  const int lt_splits = a.lt_splits;
  const int64_t lt_rows = (n + lt_splits - 1) / lt_splits;

  auto precond = [&](const double* V, double* Z, double* vz_part) {
    if (a.r > 0) {
      hipLaunchKernelGGL((pc_lt_kernel<C>), dim3((unsigned)((a.r + 63) / 64), (unsigned)lt_splits), dim3(PC_TPB), 0, s,
                         a.Ur, n, a.r, V, lt_rows, a.wpart, a.any);
      hipLaunchKernelGGL((pc_w_reduce_kernel<C>), dim3((unsigned)((a.r * C + PC_TPB - 1) / PC_TPB)), dim3(PC_TPB), 0,
                         s, a.wpart, lt_splits, a.r, a.W, a.any);
    }
    hipLaunchKernelGGL((pc_z_kernel<C>), dim3(nbz), dim3(PC_TPB), 0, s, a.U, n, a.r, a.W, V, a.lam, Z, vz_part,
                       a.any);
  };

  hipLaunchKernelGGL((pcg_init_kernel<C>), dim3(nb), dim3(PC_TPB), 0, s, a.Y, a.ldy, c0, n, a.R, a.X, a.part1);
  hipLaunchKernelGGL((pcg_init_state_kernel<C>), dim3(1), dim3(PC_TPB), 0, s, a.part1, nb, st);
  precond(a.R, a.Z, a.part2);
  hipLaunchKernelGGL((pcg_beta_kernel<C>), dim3(1), dim3(PC_TPB), 0, s, a.part2, nbz, st, 1);
  hipLaunchKernelGGL((pcg_direction_kernel<C>), dim3(gv), dim3(PC_TPB), 0, s, n, st, a.Z, a.P, 1);
  if (hipGetLastError() != hipSuccess) return -3;

  int rc = 0;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (int e = 0; e < 3 && rc == 0; ++e)
    if (hipEventCreateWithFlags(&ev[e], hipEventDisableTiming) != hipSuccess) rc = -3;
  for (int it = 0; it < a.max_iter && rc == 0; ++it) {
    if (it >= 2) {
      if (hipEventSynchronize(ev[(it - 2) % 3]) != hipSuccess) {
        rc = -3;
        break;
      }
      if (a.host_any[(it - 2) % 3] == 0) break;
    }
    if (launch_kmv_c<C>(a.K, n, a.ldk, a.P, a.lam, a.kpart, a.Q, a.part1, a.any, s, a.hook)) {
      rc = -3;
      break;
    }
    hipLaunchKernelGGL((pcg_update_kernel<C>), dim3(nb), dim3(PC_TPB), 0, s, n, a.part1, nb, st, a.P, a.Q, a.X, a.R,
                       a.part2);
    hipLaunchKernelGGL((pcg_residual_kernel<C>), dim3(1), dim3(PC_TPB), 0, s, a.part2, nb, st, it, a.tol);
    precond(a.R, a.Z, a.part1);
    hipLaunchKernelGGL((pcg_beta_kernel<C>), dim3(1), dim3(PC_TPB), 0, s, a.part1, nbz, st, 0);
    hipLaunchKernelGGL((pcg_direction_kernel<C>), dim3(gv), dim3(PC_TPB), 0, s, n, st, a.Z, a.P, 0);
    if (hipMemcpyAsync(&a.host_any[it % 3], a.any, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(ev[it % 3], s) != hipSuccess || hipGetLastError() != hipSuccess)
      rc = -3;
  }
  for (int e = 0; e < 3; ++e)
    if (ev[e]) (void)hipEventDestroy(ev[e]);
  if (rc) return rc;
  hipLaunchKernelGGL((pcg_store_kernel<C>), dim3(gv), dim3(PC_TPB), 0, s, n, a.X, a.Xout, a.ldx, c0);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_pcg_group(const PcgArgs& a, int64_t c0, int C, hipStream_t s) {
  switch (C) {
    case 1: return pcg_group<1>(a, c0, s);
    case 2: return pcg_group<2>(a, c0, s);
    case 3: return pcg_group<3>(a, c0, s);
    case 4: return pcg_group<4>(a, c0, s);
    case 5: return pcg_group<5>(a, c0, s);
    case 6: return pcg_group<6>(a, c0, s);
    case 7: return pcg_group<7>(a, c0, s);
    case 8: return pcg_group<8>(a, c0, s);
    case 9: return pcg_group<9>(a, c0, s);
    case 10: return pcg_group<10>(a, c0, s);
    case 11: return pcg_group<11>(a, c0, s);
    case 12: return pcg_group<12>(a, c0, s);
    case 13: return pcg_group<13>(a, c0, s);
    case 14: return pcg_group<14>(a, c0, s);
    case 15: return pcg_group<15>(a, c0, s);
    case 16: return pcg_group<16>(a, c0, s);
    default: return -1;
  }
}

int launch_kmv(const float* K, int64_t n, int64_t ldk, const double* P, int C, double lam, double* part, double* Q,
               double* pq_part, hipStream_t s, ProfHook* hook) {
  switch (C) {
#define NK_KMV_CASE(c) \
  case c:              \
    return launch_kmv_c<c>(K, n, ldk, P, lam, part, Q, pq_part, nullptr, s, hook);
    NK_KMV_CASE(1) NK_KMV_CASE(2) NK_KMV_CASE(3) NK_KMV_CASE(4) NK_KMV_CASE(5) NK_KMV_CASE(6) NK_KMV_CASE(7)
    NK_KMV_CASE(8) NK_KMV_CASE(9) NK_KMV_CASE(10) NK_KMV_CASE(11) NK_KMV_CASE(12) NK_KMV_CASE(13)
    NK_KMV_CASE(14) NK_KMV_CASE(15) NK_KMV_CASE(16)
#undef NK_KMV_CASE
    default:
      return -1;
  }
}

// out[0] = mean(diag K)
__global__ __launch_bounds__(PC_TPB) void pc_diag_mean_kernel(const float* __restrict__ K, int64_t n, int64_t ldk,
                                                              double* __restrict__ out) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += PC_TPB) s += (double)K[i * ldk + i];
  pc_block_sum_store(s, out);
  if (threadIdx.x == 0) out[0] = out[0] / (double)n;
}

int launch_diag_mean(const float* K, int64_t n, int64_t ldk, double* out, hipStream_t s) {
  hipLaunchKernelGGL(pc_diag_mean_kernel, dim3(1), dim3(PC_TPB), 0, s, K, n, ldk, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace nk
