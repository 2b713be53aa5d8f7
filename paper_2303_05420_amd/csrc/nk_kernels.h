// Kernel argument blocks and launchers shared between the HIP translation
// units of libnk and its host API.
#pragma once
#include <atomic>

#include "nk_common.h"

namespace nk {

// Dynamic LDS beyond 64 KiB has to be allowed per kernel, and per device.
// `seen` is one kernel's record of the largest size already allowed on each
// device (a zero-initialised static array of kMaxDevices in its launcher);
// devices beyond kMaxDevices are set on every call.  Returns 0 or -3.
constexpr int kMaxDevices = 64;
inline int allow_dyn_lds(const void* fn, size_t lds, std::atomic<size_t>* seen) {
  if (lds <= 64 * 1024) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -3;
  std::atomic<size_t>* rec = (dev >= 0 && dev < kMaxDevices) ? &seen[dev] : nullptr;
  if (rec && rec->load(std::memory_order_acquire) >= lds) return 0;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return -3;
  if (rec) {
    size_t cur = rec->load(std::memory_order_relaxed);
    while (cur < lds && !rec->compare_exchange_weak(cur, lds, std::memory_order_acq_rel)) {
    }
  }
  return 0;
}

struct PrepArgs {
  const float* x;     // images NHWC
  int64_t n;          // images in this launch
  NetDesc net;
  float2* tab;        // n * table_len float2
  double* scratch;    // n_blocks * scratch_per_img doubles (one region per workgroup)
  int64_t scratch_per_img;
};

// One Gram tile of a batched pass, in device memory.  Its pairs are global
// pairs [p_begin, p_begin + pair_count(n1, n2, sym)) of the pass; its images'
// tables are rows t1 + a and t2 + b of the pass's table array.
struct TileDesc {
  int64_t p_begin;
  int64_t n1, n2;
  int64_t t1, t2;
  const float* x1;
  const float* x2;
  float* K;
  int64_t ldk;
  int sym, pad;
};

struct StageArgs {
  int64_t n1, n2;
  int sym, T;
  int64_t p0, np;  // chunk = pairs [p0, p0 + np) of the block order
  const TileDesc* tiles;  // batched pass: tile table (NULL: one block given by n1, n2, x1, x2, K)
  int ntiles;
  int persist;     // > 0: grid of `persist` workgroups looping over the chunk
  const float* x1;
  const float* x2;
  const float2* tab1;
  const float2* tab2;
  int tablen, taboff;
  int C, D;
  float sb2, seed_scale;
  int64_t img_floats;  // floats per input image (H W C): the tangent kernel compares the two images of a pair
  const float* in;  // [np][N][N][N][N]      (stages after the first)
  float* out;       // [np][N/2][N/2][N/2][N/2] (pooling stages)
  float* K;         // final stage (NULL: not written)
  int64_t ldk;
  // tangent kernel (NTK launches only): the carried C tiles in and out, the
  // NTK block (same ldk), kappa / 2 of each layer of the stage
  const float* in2;
  float* out2;
  float* K2;
  float kh[NK_MAX_DEPTH];
};

struct StageBwdArgs {
  int64_t n1, n2;
  int sym, T;
  int64_t p0, np;
  const float* x1;
  const float* x2;
  const float2* tab1;
  const float2* tab2;
  int tablen, taboff;
  int C, D;
  float sb2, seed_scale;
  int64_t img_floats;  // floats per input image (H W C), for the identical-image test of a pair
  const float* in;    // stage input [np][N]^4 (stages after the first)
  const float* gin;   // adjoint of the next stage's input [np][N/2]^4 (all but the last stage)
  float* gout;        // adjoint of this stage's input [np][N]^4 (stages after the first)
  const float* dK;    // cotangent of the block (last stage)
  int64_t lddk;
  int last;           // 1 for the last stage (adjoint from dK), else from gin
  double* W1;         // per image w sums, table layout [img][tablen]
  double* W2;
  double* xbar1;      // per image seed gradients [img][N N C] (first stage)
  double* xbar2;
  int xj;             // 1: accumulate xbar2; 0: x2's seed gradients are not wanted (xbar2 may be null at 32x32)
  int dk_t;           // 1: dK is stored transposed, dK[x2 row * lddk + x1 row]
  double* sums;       // [0]: sigma_w2 * dL/dsigma_w2 terms, [1]: dL/dsigma_b2 terms
};

struct PrepBwdArgs {
  const float* x;
  int64_t n;
  NetDesc net;
  const double* W;    // w sums of these images [n][tablen]
  int tablen;
  double* xbar;       // += image gradients [n][H W C]
  double* sums;
  double* scratch;
  int64_t scratch_per_img;
};

struct FcArgs {
  const float* x1;
  const float* x2;
  int64_t n1, n2;
  int d, depth;
  float sw2, sb2;
  const float* d1;  // first-layer diagonals
  const float* d2;
  float* K;
  int64_t ldk;
  int sym;  // x1 and x2 are the same images: upper-triangle tiles, mirrored
};

int64_t prep_scratch_doubles(const NetDesc& net);
int launch_prepare(const float* x, int64_t n, const NetDesc& net, float2* tab, double* scratch,
                   int64_t max_blocks, hipStream_t stream);
size_t stage_lds_bytes(int N, int D, bool pool, bool seed);
// ppm: pairs-per-workgroup multiplier (1 or 2) of the stage kernels of tiles
// of at most 16 x 16 (a kernel-shape choice of the batched pass; results do
// not depend on it); ignored for larger tiles.
int launch_stage(int N, const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s, int ppm = 1);
// first stage at 64x64 (seed, D <= 2 layers, pool; plain blocks only)
size_t stage64_lds_bytes(int D, int C);
int launch_stage64(const StageArgs& a, bool bias, hipStream_t s);
size_t stage_ntk_lds_bytes(int N, int D, bool pool, bool seed);
int launch_stage_ntk(int N, const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s);
int prime_stage(int N, int D, bool seed, bool pool, bool bias, int C, int ppm = 1);  // kernel attributes, no launch
int launch_put_tiles(const TileDesc* host, int n, TileDesc* dst, hipStream_t stream);
int stage_occupancy(int N, int D, bool seed, bool pool, bool bias, int C, int ppm = 1);  // resident workgroups per CU
int stage_pairs_per_wg(int N, bool pool, int ppm);  // pairs per workgroup of the stage kernel
// the 32x32 pooling stage with two tile columns per lane (stage32.hip)
size_t stage32_lds_bytes(int D, bool seed);
int launch_stage32(const StageArgs& a, bool seed, bool bias, hipStream_t s);
int stage32_occupancy(int D, bool seed, bool bias, int C);
int launch_fc(const FcArgs& a, float* d1, float* d2, hipStream_t stream);
size_t stage_bwd_lds_bytes(int N, int D, bool seed);
int launch_stage_bwd(int N, const StageBwdArgs& a, bool seed, hipStream_t s);
int launch_stage_bwd_32(const StageBwdArgs& a, bool seed, hipStream_t s);
int launch_stage_bwd_16(const StageBwdArgs& a, bool seed, hipStream_t s);
int launch_stage_bwd_small(int N, const StageBwdArgs& a, bool seed, hipStream_t s);
int64_t prep_bwd_scratch_doubles(const NetDesc& net);
int launch_prepare_bwd(const float* x, int64_t n, const NetDesc& net, const double* W, int tablen, double* xbar,
                       double* sums, double* scratch, int64_t max_blocks, hipStream_t stream);
int launch_cast_grad(const double* src, float* dst, int64_t n, hipStream_t s);
int launch_finish_sigma(const double* sums, double sw2, float* dsigma, hipStream_t s);
// out (cols x rows) = in^T (rows x cols), both dense; rows <= 65535 * 32.
int launch_transpose_f32(const float* in, int64_t rows, int64_t cols, float* out, hipStream_t s);
int launch_zero_f64(double* p, int64_t n, hipStream_t s);
int launch_cholesky(double* A, int64_t n, int* info, hipStream_t s);
// In place X (n x c, row-major) <- L^{-1} X (upper = false) or L^{-T} X
// (upper = true), L the factor launch_cholesky left in A.
int launch_tri_solve(const double* A, int64_t n, double* X, int64_t c, bool upper, hipStream_t s);
int launch_chol_solve(const double* A, int64_t n, const float* Bf, const double* Bd, int64_t c, double* X,
                      hipStream_t s);
int launch_krr_build(const float* K, int64_t n, double ridge_rel, double lam_abs, double* mean, double* A,
                     int* info, hipStream_t s);
int launch_krr_mse_bwd(const float* Kts, int64_t m, int64_t n, const double* alpha, int64_t c, const float* Yt,
                       double* G, double* sq, double* loss, double* B, hipStream_t s);
int launch_krr_outer(const double* U, int64_t rows, const double* V, int64_t cols, int64_t c, double scale,
                     float* out, hipStream_t s);
int launch_krr_matmul(const float* K, int64_t m, int64_t n, int64_t ld, const double* X, int64_t c, float* out,
                      hipStream_t s);

// Event bracket around one launch (the host API times the product that
// dominates a conjugate-gradient iteration through it).
struct ProfHook {
  virtual void begin(hipStream_t s) = 0;
  virtual void end(hipStream_t s) = 0;
  virtual ~ProfHook() {}
};

// One preconditioned conjugate-gradient solve (pcg.hip).  All arrays are
// device memory; n x C blocks are row-major with leading dim C.
struct PcgArgs {
  const float* K;
  int64_t n, ldk;
  const double* Y;  // n x ldy, columns c0 .. c0 + C of this group
  int64_t ldy;
  double* Xout;     // n x ldx
  int64_t ldx;
  double lam, tol;
  int max_iter;
  int r;                 // preconditioner rank (0: Ph = lam I)
  const double* U;       // n x r, column major: L R^{-T}, R R^T = lam I + L^T L
  const double* Ur;      // the same, row major
  double* W;             // r x 16
  double* wpart;         // lt_splits x r x 16
  int lt_splits;
  double *R, *X, *Z, *P, *Q;  // n x 16
  double* kpart;              // kmv_splits(n) x n x 16
  double *part1, *part2;      // ceil(n / 64) x 16 (per-workgroup partial sums)
  double *gamma, *beta, *ynorm, *relres;  // 16 each
  int *active, *iters;                    // 16 each
  int* any;                               // 1 device int: some column still iterates
  int* host_any;                          // 3 ints of pinned host memory
  ProfHook* hook;
};

int launch_pchol(const float* K, int64_t n, int64_t ldk, int rank, double pivot_tol, double* L, int* piv,
                 double* d, double* pv, int* pi, double* dpiv, hipStream_t s);
int launch_pc_setup(double* LU, int64_t n, int r, double lam, double* Ur, double* M, int* info, hipStream_t s);
int launch_pcg_group(const PcgArgs& a, int64_t c0, int C, hipStream_t s);
int kmv_splits(int64_t n);
int launch_kmv(const float* K, int64_t n, int64_t ldk, const double* P, int C, double lam, double* part, double* Q,
               double* pq_part, hipStream_t s, ProfHook* hook);
int launch_diag_mean(const float* K, int64_t n, int64_t ldk, double* out, hipStream_t s);

// Dense float64 helpers of the approximate solvers (dense.hip).  GEMM:
// C (M x N, ldc) = beta C + alpha op(A) B, op(A) = A (M x K) or A^T (A is
// K x M); comp carries each sum's rounding error (compensated).
int dn_gemm_ff(const float* A, int64_t lda, bool a_t, const float* B, int64_t ldb, double* C, int64_t ldc, int64_t M,
               int64_t N, int64_t K, double alpha, double beta, bool comp, hipStream_t s);
int dn_gemm_fd(const float* A, int64_t lda, bool a_t, const double* B, int64_t ldb, double* C, int64_t ldc,
               int64_t M, int64_t N, int64_t K, double alpha, double beta, bool comp, hipStream_t s);
int dn_gemm_dd(const double* A, int64_t lda, bool a_t, const double* B, int64_t ldb, double* C, int64_t ldc,
               int64_t M, int64_t N, int64_t K, double alpha, double beta, bool comp, hipStream_t s);
int dn_load_shift(const float* S, int64_t lds, int64_t n, double shift, double* D, int* info, hipStream_t s);
int dn_shift(double* D, int64_t n, double shift, int* info, hipStream_t s);
int dn_identity(double* I, int64_t n, hipStream_t s);
int dn_copy_f(const float* in, int64_t ldi, int64_t rows, int64_t cols, bool trans, double* out, int64_t ldo,
              hipStream_t s);
int dn_residual_scale(const float* Y, int64_t ldy, int64_t n, int64_t c, double scale, double* X, hipStream_t s);
int dn_cast(const double* in, int64_t rows, int64_t cols, float* out, int64_t ldo, hipStream_t s);
int dn_axpby(double* D, const double* E, int64_t n, double alpha, double beta, hipStream_t s);

// CNN-VEC NNGP (cv.hip): per-image tables [img][layer][pixel] float2 and
// K(x, x), then one N-lane segment per pair.
int launch_cv_prepare(const float* x, int64_t n, int N, int C, int D, double sw2, double sb2, float2* tab,
                      float* kdiag, hipStream_t s);
int launch_cv_pairs(int N, const float* x1, const float* x2, int64_t n1, int64_t n2, int sym, int T, int C, int D,
                    const float2* tab1, const float2* tab2, float* K, int64_t ldk, float sb2, float seed_scale,
                    hipStream_t s);

}  // namespace nk
