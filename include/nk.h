/*
 * nk.h -- C ABI of libnk, infinite-width neural-network (NNGP) kernels on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations are those the paper scales up (Adlam et al. 2023, "Kernel
 * Regression with Infinite-Width Neural Networks on Millions of Examples"):
 * entries of the NNGP kernel of the FC3 and Myrtle networks of App. A, one
 * rectangular block of the Gram matrix per call (the unit each device owns
 * in the blockwise scheme of Fig. 1), and kernel ridge regression with those
 * kernels (the linear system of Sec. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named x*, K, dK, dx*, Y, pred, ws are DEVICE pointers owned by
 *    the caller; config structs and nk_tile arrays are HOST memory read
 *    during the call only.  Inputs are never written.
 *  - Images are float32, NHWC, contiguous: x[((n * H + y) * W + x) * C + c].
 *  - K blocks are float32 row-major with leading dimension ldk (elements):
 *    K[a * ldk + b] = k(x1[a], x2[b]).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and
 *    is asynchronous unless stated otherwise; device faults surface at the
 *    caller's next synchronisation.  The call returns once the work is
 *    enqueued.
 *  - `ws` is caller-owned device scratch of at least nk_workspace_size()
 *    bytes (256-byte aligned).  Its contents are undefined on return and it
 *    must not be reused by another call until the stream has passed this
 *    call's work.
 *  - Outputs are fully overwritten; nothing accumulates into them.
 *  - Symmetric blocks: x1 == x2 and n1 == n2 selects the upper-triangle
 *    path (each unordered pair is computed once and mirrored).
 *  - Return codes: NK_OK on success, otherwise a negative code; no
 *    exception crosses the ABI; nk_last_error() holds a message (thread
 *    local) for the last failing call of the calling thread.
 *  - Thread safety: calls on different streams with different workspaces
 *    may run concurrently.
 */
#ifndef NK_H
#define NK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NK_OK = 0,
  NK_EINVAL = -1,       /* invalid argument (null pointer, bad size, ldk < n2, workspace too small, ...) */
  NK_EUNSUPPORTED = -2, /* valid but unsupported shape (see each config) */
  NK_EHIP = -3,         /* a HIP runtime call failed; message in nk_last_error() */
  NK_ENOMEM = -4,       /* host allocation failed */
  NK_ENOTPD = -5        /* kernel ridge system not positive definite */
};

/* Operation ids for nk_workspace_size. */
enum {
  NK_OP_FC = 0,
  NK_OP_MYRTLE = 1,
  NK_OP_MYRTLE_BWD = 2,
  NK_OP_KRR = 3,
  NK_OP_MYRTLE_BATCHED = 4,
  NK_OP_MYRTLE_NTK = 5,
  NK_OP_PCG = 6,          /* cfg: nk_pcg_cfg; n1 = n, n2 = c */
  NK_OP_PIVOTED_CHOL = 7, /* cfg: NULL; n1 = n, n2 = rank */
  NK_OP_GRAM_MATVEC = 8,  /* cfg: NULL; n1 = n, n2 = c */
  NK_OP_CV = 9,           /* cfg: nk_cv_cfg; n1, n2 = block sizes (n2 = 0 for a symmetric block) */
  NK_OP_APPROX = 10       /* cfg: nk_approx_dims; n1, n2 unused */
};

/*
 * Myrtle network (App. A, Myrtle listing): n_stages stages; stage s runs
 * depth[s] blocks of [3x3 SAME conv, ReLU] at resolution (H >> s) x (W >> s),
 * stages are separated by 2x2/stride-2 average pools, and the network ends in
 * a global average pool and a Dense readout.  Conv weights have variance
 * sigma_w2 / (9 C_in) and biases sigma_b2; the readout has weight variance
 * sigma_w2 / C_in and bias sigma_b2.  Myrtle-5 = {2,1,1}, Myrtle-7 =
 * {2,2,2}, Myrtle-10 = {3,3,3}.
 *
 * Supported: H == W a power of two with 2 <= H <= 32 and every stage at
 * least 2 x 2 (H >> (n_stages-1) >= 2), filter == 3, 1 <= n_stages <= 4,
 * 0 <= depth[s] <= 4 with depth[0] >= 1 (depth[0] <= 3 when H == 32: the
 * first stage keeps its tables and both images in LDS), 1 <= C <= 4,
 * sigma_w2 > 0, sigma_b2 >= 0.  H == 64 is also accepted by nk_myrtle_nngp
 * (and its workspace query) when n_stages >= 2 and depth[0] <= 2 (e.g.
 * Myrtle-7 at 64x64x3); the tangent kernel, the adjoint and the batched
 * pass return NK_EUNSUPPORTED for it.  Anything else returns
 * NK_EUNSUPPORTED (or NK_EINVAL for values that define no network).
 */
typedef struct {
  int32_t H, W, C, n_stages;
  int32_t depth[4];
  int32_t filter;
  float sigma_w2, sigma_b2;
} nk_myrtle_cfg;

/*
 * Fully connected network (App. A, FC listing): Flatten, `depth` blocks of
 * [Dense, ReLU], Dense readout; weight variance sigma_w2 / fan_in, bias
 * sigma_b2.  FC3 = {d = H*W*C, depth = 3}.
 */
typedef struct {
  int32_t d, depth;
  float sigma_w2, sigma_b2;
} nk_fc_cfg;

/* One Gram tile for the batched entry point. */
typedef struct {
  const float *x1, *x2; /* device, NHWC images */
  int64_t n1, n2;
  float* K; /* device, row-major, leading dimension ldk */
  int64_t ldk;
} nk_tile;

/*
 * Workspace bytes needed by an operation.  cfg points at the op's config
 * struct (nk_fc_cfg for NK_OP_FC, nk_myrtle_cfg for the Myrtle ops, NULL for
 * NK_OP_KRR).  n1/n2: block sizes (KRR: n1 = n train, n2 = max(m test, c
 * targets)); for NK_OP_MYRTLE_BATCHED n1 = image rows to prepare (summed
 * over distinct image arrays), n2 = number of tiles, sized for chunks of
 * 16384 pairs.  Returns 0 for invalid arguments.
 */
size_t nk_workspace_size(int op, const void* cfg, int64_t n1, int64_t n2);

/*
 * FC NNGP block: K[a, b] = k_FC(x1[a], x2[b]) with x* (n*, d) float32
 * row-major.  The first layer's dot products run on MFMA in fp32.  x2 == x1
 * with n2 == n1 is the symmetric block: only the 128 x 128 tiles on and above
 * the diagonal are computed and the others written as their mirror (K comes
 * out exactly symmetric).
 */
int nk_fc_nngp(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_fc_cfg* cfg, float* K,
               int64_t ldk, void* ws, size_t ws_bytes, void* stream);

/*
 * nk_fc_nngp for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): no workspace argument
 * and no allocation of any kind.  Its only scratch, the first-layer
 * diagonals of both sets (n1 + n2 floats), lives in a static device array of
 * 2^21 floats (8 MiB) that each device holds until the process ends; the
 * device address of the current device's copy is looked up on its first
 * call.  n1 + n2 > 2^21 returns NK_EINVAL.  Same arguments, layout, stream
 * semantics and results (bitwise) as nk_fc_nngp.  Every call on a device
 * shares that device's array: calls that overlap in time on one device
 * (different streams, or host threads) race on it and must be serialised by
 * the caller.
 */
int nk_fc_nngp_static(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_fc_cfg* cfg, float* K,
                      int64_t ldk, void* stream);

/*
 * Myrtle NNGP block: K[a, b] = k_Myrtle(x1[a], x2[b]) with x* (n*, H, W, C).
 * Accuracy: float32 arithmetic; |K - K_exact| / sqrt(K(x,x) K(x',x')) is of
 * order 1e-6 for the networks above.  Deterministic: the same inputs give
 * bitwise identical K on the same device.
 */
int nk_myrtle_nngp(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_myrtle_cfg* cfg, float* K,
                   int64_t ldk, void* ws, size_t ws_bytes, void* stream);

/*
 * Myrtle neural tangent kernel block, the kernel of the paper's large-scale
 * runs (Sec. "Approaches to large-scale kernel methods": the 10-layer Myrtle
 * NTK), for the network of nk_myrtle_nngp in the parameterisation where each
 * layer scales N(0, 1) weights by sqrt(sigma_w2 / fan_in) and N(0, 1) biases
 * by sqrt(sigma_b2): K_ntk[a, b] = sum over all parameters of the products of
 * the derivatives of the network output at x1[a] and x2[b], in the
 * infinite-width limit.  The same pass yields the NNGP, written to K_nngp if
 * it is not NULL (both blocks share ldk).  Same shapes, symmetric-block rule,
 * workspace convention (op NK_OP_MYRTLE_NTK) and stream semantics as
 * nk_myrtle_nngp.  Where a pair's two images are identical (the diagonal of
 * a symmetric block, or two arrays holding the same image element for
 * element) its displacement-0 correlation is taken as exactly 1 at every
 * layer: the derivative of the ReLU map has an infinite slope there, so a
 * rounded correlation would cost about 1e-4 of relative accuracy.
 */
int nk_myrtle_ntk(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_myrtle_cfg* cfg, float* K_ntk,
                  float* K_nngp, int64_t ldk, void* ws, size_t ws_bytes, void* stream);

/*
 * Adjoint of nk_myrtle_nngp: given the cotangent dK (n1 x n2, leading
 * dimension lddk) of L(K), writes
 *   dx1 = dL/dx1 (n1, H, W, C), dx2 = dL/dx2 (n2, H, W, C),
 *   dsigma[0] = dL/dsigma_w2, dsigma[1] = dL/dsigma_b2 (device, 2 floats).
 * Any of dx1, dx2, dsigma may be NULL (not computed).  For a symmetric
 * block (x1 == x2, n1 == n2) the full dK is used (entries (a, b) and (b, a)
 * both contribute) and the gradient for the shared images goes to dx1; dx2
 * must then be NULL or equal to dx1.  Covariances are recomputed from the
 * inputs (no state is kept from the forward call).  The per-image sums are
 * accumulated in float64 with atomic adds (one per workgroup and pixel, in
 * no fixed order) and rounded to float32 at the end, so gradients are
 * reproducible up to float64 rounding order.  Where a pair's two images are
 * identical (the diagonal of a symmetric block, or two arrays holding the
 * same image element for element) the displacement-0 correlation is taken
 * as exactly 1, where d/drho of the ReLU map has an infinite slope.
 */
int nk_myrtle_nngp_backward(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_myrtle_cfg* cfg,
                            const float* dK, int64_t lddk, float* dx1, float* dx2, float* dsigma, void* ws,
                            size_t ws_bytes, void* stream);

/*
 * Kernel ridge regression (the system of Sec. 2, solved directly):
 *   lambda = ridge_rel * mean(diag(K_train)),
 *   alpha  = (K_train + lambda I)^{-1} Y,    pred = K_test alpha,
 * with K_train (n x n, leading dim n), K_test (m x n, leading dim n), Y and
 * pred (n x c / m x c, row-major) float32 on the device; the factorisation
 * and solves run in float64.  Synchronises `stream` before returning so it
 * can report NK_ENOTPD when the Cholesky factorisation meets a non-positive
 * pivot (pred is then undefined).
 */
int nk_krr_predict(const float* K_train, int64_t n, const float* K_test, int64_t m, const float* Y, int64_t c,
                   double ridge_rel, float* pred, void* ws, size_t ws_bytes, void* stream);

/*
 * Cotangents of the held-out squared error of kernel ridge regression,
 *   L = mean((K_ts alpha - Y_t)^2),  alpha = (K_ss + lambda I)^{-1} Y_s,
 * with lambda held fixed (not differentiated):
 *   dK_ts = G alpha^T,  dK_ss = -(A^{-1} K_ts^T G) alpha^T,  G = dL/dpred,
 *   A = K_ss + lambda I.
 * ridge >= 0 with ridge_is_relative == 0 gives lambda = ridge; with
 * ridge_is_relative != 0, lambda = ridge * mean(diag K_ss).
 * K_ss (n x n), K_ts (m x n), Y_s (n x c), Y_t (m x c) float32 device;
 * dK_ss (n x n), dK_ts (m x n) float32 device outputs (dK_ss is the full,
 * unsymmetrised cotangent); *loss and *lambda_used (host doubles,
 * lambda_used may be NULL) receive L and lambda.  Float64 inside.
 * Synchronises `stream`; NK_ENOTPD if A is not positive definite.
 */
int nk_krr_mse_backward(const float* K_ss, int64_t n, const float* K_ts, int64_t m, const float* Y_s,
                        const float* Y_t, int64_t c, double ridge, int ridge_is_relative, float* dK_ss,
                        float* dK_ts, double* loss, double* lambda_used, void* ws, size_t ws_bytes, void* stream);

/*
 * Gradient of the held-out kernel-ridge-regression error through the Myrtle
 * NNGP, with respect to learnable support images and both variances (the
 * differentiable use of the kernel: support images regressed onto target
 * images):
 *   K_ss = k(x_s, x_s), K_ts = k(x_t, x_s),  alpha = (K_ss + lambda I)^{-1} Y_s,
 *   L = mean((K_ts alpha - Y_t)^2),  lambda = ridge (or ridge * mean diag
 *   K_ss with ridge_is_relative != 0), held fixed (not differentiated).
 * One call runs the whole step in the library: both Gram blocks
 * (nk_myrtle_nngp), the float64 solve and its cotangents
 * (nk_krr_mse_backward), the adjoint of both blocks (nk_myrtle_nngp_backward)
 * with the support images' contributions of the two blocks summed on the
 * device before the self-chain reverse, and the casts.
 *   x_s (n, H, W, C), x_t (m, H, W, C): float32 device images, different
 *   arrays; Y_s (n x c), Y_t (m x c) float32 device, row-major.
 *   dx_s (n, H, W, C) float32 device output = dL/dx_s (may be NULL);
 *   dsigma (2 floats, device) = dL/dsigma_w2, dL/dsigma_b2 (may be NULL);
 *   *loss (host) = L; *lambda_used (host, may be NULL) = lambda.
 * 1 <= n <= 16384.  Workspace: nk_krr_mse_grad_workspace(cfg, n, m, c)
 * bytes (a smaller one, down to one pair per pass, runs in more passes).
 * Synchronises `stream` (the loss is read on the host between the solve and
 * the adjoint); NK_ENOTPD if K_ss + lambda I is not positive definite.
 */
int nk_krr_mse_grad(const float* x_s, int64_t n, const float* x_t, int64_t m, const float* Y_s, const float* Y_t,
                    int64_t c, const nk_myrtle_cfg* cfg, double ridge, int ridge_is_relative, float* dx_s,
                    float* dsigma, double* loss, double* lambda_used, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for nk_krr_mse_grad (0 if the arguments are invalid). */
size_t nk_krr_mse_grad_workspace(const nk_myrtle_cfg* cfg, int64_t n, int64_t m, int64_t c);

/*
 * nk_krr_mse_grad keeping the first stage's output of every pair (the pooled
 * covariance the second stage reads, (H/2)^4 floats per pair) from the
 * forward pass for the adjoint instead of re-running the first stage there:
 * the stage-boundary checkpoints of the recomputation strategy, held for the
 * whole step (the gradient through the kernel that data distillation, named
 * in Sec. 1's related work, takes).  The cross block's forward then runs as (support, targets) and is transposed
 * into K_ts, which can move K_ts, and so the loss and the gradients, by
 * float32 rounding against nk_krr_mse_grad (the kernel is symmetric in exact
 * arithmetic).  Arguments as nk_krr_mse_grad; the workspace must hold at
 * least nk_krr_mse_grad_workspace_keep(cfg, n, m, c) bytes (NK_EINVAL
 * otherwise).  A one-stage network has nothing to keep and runs as
 * nk_krr_mse_grad.
 */
int nk_krr_mse_grad_kept(const float* x_s, int64_t n, const float* x_t, int64_t m, const float* Y_s,
                         const float* Y_t, int64_t c, const nk_myrtle_cfg* cfg, double ridge, int ridge_is_relative,
                         float* dx_s, float* dsigma, double* loss, double* lambda_used, void* ws, size_t ws_bytes,
                         void* stream);

/* Workspace bytes for nk_krr_mse_grad_kept: the default workspace plus
 * (n (n + 1) / 2 + n m) (H/2)^4 floats (about 146 GB at H = 32, n = 256,
 * m = 2048), less one chunk buffer of the first stage; the same as
 * nk_krr_mse_grad_workspace for a one-stage network.  0 if the arguments
 * are invalid. */
size_t nk_krr_mse_grad_workspace_keep(const nk_myrtle_cfg* cfg, int64_t n, int64_t m, int64_t c);

/*
 * Many Myrtle Gram tiles of uneven size in one scheduled pass (the paper
 * computes a large kernel as many independent blocks, Sec. "Approaches to
 * large-scale kernel methods").  The variance tables of every distinct
 * image array are prepared once (tiles that pass the same x pointer share
 * them; the rows used are the largest n of the tiles naming that pointer),
 * and the pairs of all tiles form one work list that runs in full chunks
 * through the stage kernels, so no tile pays its own launch tail.  A tile
 * with x1 == x2 and n1 == n2 is symmetric (upper triangle computed and
 * mirrored).  Tiles must not overlap in their K outputs.  K values are
 * bitwise identical to nk_myrtle_nngp on the same tile.
 *
 * Schedule.  On the first call for a network configuration the library
 * times the first stage kernel on the pass's own first pairs under each
 * candidate schedule -- pairs per stage pass (8192, 16384, 32768, as far as
 * the workspace allows), side of the image tile that orders pairs (8, 16,
 * 32), and a persistent grid (all workgroups resident, the workgroups of
 * each XCD walking one contiguous range of the work list) or one workgroup
 * per work unit -- and keeps the fastest; under that schedule it then
 * times the stage kernels of tiles of at most 16 x 16 (the later stages of
 * a 32 x 32 network) with one and with two pairs-per-workgroup multiples and
 * keeps the faster kernel shape, for the process (nk_myrtle_batched_tuning
 * reports the timings).  Results do not depend on the choices.  That call
 * synchronises `stream`; later calls do not.
 *
 * If `graph` is non-zero the pass (table preparation and all stage
 * launches) is captured into a hipGraph the first time this exact pass is
 * seen (same tiles, configuration, workspace pointer and size) and replayed
 * on `stream` afterwards; the tile table is uploaded into the workspace on
 * every call before the launch.  Graphs are cached per process (the 8 most
 * recent).  ws: at least nk_myrtle_nngp_batched_workspace(...) bytes.
 */
int nk_myrtle_nngp_batched(const nk_tile* tiles, int32_t ntiles, const nk_myrtle_cfg* cfg, void* ws,
                           size_t ws_bytes, void* stream, int32_t graph);

/* Workspace bytes for nk_myrtle_nngp_batched on this tile list (0 if the
 * arguments are invalid). */
size_t nk_myrtle_nngp_batched_workspace(const nk_tile* tiles, int32_t ntiles, const nk_myrtle_cfg* cfg);

/* One timed candidate of the batched pass: a schedule (kind 0, first stage
 * timed) or, under the chosen schedule, a kernel shape of the stages of tiles
 * of at most 16 x 16 (kind 1, those stages timed together). */
typedef struct {
  int64_t chunk;         /* pairs per stage pass */
  int32_t pair_tile;     /* image-tile side of the pair order */
  int32_t persistent;    /* 1: persistent XCD-ordered grid, 0: one workgroup per unit */
  double us_per_pair;    /* measured time per pair of the stages timed */
  int32_t kind;          /* 0: schedule candidate, 1: kernel-shape candidate */
  int32_t wg_pairs_mult; /* pairs per workgroup of the stage kernels of tiles of at most 16 x 16, as a
                            multiple (1 or 2) of their smallest workgroup (256 threads); in `chosen`: the
                            tuned multiple */
} nk_batched_candidate;

/* Timings of the candidates tried for this network (up to max_entries into
 * out, may be NULL) and the chosen schedule and shape (into *chosen, may be
 * NULL; its us_per_pair is the chosen schedule's first-stage time).  Returns
 * the number of candidates, or NK_EINVAL if no batched pass has been tuned
 * for this configuration in this process. */
int nk_myrtle_batched_tuning(const nk_myrtle_cfg* cfg, nk_batched_candidate* out, int max_entries,
                             nk_batched_candidate* chosen);

/* Fixes the schedule and kernel shape of the batched pass for this network
 * configuration for the rest of the process, in place of tuning (no timing
 * is done; nk_myrtle_batched_tuning then reports no candidates and this
 * choice).  Read from *choice: chunk in [1, 32768] (cut to what the
 * workspace holds at each call), pair_tile in [1, 256], persistent 0 or 1,
 * wg_pairs_mult 1 or 2; the other fields are ignored.  Results do not depend
 * on the choice.  NK_EINVAL on other values or a NULL pointer; no GPU call. */
int nk_myrtle_batched_set_schedule(const nk_myrtle_cfg* cfg, const nk_batched_candidate* choice);

/*
 * CNN-VEC network (App. "Neural Kernel Architecture", CNN-VEC listing; CV8 =
 * depth 8): `depth` blocks of [3x3 SAME conv, ReLU] at full resolution
 * H x W, Flatten, Dense readout; conv weight variance sigma_w2 / (9 C_in),
 * biases sigma_b2, readout weight variance sigma_w2 / (H W C_in).
 * Supported: H == W a power of two with 2 <= H <= 32, 1 <= C <= 4,
 * 1 <= depth <= 16, sigma_w2 > 0, sigma_b2 >= 0.
 */
typedef struct {
  int32_t H, W, C, depth;
  float sigma_w2, sigma_b2;
} nk_cv_cfg;

/*
 * CNN-VEC NNGP block: K[a * ldk + b] = k_CV(x1[a], x2[b]).  The flatten
 * readout averages the covariance of each pixel with the same pixel of the
 * other image, so only those n^2 entries per pair are propagated.  x1, x2:
 * NHWC float32 device images; K float32 device, row-major, ldk >= n2.
 * x1 == x2 && n1 == n2 selects the symmetric path (upper triangle computed,
 * mirrored).  Workspace: nk_workspace_size(NK_OP_CV, cfg, n1, n2) (pass n2
 * = 0 for a symmetric block).  Asynchronous on `stream`.
 */
int nk_cv_nngp(const float* x1, int64_t n1, const float* x2, int64_t n2, const nk_cv_cfg* cfg, float* K,
               int64_t ldk, void* ws, size_t ws_bytes, void* stream);

/*
 * Partial pivoted Cholesky factor of a symmetric positive semi-definite
 * Gram matrix, the preconditioner of the paper's conjugate-gradient solver
 * (Sec. 2, "Iterative solvers"; Sec. 1, related work).  Greedy diagonal
 * pivoting: with d the diagonal of the current Schur complement (diag K at
 * the start), step m picks the not-yet-picked index p of largest d (lowest
 * index on ties), stops if d_p <= 0 or d_p <= pivot_tol * max(diag K), and
 * otherwise appends column m of L:
 *   L[p][m] = sqrt(d_p),
 *   L[i][m] = (K[p][i] - sum_{k<m} L[p][k] L[i][k]) / sqrt(d_p)  (i not picked),
 *   L[i][m] = 0 at indices picked earlier;  then d_i -= L[i][m]^2.
 * K: n x n float32 device, row-major, leading dim ldk >= n (read, symmetric;
 * the row of each pivot is read).  L: n x rank float64 device, COLUMN-major
 * (column m at L + m n); columns past the rank reached are zero.  piv: rank
 * int32 device (pivot of each column, -1 past the rank reached).
 * *rank_used (host, may be NULL): columns produced.  0 <= rank <= min(n,
 * 8192).  Workspace: nk_workspace_size(NK_OP_PIVOTED_CHOL, NULL, n, rank).
 * Float64 throughout; synchronises `stream`.
 */
int nk_pivoted_cholesky(const float* K, int64_t n, int64_t ldk, int32_t rank, double pivot_tol, double* L,
                        int32_t* piv, int32_t* rank_used, void* ws, size_t ws_bytes, void* stream);

/*
 * Kernel-vector products of the solver: Q = (K + lambda I) P, the one place
 * the kernel enters conjugate gradients (Sec. 2, "Iterative solvers";
 * Fig. 1 splits this product over workers).  K: n x n float32 device,
 * row-major, leading dim ldk >= n, SYMMETRIC (the product reads K by rows
 * and uses K = K^T); P, Q: n x c float64 device, row-major (leading dim c);
 * 1 <= c <= 16.  Float64 products and sums, in a fixed order (bitwise
 * reproducible).  Workspace: nk_workspace_size(NK_OP_GRAM_MATVEC, NULL, n,
 * c).  Asynchronous on `stream`.
 */
int nk_gram_matvec(const float* K, int64_t n, int64_t ldk, const double* P, int64_t c, double lambda, double* Q,
                   void* ws, size_t ws_bytes, void* stream);

/*
 * Solver settings of nk_krr_pcg.
 *   rank      preconditioner rank r >= 0 (0: no preconditioner, plain CG);
 *             at most min(n, 8192)
 *   max_iter  iteration cap >= 1
 *   tol       column j stops once ||r_j|| <= tol ||y_j|| (recursive residual)
 *   pivot_tol the pivoted Cholesky stops early when the largest residual
 *             diagonal is <= pivot_tol * max(diag K) (0: only at d <= 0)
 */
typedef struct {
  int32_t rank;
  int32_t max_iter;
  double tol;
  double pivot_tol;
} nk_pcg_cfg;

/* Outcome of nk_krr_pcg. */
typedef struct {
  int32_t rank;       /* preconditioner rank reached */
  int32_t iterations; /* largest iteration count over the columns */
  double lambda;      /* ridge used */
} nk_pcg_stats;

/*
 * Kernel ridge regression by preconditioned conjugate gradients in float64
 * (Sec. 2, "Iterative solvers", with the partial pivoted Cholesky
 * preconditioner; the paper solves in high precision, Sec. 1): solves
 * (K + lambda I) X = Y column by column, lambda = ridge, or ridge *
 * mean(diag K) when ridge_is_relative != 0 (lambda must come out > 0).
 * Preconditioner Ph = L L^T + lambda I with L = nk_pivoted_cholesky(K,
 * cfg->rank), applied by the Woodbury identity.  Each column runs the
 * textbook PCG recursion from X = 0 and stops (its X frozen) after the
 * first update that brings ||r|| <= tol ||y||; a zero column of Y gives
 * X = 0 after 0 iterations.
 * K: n x n float32 device, row-major, ldk >= n, symmetric.  Y: n x c
 * float64 device, row-major (leading dim c).  X: n x c float64 device
 * output.  iters (c int32) and relres (c doubles, ||r||/||y|| at the
 * column's last update) are host arrays, may be NULL; stats (host) may be
 * NULL.  Columns are solved in groups of 16.  Workspace:
 * nk_workspace_size(NK_OP_PCG, cfg, n, c).  Synchronises `stream` (it reads
 * lambda, the rank reached and the convergence flags on the host).
 * NK_ENOTPD if lambda I + L^T L cannot be factored.
 */
int nk_krr_pcg(const float* K, int64_t n, int64_t ldk, const double* Y, int64_t c, double ridge,
               int ridge_is_relative, const nk_pcg_cfg* cfg, double* X, int32_t* iters, double* relres,
               nk_pcg_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * Approximate kernel ridge regression: the four approximations to the
 * linear system the paper compares with CG (Sec. 2, "Approximations to the
 * linear system"), in the forms of Rasmussen and Williams, "Gaussian
 * Processes for Machine Learning", ch. 8 (which the paper cites).  None of
 * them needs the whole training Gram.  The subset (Nystrom, subset of
 * regressors) or the partition (block-diagonal, committee machine) is the
 * caller's choice -- the paper draws it uniformly at random -- and is given
 * through the kernel blocks passed in: a subset as its kernel columns, a
 * partition by ordering the training points block by block.
 *
 * All kernel blocks and Y are float32 device arrays, row-major with the
 * given leading dimensions (Y: n x c, leading dim c); pred is m x c float32
 * (leading dim c).  Sums and solves run in float64; the sums whose results
 * are later subtracted from nearly equal quantities are compensated.
 * lambda > 0 is the ridge; jitter >= 0 is added to the diagonal of the
 * matrix a method inverts besides its ridge system (K_rr, or the committee
 * machine's test covariances).  Each call synchronises `stream` and returns
 * NK_ENOTPD if a Cholesky factorisation meets a non-positive pivot.
 * Workspace: nk_workspace_size(NK_OP_APPROX, &dims, 0, 0) with
 * dims = {n, r, m, c, largest block}.
 */
typedef struct {
  int64_t n, r, m, c, max_block;
} nk_approx_dims;

/* Nystrom: the training kernel replaced by K_nr (K_rr + jitter I)^{-1} K_rn;
 * pred = K_mn (K~ + lambda I)^{-1} Y, through the Woodbury identity in
 * O(n r^2).  K_nr: n x r (training vs subset), K_rr: r x r, K_mn: m x n
 * (test vs all training points). */
int nk_krr_nystrom(const float* K_nr, int64_t n, int64_t r, int64_t ld_nr, const float* K_rr, int64_t ld_rr,
                   const float* K_mn, int64_t m, int64_t ld_mn, const float* Y, int64_t c, double lambda,
                   double jitter, float* pred, void* ws, size_t ws_bytes, void* stream);

/* Subset of regressors: pred = K_mr (K_rn K_nr + lambda (K_rr + jitter I))^{-1}
 * K_rn Y.  K_mr: m x r (test vs subset). */
int nk_krr_sor(const float* K_nr, int64_t n, int64_t r, int64_t ld_nr, const float* K_rr, int64_t ld_rr,
               const float* K_mr, int64_t m, int64_t ld_mr, const float* Y, int64_t c, double lambda, double jitter,
               float* pred, void* ws, size_t ws_bytes, void* stream);

/* Block-diagonal: p blocks of sizes[i] consecutive training points;
 * alpha_i = (K_ii + lambda I)^{-1} Y_i; pred = K_mn alpha.  K_blocks: host
 * array of p device pointers, block i sizes[i] x sizes[i] (leading dim
 * sizes[i]); sizes: host array summing to n; K_mn: m x n (columns in block
 * order). */
int nk_krr_block_diag(int32_t p, const float* const* K_blocks, const int64_t* sizes, const float* K_mn, int64_t m,
                      int64_t ld_mn, const float* Y, int64_t c, double lambda, float* pred, void* ws,
                      size_t ws_bytes, void* stream);

/* Bayesian committee machine, posterior mean of the m test points taken
 * jointly: per block mu_i = K_mi (K_ii + lambda I)^{-1} Y_i and
 * S_i = K_mm - K_mi (K_ii + lambda I)^{-1} K_im;
 * S^{-1} = sum_i (S_i + jitter I)^{-1} - (p - 1) (K_mm + jitter I)^{-1};
 * pred = S sum_i (S_i + jitter I)^{-1} mu_i.  Blocks as in
 * nk_krr_block_diag; K_mm: m x m test-test kernel. */
int nk_krr_bcm(int32_t p, const float* const* K_blocks, const int64_t* sizes, const float* K_mn, int64_t m,
               int64_t ld_mn, const float* K_mm, int64_t ld_mm, const float* Y, int64_t c, double lambda,
               double jitter, float* pred, void* ws, size_t ws_bytes, void* stream);

/*
 * Kernel timing (tracing).  After nk_profile_enable(1), every launch of the
 * library's kernels is bracketed by HIP events recorded on the caller's
 * stream (no host synchronisation).  nk_profile_read() waits for those
 * events and writes, per kernel kind, the launch count and summed elapsed
 * milliseconds into out[0 .. max_entries); it returns the number of kinds
 * (or a negative code) and clears the records when reset != 0.
 * nk_profile_enable(0) stops recording.  Process-wide; thread safe.
 */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} nk_profile_entry;

int nk_profile_enable(int on);
int nk_profile_read(nk_profile_entry* out, int max_entries, int reset);

/* Message for the last non-zero return on this thread ("" if none). */
const char* nk_last_error(void);

/* Library version string. */
const char* nk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NK_H */
