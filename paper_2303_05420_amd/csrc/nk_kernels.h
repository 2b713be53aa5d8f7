// Kernel argument blocks and launchers shared between the HIP translation
// units of libnk and its host API.
#pragma once
#include "nk_common.h"

namespace nk {

struct PrepArgs {
  const float* x;     // images NHWC
  int64_t n;          // images in this launch
  NetDesc net;
  float2* tab;        // n * table_len float2
  double* scratch;    // n_blocks * scratch_per_img doubles (one region per workgroup)
  int64_t scratch_per_img;
};

struct StageArgs {
  int64_t n1, n2;
  int sym, T;
  int64_t p0, np;  // chunk = pairs [p0, p0 + np) of the block order
  const float* x1;
  const float* x2;
  const float2* tab1;
  const float2* tab2;
  int tablen, taboff;
  int C, D;
  float sb2, seed_scale;
  const float* in;  // [np][N][N][N][N]      (stages after the first)
  float* out;       // [np][N/2][N/2][N/2][N/2] (pooling stages)
  float* K;         // final stage
  int64_t ldk;
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
};

int64_t prep_scratch_doubles(const NetDesc& net);
int launch_prepare(const float* x, int64_t n, const NetDesc& net, float2* tab, double* scratch,
                   int64_t max_blocks, hipStream_t stream);
size_t stage_lds_bytes(int N, int D, bool pool, bool seed);
int launch_stage(int N, const StageArgs& a, bool seed, bool pool, bool bias, hipStream_t s);
int launch_fc(const FcArgs& a, float* d1, float* d2, hipStream_t stream);
int launch_cholesky(double* A, int64_t n, int* info, hipStream_t s);
int launch_chol_solve(const double* A, int64_t n, const float* Bf, const double* Bd, int64_t c, double* X,
                      hipStream_t s);
int launch_krr_build(const float* K, int64_t n, double ridge_rel, double lam_abs, double* mean, double* A,
                     int* info, hipStream_t s);
int launch_krr_matmul(const float* K, int64_t m, int64_t n, int64_t ld, const double* X, int64_t c, float* out,
                      hipStream_t s);

}  // namespace nk
