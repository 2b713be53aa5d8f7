// Per-image variance tables for the Myrtle NNGP (float64 inside).
//
// Every ReLU of a pair (x, x') needs the variances q(i) = S_xx(i, i) and
// q'(j) of the two images at that layer: the diagonal of each image's own
// recursion (App. A Myrtle network; the ReLU map takes the two marginal
// variances and the covariance).  Inside a stage a 3x3 conv keeps the pixel
// displacement delta = j - i, and on the delta = 0 slice the ReLU map is
// F(q, q, q) = q / 2, so within a stage
//   q_1 = c box(base) + b,   q_{l+1} = c box(q_l / 2) + b,   c = sigma_w2 / 9,
// with base the diagonal of the stage input.  A 2x2 pool mixes the slices
// delta = 2 Delta + {-1, 0, 1}^2, so the diagonal after a pool needs the
// previous stage's slices |delta| <= 1, which need the stage before's
// |delta| <= 3, and so on: stage s of S uses slices |delta| <= 2^(S-1-s) - 1.
// This kernel runs exactly those slices of the self recursion (a few
// percent of one pair's work per image) and writes, per stage, layer and
// pixel,
//   alpha = 1 / sqrt(q)         (0 where q == 0),
//   beta  = sqrt(q * kappa / 2),
// where kappa is the factor the next linear step applies to the ReLU output
// (c inside a stage, c / 16 before a pool, sigma_w2 / n^4 before the final
// global-average readout).  The pair kernels then form
// rho = S alpha(i) alpha'(j) and kappa F = beta(i) beta'(j) J1(rho).
#include "nk_kernels.h"

namespace nk {



__host__ __device__ inline int prep_R(const NetDesc& net, int s) { return (1 << (net.S - 1 - s)) - 1; }

// doubles of scratch per workgroup
int64_t prep_scratch_doubles(const NetDesc& net) {
  int64_t tot = 0;
  int n0 = net.hw;
  // q maps (all stages)
  for (int s = 0; s < net.S; ++s) tot += (int64_t)net.depth[s] * stage_res(net, s) * stage_res(net, s);
  // two work slices at the largest resolution
  tot += 2LL * n0 * n0;
  // input slices of the current stage and output slices of the next (both at most stage 1 / stage 2 sizes)
  int64_t in_max = 0, out_max = 0;
  for (int s = 0; s < net.S; ++s) {
    int R = prep_R(net, s), n = stage_res(net, s);
    int64_t v = (int64_t)(2 * R + 1) * (2 * R + 1) * n * n;
    if (s > 0 && v > in_max) in_max = v;
    if (s > 0 && v > out_max) out_max = v;
  }
  tot += in_max + out_max;
  tot += (int64_t)n0 * n0;  // base map
  return (tot + 31) & ~31LL;
}

__device__ inline double relu_map64(double s, double q1, double q2) {
  double qq = q1 * q2;
  if (!(qq > 0.0)) return 0.0;
  double nrm = sqrt(qq);
  double rho = s / nrm;
  rho = rho > 1.0 ? 1.0 : (rho < -1.0 ? -1.0 : rho);
  double th = acos(rho);
  return nrm * (sqrt(fmax(1.0 - rho * rho, 0.0)) + (M_PI - th) * rho) * (0.5 / M_PI);
}

// 3x3 box sum with zero padding over an n x n map.
__device__ inline double box9(const double* m, int n, int y, int x) {
  double s = 0.0;
  for (int dy = -1; dy <= 1; ++dy) {
    int yy = y + dy;
    if (yy < 0 || yy >= n) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      int xx = x + dx;
      if (xx < 0 || xx >= n) continue;
      s += m[yy * n + xx];
    }
  }
  return s;
}

__global__ __launch_bounds__(256) void prepare_kernel(const PrepArgs args) {
  const int64_t img = blockIdx.x;
  if (img >= args.n) return;
  const NetDesc& net = args.net;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int C = net.C;
  const float* x = args.x + img * (int64_t)net.hw * net.hw * C;
  const double c = (double)net.sw2 / 9.0, b = (double)net.sb2;

  double* sc = args.scratch + (int64_t)blockIdx.x * args.scratch_per_img;
  double* qm = sc;  // all q maps
  int64_t qlen = 0;
  for (int s = 0; s < net.S; ++s) qlen += (int64_t)net.depth[s] * stage_res(net, s) * stage_res(net, s);
  const int n0 = net.hw;
  double* w0 = qm + qlen;
  double* w1 = w0 + (int64_t)n0 * n0;
  int64_t in_max = 0;
  for (int s = 1; s < net.S; ++s) {
    int R = prep_R(net, s), n = stage_res(net, s);
    int64_t v = (int64_t)(2 * R + 1) * (2 * R + 1) * n * n;
    if (v > in_max) in_max = v;
  }
  double* sl_in = w1 + (int64_t)n0 * n0;
  double* sl_out = sl_in + in_max;
  double* base = sl_out + in_max;

  float2* tab = args.tab + img * (int64_t)table_len(net);

  int64_t qoff = 0;
  for (int s = 0; s < net.S; ++s) {
    const int n = stage_res(net, s), D = net.depth[s];
    const int R = prep_R(net, s);
    // base map: diagonal of the stage input
    for (int i = tid; i < n * n; i += nt) {
      double v;
      if (s == 0) {
        v = 0.0;
        for (int k = 0; k < C; ++k) v += (double)x[i * C + k] * (double)x[i * C + k];
        v /= C;
      } else {
        // input slices of stage s carry radius R; delta = 0 is the centre one
        const int side = 2 * R + 1;
        v = sl_in[(int64_t)(R * side + R) * n * n + i];
      }
      base[i] = v;
    }
    __syncthreads();
    // q maps of this stage
    for (int l = 0; l < D; ++l) {
      double* q = qm + qoff + (int64_t)l * n * n;
      const double* src = l == 0 ? base : qm + qoff + (int64_t)(l - 1) * n * n;
      const double f = l == 0 ? 1.0 : 0.5;
      for (int i = tid; i < n * n; i += nt) q[i] = c * f * box9(src, n, i / n, i % n) + b;
      __syncthreads();
    }
    // tables
    for (int l = 0; l < D; ++l) {
      const double* q = qm + qoff + (int64_t)l * n * n;
      // scale of the next linear step on this ReLU output: the next conv (c),
      // through the pools in between (1/16 each; stages without layers only
      // pool), or the global-average readout (sigma_w2 / n^4)
      double kappa = c;
      if (l + 1 == D) {
        int s2 = s + 1;
        double f = 1.0 / 16.0;
        while (s2 < net.S && net.depth[s2] == 0) {
          f /= 16.0;
          ++s2;
        }
        kappa = s2 < net.S ? c * f : (double)net.sw2 / ((double)n * n * n * n);
      }
      float2* t = tab + table_off(net, s) + l * n * n;
      for (int i = tid; i < n * n; i += nt) {
        double qi = q[i];
        float al = qi > 0.0 ? (float)(1.0 / sqrt(qi)) : 0.0f;
        float be = qi > 0.0 ? (float)sqrt(qi * kappa * 0.5) : 0.0f;
        t[i] = make_float2(al, be);
      }
    }
    if (s + 1 == net.S) break;

    // run the slices |delta| <= R through this stage and pool them into the
    // next stage's slices |Delta| <= Rn
    const int Rn = prep_R(net, s + 1);
    const int nn = n / 2, side_n = 2 * Rn + 1, side = 2 * R + 1;
    for (int i = tid; i < side_n * side_n * nn * nn; i += nt) sl_out[i] = 0.0;
    __syncthreads();
    for (int dyi = -R; dyi <= R; ++dyi) {
      for (int dxi = -R; dxi <= R; ++dxi) {
        // stage input slice: valid where i and i + delta are in the image
        for (int i = tid; i < n * n; i += nt) {
          const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
          double v = 0.0;
          if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) {
            if (s == 0) {
              for (int k = 0; k < C; ++k) v += (double)x[i * C + k] * (double)x[(y2 * n + x2) * C + k];
              v /= C;
            } else {
              v = sl_in[(int64_t)((dyi + R) * side + (dxi + R)) * n * n + i];
            }
          }
          w0[i] = v;
        }
        __syncthreads();
        for (int l = 0; l < D; ++l) {
          const double* q = qm + qoff + (int64_t)l * n * n;
          for (int i = tid; i < n * n; i += nt) {
            const int y = i / n, xx = i % n, y2 = y + dyi, x2 = xx + dxi;
            double v = 0.0;
            if (y2 >= 0 && y2 < n && x2 >= 0 && x2 < n) {
              double sg = c * box9(w0, n, y, xx) + b;
              v = relu_map64(sg, q[i], q[y2 * n + x2]);
            }
            w1[i] = v;
          }
          __syncthreads();
          double* t = w0;
          w0 = w1;
          w1 = t;
        }
        // pool into next-stage slices: coarse (Delta, I) gathers fine i = 2I + a
        // with (i + delta) >> 1 == I + Delta in each dimension
        for (int e = tid; e < side_n * side_n * nn * nn; e += nt) {
          const int Ii = e % (nn * nn), sl = e / (nn * nn);
          const int DY = sl / side_n - Rn, DX = sl % side_n - Rn;
          const int IY = Ii / nn, IX = Ii % nn;
          double acc = 0.0;
          for (int ay = 0; ay < 2; ++ay) {
            const int fy = 2 * IY + ay, gy = fy + dyi;
            if (gy < 0 || gy >= n || (gy >> 1) != IY + DY) continue;
            for (int ax = 0; ax < 2; ++ax) {
              const int fx = 2 * IX + ax, gx = fx + dxi;
              if (gx < 0 || gx >= n || (gx >> 1) != IX + DX) continue;
              acc += w0[fy * n + fx];
            }
          }
          sl_out[e] += acc / 16.0;
        }
        __syncthreads();
      }
    }
    // next stage input
    for (int i = tid; i < side_n * side_n * nn * nn; i += nt) sl_in[i] = sl_out[i];
    __syncthreads();
    qoff += (int64_t)D * n * n;
  }
}

int launch_prepare(const float* x, int64_t n, const NetDesc& net, float2* tab, double* scratch,
                   int64_t max_blocks, hipStream_t stream) {
  const int64_t per = prep_scratch_doubles(net);
  for (int64_t s = 0; s < n; s += max_blocks) {
    int64_t cnt = n - s < max_blocks ? n - s : max_blocks;
    PrepArgs a;
    a.x = x + s * (int64_t)net.hw * net.hw * net.C;
    a.n = cnt;
    a.net = net;
    a.tab = tab + s * (int64_t)table_len(net);
    a.scratch = scratch;
    a.scratch_per_img = per;
    hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)cnt), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return -3;
  }
  return 0;
}

}  // namespace nk
