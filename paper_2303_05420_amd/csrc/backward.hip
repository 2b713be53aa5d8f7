// Adjoint of the Myrtle NNGP (gradients with respect to the input images and
// both sigmas), hand-written reverse mode of the forward in stage.hip and
// prepare.hip.  The cross-pair stage adjoints are in stage_bwd.h (one
// translation unit per tile side); this file holds the reverse of the self
// recursions and the small kernels around them.
//
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
#include "stage_bwd.h"

namespace nk {

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

size_t stage_bwd_lds_bytes(int N, int D, bool seed) {
  switch (N) {
    case 2: return BCfg<2>::PPWG * bwd_slot_lds_bytes<2>(D, seed);
    case 4: return BCfg<4>::PPWG * bwd_slot_lds_bytes<4>(D, seed);
    case 8: return BCfg<8>::PPWG * bwd_slot_lds_bytes<8>(D, seed);
    case 16: return BCfg<16>::PPWG * bwd_slot_lds_bytes<16>(D, seed);
    case 32: return BCfg<32>::PPWG * bwd_slot_lds_bytes<32>(D, seed);
  }
  return 0;
}

int launch_stage_bwd(int N, const StageBwdArgs& a, bool seed, hipStream_t s) {
  if (N == 32) return launch_stage_bwd_32(a, seed, s);
  if (N == 16) return launch_stage_bwd_16(a, seed, s);
  return launch_stage_bwd_small(N, a, seed, s);
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

// out (cols x rows, dense) = in^T (rows x cols, dense), through a 32 x 33
// LDS tile so that both the reads and the writes are coalesced.
__global__ __launch_bounds__(256) void transpose_f32_kernel(const float* __restrict__ in, int64_t rows, int64_t cols,
                                                            float* __restrict__ out) {
  __shared__ float t[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) t[k][tx] = in[r * cols + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) out[c * rows + r] = t[tx][k];
  }
}

int launch_transpose_f32(const float* in, int64_t rows, int64_t cols, float* out, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return 0;
  if ((rows + 31) / 32 > 65535) return -1;
  hipLaunchKernelGGL(transpose_f32_kernel, dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)), dim3(256),
                     0, s, in, rows, cols, out);
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
