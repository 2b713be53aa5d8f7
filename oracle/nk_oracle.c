/*
 * FP64 CPU oracle for infinite-width neural-network Gaussian-process kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path links, loads or
 * calls this file; it exists so tests and the CPU-baseline leg of the
 * benchmark can check the GPU results against a plain, slow, obviously
 * correct recursion.  It shares no code with the GPU library.
 *
 * What it computes (Adlam et al. 2023, "Kernel Regression with Infinite-Width
 * Neural Networks on Millions of Examples"):
 *   - the NNGP kernel of the fully-connected FC3 network of App. A (Flatten,
 *     3 x [Dense, ReLU], Dense);
 *   - the NNGP kernel of the Myrtle convolutional network of App. A (stages of
 *     [3x3 SAME conv, ReLU] separated by 2x2 average pools, then global
 *     average pooling and a Dense readout).
 * The paper names these networks and computes their kernels with Neural
 * Tangents; it prints no kernel formula.  The recursion below is the
 * standard NNGP covariance propagation for these layers (the infinite-width
 * correspondence introduced in Sec. 1 and the related-work paragraph on
 * fully-connected and convolutional NNGPs), written out as plain loops:
 *
 *   seed        S0(i,j)  = (1/C) sum_c x(i,c) x'(j,c)        (i, j pixels)
 *   conv 3x3    S(i,j)   = (sw2/9) sum_{d in {-1,0,1}^2} A(i+d, j+d) + sb2
 *                          (terms with i+d or j+d outside the image are 0;
 *                           the divisor stays 9 - fan-in of the filter)
 *   ReLU        A(i,j)   = F(S(i,j), q(i), q'(j)),  q = own-image variance
 *                          F(s,q,q') = sqrt(q q')/(2 pi) (sin t + (pi - t) cos t),
 *                          cos t = s / sqrt(q q') clamped to [-1, 1]
 *   avg pool    P(I,J)   = (1/16) sum_{a,a' in {0,1}^2} A(2I+a, 2J+a')
 *   readout     K        = sw2 * mean_{i,j} A(i,j) + sb2
 *   FC          K1 = sw2 x.x'/d + sb2;  K_{l+1} = sw2 F(K_l, K_l(x,x), K_l(x',x')) + sb2
 *
 * q(i) is the diagonal S_xx(i,i) of the image's own (self) recursion at the
 * same layer, so every image first runs the full pair recursion against
 * itself.  All arithmetic is float64; inputs are the float32 arrays the GPU
 * reads, promoted once.
 *
 * Neural tangent kernel of the same Myrtle network (the kernel the paper's
 * large-scale runs use, e.g. the 10-layer Myrtle NTK of the section on
 * approaches to large-scale kernel methods), in the parameterisation where
 * every layer scales its N(0,1) weights by sigma_w / sqrt(fan-in) and its
 * N(0,1) biases by sigma_b.  Beside the covariance S of the pre-activations
 * it carries their tangent kernel T (sum over all parameters below the layer
 * of the products of derivatives), and beside A the post-activation tangent
 * kernel B:
 *   seed        B0 = 0 (the input has no parameters)
 *   conv 3x3    T(i,j) = S(i,j) + (sw2/9) sum_d B(i+d, j+d)   (same padding
 *                        rule; S already holds the weight and bias terms)
 *   ReLU        B(i,j) = Fdot(S(i,j), q(i), q'(j)) T(i,j),
 *               Fdot = E[relu'(u) relu'(v)] = (pi - t) / (2 pi)
 *   avg pool    pools B like A
 *   readout     Theta = K + sw2 * mean_{i,j} B(i,j)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NKO_PI 3.14159265358979323846264338327950288

/* E[relu(u) relu(v)] for (u, v) ~ N(0, [[q1, s], [s, q2]]) (arc-cosine map). */
static double relu_map(double s, double q1, double q2) {
  double qq = q1 * q2;
  if (!(qq > 0.0)) return 0.0;
  double nrm = sqrt(qq);
  double rho = s / nrm;
  if (rho > 1.0) rho = 1.0;
  if (rho < -1.0) rho = -1.0;
  double th = acos(rho);
  return nrm / (2.0 * NKO_PI) * (sin(th) + (NKO_PI - th) * rho);
}

/* ------------------------------------------------------------------------ */
/* Myrtle                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int H, W, C, n_stages;
  int depth[8];
  double sw2, sb2;
} nko_myrtle;

/* index of entry (iy, ix, jy, jx) of an h x w pair tensor */
#define IDX4(iy, ix, jy, jx, h, w) ((((size_t)(iy) * (w) + (ix)) * (h) + (jy)) * (w) + (jx))

static void seed4(const double* x1, const double* x2, int h, int w, int c, double* S) {
  for (int iy = 0; iy < h; ++iy)
    for (int ix = 0; ix < w; ++ix)
      for (int jy = 0; jy < h; ++jy)
        for (int jx = 0; jx < w; ++jx) {
          double s = 0.0;
          for (int k = 0; k < c; ++k) s += x1[((size_t)iy * w + ix) * c + k] * x2[((size_t)jy * w + jx) * c + k];
          S[IDX4(iy, ix, jy, jx, h, w)] = s / c;
        }
}

static void conv4(const double* A, double* S, int h, int w, double sw2, double sb2) {
  for (int iy = 0; iy < h; ++iy)
    for (int ix = 0; ix < w; ++ix)
      for (int jy = 0; jy < h; ++jy)
        for (int jx = 0; jx < w; ++jx) {
          double s = 0.0;
          for (int dy = -1; dy <= 1; ++dy) {
            int ay = iy + dy, by = jy + dy;
            if (ay < 0 || ay >= h || by < 0 || by >= h) continue;
            for (int dx = -1; dx <= 1; ++dx) {
              int ax = ix + dx, bx = jx + dx;
              if (ax < 0 || ax >= w || bx < 0 || bx >= w) continue;
              s += A[IDX4(ay, ax, by, bx, h, w)];
            }
          }
          S[IDX4(iy, ix, jy, jx, h, w)] = sw2 / 9.0 * s + sb2;
        }
}

static void relu4(const double* S, double* A, int h, int w, const double* q1, const double* q2) {
  for (int iy = 0; iy < h; ++iy)
    for (int ix = 0; ix < w; ++ix)
      for (int jy = 0; jy < h; ++jy)
        for (int jx = 0; jx < w; ++jx) {
          size_t e = IDX4(iy, ix, jy, jx, h, w);
          A[e] = relu_map(S[e], q1[iy * w + ix], q2[jy * w + jx]);
        }
}

static void pool4(const double* A, double* P, int h, int w) {
  int H2 = h / 2, W2 = w / 2;
  for (int Iy = 0; Iy < H2; ++Iy)
    for (int Ix = 0; Ix < W2; ++Ix)
      for (int Jy = 0; Jy < H2; ++Jy)
        for (int Jx = 0; Jx < W2; ++Jx) {
          double s = 0.0;
          for (int ay = 0; ay < 2; ++ay)
            for (int ax = 0; ax < 2; ++ax)
              for (int by = 0; by < 2; ++by)
                for (int bx = 0; bx < 2; ++bx)
                  s += A[IDX4(2 * Iy + ay, 2 * Ix + ax, 2 * Jy + by, 2 * Jx + bx, h, w)];
          P[IDX4(Iy, Ix, Jy, Jx, H2, W2)] = s / 16.0;
        }
}

static int myrtle_layers(const nko_myrtle* m) {
  int L = 0;
  for (int s = 0; s < m->n_stages; ++s) L += m->depth[s];
  return L;
}

/* Number of doubles in all variance maps of one image (one map per ReLU). */
static size_t qmaps_len(const nko_myrtle* m) {
  size_t n = 0;
  int h = m->H, w = m->W;
  for (int s = 0; s < m->n_stages; ++s) {
    n += (size_t)m->depth[s] * h * w;
    h /= 2;
    w /= 2;
  }
  return n;
}

/*
 * Pair recursion for images x1, x2 (h*w*c float64, NHWC).
 * Self mode (q1 == NULL): x2 must equal x1; the variance map of each layer is
 * read off the diagonal of S before its ReLU and written to qout.
 * Cross mode: q1 and q2 hold the two images' variance maps (self mode output).
 * Returns the readout K(x1, x2).  buf0/buf1 hold H*W*H*W doubles each.
 */
static double myrtle_pair(const nko_myrtle* m, const double* x1, const double* x2, const double* q1,
                          const double* q2, double* qout, double* buf0, double* buf1) {
  int h = m->H, w = m->W;
  double* A = buf0; /* current input of the next conv */
  double* S = buf1;
  seed4(x1, x2, h, w, m->C, A);
  size_t qoff = 0;
  for (int s = 0; s < m->n_stages; ++s) {
    for (int l = 0; l < m->depth[s]; ++l) {
      conv4(A, S, h, w, m->sw2, m->sb2);
      const double *qa, *qb;
      if (q1 == NULL) {
        double* qd = qout + qoff;
        for (int iy = 0; iy < h; ++iy)
          for (int ix = 0; ix < w; ++ix) qd[iy * w + ix] = S[IDX4(iy, ix, iy, ix, h, w)];
        qa = qb = qd;
      } else {
        qa = q1 + qoff;
        qb = q2 + qoff;
      }
      relu4(S, A, h, w, qa, qb);
      qoff += (size_t)h * w;
    }
    if (s + 1 < m->n_stages) {
      pool4(A, S, h, w);
      double* t = A;
      A = S;
      S = t;
      h /= 2;
      w /= 2;
    }
  }
  /* global average pool + dense readout */
  size_t n4 = (size_t)h * w * h * w;
  double acc = 0.0;
  for (size_t e = 0; e < n4; ++e) acc += A[e];
  return m->sw2 * (acc / (double)n4) + m->sb2;
}

static int check_myrtle(const nko_myrtle* m) {
  if (m->H <= 0 || m->W <= 0 || m->C <= 0 || m->n_stages <= 0 || m->n_stages > 8) return -1;
  int h = m->H, w = m->W;
  for (int s = 0; s < m->n_stages; ++s) {
    if (m->depth[s] < 0) return -1;
    if (s + 1 < m->n_stages) {
      if ((h % 2) || (w % 2)) return -1;
      h /= 2;
      w /= 2;
    }
  }
  if (myrtle_layers(m) <= 0) return -1;
  if (!(m->sw2 > 0.0) || m->sb2 < 0.0) return -1;
  return 0;
}

static void promote(const float* src, double* dst, size_t n) {
  for (size_t i = 0; i < n; ++i) dst[i] = (double)src[i];
}

/*
 * Variance maps and self kernel of n images.
 * qmaps: n * qmaps_len doubles (per image: stage-major, layer-major, h*w row-major).
 * kself: n doubles, K(x, x).  Either may be NULL.
 */
int nko_myrtle_self(const float* x, int64_t n, int H, int W, int C, int n_stages, const int* depth,
                    double sw2, double sb2, double* qmaps, double* kself, int nthreads) {
  nko_myrtle m;
  memset(&m, 0, sizeof m);
  m.H = H; m.W = W; m.C = C; m.n_stages = n_stages; m.sw2 = sw2; m.sb2 = sb2;
  if (n_stages <= 0 || n_stages > 8) return -1;
  for (int s = 0; s < n_stages; ++s) m.depth[s] = depth[s];
  if (check_myrtle(&m) || n < 0) return -1;
  size_t qlen = qmaps_len(&m), npix = (size_t)H * W, n4 = npix * npix;
  int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    double* xb = (double*)malloc(npix * C * sizeof(double));
    double* b0 = (double*)malloc(n4 * sizeof(double));
    double* b1 = (double*)malloc(n4 * sizeof(double));
    double* qb = (double*)malloc(qlen * sizeof(double));
    if (!xb || !b0 || !b1 || !qb) {
#pragma omp atomic write
      err = -4;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t a = 0; a < n; ++a) {
        promote(x + (size_t)a * npix * C, xb, npix * C);
        double k = myrtle_pair(&m, xb, xb, NULL, NULL, qb, b0, b1);
        if (qmaps) memcpy(qmaps + (size_t)a * qlen, qb, qlen * sizeof(double));
        if (kself) kself[a] = k;
      }
    }
    free(xb); free(b0); free(b1); free(qb);
  }
  return err;
}

/*
 * K(x1[a], x2[b]) for a list of (a, b) pairs.
 * pairs: npairs * 2 int64 (a, b).  out: npairs doubles.
 * q1/q2: variance maps of x1/x2 from nko_myrtle_self (n1 / n2 images).
 */
int nko_myrtle_pairs(const float* x1, const double* q1, const float* x2, const double* q2, int H, int W,
                     int C, int n_stages, const int* depth, double sw2, double sb2, const int64_t* pairs,
                     int64_t npairs, double* out, int nthreads) {
  nko_myrtle m;
  memset(&m, 0, sizeof m);
  m.H = H; m.W = W; m.C = C; m.n_stages = n_stages; m.sw2 = sw2; m.sb2 = sb2;
  if (n_stages <= 0 || n_stages > 8) return -1;
  for (int s = 0; s < n_stages; ++s) m.depth[s] = depth[s];
  if (check_myrtle(&m) || npairs < 0) return -1;
  size_t qlen = qmaps_len(&m), npix = (size_t)H * W, n4 = npix * npix;
  int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    double* xa = (double*)malloc(npix * C * sizeof(double));
    double* xb = (double*)malloc(npix * C * sizeof(double));
    double* b0 = (double*)malloc(n4 * sizeof(double));
    double* b1 = (double*)malloc(n4 * sizeof(double));
    if (!xa || !xb || !b0 || !b1) {
#pragma omp atomic write
      err = -4;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t p = 0; p < npairs; ++p) {
        int64_t a = pairs[2 * p], b = pairs[2 * p + 1];
        promote(x1 + (size_t)a * npix * C, xa, npix * C);
        promote(x2 + (size_t)b * npix * C, xb, npix * C);
        out[p] = myrtle_pair(&m, xa, xb, q1 + (size_t)a * qlen, q2 + (size_t)b * qlen, NULL, b0, b1);
      }
    }
    free(xa); free(xb); free(b0); free(b1);
  }
  return err;
}


/* E[relu'(u) relu'(v)] for (u, v) ~ N(0, [[q1, s], [s, q2]]). */
static double relu_dot(double s, double q1, double q2) {
  double qq = q1 * q2;
  if (!(qq > 0.0)) return 0.0;
  double rho = s / sqrt(qq);
  if (rho > 1.0) rho = 1.0;
  if (rho < -1.0) rho = -1.0;
  return (NKO_PI - acos(rho)) / (2.0 * NKO_PI);
}

/* T = S + (sw2/9) sum_d B(i+d, j+d), with the conv's padding rule. */
static void conv_tangent4(const double* B, const double* S, double* T, int h, int w, double sw2) {
  for (int iy = 0; iy < h; ++iy)
    for (int ix = 0; ix < w; ++ix)
      for (int jy = 0; jy < h; ++jy)
        for (int jx = 0; jx < w; ++jx) {
          double s = 0.0;
          for (int dy = -1; dy <= 1; ++dy) {
            int ay = iy + dy, by = jy + dy;
            if (ay < 0 || ay >= h || by < 0 || by >= h) continue;
            for (int dx = -1; dx <= 1; ++dx) {
              int ax = ix + dx, bx = jx + dx;
              if (ax < 0 || ax >= w || bx < 0 || bx >= w) continue;
              s += B[IDX4(ay, ax, by, bx, h, w)];
            }
          }
          size_t e = IDX4(iy, ix, jy, jx, h, w);
          T[e] = S[e] + sw2 / 9.0 * s;
        }
}

/* B = Fdot(S, q, q') * T */
static void relu_tangent4(const double* S, const double* T, double* B, int h, int w, const double* q1,
                          const double* q2) {
  for (int iy = 0; iy < h; ++iy)
    for (int ix = 0; ix < w; ++ix)
      for (int jy = 0; jy < h; ++jy)
        for (int jx = 0; jx < w; ++jx) {
          size_t e = IDX4(iy, ix, jy, jx, h, w);
          B[e] = relu_dot(S[e], q1[iy * w + ix], q2[jy * w + jx]) * T[e];
        }
}

/*
 * NNGP and NTK of one pair (cross mode: q1, q2 from the self recursion).
 * buf0..buf4 hold H*W*H*W doubles each.
 */
static void myrtle_pair_ntk(const nko_myrtle* m, const double* x1, const double* x2, const double* q1,
                            const double* q2, double* bufs[5], double* k_nngp, double* k_ntk) {
  int h = m->H, w = m->W;
  double* A = bufs[0];
  double* B = bufs[1];
  double* S = bufs[2];
  double* T = bufs[3];
  double* P = bufs[4];
  seed4(x1, x2, h, w, m->C, A);
  memset(B, 0, sizeof(double) * (size_t)h * w * h * w);
  size_t qoff = 0;
  for (int s = 0; s < m->n_stages; ++s) {
    for (int l = 0; l < m->depth[s]; ++l) {
      conv4(A, S, h, w, m->sw2, m->sb2);
      conv_tangent4(B, S, T, h, w, m->sw2);
      relu4(S, A, h, w, q1 + qoff, q2 + qoff);
      relu_tangent4(S, T, B, h, w, q1 + qoff, q2 + qoff);
      qoff += (size_t)h * w;
    }
    if (s + 1 < m->n_stages) {
      pool4(A, P, h, w);
      pool4(B, S, h, w);
      double* t = A;
      A = P;
      P = t;
      t = B;
      B = S;
      S = t;
      h /= 2;
      w /= 2;
    }
  }
  size_t n4 = (size_t)h * w * h * w;
  double ka = 0.0, kb = 0.0;
  for (size_t e = 0; e < n4; ++e) {
    ka += A[e];
    kb += B[e];
  }
  *k_nngp = m->sw2 * (ka / (double)n4) + m->sb2;
  *k_ntk = *k_nngp + m->sw2 * (kb / (double)n4);
}

/*
 * NNGP and NTK for a list of (a, b) pairs (as nko_myrtle_pairs); out_nngp may
 * be NULL.
 */
int nko_myrtle_ntk_pairs(const float* x1, const double* q1, const float* x2, const double* q2, int H, int W,
                         int C, int n_stages, const int* depth, double sw2, double sb2, const int64_t* pairs,
                         int64_t npairs, double* out_nngp, double* out_ntk, int nthreads) {
  nko_myrtle m;
  memset(&m, 0, sizeof m);
  m.H = H; m.W = W; m.C = C; m.n_stages = n_stages; m.sw2 = sw2; m.sb2 = sb2;
  if (n_stages <= 0 || n_stages > 8) return -1;
  for (int s = 0; s < n_stages; ++s) m.depth[s] = depth[s];
  if (check_myrtle(&m) || npairs < 0) return -1;
  size_t qlen = qmaps_len(&m), npix = (size_t)H * W, n4 = npix * npix;
  int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    double* xa = (double*)malloc(npix * C * sizeof(double));
    double* xb = (double*)malloc(npix * C * sizeof(double));
    double* bufs[5];
    int ok = xa && xb;
    for (int k = 0; k < 5; ++k) {
      bufs[k] = (double*)malloc(n4 * sizeof(double));
      ok = ok && bufs[k];
    }
    if (!ok) {
#pragma omp atomic write
      err = -4;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t p = 0; p < npairs; ++p) {
        int64_t a = pairs[2 * p], b = pairs[2 * p + 1];
        promote(x1 + (size_t)a * npix * C, xa, npix * C);
        promote(x2 + (size_t)b * npix * C, xb, npix * C);
        double kn, kt;
        myrtle_pair_ntk(&m, xa, xb, q1 + (size_t)a * qlen, q2 + (size_t)b * qlen, bufs, &kn, &kt);
        if (out_nngp) out_nngp[p] = kn;
        out_ntk[p] = kt;
      }
    }
    free(xa); free(xb);
    for (int k = 0; k < 5; ++k) free(bufs[k]);
  }
  return err;
}

/* E[relu' relu'] itself, exposed for the quadrature pin. */
double nko_relu_dot(double s, double q1, double q2) { return relu_dot(s, q1, q2); }

size_t nko_myrtle_qmaps_len(int H, int W, int n_stages, const int* depth) {
  nko_myrtle m;
  memset(&m, 0, sizeof m);
  m.H = H; m.W = W; m.n_stages = n_stages;
  for (int s = 0; s < n_stages && s < 8; ++s) m.depth[s] = depth[s];
  return qmaps_len(&m);
}

/* ------------------------------------------------------------------------ */
/* Fully connected (FC3 of App. A)                                           */
/* ------------------------------------------------------------------------ */

/*
 * K (n1 x n2, row-major) of a depth-ReLU fully connected network on
 * flattened d-dim inputs: K1 = sw2 x.x'/d + sb2, then depth times
 * K <- sw2 F(K, Kxx, Kx'x') + sb2, where the diagonals follow the same map.
 */
int nko_fc_nngp(const float* x1, int64_t n1, const float* x2, int64_t n2, int d, int depth, double sw2,
                double sb2, double* K, int nthreads) {
  if (n1 < 0 || n2 < 0 || d <= 0 || depth < 0 || !(sw2 > 0.0) || sb2 < 0.0) return -1;
  double* d1 = (double*)malloc((size_t)(n1 > 0 ? n1 : 1) * sizeof(double));
  double* d2 = (double*)malloc((size_t)(n2 > 0 ? n2 : 1) * sizeof(double));
  if (!d1 || !d2) { free(d1); free(d2); return -4; }
  for (int64_t a = 0; a < n1; ++a) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += (double)x1[(size_t)a * d + k] * (double)x1[(size_t)a * d + k];
    d1[a] = s;
  }
  for (int64_t b = 0; b < n2; ++b) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += (double)x2[(size_t)b * d + k] * (double)x2[(size_t)b * d + k];
    d2[b] = s;
  }
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static)
  for (int64_t a = 0; a < n1; ++a) {
    for (int64_t b = 0; b < n2; ++b) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += (double)x1[(size_t)a * d + k] * (double)x2[(size_t)b * d + k];
      double k12 = sw2 * s / d + sb2;
      double k11 = sw2 * d1[a] / d + sb2;
      double k22 = sw2 * d2[b] / d + sb2;
      for (int l = 0; l < depth; ++l) {
        double n12 = sw2 * relu_map(k12, k11, k22) + sb2;
        double n11 = sw2 * relu_map(k11, k11, k11) + sb2;
        double n22 = sw2 * relu_map(k22, k22, k22) + sb2;
        k12 = n12; k11 = n11; k22 = n22;
      }
      K[(size_t)a * n2 + b] = k12;
    }
  }
  free(d1);
  free(d2);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* CNN-VEC (App. "Neural Kernel Architecture", CNN-VEC listing)              */
/* ------------------------------------------------------------------------ */
/*
 * depth blocks of [3x3 SAME conv, ReLU] at full resolution, Flatten, Dense.
 * The flatten readout averages the covariance of each pixel of x with the
 * SAME pixel of x': K = sw2 mean_i A(i, i) + sb2.  A conv only couples
 * (i, j) to (i + d, j + d), so the entries (i, i) form a closed recursion
 * over one h x w map per pair:
 *   S(i) = x(i).x'(i) / C,
 *   per block: V(i) = sw2 / 9 sum_{|d| <= 1, i + d inside} S(i + d) + sb2,
 *              S(i) = F(V(i), q_x(i), q_x'(i)),
 * with q_x the same recursion run on the pair (x, x) (whose V is its own
 * variance map).
 */

/* one block: V = conv of S (zero padding, /9 always), then S = F(V, q1, q2) */
static void cv_block(double* S, double* V, int h, int w, double sw2, double sb2) {
  for (int iy = 0; iy < h; ++iy)
    for (int ix = 0; ix < w; ++ix) {
      double s = 0.0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int y = iy + dy, x = ix + dx;
          if (y < 0 || y >= h || x < 0 || x >= w) continue;
          s += S[(size_t)y * w + x];
        }
      V[(size_t)iy * w + ix] = sw2 / 9.0 * s + sb2;
    }
}

static void cv_seed(const float* x1, const float* x2, int hw, int c, double* S) {
  for (int i = 0; i < hw; ++i) {
    double s = 0.0;
    for (int k = 0; k < c; ++k) s += (double)x1[(size_t)i * c + k] * (double)x2[(size_t)i * c + k];
    S[i] = s / c;
  }
}

/* Variance maps q[img][block][pixel] (the pre-activation variance at each
 * ReLU) and K(x, x) of each image. */
int nko_cv_self(const float* x, int64_t n, int H, int W, int C, int depth, double sw2, double sb2, double* q,
                double* kdiag, int nthreads) {
  if (n < 0 || H <= 0 || W <= 0 || C <= 0 || depth < 1 || !(sw2 > 0.0) || sb2 < 0.0) return -1;
  const int hw = H * W;
  int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    double* S = (double*)malloc(sizeof(double) * hw);
    double* V = (double*)malloc(sizeof(double) * hw);
    if (!S || !V) {
#pragma omp atomic write
      err = -4;
    } else {
#pragma omp for schedule(static)
      for (int64_t a = 0; a < n; ++a) {
        const float* xa = x + (size_t)a * hw * C;
        cv_seed(xa, xa, hw, C, S);
        for (int l = 0; l < depth; ++l) {
          cv_block(S, V, H, W, sw2, sb2);
          double* qa = q + ((size_t)a * depth + l) * hw;
          for (int i = 0; i < hw; ++i) {
            qa[i] = V[i];
            S[i] = relu_map(V[i], V[i], V[i]);
          }
        }
        double m = 0.0;
        for (int i = 0; i < hw; ++i) m += S[i];
        kdiag[a] = sw2 * m / hw + sb2;
      }
    }
    free(S);
    free(V);
  }
  return err;
}

/* K(x1[a], x2[b]) for each listed pair, given both images' variance maps. */
int nko_cv_pairs(const float* x1, const double* q1, const float* x2, const double* q2, int H, int W, int C,
                 int depth, double sw2, double sb2, const int64_t* pairs, int64_t np, double* out, int nthreads) {
  if (H <= 0 || W <= 0 || C <= 0 || depth < 1 || !(sw2 > 0.0) || sb2 < 0.0 || np < 0) return -1;
  const int hw = H * W;
  int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    double* S = (double*)malloc(sizeof(double) * hw);
    double* V = (double*)malloc(sizeof(double) * hw);
    if (!S || !V) {
#pragma omp atomic write
      err = -4;
    } else {
#pragma omp for schedule(static)
      for (int64_t p = 0; p < np; ++p) {
        const int64_t a = pairs[2 * p], b = pairs[2 * p + 1];
        cv_seed(x1 + (size_t)a * hw * C, x2 + (size_t)b * hw * C, hw, C, S);
        for (int l = 0; l < depth; ++l) {
          cv_block(S, V, H, W, sw2, sb2);
          const double* qa = q1 + ((size_t)a * depth + l) * hw;
          const double* qb = q2 + ((size_t)b * depth + l) * hw;
          for (int i = 0; i < hw; ++i) S[i] = relu_map(V[i], qa[i], qb[i]);
        }
        double m = 0.0;
        for (int i = 0; i < hw; ++i) m += S[i];
        out[p] = sw2 * m / hw + sb2;
      }
    }
    free(S);
    free(V);
  }
  return err;
}

/* The ReLU map itself, exposed for the quadrature pin. */
double nko_relu_map(double s, double q1, double q2) { return relu_map(s, q1, q2); }

int nko_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
