// Kernels of the C_l emulator: a small MLP (FP32 on the matrix cores) from
// the 5 source parameters to whitened PCA coefficients of the transformed
// spectra, its training (backprop + Adam), the PCA fit (FP64) and the
// ensemble reconstruction with an error estimate.  Definitions of every
// quantity are in emu_api.cpp.
#include <hip/hip_runtime.h>

#include "emu_internal.hpp"

namespace los {
namespace emu {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) +
         x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// C(m, n) = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn], C row-major with leading dimension ldc.
// Workgroup: 64 x 64 of C, 4 waves in a 2 x 2 arrangement, each wave 32 x 32
// (2 x 2 MFMA 16x16x4 blocks); rows and columns outside [M, N) and K beyond K
// read 0.  K goes in tiles of 32: the workgroup stages the 64 x 32 slice of A
// and the 32 x 64 slice of B in LDS, each loaded along whichever of its
// strides is 1 (consecutive lanes, consecutive addresses), and loads the next
// tile into registers while the matrix cores work on this one.  Every wave
// issues its products in increasing k, 4 at a time.
template <int EPI>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmF32 g) {
  constexpr int KT = 32, LD = 80;  // row pitch: the 4 k rows of a read hit distinct banks
  __shared__ float As[KT][LD], Bs[KT][LD];
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, kq = lane >> 4;
  const int64_t mb = (int64_t)blockIdx.y * 64, nb = (int64_t)blockIdx.x * 64;
  const int mw = (w >> 1) * 32, nw = (w & 1) * 32;
  const int64_t m0 = mb + mw, n0 = nb + nw;
  const bool a_k = g.sak == 1, b_n = g.sbn == 1;  // contiguous axis of each operand
  // element it * 256 + tid of a tile: (row of A, k) and (k, column of B)
  auto a_at = [&](int e, int &mm, int &kk) {
    if (a_k) { kk = e & 31; mm = e >> 5; } else { mm = e & 63; kk = e >> 6; }
  };
  auto b_at = [&](int e, int &kk, int &nn) {
    if (b_n) { nn = e & 63; kk = e >> 6; } else { kk = e & 31; nn = e >> 5; }
  };
  float ra[8], rb[8];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int e = it * 256 + tid;
      int mm, kk, nn, kb;
      a_at(e, mm, kk);
      b_at(e, kb, nn);
      const int64_t m = mb + mm, ka = k0 + kk, n = nb + nn, kB = k0 + kb;
      ra[it] = (m < g.M && ka < g.K) ? g.A[m * g.sam + ka * g.sak] : 0.f;
      rb[it] = (n < g.N && kB < g.K) ? g.B[kB * g.sbk + n * g.sbn] : 0.f;
    }
  };
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  if (g.K > 0) load(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += KT) {
    __syncthreads();  // the previous tile is consumed
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int e = it * 256 + tid;
      int mm, kk, nn, kb;
      a_at(e, mm, kk);
      b_at(e, kb, nn);
      As[kk][mm] = ra[it];
      Bs[kb][nn] = rb[it];
    }
    __syncthreads();
    if (k0 + KT < g.K) load(k0 + KT);
    const int kn = g.K - k0 < KT ? (int)(g.K - k0) : KT;
    for (int kk = 0; kk < kn; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = As[kk + kq][mw + 16 * i + r16];
        b[i] = Bs[kk + kq][nw + 16 * i + r16];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t n = n0 + 16 * j + r16;
      if (n >= g.N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + 16 * i + 4 * kq + v;
        if (m >= g.M) continue;
        float x = acc[i][j][v];
        float *c = g.C + m * g.ldc + n;
        if (EPI == kEpiStore) {
          *c = x;
        } else if (EPI == kEpiAccumulate) {
          *c += x;
        } else if (EPI == kEpiBias) {
          *c = x + g.bias[n];
        } else {  // kEpiBiasGelu: keep the pre-activation in Z
          x += g.bias[n];
          g.Z[m * g.ldc + n] = x;
          *c = gelu_f(x);
        }
      }
    }
}

// FP64 C = A B (same strides as above), LDS-tiled 64 x 64 with a 4 x 4
// register tile per thread; used for the PCA fit only.
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmF64 g) {
  __shared__ double As[16][65], Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < g.K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, mm = e % 64;
      const int64_t m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.M && k < g.K) ? g.A[m * g.sam + k * g.sak] : 0.0;
      const int64_t n = n0 + mm;
      Bs[kk][mm] = (n < g.N && k < g.K) ? g.B[k * g.sbk + n * g.sbn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t m = m0 + ty + 16 * i, n = n0 + tx + 16 * j;
      if (m < g.M && n < g.N) g.C[m * g.ldc + n] = acc[i][j];
    }
}

// G <- G * gelu'(Z), elementwise.
__global__ void gelu_backward_kernel(float *G, const float *Z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) G[i] *= gelu_grad_f(Z[i]);
}

// out[c] = sum_r X[r * ld + c] (one thread per column, fixed order).
__global__ void colsum_f32_kernel(const float *X, int64_t rows, int64_t cols, float *out) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int64_t r = 0; r < rows; ++r) s += X[r * cols + c];
  out[c] = s;
}

// MSE gradient: G = 2 (out - z) / (n m); loss[0] = sum (out - z)^2 / (n m),
// summed per block then added in block order by a single thread (fixed order).
__global__ __launch_bounds__(256) void mse_grad_kernel(const float *out, const float *z, int64_t cnt,
                                                       float scale, float *G, float *partial) {
  __shared__ float red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float d = 0.f;
  if (i < cnt) {
    d = out[i] - z[i];
    G[i] = 2.f * scale * d;
  }
  red[threadIdx.x] = d * d;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * scale;
}

__global__ void sum_partials_kernel(const float *partial, int nb, float *loss, int accumulate) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += partial[b];
  loss[0] = accumulate ? loss[0] + s : s;
}

// Adam with bias correction; lr already includes the schedule.
__global__ void adam_kernel(float *w, const float *g, float *m, float *v, int64_t n, float lr,
                            float b1, float b2, float c1, float c2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// dst[r][:] = src[idx[r]][:], float rows of length cols.
__global__ void gather_rows_kernel(const float *src, const int64_t *idx, int64_t rows, int64_t cols,
                                   float *dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols, c = i % cols;
  dst[i] = src[idx[r] * cols + c];
}

// u = 2 (p - lo) / (hi - lo) - 1 in FP32.
__global__ void scale_params_kernel(const double *p, int64_t n, int np, const double *lo,
                                    const double *hi, float *u) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * np) return;
  const int j = (int)(i % np);
  u[i] = (float)(2.0 * (p[i] - lo[j]) / (hi[j] - lo[j]) - 1.0);
}

// y[r][s][l] from cl[r][s][l]: log for TT, EE, PP, asinh(TE / t_l) for TE.
__global__ void transform_kernel(const double *cl, int64_t n, int nl, const double *t, double *y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * 4 * nl) return;
  const int l = (int)(i % nl);
  const int s = (int)((i / nl) % 4);
  const double c = cl[i];
  y[i] = s == 2 ? asinh(c / t[l]) : log(c);
}

// t_l = lower median over samples of |TE_l| (1 if that is 0), from at most
// 8192 evenly strided samples (all of them when n <= 8192): bitonic sort in LDS.
__global__ __launch_bounds__(1024) void te_median_kernel(const double *cl, int64_t n, int nl,
                                                          double *t) {
  __shared__ double v[8192];
  const int l = blockIdx.x;
  const int64_t cnt = n < 8192 ? n : 8192;
  const double step = (double)n / (double)cnt;
  for (int i = threadIdx.x; i < 8192; i += 1024) {
    double x = __builtin_huge_val();
    if (i < cnt) {
      const int64_t r = cnt == n ? i : (int64_t)(i * step);
      x = fabs(cl[(r * 4 + 2) * nl + l]);
    }
    v[i] = x;
  }
  __syncthreads();
  for (int size = 2; size <= 8192; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < 8192; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const double a = v[i], b = v[j];
          if ((a > b) == up) {
            v[i] = b;
            v[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const double med = v[(cnt - 1) / 2];
    t[l] = med > 0.0 ? med : 1.0;  // a zero median: asinh(0 / t) = 0 for any t
  }
}

// Column means of X [rows][cols] (FP64, fixed order), then X -= mean.
__global__ void center_kernel(double *X, int64_t rows, int64_t cols, int64_t ld, double *mean) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int64_t r = 0; r < rows; ++r) s += X[r * ld + c];
  s /= (double)rows;
  mean[c] = s;
  for (int64_t r = 0; r < rows; ++r) X[r * ld + c] -= s;
}

// Cholesky-QR step on a q x q Gram matrix G (one workgroup, q <= kMaxQ):
// R^T R = G with R upper triangular (in LDS), then Rinv = R^{-1} written to
// global memory column by column (thread c owns column c, so its own earlier
// writes are the only values it reads back).  status[0] = 1 if G is not
// numerically positive definite.
__global__ __launch_bounds__(256) void chol_inv_kernel(const double *G, int q, double shift_rel,
                                                       double *Rinv, int *status) {
  __shared__ double R[kMaxQ][kMaxQ + 1];
  __shared__ double shift;
  for (int e = threadIdx.x; e < q * q; e += 256) R[e / q][e % q] = G[e];
  __syncthreads();
  if (threadIdx.x == 0) {  // shift = shift_rel * trace(G)
    double tr = 0.0;
    for (int j = 0; j < q; ++j) tr += R[j][j];
    shift = shift_rel * tr;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < q; j += 256) R[j][j] += shift;
  __syncthreads();
  for (int j = 0; j < q; ++j) {
    if (threadIdx.x == 0) {
      const double d = R[j][j];
      if (!(d > 0.0)) status[0] = 1;
      R[j][j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    for (int c = j + 1 + threadIdx.x; c < q; c += 256) R[j][c] /= R[j][j];
    __syncthreads();
    const int w = q - j - 1;
    for (int e = threadIdx.x; e < w * w; e += 256) {
      const int r = j + 1 + e / w, c = j + 1 + e % w;
      if (c >= r) R[r][c] -= R[j][r] * R[j][c];
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < q; c += 256) {
    for (int r = q - 1; r > c; --r) Rinv[r * q + c] = 0.0;
    for (int r = c; r >= 0; --r) {
      double s = r == c ? 1.0 : 0.0;
      for (int k = r + 1; k <= c; ++k) s -= R[r][k] * Rinv[k * q + c];
      Rinv[r * q + c] = s / R[r][r];
    }
  }
}

// Symmetric eigen-decomposition of a q x q matrix (one workgroup, q <= kMaxQ)
// by cyclic Jacobi rotations.  The matrix lives in LDS; the accumulated
// rotations V [q][q] in global memory (thread k owns row k of V).  On exit
// evals are sorted decreasing and U's columns are the matching eigenvectors.
__global__ __launch_bounds__(256) void jacobi_eig_kernel(const double *A, int q, int sweeps,
                                                         double *V, double *evals, double *U) {
  __shared__ double W[kMaxQ][kMaxQ + 1];
  __shared__ double cs[2];
  __shared__ int order[kMaxQ];
  for (int e = threadIdx.x; e < q * q; e += 256) {
    W[e / q][e % q] = A[e];
    V[e] = (e / q == e % q) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int p = 0; p < q - 1; ++p) {
      for (int r = p + 1; r < q; ++r) {
        if (threadIdx.x == 0) {
          const double apq = W[p][r];
          double c = 1.0, s = 0.0;
          if (fabs(apq) > 1e-300) {
            const double tau = (W[r][r] - W[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
          cs[0] = c;
          cs[1] = s;
        }
        __syncthreads();
        const double c = cs[0], s = cs[1];
        if (s != 0.0) {
          for (int k = threadIdx.x; k < q; k += 256) {  // rows p and r
            const double wp = W[p][k], wr = W[r][k];
            W[p][k] = c * wp - s * wr;
            W[r][k] = s * wp + c * wr;
          }
          __syncthreads();
          for (int k = threadIdx.x; k < q; k += 256) {  // columns p and r, and V
            const double wp = W[k][p], wr = W[k][r];
            W[k][p] = c * wp - s * wr;
            W[k][r] = s * wp + c * wr;
            const double vp = V[k * q + p], vr = V[k * q + r];
            V[k * q + p] = c * vp - s * vr;
            V[k * q + r] = s * vp + c * vr;
          }
        }
        __syncthreads();
      }
    }
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < q; ++i) order[i] = i;
    for (int i = 1; i < q; ++i) {  // insertion sort, decreasing eigenvalue
      const int o = order[i];
      int j = i - 1;
      while (j >= 0 && W[order[j]][order[j]] < W[o][o]) {
        order[j + 1] = order[j];
        --j;
      }
      order[j + 1] = o;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < q * q; e += 256) U[e] = V[(e / q) * q + order[e % q]];
  for (int i = threadIdx.x; i < q; i += 256) evals[i] = W[order[i]][order[i]];
}

// Scaled targets of spectrum s: sigma_s = sqrt(sum_j mean_r c[r][j]^2) (the
// variance the kept components explain; coefficients have zero mean), stored
// for every component j, and z[r][s * ncomp + j] = c[r][j] / sigma_s (FP32).
// One workgroup, one thread per component (ncomp <= 256).
__global__ __launch_bounds__(256) void whiten_kernel(const double *c, int64_t n, int ncomp, int s,
                                                     int nout, double *sigma, float *z) {
  __shared__ double var[256];
  __shared__ double scale;
  const int j = threadIdx.x;
  double q = 0.0;
  if (j < ncomp)
    for (int64_t r = 0; r < n; ++r) q += c[r * ncomp + j] * c[r * ncomp + j];
  var[j] = q / (double)n;
  __syncthreads();
  if (j == 0) {
    double tot = 0.0;
    for (int i = 0; i < ncomp; ++i) tot += var[i];
    scale = tot > 0.0 ? sqrt(tot) : 1.0;
  }
  __syncthreads();
  if (j >= ncomp) return;
  sigma[s * ncomp + j] = scale;
  for (int64_t r = 0; r < n; ++r) z[r * nout + s * ncomp + j] = (float)(c[r * ncomp + j] / scale);
}

// coefficient rows for reconstruction: cz[r][j] = out[r][s * ncomp + j] * sigma[s][j]
__global__ void unwhiten_kernel(const float *out, int64_t n, int ncomp, int s, int nout,
                                const double *sigma, float *cz) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * ncomp) return;
  const int64_t r = i / ncomp;
  const int j = (int)(i % ncomp);
  cz[i] = (float)((double)out[r * nout + s * ncomp + j] * sigma[s * ncomp + j]);
}

// Ensemble mean of C_l and error estimate.  y holds every member's
// reconstructed transformed spectra, y[e][r][s][l] (float).  One thread per
// (r, l): writes cl[r][s][l] (mean over members) for the 4 spectra and folds
// the largest scaled deviation into err[r] (float bits, atomic max of
// non-negative values: independent of order).
// Member mean of every C_l and, per (row, spectrum), the largest member
// deviation relative to the spectrum's scale (err_bits[r][4], float bits,
// order-independent atomicMax).  Workgroup = one row r (blockIdx.x) and 256
// multipoles (blockIdx.y): the deviations are reduced over the workgroup
// first (max of the float bits, exact in any order), so each workgroup issues
// four atomics instead of four per multipole on the same four addresses.
__global__ __launch_bounds__(256) void ensemble_kernel(const float *y, int members, int64_t n,
                                                       int nl, const double *t, double *cl,
                                                       unsigned int *err_bits) {
  __shared__ unsigned int red[4][4];
  const int64_t r = blockIdx.x;
  const int l = blockIdx.y * 256 + threadIdx.x;
  unsigned int bits[4] = {0u, 0u, 0u, 0u};
  if (l < nl) {
    double mean[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = 0; e < members; ++e)
      for (int s = 0; s < 4; ++s) {
        const double v = (double)y[(((int64_t)e * n + r) * 4 + s) * nl + l];
        mean[s] += s == 2 ? t[l] * sinh(v) : exp(v);
      }
    for (int s = 0; s < 4; ++s) {
      mean[s] /= members;
      cl[(r * 4 + s) * nl + l] = mean[s];
    }
    double scale[4] = {fabs(mean[0]), fabs(mean[1]), sqrt(mean[0] * mean[1]), fabs(mean[3])};
    double dev[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = 0; e < members; ++e)
      for (int s = 0; s < 4; ++s) {
        const double v = (double)y[(((int64_t)e * n + r) * 4 + s) * nl + l];
        const double c = s == 2 ? t[l] * sinh(v) : exp(v);
        dev[s] = fmax(dev[s], fabs(c - mean[s]) / scale[s]);
      }
    for (int s = 0; s < 4; ++s) bits[s] = __float_as_uint((float)dev[s]);
  }
  for (int s = 0; s < 4; ++s)
    for (int o = 32; o >= 1; o >>= 1) {
      const unsigned int u = __shfl_xor(bits[s], o, 64);
      bits[s] = u > bits[s] ? u : bits[s];
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int s = 0; s < 4; ++s) red[w][s] = bits[s];
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned int m = 0u;
    for (int v = 0; v < 4; ++v) m = red[v][threadIdx.x] > m ? red[v][threadIdx.x] : m;
    atomicMax(err_bits + r * 4 + threadIdx.x, m);
  }
}

// Per row (err, flag: the largest of its four spectra) and / or per
// (row, spectrum) (err4, flag4); any of the four may be NULL.
__global__ void flag_kernel(const unsigned int *err_bits, int64_t n, float thr, float *err,
                            unsigned char *flag, float *err4, unsigned char *flag4) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  float emax = 0.f;
  for (int s = 0; s < 4; ++s) {
    const float e = __uint_as_float(err_bits[r * 4 + s]);
    emax = fmaxf(emax, e);
    if (err4) err4[r * 4 + s] = e;
    if (flag4) flag4[r * 4 + s] = !(e <= thr);
  }
  if (err) err[r] = emax;
  if (flag) flag[r] = !(emax <= thr);
}

__global__ void zero_u32_kernel(unsigned int *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t gemm_f32(const GemmF32 &g, int epi, hipStream_t s) {
  dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64));
  switch (epi) {
    case kEpiStore: hipLaunchKernelGGL(gemm_f32_kernel<kEpiStore>, grid, dim3(256), 0, s, g); break;
    case kEpiAccumulate:
      hipLaunchKernelGGL(gemm_f32_kernel<kEpiAccumulate>, grid, dim3(256), 0, s, g);
      break;
    case kEpiBias: hipLaunchKernelGGL(gemm_f32_kernel<kEpiBias>, grid, dim3(256), 0, s, g); break;
    default: hipLaunchKernelGGL(gemm_f32_kernel<kEpiBiasGelu>, grid, dim3(256), 0, s, g); break;
  }
  return hipGetLastError();
}

hipError_t gemm_f64(const GemmF64 &g, hipStream_t s) {
  dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64));
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t gelu_backward(float *G, const float *Z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(gelu_backward_kernel, dim3(blocks(n)), dim3(256), 0, s, G, Z, n);
  return hipGetLastError();
}

hipError_t colsum_f32(const float *X, int64_t rows, int64_t cols, float *out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_f32_kernel, dim3(blocks(cols)), dim3(256), 0, s, X, rows, cols, out);
  return hipGetLastError();
}

hipError_t mse_grad(const float *out, const float *z, int64_t cnt, float *G, float *partial,
                    float *loss, int accumulate, hipStream_t s) {
  const unsigned nb = blocks(cnt);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nb), dim3(256), 0, s, out, z, cnt, 1.f / (float)cnt, G,
                     partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, partial, (int)nb, loss,
                     accumulate);
  return hipGetLastError();
}

hipError_t adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, int64_t t,
                hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - pow(0.9, (double)t)), c2 = (float)(1.0 - pow(0.999, (double)t));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, c1,
                     c2, 1e-8f);
  return hipGetLastError();
}

hipError_t gather_rows(const float *src, const int64_t *idx, int64_t rows, int64_t cols,
                       float *dst, hipStream_t s) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks(rows * cols)), dim3(256), 0, s, src, idx,
                     rows, cols, dst);
  return hipGetLastError();
}

hipError_t scale_params(const double *p, int64_t n, int np, const double *lo, const double *hi,
                        float *u, hipStream_t s) {
  hipLaunchKernelGGL(scale_params_kernel, dim3(blocks(n * np)), dim3(256), 0, s, p, n, np, lo, hi,
                     u);
  return hipGetLastError();
}

hipError_t transform(const double *cl, int64_t n, int nl, const double *t, double *y,
                     hipStream_t s) {
  hipLaunchKernelGGL(transform_kernel, dim3(blocks(n * 4 * nl)), dim3(256), 0, s, cl, n, nl, t, y);
  return hipGetLastError();
}

hipError_t te_median(const double *cl, int64_t n, int nl, double *t, hipStream_t s) {
  hipLaunchKernelGGL(te_median_kernel, dim3(nl), dim3(1024), 0, s, cl, n, nl, t);
  return hipGetLastError();
}

hipError_t center(double *X, int64_t rows, int64_t cols, int64_t ld, double *mean, hipStream_t s) {
  hipLaunchKernelGGL(center_kernel, dim3(blocks(cols)), dim3(256), 0, s, X, rows, cols, ld, mean);
  return hipGetLastError();
}

hipError_t chol_inv(const double *G, int q, double shift_rel, double *Rinv, int *status,
                    hipStream_t s) {
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(256), 0, s, G, q, shift_rel, Rinv, status);
  return hipGetLastError();
}

hipError_t jacobi_eig(const double *A, int q, int sweeps, double *V, double *evals, double *U,
                      hipStream_t s) {
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(1), dim3(256), 0, s, A, q, sweeps, V, evals, U);
  return hipGetLastError();
}

hipError_t whiten(const double *c, int64_t n, int ncomp, int s_idx, int nout, double *sigma,
                  float *z, hipStream_t s) {
  hipLaunchKernelGGL(whiten_kernel, dim3(1), dim3(256), 0, s, c, n, ncomp, s_idx, nout, sigma, z);
  return hipGetLastError();
}

hipError_t unwhiten(const float *out, int64_t n, int ncomp, int s_idx, int nout,
                    const double *sigma, float *cz, hipStream_t s) {
  hipLaunchKernelGGL(unwhiten_kernel, dim3(blocks(n * ncomp)), dim3(256), 0, s, out, n, ncomp,
                     s_idx, nout, sigma, cz);
  return hipGetLastError();
}

hipError_t ensemble(const float *y, int members, int64_t n, int nl, const double *t, double *cl,
                    unsigned int *err_bits, float thr, float *err, unsigned char *flag,
                    float *err4, unsigned char *flag4, hipStream_t s) {
  hipLaunchKernelGGL(zero_u32_kernel, dim3(blocks(4 * n)), dim3(256), 0, s, err_bits, 4 * n);
  if (n > 0x7fffffff) return hipErrorInvalidValue;  // one workgroup row per model row
  if (n > 0 && nl > 0)
    hipLaunchKernelGGL(ensemble_kernel, dim3((unsigned)n, (unsigned)((nl + 255) / 256)), dim3(256), 0,
                       s, y, members, n, nl, t, cl, err_bits);
  hipLaunchKernelGGL(flag_kernel, dim3(blocks(n)), dim3(256), 0, s, err_bits, n, thr, err, flag,
                     err4, flag4);
  return hipGetLastError();
}

// Fallback merge: row rows[i] of cl [n][row_len] takes src[i][row_len]; its
// error estimate becomes 0 and its fallback flag 0 (err, flag optional).
__global__ __launch_bounds__(256) void merge_rows_kernel(const int64_t *rows, int64_t nf,
                                                         const double *src, int64_t row_len,
                                                         double *cl, float *err,
                                                         unsigned char *flag) {
  const int64_t total = nf * row_len;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / row_len, c = t - i * row_len;
    const int64_t r = rows[i];
    cl[r * row_len + c] = src[t];
    if (c == 0) {
      if (err) err[r] = 0.f;
      if (flag) flag[r] = 0;
    }
  }
}

hipError_t merge_rows(const int64_t *rows, int64_t nf, const double *src, int64_t row_len,
                      double *cl, float *err, unsigned char *flag, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  int64_t b = (nf * row_len + 255) / 256;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(merge_rows_kernel, dim3((unsigned)b), dim3(256), 0, s, rows, nf, src, row_len,
                     cl, err, flag);
  return hipGetLastError();
}

// One spectrum of the fallback rows: cl[rows[i]][spec][l] = src[i][l] for
// l < nl; err4 / flag4 of (rows[i], spec) become 0 (both optional).
__global__ __launch_bounds__(256) void merge_spectrum_kernel(const int64_t *rows, int64_t nf,
                                                             const double *src, int nl, int spec,
                                                             double *cl, float *err4,
                                                             unsigned char *flag4) {
  const int64_t total = nf * nl;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / nl, l = t - i * nl;
    const int64_t r = rows[i];
    cl[(r * 4 + spec) * nl + l] = src[t];
    if (l == 0) {
      if (err4) err4[r * 4 + spec] = 0.f;
      if (flag4) flag4[r * 4 + spec] = 0;
    }
  }
}

hipError_t merge_spectrum(const int64_t *rows, int64_t nf, const double *src, int nl, int spec,
                          double *cl, float *err4, unsigned char *flag4, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  int64_t b = (nf * nl + 255) / 256;
  if (b > 16384) b = 16384;
  hipLaunchKernelGGL(merge_spectrum_kernel, dim3((unsigned)b), dim3(256), 0, s, rows, nf, src, nl,
                     spec, cl, err4, flag4);
  return hipGetLastError();
}

}  // namespace emu
}  // namespace los
