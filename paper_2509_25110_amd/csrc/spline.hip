// Source preparation on the integration grid (gCAMB paper Sec. 3.2: the
// InterpolateSources step runs before the line-of-sight integrals).  The
// sources are given on a coarse wavenumber grid q_0 < ... < q_{N-1} at the
// projection's tau nodes and are carried to the projection's k grid by the
// natural cubic spline in k, one spline per (source, tau node) column:
//
//   on [q_j, q_{j+1}], h_j = q_{j+1} - q_j, A = (q_{j+1} - k) / h_j,
//   B = (k - q_j) / h_j:
//     s(k) = A y_j + B y_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) h_j^2 / 6
//
// with the second derivatives M from the tridiagonal system (j = 1 .. N-2)
//     h_{j-1}/6 M_{j-1} + (h_{j-1} + h_j)/3 M_j + h_j/6 M_{j+1}
//         = (y_{j+1} - y_j)/h_j - (y_j - y_{j-1})/h_{j-1},   M_0 = M_{N-1} = 0.
//
// Solve: the matrix depends on the knots only and is shared by all
// nsrc * ntau columns.  Rows are cut into segments of SEG = 16; a thread owns
// one segment of one column and keeps its 16 unknowns in registers.  Within a
// segment the system is solved with the coupling to the neighbouring
// segments left out (y), and the two "spikes" v, w (the segment's response to
// its outside neighbours) are column-independent, so
//   x = y - v * x_{first-1} - w * x_{last+1}.
// The boundary unknowns (first F_p and last L_p of every segment) satisfy a
// 2x2-block tridiagonal system; its elimination factors are again
// column-independent.  One factor kernel builds every table from q; one
// solve kernel per group of C columns x P segments runs local solve -> LDS
// -> reduced solve by one thread per column -> correction, reading each
// source value once and writing each M once.  The system is strictly
// diagonally dominant (off-diagonal sum = half the diagonal), so no pivoting.
#include "los.h"
#include "los_internal.hpp"

namespace los {
namespace {

constexpr int SEG = 16;
constexpr int kRed = 6;  // per-segment reduced factors: v0, v15, inv_d, eF, eL, v15 * eL_prev

__global__ __launch_bounds__(256) void spline_factor_kernel(const double *__restrict__ q,
                                                             int64_t N, int P, SplineTabs t) {
  extern __shared__ double ends[];  // [P][4]: v0, v15, w0, w15 -> the reduced factors [P][6]
  const int64_t n = N - 2;  // interior unknowns i = 0 .. n-1 (knot i + 1)
  for (int64_t j = threadIdx.x; j < N - 1; j += blockDim.x) t.ih[j] = 1.0 / (q[j + 1] - q[j]);
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    double sub[SEG], dg[SEG], sup[SEG];
#pragma unroll
    for (int r = 0; r < SEG; ++r) {
      const int64_t i = (int64_t)p * SEG + r;
      if (i < n) {
        const double h0 = q[i + 1] - q[i], h1 = q[i + 2] - q[i + 1];
        sub[r] = i > 0 ? h0 / 6.0 : 0.0;  // row 0 couples to M_0 = 0
        dg[r] = (h0 + h1) / 3.0;
        sup[r] = i < n - 1 ? h1 / 6.0 : 0.0;  // last row couples to M_{N-1} = 0
      } else {  // padding row: x = 0, decoupled
        sub[r] = 0.0;
        dg[r] = 1.0;
        sup[r] = 0.0;
      }
    }
    // local Thomas factors (row 0's sub and row 15's sup are the couplings)
    double iden[SEG], cp[SEG];
    iden[0] = 1.0 / dg[0];
    cp[0] = sup[0] * iden[0];
#pragma unroll
    for (int r = 1; r < SEG; ++r) {
      iden[r] = 1.0 / (dg[r] - sub[r] * cp[r - 1]);
      cp[r] = sup[r] * iden[r];
    }
    // spike v: T v = sub[0] e_0
    double v[SEG], w[SEG];
    v[0] = sub[0] * iden[0];
#pragma unroll
    for (int r = 1; r < SEG; ++r) v[r] = -sub[r] * v[r - 1] * iden[r];
#pragma unroll
    for (int r = SEG - 2; r >= 0; --r) v[r] -= cp[r] * v[r + 1];
    // spike w: T w = sup[15] e_15
    w[SEG - 1] = sup[SEG - 1] * iden[SEG - 1];
#pragma unroll
    for (int r = SEG - 2; r >= 0; --r) w[r] = -cp[r] * w[r + 1];
#pragma unroll
    for (int r = 0; r < SEG; ++r) {
      const int64_t i = (int64_t)p * SEG + r;
      t.sub[i] = r > 0 ? sub[r] : 0.0;
      t.iden[i] = iden[r];
      t.cp[i] = cp[r];
      t.v[i] = v[r];
      t.w[i] = w[r];
    }
    ends[4 * p + 0] = v[0];
    ends[4 * p + 1] = v[SEG - 1];
    ends[4 * p + 2] = w[0];
    ends[4 * p + 3] = w[SEG - 1];
  }
  __syncthreads();
  double *red = ends + 4 * P;  // [P][kRed]
  if (threadIdx.x == 0) {
    // 2x2-block elimination of z_p = (F_p, L_p):
    //   z_p + (v0, v15) L_{p-1} + (w0, w15) F_{p+1} = (y_0, y_15)
    // gives z_p = g_p - e_p F_{p+1} with e_p column-independent.
    double eL = 0.0;  // eL_{p-1}
    for (int p = 0; p < P; ++p) {
      const double v0 = ends[4 * p], v15 = ends[4 * p + 1], w0 = ends[4 * p + 2],
                   w15 = ends[4 * p + 3];
      const double inv_d = 1.0 / (1.0 - v0 * eL);
      const double eF = w0 * inv_d;
      const double v15eL = v15 * eL;
      const double eLn = w15 + v15eL * eF;
      double *rf = red + p * kRed;
      rf[0] = v0;
      rf[1] = v15;
      rf[2] = inv_d;
      rf[3] = eF;
      rf[4] = eLn;
      rf[5] = v15eL;
      eL = eLn;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < P * kRed; e += blockDim.x) t.red[e] = red[e];
}

template <int C>
__global__ __launch_bounds__(1024) void spline_solve_kernel(const double *__restrict__ Sc,
                                                            double *__restrict__ M, int64_t N,
                                                            int64_t ncols, int64_t ntau, int P,
                                                            SplineTabs t) {
  extern __shared__ double zb[];  // [P][C][2]: (y_0, y_15) -> (gF, gL) -> (F, L); then [P][6]
  double *red = zb + 2 * C * P;
  for (int e = threadIdx.x; e < P * kRed; e += blockDim.x) red[e] = t.red[e];
  const int c = threadIdx.x % C, p = threadIdx.x / C;
  const int64_t col = (int64_t)blockIdx.x * C + c;
  const bool live = col < ncols && p < P;
  const int64_t n = N - 2;
  const int64_t s = col / ntau, nn = col - s * ntau;
  const int64_t base = s * N * ntau + nn;  // knot j of this column at base + j * ntau
  double y[SEG];
  if (live) {
    const int64_t i0 = (int64_t)p * SEG;
    // knots i0 .. i0 + SEG + 1 feed the right-hand sides of rows i0 .. i0 + SEG - 1
    double yk[SEG + 2], ih[SEG + 1];
#pragma unroll
    for (int r = 0; r < SEG + 2; ++r) {
      const int64_t j = i0 + r;
      yk[r] = j < N ? Sc[base + j * ntau] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < SEG + 1; ++r) {
      const int64_t j = i0 + r;
      ih[r] = j < N - 1 ? t.ih[j] : 0.0;
    }
    double g = 0.0;
#pragma unroll
    for (int r = 0; r < SEG; ++r) {
      const int64_t i = i0 + r;
      const double rhs =
          i < n ? (yk[r + 2] - yk[r + 1]) * ih[r + 1] - (yk[r + 1] - yk[r]) * ih[r] : 0.0;
      g = (rhs - t.sub[i] * g) * t.iden[i];
      y[r] = g;
    }
#pragma unroll
    for (int r = SEG - 2; r >= 0; --r) y[r] -= t.cp[i0 + r] * y[r + 1];
    zb[(p * C + c) * 2 + 0] = y[0];
    zb[(p * C + c) * 2 + 1] = y[SEG - 1];
  }
  __syncthreads();
  if (p == 0 && col < ncols) {
    double gL = 0.0;
    for (int pp = 0; pp < P; ++pp) {
      const double *rf = red + pp * kRed;
      double *z = zb + (pp * C + c) * 2;
      const double gF = (z[0] - rf[0] * gL) * rf[2];
      const double gLn = z[1] - rf[1] * gL + rf[5] * gF;
      z[0] = gF;
      z[1] = gLn;
      gL = gLn;
    }
    double F = 0.0;  // F_P = 0
    for (int pp = P - 1; pp >= 0; --pp) {
      const double *rf = red + pp * kRed;
      double *z = zb + (pp * C + c) * 2;
      const double Fp = z[0] - rf[3] * F;
      const double Lp = z[1] - rf[4] * F;
      z[0] = Fp;
      z[1] = Lp;
      F = Fp;
    }
  }
  __syncthreads();
  if (live) {
    const int64_t i0 = (int64_t)p * SEG;
    const double xl = p > 0 ? zb[((p - 1) * C + c) * 2 + 1] : 0.0;
    const double xr = p < P - 1 ? zb[((p + 1) * C + c) * 2 + 0] : 0.0;
#pragma unroll
    for (int r = 0; r < SEG; ++r) {
      const int64_t i = i0 + r;
      if (i < n) M[base + (i + 1) * ntau] = y[r] - t.v[i] * xl - t.w[i] * xr;
    }
    if (p == 0) {
      M[base] = 0.0;
      M[base + (N - 1) * ntau] = 0.0;
    }
  }
}

// One workgroup per group of ER = 4 consecutive k rows: each row's interval
// and weights are uniform, and rows that share an interval (most of them:
// the LOS grid is finer than the coarse one) reuse the coarse values already
// in registers instead of reading them again.  Row groups are dealt to the 8
// XCDs (workgroup L runs on XCD L % 8) in contiguous ranges, group =
// (L % 8) * per + L / 8, so neighbouring groups read their shared coarse rows
// from the same L2.
constexpr int ER = 4;

template <typename TO>
__global__ __launch_bounds__(256) void spline_eval_kernel(const double *__restrict__ q, int64_t N,
                                                          const double *__restrict__ Sc,
                                                          const double *__restrict__ M,
                                                          const double *__restrict__ k, int64_t nk,
                                                          int nsrc, int64_t ntau,
                                                          TO *__restrict__ out) {
  const int64_t groups = (nk + ER - 1) / ER;
  const int64_t L = blockIdx.x, per = (groups + 7) / 8;
  const int64_t g = (L % 8) * per + L / 8;
  if (g >= groups) return;
  const int64_t i0 = g * ER;
  const int nr = (int)min((int64_t)ER, nk - i0);
  int64_t jr[ER];
  double wA[ER], wB[ER], cA[ER], cB[ER];
#pragma unroll
  for (int r = 0; r < ER; ++r) {
    const double kk = k[i0 + (r < nr ? r : 0)];
    // largest j in [0, N-2] with q_j <= k (0 when k < q_0)
    int64_t lo = 0, hi = N - 2;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (q[mid] <= kk)
        lo = mid;
      else
        hi = mid - 1;
    }
    const double q0 = q[lo], q1 = q[lo + 1];
    const double h = q1 - q0;
    const double A = (q1 - kk) / h, B = (kk - q0) / h;
    const double h26 = h * h / 6.0;
    jr[r] = lo;
    wA[r] = A;
    wB[r] = B;
    cA[r] = (A * A * A - A) * h26;
    cB[r] = (B * B * B - B) * h26;
  }
  for (int s = 0; s < nsrc; ++s) {
    const double *ys = Sc + (int64_t)s * N * ntau;
    const double *ms = M + (int64_t)s * N * ntau;
    TO *o = out + ((int64_t)s * nk + i0) * ntau;
    for (int64_t n = threadIdx.x; n < ntau; n += blockDim.x) {
      int64_t jc = -1;
      double y0 = 0.0, y1 = 0.0, m0 = 0.0, m1 = 0.0;
#pragma unroll
      for (int r = 0; r < ER; ++r) {
        if (r < nr) {
          if (jr[r] != jc) {  // uniform
            jc = jr[r];
            y0 = ys[jc * ntau + n];
            y1 = ys[(jc + 1) * ntau + n];
            m0 = ms[jc * ntau + n];
            m1 = ms[(jc + 1) * ntau + n];
          }
          o[r * ntau + n] = (TO)(wA[r] * y0 + wB[r] * y1 + cA[r] * m0 + cB[r] * m1);
        }
      }
    }
  }
}

}  // namespace

int64_t spline_segments(int64_t N) { return N > 2 ? (N - 2 + SEG - 1) / SEG : 0; }

size_t spline_tab_doubles(int64_t N) {
  const int64_t P = spline_segments(N);
  return (size_t)(5 * P * SEG + (N - 1) + kRed * P);
}

SplineTabs spline_tabs_at(double *ws, int64_t N) {
  const int64_t P = spline_segments(N);
  const int64_t R = P * SEG;
  SplineTabs t;
  t.sub = ws;
  t.iden = ws + R;
  t.cp = ws + 2 * R;
  t.v = ws + 3 * R;
  t.w = ws + 4 * R;
  t.ih = ws + 5 * R;
  t.red = t.ih + (N - 1);
  return t;
}

template <int C>
static hipError_t solve_t(const double *Sc, double *M, int64_t N, int64_t ncols, int64_t ntau,
                          int P, const SplineTabs &t, hipStream_t s) {
  const int threads = ((C * P + 63) / 64) * 64;
  const int64_t groups = (ncols + C - 1) / C;
  const size_t lds = sizeof(double) * (2 * (size_t)C * P + kRed * (size_t)P);  // <= 64 KiB
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)spline_solve_kernel<C>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(spline_solve_kernel<C>, dim3((unsigned)groups), dim3(threads), lds, s, Sc, M,
                     N, ncols, ntau, P, t);
  return hipGetLastError();
}

hipError_t spline_solve_launch(const double *q, const double *Sc, double *M, int64_t N,
                               int64_t ncols, int64_t ntau, const SplineTabs &t, hipStream_t s) {
  const int64_t P = spline_segments(N);
  if (P == 0) return fill_zero_launch(M, ncols * N, s);  // N == 2: straight lines
  if (P > kSplineMaxSegments) return hipErrorInvalidValue;
  if (ncols > 0x7fffffff) return hipErrorInvalidValue;
  const size_t flds = sizeof(double) * (4 + kRed) * (size_t)P;  // <= 80 KiB
  hipError_t e = hipSuccess;
  if (flds > 64 * 1024) {  // a per-device function attribute: set on every such launch
    e = hipFuncSetAttribute((const void *)spline_factor_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)flds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(spline_factor_kernel, dim3(1), dim3(256), flds, s, q, N, (int)P, t);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int Pi = (int)P;
  // about 512 threads per workgroup, so that two share a CU and one's serial
  // reduced solve overlaps the other's loads and stores
  if (Pi * 16 <= 512) return solve_t<16>(Sc, M, N, ncols, ntau, Pi, t, s);
  if (Pi * 8 <= 512) return solve_t<8>(Sc, M, N, ncols, ntau, Pi, t, s);
  if (Pi * 4 <= 512) return solve_t<4>(Sc, M, N, ncols, ntau, Pi, t, s);
  if (Pi * 2 <= 512) return solve_t<2>(Sc, M, N, ncols, ntau, Pi, t, s);
  return solve_t<1>(Sc, M, N, ncols, ntau, Pi, t, s);
}

hipError_t spline_eval_launch(const double *q, int64_t N, const double *Sc, const double *M,
                              const double *k, int64_t nk, int nsrc, int64_t ntau, int out_prec,
                              void *out, hipStream_t s) {
  const int64_t grid = (((nk + ER - 1) / ER + 7) / 8) * 8;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (out_prec == LOS_FP32)
    hipLaunchKernelGGL(spline_eval_kernel<float>, dim3((unsigned)grid), dim3(256), 0, s, q, N, Sc,
                       M, k, nk, nsrc, ntau, (float *)out);
  else
    hipLaunchKernelGGL(spline_eval_kernel<double>, dim3((unsigned)grid), dim3(256), 0, s, q, N,
                       Sc, M, k, nk, nsrc, ntau, (double *)out);
  return hipGetLastError();
}

}  // namespace los
