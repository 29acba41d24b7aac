// Spherical Bessel table out[(l - lmin) * nx + i] = j_l(x[i]): the radial
// kernel of the LOS integrals (gCAMB paper Sec. 2.1, Eq. 2-3, flat space).
//
// One lane per x.  Upward recurrence from j_{-1} = cos x / x, j_0 = sin x / x
// for l <= m = floor(x); Miller recurrence started at ltop(x) + 2 and scaled to
// meet j_m for m < l <= ltop(x); zero above ltop(x).  Stores of one l row are
// coalesced across lanes.
#include "bessel_dev.hpp"
#include "los_internal.hpp"

namespace los {
namespace {

__global__ void __launch_bounds__(256) bessel_table_kernel(const double *__restrict__ xs, int64_t nx,
                                                           int lmin, int lmax,
                                                           double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  const double x = xs[i];
  if (!(x >= kXTiny)) {
    // x < 1e-9 (or NaN / negative: NaN out): power series j_l(x) = x^l/(2l+1)!! (1 - ...)
    const bool bad = !(x >= 0.0);
    for (int l = lmin; l <= lmax; ++l) {
      double v = 0.0;
      if (l == 0) v = 1.0 - x * x / 6.0;
      if (l == 1) v = x / 3.0;
      if (l == 2) v = x * x / 15.0;
      out[(int64_t)(l - lmin) * nx + i] = bad ? __builtin_nan("") : v;
    }
    return;
  }
  const double ix = 1.0 / x;
  double sn, cs;
  sincos(x, &sn, &cs);
  const double fx = floor(x);
  const int m = fx >= (double)lmax ? lmax : (int)fx;
  // upward: (p, c) = (j_{l-1}, j_l)
  double p = cs * ix, c = sn * ix, jm = c;
  for (int l = 0; l <= m; ++l) {
    if (l >= lmin) out[(int64_t)(l - lmin) * nx + i] = c;
    if (l == m) jm = c;
    const double nx_ = rec_step((double)(2 * l + 1) * ix, c, p);
    p = c;
    c = nx_;
  }
  if (m >= lmax) return;
  const int lt = ltop_of(x);
  const int ls = lt + 2;
  // zeros above the cut
  for (int l = (lt + 1 > m + 1 ? lt + 1 : m + 1); l <= lmax; ++l)
    if (l >= lmin) out[(int64_t)(l - lmin) * nx + i] = 0.0;
  // Miller: value reached at m from (j~_{ls+1}, j~_ls) = (0, 1)
  double jp = 0.0, jc = 1.0;
  for (int l = ls; l > m; --l) {
    const double nx_ = rec_step((double)(2 * l + 1) * ix, jc, jp);
    jp = jc;
    jc = nx_;
  }
  const double seed = jm / jc;
  jp = 0.0;
  jc = seed;
  for (int l = ls; l > m; --l) {
    if (l <= lt && l <= lmax && l >= lmin) out[(int64_t)(l - lmin) * nx + i] = jc;
    const double nx_ = rec_step((double)(2 * l + 1) * ix, jc, jp);
    jp = jc;
    jc = nx_;
  }
}

}  // namespace

hipError_t bessel_table_launch(const double *x, int64_t nx, int lmin, int lmax, double *out,
                               hipStream_t s) {
  if (nx == 0) return hipSuccess;
  const int tpb = 256;
  const int64_t nb = (nx + tpb - 1) / tpb;
  hipLaunchKernelGGL(bessel_table_kernel, dim3((unsigned)nb), dim3(tpb), 0, s, x, nx, lmin, lmax,
                     out);
  return hipGetLastError();
}

}  // namespace los
