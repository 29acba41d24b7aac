// C_l at every multipole from its values at sampled multipoles (gCAMB paper
// Sec. 3.1: the output l-sampling density sets how many multipoles are
// computed explicitly; the others are interpolated).  For each spectrum the
// natural cubic spline in l of D_l = l (l + 1) C_l through the sampled points
// (L_j, D_j) is evaluated at every l of [lmin, lmax] and divided by l (l + 1):
//
//   on [L_j, L_{j+1}], h = L_{j+1} - L_j, A = (L_{j+1} - l)/h, B = (l - L_j)/h:
//   D(l) = A D_j + B D_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) h^2 / 6,
//
// M the second derivatives (continuous D'' at the knots, M = 0 at both
// ends).  The work is tiny (a few hundred knots per spectrum): one workgroup
// per spectrum, the tridiagonal system solved by one thread in LDS (Thomas;
// the matrix is strictly diagonally dominant), then every thread evaluates a
// share of the multipoles.
#include "los_internal.hpp"

namespace los {
namespace {

__global__ __launch_bounds__(256) void cl_interp_kernel(const double *__restrict__ knots, int nls,
                                                        const double *__restrict__ cls, int lmin,
                                                        int lmax, double *__restrict__ cl) {
  extern __shared__ double sh[];  // [nls] L, [nls] D, [nls] M, [nls] c'
  double *L = sh, *D = sh + nls, *M = sh + 2 * nls, *cp = sh + 3 * nls;
  const int p = blockIdx.x;
  const int nl = lmax - lmin + 1;
  for (int j = threadIdx.x; j < nls; j += blockDim.x) {
    const double lj = knots[j];
    L[j] = lj;
    D[j] = lj * (lj + 1.0) * cls[(int64_t)p * nls + j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    M[0] = 0.0;
    M[nls - 1] = 0.0;
    cp[0] = 0.0;
    // forward elimination over the interior knots 1 .. nls-2 (M holds d')
    for (int j = 1; j + 1 < nls; ++j) {
      const double h0 = L[j] - L[j - 1], h1 = L[j + 1] - L[j];
      const double a = j > 1 ? h0 / 6.0 : 0.0;         // couples to M_{j-1} (M_0 = 0)
      const double c = j + 2 < nls ? h1 / 6.0 : 0.0;   // couples to M_{j+1} (M_{nls-1} = 0)
      const double rhs = (D[j + 1] - D[j]) / h1 - (D[j] - D[j - 1]) / h0;
      const double den = (h0 + h1) / 3.0 - a * cp[j - 1];
      cp[j] = c / den;
      M[j] = (rhs - a * M[j - 1]) / den;
    }
    for (int j = nls - 3; j >= 1; --j) M[j] -= cp[j] * M[j + 1];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nl; i += blockDim.x) {
    const double l = (double)(lmin + i);
    // largest j in [0, nls-2] with L_j <= l
    int lo = 0, hi = nls - 2;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L[mid] <= l)
        lo = mid;
      else
        hi = mid - 1;
    }
    const double h = L[lo + 1] - L[lo];
    const double A = (L[lo + 1] - l) / h, B = (l - L[lo]) / h;
    const double d = A * D[lo] + B * D[lo + 1] +
                     ((A * A * A - A) * M[lo] + (B * B * B - B) * M[lo + 1]) * (h * h / 6.0);
    cl[(int64_t)p * nl + i] = d / (l * (l + 1.0));
  }
}

}  // namespace

hipError_t cl_interp_launch(const double *knots, int nls, const double *cls, int npairs, int lmin,
                            int lmax, double *cl, hipStream_t s) {
  hipLaunchKernelGGL(cl_interp_kernel, dim3((unsigned)npairs), dim3(256),
                     sizeof(double) * 4 * (size_t)nls, s, knots, nls, cls, lmin, lmax, cl);
  return hipGetLastError();
}

}  // namespace los
