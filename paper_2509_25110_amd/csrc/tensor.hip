// Tensor-mode line-of-sight transfer functions (gCAMB paper, Sec. 2.1: tensor
// perturbations and B modes lead to equations of the Eq. 2-3 kind; the radial
// kernels are the published tensor kernels of the line-of-sight method the
// paper builds on):
//   K^T_l = sqrt((l+2)!/(l-2)!) j_l / x^2
//   K^E_l = -j_l + j_l'' + 2 j_l / x^2 + 4 j_l' / x
//   K^B_l = 2 j_l' + 4 j_l / x.
// With j_l' = j_{l-1} - (l+1) j_l / x and j_l'' from Bessel's equation,
// j_l'' = -(2/x) j_l' - (1 - l(l+1)/x^2) j_l, they become
//   K^E_l = -2 j_l + 2 j_{l-1} / x + l (l-1) j_l / x^2
//   K^B_l =  2 j_{l-1} - 2 (l-1) j_l / x,
// so the tensor projection is the FP64 sweep over four columns on the rows
// lmin-1 .. lmax,
//   c0: P0_m = sum_n w S_P j_m        c1: P1_m = sum_n w S_P j_m / x
//   c2: P2_m = sum_n w S_P j_m / x^2  c3: T2_m = sum_n w S_T j_m / x^2,
// followed by this combination of neighbouring rows:
//   Delta^T_l = sqrt((l-1) l (l+1) (l+2)) T2_l
//   Delta^E_l = -2 P0_l + 2 P1_{l-1} + l (l-1) P2_l
//   Delta^B_l =  2 P0_{l-1} - 2 (l-1) P1_l.
#include "los_internal.hpp"

namespace los {
namespace {

__global__ __launch_bounds__(256) void tensor_combine_kernel(const double *__restrict__ d4,
                                                             double *__restrict__ out, int lmin,
                                                             int nl, int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t ki = t / nl;
    const int r = (int)(t - ki * nl);  // l - lmin
    const double l = (double)(lmin + r);
    // rows of the sweep output start at lmin - 1: row l is r + 1, row l - 1 is r
    const double *hi = d4 + (ki * (nl + 1) + r + 1) * 4;
    const double *lo = hi - 4;
    const double p0 = hi[0], p1 = hi[1], p2 = hi[2], t2 = hi[3];
    const double q0 = lo[0], q1 = lo[1];
    double *o = out + t * 3;
    o[0] = sqrt((l - 1.0) * l * (l + 1.0) * (l + 2.0)) * t2;
    o[1] = -2.0 * p0 + 2.0 * q1 + l * (l - 1.0) * p2;
    o[2] = 2.0 * q0 - 2.0 * (l - 1.0) * p1;
  }
}

}  // namespace

hipError_t tensor_combine_launch(const double *d4, double *out, int lmin, int nl, int64_t nk,
                                 hipStream_t s) {
  const int64_t total = nk * (int64_t)nl;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(tensor_combine_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d4, out, lmin,
                     nl, total);
  return hipGetLastError();
}

}  // namespace los
