// Per-model angular power spectra of a batch (gCAMB paper, Sec. 2.1 Eq. 1 for
// each model m on its own k grid, a subset of the shared master grid):
//
//   cl[m][p][l - lmin] = 4 pi sum_j w_lnk[m][j] P[m][j] Delta^{a_p}_l Delta^{b_p}_l
//
// evaluated one chunk of master rows at a time: each call adds the chunk's
// terms (FP64 accumulation, in increasing j) to cl.  Chunks are issued in
// order on one stream, so the result is bitwise reproducible.
#include "los_internal.hpp"

namespace los {
namespace {

__global__ __launch_bounds__(256) void fill_zero_kernel(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

template <int NSRC>
__global__ __launch_bounds__(256) void batch_cl_kernel(BatchClArgs a) {
  const int m = a.order[blockIdx.y];  // longest workgroups dispatched first
  const int lr = blockIdx.x * 256 + threadIdx.x;  // l - lmin
  if (lr + a.lmin > a.lmax[m]) return;
  const int64_t *jr = a.jr + ((int64_t)a.chunk * a.nmodels + m) * 2;
  const int64_t jlo = jr[0], jhi = jr[1];
  if (jlo >= jhi) return;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  const int64_t p0 = a.koff[m];
  auto add_term = [&](const double wp, const double (&v)[NSRC]) {
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (q < a.npairs) acc[q] += wp * v[a.pa[q]] * v[a.pb[q]];
  };
  int64_t j = jlo;
  // four k at a time: every load of the four issued before the first term is
  // added; the terms are added in increasing j as in the plain loop
  for (; j + 4 <= jhi; j += 4) {
    double v[4][NSRC], wp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t p = p0 + j + u;
      const float *d = a.D + (a.pos_col[p] - a.col_base) * (int64_t)a.nl + lr;
#pragma unroll
      for (int s = 0; s < NSRC; ++s) v[u][s] = (double)d[(int64_t)s * a.nl];
      wp[u] = a.w_lnk[p] * a.Pk[p];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) add_term(wp[u], v[u]);
  }
  for (; j < jhi; ++j) {
    const int64_t p = p0 + j;
    const float *d = a.D + (a.pos_col[p] - a.col_base) * (int64_t)a.nl + lr;
    double v[NSRC];
#pragma unroll
    for (int s = 0; s < NSRC; ++s) v[s] = (double)d[(int64_t)s * a.nl];
    add_term(a.w_lnk[p] * a.Pk[p], v);
  }
  const double four_pi = 12.566370614359172954;
  double *out = a.cl + (int64_t)m * a.npairs * a.nl + lr;
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q < a.npairs) out[(int64_t)q * a.nl] += four_pi * acc[q];
}

}  // namespace

hipError_t fill_zero_launch(double *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t batch_cl_launch(const BatchClArgs &a, hipStream_t s) {
  dim3 grid((unsigned)((a.nl + 255) / 256), (unsigned)a.nmodels);
  switch (a.nsrc) {
    case 1: hipLaunchKernelGGL(batch_cl_kernel<1>, grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(batch_cl_kernel<2>, grid, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(batch_cl_kernel<3>, grid, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(batch_cl_kernel<4>, grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace los
