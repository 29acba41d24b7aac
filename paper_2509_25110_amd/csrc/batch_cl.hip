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

// One workgroup per (256 multipoles, model).  The model's k rows of the chunk
// go in runs of up to 256: each run's Delta column offsets and w P factors are
// staged in LDS by one coalesced load, so the Delta loads of the run depend on
// no other global load; the Delta values of four k are loaded before the first
// of their terms is added.  Terms are accumulated per ordered source pair
// (s, t) that some output pair uses, as (w P Delta_s) Delta_t in increasing j,
// and each output pair reads its (s, t) sum at the end.
template <int NSRC>
__global__ __launch_bounds__(256) void batch_cl_kernel(BatchClArgs a) {
  __shared__ int64_t s_col[256];
  __shared__ double s_wp[256];
  const int m = a.order[blockIdx.y];  // longest workgroups dispatched first
  const int lmax = a.lmax[m];
  if ((int)blockIdx.x * 256 + a.lmin > lmax) return;  // no multipole of this block
  const int lr = blockIdx.x * 256 + threadIdx.x;  // l - lmin
  const bool live = lr + a.lmin <= lmax;
  const int64_t *jr = a.jr + ((int64_t)a.chunk * a.nmodels + m) * 2;
  const int64_t jlo = jr[0], jhi = jr[1];
  if (jlo >= jhi) return;
  // ordered source pairs in use (bit s * NSRC + t)
  uint32_t used = 0;
  for (int q = 0; q < a.npairs; ++q) used |= 1u << (a.pa[q] * NSRC + a.pb[q]);
  double acc[NSRC][NSRC];
#pragma unroll
  for (int s = 0; s < NSRC; ++s)
#pragma unroll
    for (int t = 0; t < NSRC; ++t) acc[s][t] = 0.0;
  auto add_term = [&](const double wp, const double (&v)[NSRC]) {
#pragma unroll
    for (int s = 0; s < NSRC; ++s) {
      const double ws = wp * v[s];
#pragma unroll
      for (int t = 0; t < NSRC; ++t)
        if ((used >> (s * NSRC + t)) & 1u) acc[s][t] += ws * v[t];
    }
  };
  const int64_t p0 = a.koff[m] + jlo;
  const float *D = a.D + lr;
  for (int64_t j0 = 0; j0 < jhi - jlo; j0 += 256) {
    const int nb = (int)(jhi - jlo - j0 < 256 ? jhi - jlo - j0 : 256);
    __syncthreads();  // the previous run's entries are consumed
    if ((int)threadIdx.x < nb) {
      const int64_t p = p0 + j0 + threadIdx.x;
      s_col[threadIdx.x] = (a.pos_col[p] - a.col_base) * (int64_t)a.nl;
      s_wp[threadIdx.x] = a.w_lnk[p] * a.Pk[p];
    }
    __syncthreads();
    if (!live) continue;
    int i = 0;
    for (; i + 4 <= nb; i += 4) {
      double v[4][NSRC];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float *d = D + s_col[i + u];
#pragma unroll
        for (int s = 0; s < NSRC; ++s) v[u][s] = (double)d[(int64_t)s * a.nl];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) add_term(s_wp[i + u], v[u]);
    }
    for (; i < nb; ++i) {
      const float *d = D + s_col[i];
      double v[NSRC];
#pragma unroll
      for (int s = 0; s < NSRC; ++s) v[s] = (double)d[(int64_t)s * a.nl];
      add_term(s_wp[i], v);
    }
  }
  if (!live) return;
  const double four_pi = 12.566370614359172954;
  double *out = a.cl + (int64_t)m * a.npairs * a.nl + lr;
  for (int q = 0; q < a.npairs; ++q) {
    double c = 0.0;
#pragma unroll
    for (int s = 0; s < NSRC; ++s)
#pragma unroll
      for (int t = 0; t < NSRC; ++t)
        if (a.pa[q] == s && a.pb[q] == t) c = acc[s][t];
    out[(int64_t)q * a.nl] += four_pi * c;
  }
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
