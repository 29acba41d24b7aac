// Angular power spectra (gCAMB paper Sec. 2.1, Eq. 1, with dk/k = d ln k):
//
//   cl[p][l] = 4 pi sum_k w_k P_k delta[k][l][a_p] delta[k][l][b_p]
//
// HBM-bound reduction over k.  Pass 1: a grid of (l tile of 64, k segment)
// single-wave workgroups; lane = l, loop over the segment's k in order,
// FP64 accumulators per pair; coalesced reads of delta[k][l0..l0+63][*].
// Pass 2: one wave per (p, l) sums the segment partials (each lane a stride
// of them, then a fixed butterfly) and applies 4 pi.  Fixed summation order
// -> bitwise reproducible.
#include "los_internal.hpp"

namespace los {
namespace {

constexpr int kLTile = 64;
constexpr int kMaxPairs = 16;

template <typename DT, int NSRC>
__global__ void __launch_bounds__(64) cl_partial_kernel(ClArgs a) {
  const int l = blockIdx.x * kLTile + threadIdx.x;
  const int seg = blockIdx.y;
  const int64_t per = (a.nk + a.nseg - 1) / a.nseg;
  const int64_t k0 = seg * per;
  const int64_t k1 = k0 + per < a.nk ? k0 + per : a.nk;
  if (l >= a.nl) return;
  double acc[kMaxPairs];
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) acc[p] = 0.0;
  const DT *d = (const DT *)a.delta;
  for (int64_t k = k0; k < k1; ++k) {
    const DT *row = d + (k * a.nl + l) * NSRC;
    double v[NSRC];
#pragma unroll
    for (int s = 0; s < NSRC; ++s) v[s] = (double)row[s];
    const double wp = a.w[k] * a.P[k];
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
      if (p < a.npairs) {
        double va = 0.0, vb = 0.0;
#pragma unroll
        for (int s = 0; s < NSRC; ++s) {
          va = s == a.pa[p] ? v[s] : va;
          vb = s == a.pb[p] ? v[s] : vb;
        }
        acc[p] = fma(wp * va, vb, acc[p]);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p)
    if (p < a.npairs) a.partial[((int64_t)seg * a.npairs + p) * a.nl + l] = acc[p];
}

// One wave per output: lane i sums the partials of segments i, i + 64, ...
// in increasing order, then the 64 lane sums are combined by a fixed
// butterfly (xor 32, 16, ..., 1), so the result is the same on every run.
__global__ void __launch_bounds__(256) cl_final_kernel(ClArgs a) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= (int64_t)a.npairs * a.nl) return;  // whole wave: t is uniform
  double s = 0.0;
  for (int seg = lane; seg < a.nseg; seg += 64)
    s += a.partial[(int64_t)seg * a.npairs * a.nl + t];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) a.cl[t] = 4.0 * 3.14159265358979323846 * s;
}

template <typename DT>
hipError_t launch_dt(const ClArgs &a, hipStream_t st) {
  dim3 g((unsigned)((a.nl + kLTile - 1) / kLTile), (unsigned)a.nseg);
  switch (a.nsrc) {
    case 1: hipLaunchKernelGGL((cl_partial_kernel<DT, 1>), g, dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((cl_partial_kernel<DT, 2>), g, dim3(64), 0, st, a); break;
    case 3: hipLaunchKernelGGL((cl_partial_kernel<DT, 3>), g, dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL((cl_partial_kernel<DT, 4>), g, dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)a.npairs * a.nl;  // one wave each, four waves per workgroup
  if ((n + 3) / 4 > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cl_final_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace

int cl_segments(int64_t nk, int nl) {
  // enough single-wave workgroups to cover 256 CUs several times over
  const int64_t tiles = (nl + kLTile - 1) / kLTile;
  int64_t seg = (4096 + tiles - 1) / tiles;
  if (seg > nk) seg = nk;
  if (seg < 1) seg = 1;
  if (seg > 1024) seg = 1024;
  return (int)seg;
}

hipError_t cl_launch(const ClArgs &a, hipStream_t s) {
  return a.delta_f32 ? launch_dt<float>(a, s) : launch_dt<double>(a, s);
}

}  // namespace los
