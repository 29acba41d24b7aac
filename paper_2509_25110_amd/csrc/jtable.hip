// Weighted Bessel tables for the MFMA projection (gCAMB paper, Sec. 2.1
// Eq. 2-3, written as a matrix product per k):
//
//   J_k[l][n] = w_n * j_l(k * (tau0 - tau_n)),   so   Delta_k = J_k . S_k
//
// One lane per tau node, one workgroup column per k.  Each lane first finds
// a normalised pair (J_R, J_{R+1}) at its top row R, the top row of the
// 16-row block holding min(ltop(x), lmax):
//   * x >= lmax + 1: upward recurrence from j_0 = sin x / x, j_{-1} = cos x / x
//     (stable on the oscillatory side) up to l = R + 1;
//   * otherwise: upward to m = floor(x) for j_m, and Miller's downward
//     recurrence from max(ltop(x), R) with seeds (0, 1) down to m; the Miller
//     values are scaled by j_m / J^_m.
// It then runs the recurrence DOWNWARD from R to lmin, writing every row
// (a whole 16-row block at a time: zeros in blocks above R).
// Downward is the stable direction above the turning point and neutrally
// stable below it (both solutions oscillate with equal amplitude there), so
// a single descending sweep covers the whole band.
//
// Output, FP32 (w folded in before rounding):
//   J[(kc * nlp + (l - lmin)) * ntp + n]   rows padded to nlp = 16 * nlb,
//                                           columns to ntp = 32 * ntb,
// and top[kc * ntb + tb] = highest 16-row block holding a non-zero row in the
// 32-node block tb (-1: none).  Blocks above `top` are not written; the
// GEMM never reads them.
#include "bessel_dev.hpp"
#include "los_internal.hpp"

namespace los {
namespace {

__device__ inline int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline int half_max_i(int v) {
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ __launch_bounds__(256) void jtable_kernel(JTableArgs a) {
  const int ki = blockIdx.y;
  const int64_t i = a.row_index ? a.row_index[a.k0 + ki] : a.k0 + ki;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  if ((int64_t)blockIdx.x * 256 + (threadIdx.x & ~63) >= a.ntp) return;  // whole wave is padding

  int R = -1;
  double ix = 0.0, cur = 0.0, nxt = 0.0;
  if (n < a.ntau) {
    const double chi = a.tau0 - a.tau[n];
    const double x = a.k[i] * chi;
    const double wt = a.w[n];
    if (x >= kXTiny && wt != 0.0) {
      ix = 1.0 / x;
      // R is the top row of the 16-row block holding min(ltop_mfma(x), lmax): a
      // lane is then live either throughout a block or not at all.  Rows past
      // lmax (at most 15, inside the padded table) are never stored by the
      // product.
      R = node_top_pair(x, ix, wt, a.lmin, a.lmax, ltop_mfma_of(x), cur, nxt);
    }
  }

  const int tb_lane = R >= 0 ? (R - a.lmin) >> 4 : -1;
  const int tb_half = half_max_i(tb_lane);
  const int tb_wave = wave_max_i(tb_lane);
  if ((lane & 31) == 0) {
    const int64_t blk = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 5;
    if (blk < a.ntb) a.top[(int64_t)ki * a.ntb + blk] = tb_half;
  }

  if (n >= a.ntp) return;  // no column of its own (after the shuffles above)
  float *col = a.J + (int64_t)ki * a.nlp * a.ntp + n;
  const double d2 = ix + ix;
  for (int b = tb_wave; b >= 0; --b) {
    const int lbase = a.lmin + 16 * b;
    float *dst = col + (int64_t)(16 * b) * a.ntp;
    if (R >= lbase + 15) {  // live through the block
      double t = 0.0;
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        if (r == 15 || r == 7) t = (double)(2 * (lbase + r) + 1) * ix;  // exact every 8 rows
        dst[(int64_t)r * a.ntp] = (float)cur;
        const double pv = rec_step(t, cur, nxt);
        nxt = cur;
        cur = pv;
        t -= d2;
      }
    } else {
#pragma unroll
      for (int r = 15; r >= 0; --r) dst[(int64_t)r * a.ntp] = 0.f;
    }
  }
}

}  // namespace

hipError_t jtable_launch(const JTableArgs &a, int kcount, hipStream_t s) {
  dim3 grid((unsigned)((a.ntp + 255) / 256), (unsigned)kcount);
  hipLaunchKernelGGL(jtable_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace los
