// Device helpers shared by the FP64 projection kernels (project_fp64.hip,
// project_fp64_desc.hip): the per-block sum over tau of a workgroup's lanes
// (fixed order, bitwise reproducible), source loads and wave-uniform slot tests.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace los {
namespace fp64 {

// Sum of `a` over lanes {l, l^32} kept by the low half, of `b` by the high half.
__device__ inline double swap_add32(double a, double b) {
#if defined(LOS_REDUCE_SHFL)
  const bool hi = (threadIdx.x & 32) != 0;
  double send = hi ? a : b, keep = hi ? b : a;
  return keep + __shfl_xor(send, 32);
#else
  auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  auto up = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(up[0], lo[0]) + __hiloint2double(up[1], lo[1]);
#endif
}

// Sum of `a` over rows {r, r^1} (rows of 16 lanes) kept by even rows, of `b` by odd rows.
__device__ inline double swap_add16(double a, double b) {
#if defined(LOS_REDUCE_SHFL)
  const bool odd = (threadIdx.x & 16) != 0;
  double send = odd ? a : b, keep = odd ? b : a;
  return keep + __shfl_xor(send, 16);
#else
  auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  auto up = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(up[0], lo[0]) + __hiloint2double(up[1], lo[1]);
#endif
}

// Doubles of one wave's staging area for wg_reduce<NV>: 16 columns of NV + 1
// (the pad makes both the column writes and the lane-consecutive reads free
// of LDS bank conflicts).
constexpr int stage_doubles(int NV) { return 16 * (NV + 1); }

// Reduce v[NV] over one wave's lanes.  On return, lane L < NV holds the
// wave's total of index L (other lanes: unspecified).  `stage` is this wave's
// [16][NV + 1] LDS area.
template <int NV>
__device__ inline double wave_reduce(double (&v)[NV], double *stage, int lane) {
  static_assert(NV % 4 == 0, "NV must be a multiple of 4");
  double u[NV / 2];
#pragma unroll
  for (int p = 0; p < NV / 2; ++p) u[p] = swap_add32(v[p], v[p + NV / 2]);
  double q[NV / 4];
#pragma unroll
  for (int p = 0; p < NV / 4; ++p) q[p] = swap_add16(u[p], u[p + NV / 4]);
  // lane (r, c) now holds, for index p + r*NV/4, the sum over the 4 lanes of column c
  const int r = lane >> 4, c = lane & 15;
#pragma unroll
  for (int p = 0; p < NV / 4; ++p) stage[c * (NV + 1) + p + r * (NV / 4)] = q[p];
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  double tot = 0.0;
  if (lane < NV) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) tot += stage[cc * (NV + 1) + lane];
  }
  return tot;
}

// Reduce v[NV] over the workgroup's lanes.  On return, lane L < NV of wave 0
// holds the total of index L (other lanes: unspecified).  `stage` is this
// wave's [16][NV + 1] LDS area, `cross` the [W][NV] area of the current parity.
template <int NV>
__device__ inline double wg_reduce(double (&v)[NV], double *stage, double *cross, int W, int w,
                                   int lane, bool wave_active = true) {
  if (!wave_active) {  // uniform: this wave contributed nothing to the block
    if (lane < NV) cross[w * NV + lane] = 0.0;
  } else {
    const double tot = wave_reduce<NV>(v, stage, lane);
    if (lane < NV) cross[w * NV + lane] = tot;
  }
  __syncthreads();
  double all = 0.0;
  if (w == 0 && lane < NV) {
    for (int ww = 0; ww < W; ++ww) all += cross[ww * NV + lane];
  }
  return all;
}

// Load S[s][k][n] for this lane's node n (zeros for padding lanes).  The byte
// offset goes through an empty asm so the compiler recomputes SGPR-base +
// 32-bit offset addressing in the loop instead of keeping one 64-bit address
// per slot and source live across it.
template <int NSRC>
__device__ inline void load_s(double (&sv)[NSRC], const double *const (&srow)[NSRC], int n,
                              int ntau) {
  unsigned off = (unsigned)n * 8u;
  asm volatile("" : "+v"(off));
  if (n < ntau) {
#pragma unroll
    for (int s = 0; s < NSRC; ++s) sv[s] = *(const double *)((const char *)srow[s] + off);
  } else {
#pragma unroll
    for (int s = 0; s < NSRC; ++s) sv[s] = 0.0;
  }
}

// Wave-uniform max / min of an int (result in a scalar register).
__device__ inline int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ inline int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return __builtin_amdgcn_readfirstlane(v);
}

// Slot j's block thresholds live in lane j of a VGPR, so the set of slots to
// run in a block is one compare + ballot, and each slot test is a scalar bit test.
__device__ inline uint64_t slot_mask(bool pred) { return __ballot(pred); }
__device__ inline bool has(uint64_t mask, int j) { return (mask >> j) & 1u; }

}  // namespace fp64
}  // namespace los
