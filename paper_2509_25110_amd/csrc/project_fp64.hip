// FP64 line-of-sight projection (gCAMB paper Sec. 2.1 Eq. 2-3; Sec. 3.2 and
// Algorithm 1 for the k / l / tau loop structure):
//
//   delta[k][l][s] = sum_n w_n S[s][k][n] j_l(k (tau0 - tau_n))
//
// Mapping on CDNA4 (gfx950):
//   * one workgroup per k (the paper's "gang" loop), heaviest k first;
//   * each lane owns `T` tau nodes ("slots"); slot j of wave w covers the 64
//     consecutive nodes 64*(w + W*j) .. +63, so slots are sorted by
//     decreasing x = k chi and the lanes of one slot see nearly equal x;
//   * l advances in blocks of B = 8.  Inside a block every lane runs the
//     three-term recurrence for each of its slots and accumulates
//     j_l * w_n S_n into a private acc[B][NSRC]; the sum over tau is then a
//     cross-lane reduction per block (permlane swaps, LDS, one workgroup
//     barrier), written to delta in a fixed order (bitwise reproducible);
//   * pass 1 (ascending blocks): upward recurrence, valid for l <= m = floor(x);
//     pass 2 (descending blocks): Miller recurrence from the top of the
//     block holding ltop(x) + 2, scaled to meet j_m, for m < l <= ltop(x);
//     its contributions are added to the stored pass-1 sums by the same lanes.
//   * All arithmetic is IEEE double.  The recurrence costs one FMA plus one
//     FMA for the coefficient per (l, tau); the contraction NSRC FMAs.
#include "bessel_dev.hpp"
#include "los_internal.hpp"

#include <climits>

namespace los {
namespace {

constexpr int kB = kProjectBlock;  // the Miller start is aligned up to a block top (<= 7 extra
                                   // steps): dynamic range stays far below 1e308 for x >= kXTiny

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

// Reduce v[NV] over the workgroup's lanes.  On return, lane L < NV of wave 0
// holds the total of index L (other lanes: unspecified).  `stage` is this
// wave's [NV][16] LDS area, `cross` the [W][NV] area of the current parity.
template <int NV>
__device__ inline double wg_reduce(double (&v)[NV], double *stage, double *cross, int W, int w,
                                   int lane) {
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
  for (int p = 0; p < NV / 4; ++p) stage[(p + r * (NV / 4)) * 16 + c] = q[p];
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  double tot = 0.0;
  if (lane < NV) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) tot += stage[lane * 16 + cc];
    cross[w * NV + lane] = tot;
  }
  __syncthreads();
  double all = 0.0;
  if (w == 0 && lane < NV) {
    for (int ww = 0; ww < W; ++ww) all += cross[ww * NV + lane];
  }
  return all;
}

// Load w_n * S[s][k][n] for this lane's node n.  The byte offset is passed
// through an empty asm so the compiler recomputes SGPR-base + 32-bit offset
// addressing in the loop instead of keeping one 64-bit address per slot and
// source live across it.
template <int NSRC>
__device__ inline void load_ws(double (&sv)[NSRC], const double *const (&srow)[NSRC],
                               const double *wv, int n) {
  unsigned off = (unsigned)n * 8u;
  asm volatile("" : "+v"(off));
  const double wn = *(const double *)((const char *)wv + off);
#pragma unroll
  for (int s = 0; s < NSRC; ++s) sv[s] = wn * *(const double *)((const char *)srow[s] + off);
}

template <int NSRC, int T>
__global__ void __launch_bounds__(512) project_fp64_kernel(ProjectArgs a) {
  constexpr int B = kB;
  constexpr int NV = B * NSRC;
  extern __shared__ double lds[];

  const int W = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ki = a.nk - 1 - (int64_t)blockIdx.x;  // large k (most work) first
  const int lmin = a.lmin, lmax = a.lmax;
  const int ntau = (int)a.ntau;
  const int npad = W * 64 * T;

  double *ixs = lds;                       // [npad]  1/x per node
  double *jms = lds + npad;                // [npad]  j_m, later the Miller seed
  double *stage = lds + 2 * npad + w * NV * 16;  // per wave [NV][16]
  double *cross0 = lds + 2 * npad + W * NV * 16; // [2][W][NV]
  int *bnd = (int *)(cross0 + 2 * W * NV);       // [3]

  const double kk = a.k[ki];
  const double *srow[NSRC];  // uniform row pointers of this k
#pragma unroll
  for (int s = 0; s < NSRC; ++s) srow[s] = a.S + ((int64_t)s * a.nk + ki) * a.ntau;
  const double *__restrict__ wv = a.w;

  // ---------------- per-node setup ----------------
  uint32_t mp[T];  // (m + 1) | (sblk + 1) << 16 ; m = last upward l, sblk = Miller start block
  double Ja[T], Jb[T];
  int my_mmax = -1, my_smax = -1, my_dlo = INT_MAX;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const int n = (w + W * j) * 64 + lane;
    int m = -1, sblk = -1;
    double ix = 0.0, jm = 0.0, pa = 0.0, pc = 0.0;
    if (n < ntau) {
      const double x = kk * (a.tau0 - a.tau[n]);
      if (x >= kXTiny) {
        ix = 1.0 / x;
        double sn, cs;
        sincos(x, &sn, &cs);
        pa = cs * ix;  // j_{-1}
        pc = sn * ix;  // j_0
        const double fx = floor(x);
        m = fx >= (double)lmax ? lmax : (int)fx;
        jm = pc;
        for (int l = 0; l < lmin; ++l) {  // advance to (j_{lmin-1}, j_{lmin})
          const double nx = rec_step((double)(2 * l + 1) * ix, pc, pa);
          pa = pc;
          pc = nx;
          if (l + 1 == m) jm = pc;
        }
        if (fx < (double)lmax) {
          const int ls = ltop_of(x) + 2;
          if (ls >= lmin) sblk = (ls - lmin) / B;
        }
        if (m < lmin && sblk < 0) m = -1;  // contributes nothing for l >= lmin
      }
    }
    ixs[(w + W * j) * 64 + lane] = ix;
    jms[(w + W * j) * 64 + lane] = jm;
    mp[j] = (uint32_t)(m + 1) | ((uint32_t)(sblk + 1) << 16);
    Ja[j] = pa;
    Jb[j] = pc;
    my_mmax = m > my_mmax ? m : my_mmax;
    if (sblk >= 0) {
      my_smax = sblk > my_smax ? sblk : my_smax;
      const int lo = m + 1 > lmin ? m + 1 : lmin;
      my_dlo = lo < my_dlo ? lo : my_dlo;
    }
  }
  if (threadIdx.x == 0) {
    bnd[0] = -1;
    bnd[1] = -1;
    bnd[2] = INT_MAX;
  }
  __syncthreads();
  atomicMax(&bnd[0], my_mmax);
  atomicMax(&bnd[1], my_smax);
  atomicMin(&bnd[2], my_dlo);
  __syncthreads();
  const int mmax_wg = bnd[0], smax_wg = bnd[1], dlo_wg = bnd[2];

  double *drow = a.delta + ki * (int64_t)a.nl * NSRC;
  int parity = 0;

  // ---------------- pass 1: upward recurrence, ascending blocks ----------------
  const int asc_last = mmax_wg >= lmin ? (mmax_wg - lmin) / B : -1;
  for (int bi = 0; bi <= asc_last; ++bi) {
    const int b = lmin + bi * B;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const int nb = (w + W * j) * 64;
      if (nb >= ntau) break;
      int n = nb + lane;
      uint32_t mpj = mp[j];
      asm volatile("" : "+v"(n), "+v"(mpj));  // keep only mp[j] live across blocks
      const int m = (int)(mpj & 0xFFFFu) - 1;
      if (!__any(m >= b)) continue;
      // fully upward through the block, and j_m (if needed) lies beyond it
      const bool full = __all(m >= b + B);
      const double ix = ixs[n];
      double sv[NSRC];
      if (n < ntau) {
        load_ws<NSRC>(sv, srow, wv, n);
      } else {
#pragma unroll
        for (int s = 0; s < NSRC; ++s) sv[s] = 0.0;
      }
      double pa = Ja[j], pc = Jb[j];
      double t = (double)(2 * b + 1) * ix;
      const double d2 = ix + ix;
      if (full) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
#pragma unroll
          for (int s = 0; s < NSRC; ++s) acc[i * NSRC + s] = fma(pc, sv[s], acc[i * NSRC + s]);
          const double nx = rec_step(t, pc, pa);
          t += d2;
          pa = pc;
          pc = nx;
        }
      } else {
        int rel = m - b;  // opaque, so the compiler does not precompute m - i per slot
        asm volatile("" : "+v"(rel));
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const double o = i <= rel ? pc : 0.0;
          if (i == rel) jms[n] = pc;
#pragma unroll
          for (int s = 0; s < NSRC; ++s) acc[i * NSRC + s] = fma(o, sv[s], acc[i * NSRC + s]);
          const double nx = rec_step(t, pc, pa);
          t += d2;
          pa = pc;
          pc = nx;
        }
      }
      Ja[j] = pa;
      Jb[j] = pc;
    }
    const double tot = wg_reduce<NV>(acc, stage, cross0 + parity * W * NV, W, w, lane);
    parity ^= 1;
    if (w == 0 && lane < NV) {
      const int l = b + lane / NSRC;
      if (l <= lmax) drow[(int64_t)(b - lmin) * NSRC + lane] = tot;
    }
  }
  // blocks with no upward contribution start from zero
  if (w == 0 && lane < NV) {
    for (int bi = asc_last + 1; bi < a.nblk; ++bi) {
      const int b = lmin + bi * B;
      if (b + lane / NSRC <= lmax) drow[(int64_t)(b - lmin) * NSRC + lane] = 0.0;
    }
  }

  // ---------------- pass 2: Miller recurrence, descending blocks ----------------
  if (smax_wg < 0) return;  // uniform
  // seed = j_m / (value reached at l = m by the recurrence started with (0, 1))
#pragma unroll
  for (int j = 0; j < T; ++j) {
    Ja[j] = 0.0;
    Jb[j] = 0.0;
    const int nb = (w + W * j) * 64;
    if (nb >= ntau) break;
    const int n = nb + lane;
    const int m = (int)(mp[j] & 0xFFFFu) - 1;
    const int sb = (int)(mp[j] >> 16) - 1;
    if (sb >= 0) {
      const double ix = ixs[n];
      const int ls = lmin + sb * B + B - 1;
      double jp = 0.0, jc = 1.0;
      for (int l = ls; l > m; --l) {
        const double nx = rec_step((double)(2 * l + 1) * ix, jc, jp);
        jp = jc;
        jc = nx;
      }
      jms[n] = jms[n] / jc;
    }
  }
  const int dlo_blk = (dlo_wg - lmin) / B;
  for (int bi = smax_wg; bi >= dlo_blk; --bi) {
    const int b = lmin + bi * B;
    const int top = b + B - 1;
    const bool store = bi < a.nblk;  // uniform
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const int nb = (w + W * j) * 64;
      if (nb >= ntau) break;
      int n = nb + lane;
      uint32_t mpj = mp[j];
      asm volatile("" : "+v"(n), "+v"(mpj));
      const int m = (int)(mpj & 0xFFFFu) - 1;
      const int sb = (int)(mpj >> 16) - 1;
      if (!__any(sb >= bi && top > m)) continue;
      const double ix = ixs[n];
      double p1 = Ja[j], p0 = Jb[j];  // j_{top+1}, j_top
      if (__any(sb == bi)) {
        const double sd = jms[n];
        if (sb == bi) {
          p1 = 0.0;
          p0 = sd;
        }
      }
      double t = (double)(2 * top + 1) * ix;
      const double d2 = ix + ix;
      if (!store) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const double nx = rec_step(t, p0, p1);
          t -= d2;
          p1 = p0;
          p0 = nx;
        }
      } else {
        double sv[NSRC];
        if (n < ntau) {
          load_ws<NSRC>(sv, srow, wv, n);
        } else {
#pragma unroll
          for (int s = 0; s < NSRC; ++s) sv[s] = 0.0;
        }
        if (__all(b > m)) {
#pragma unroll
          for (int i = 0; i < B; ++i) {
            const int q = (B - 1 - i) * NSRC;
#pragma unroll
            for (int s = 0; s < NSRC; ++s) acc[q + s] = fma(p0, sv[s], acc[q + s]);
            const double nx = rec_step(t, p0, p1);
          t -= d2;
            p1 = p0;
            p0 = nx;
          }
        } else {
          int rel = top - m;  // opaque, see pass 1
          asm volatile("" : "+v"(rel));
#pragma unroll
          for (int i = 0; i < B; ++i) {
            const int q = (B - 1 - i) * NSRC;
            const double o = i < rel ? p0 : 0.0;
#pragma unroll
            for (int s = 0; s < NSRC; ++s) acc[q + s] = fma(o, sv[s], acc[q + s]);
            const double nx = rec_step(t, p0, p1);
          t -= d2;
            p1 = p0;
            p0 = nx;
          }
        }
      }
      Ja[j] = p1;
      Jb[j] = p0;
    }
    if (store) {
      const double tot = wg_reduce<NV>(acc, stage, cross0 + parity * W * NV, W, w, lane);
      parity ^= 1;
      if (w == 0 && lane < NV) {
        const int l = b + lane / NSRC;
        if (l <= lmax) drow[(int64_t)(b - lmin) * NSRC + lane] += tot;
      }
    }
  }
}

template <int NSRC, int T>
hipError_t launch_t(const ProjectArgs &a, const ProjectShape &sh, hipStream_t s) {
  auto kern = project_fp64_kernel<NSRC, T>;
  if (sh.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)a.nk), dim3(64 * sh.waves), sh.lds, s, a);
  return hipGetLastError();
}

template <int NSRC>
hipError_t launch_n(const ProjectArgs &a, const ProjectShape &sh, hipStream_t s) {
  switch (sh.slots) {
    case 4: return launch_t<NSRC, 4>(a, sh, s);
    case 8: return launch_t<NSRC, 8>(a, sh, s);
    case 12: return launch_t<NSRC, 12>(a, sh, s);
    case 16: return launch_t<NSRC, 16>(a, sh, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

ProjectShape project_fp64_shape(int nsrc, int64_t ntau, int force_waves, int force_slots) {
  // Up to 12 slots per lane keeps the kernel within 256 VGPRs (two waves per
  // SIMD); more waves per workgroup cover larger tau grids.
  ProjectShape sh{};
  int W = force_waves > 0 ? force_waves : (int)((ntau + 64 * 12 - 1) / (64 * 12));
  if (W < 1) W = 1;
  if (W > 8) return sh;
  int T = force_slots > 0 ? force_slots : (int)((ntau + 64 * W - 1) / (64 * W));
  T = (T + 3) / 4 * 4;
  if (T < 4) T = 4;
  if (T > 16 || (int64_t)64 * W * T < ntau) return sh;  // waves == 0: unsupported
  sh.waves = W;
  sh.slots = T;
  const int NV = kB * nsrc;
  const int npad = W * 64 * T;
  sh.lds = sizeof(double) * ((size_t)2 * npad + (size_t)W * NV * 16 + 2 * (size_t)W * NV) +
           4 * sizeof(int);
  return sh;
}

hipError_t project_fp64_launch(const ProjectArgs &a, int nsrc, const ProjectShape &sh,
                               hipStream_t s) {
  switch (nsrc) {
    case 1: return launch_n<1>(a, sh, s);
    case 2: return launch_n<2>(a, sh, s);
    case 3: return launch_n<3>(a, sh, s);
    case 4: return launch_n<4>(a, sh, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace los
