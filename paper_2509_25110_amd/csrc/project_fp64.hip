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
#include "fp64_common.hpp"
#include "los_internal.hpp"

#include <climits>

#ifndef LOS_IX_REG
#define LOS_IX_REG 0
#endif

namespace los {
namespace {

using fp64::has;
using fp64::load_s;
using fp64::slot_mask;
using fp64::wave_max;
using fp64::wave_min;
using fp64::wg_reduce;

constexpr int kB = kProjectBlock;  // the Miller start is aligned up to a block top (<= 7 extra
                                   // steps): dynamic range stays far below 1e308 for x >= kXTiny

// One slot of pass 1 over a block of B multipoles: outputs pc (= w j_l) for
// l = b..b+B-1 into acc and advances (pa, pc) = (w j_{l-1}, w j_l).  With MASK,
// only l <= m contributes (rel = m - b) and w j_m, the value the lane's Miller
// part is matched to (j_m is near its last maximum in l, never near a zero),
// is stored into *jm_out.
template <int NSRC, int B, bool MASK>
__device__ __forceinline__ void asc_slot(double (&acc)[B * NSRC], double &pa, double &pc,
                                         double ix, const double (&sv)[NSRC], int b, int rel,
                                         double *jm_out) {
  double t = (double)(2 * b + 1) * ix;
  const double d2 = ix + ix;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    double o = pc;
    if (MASK) {
      o = i <= rel ? pc : 0.0;
      if (i == rel) *jm_out = pc;
    }
#pragma unroll
    for (int s = 0; s < NSRC; ++s) acc[i * NSRC + s] = fma(o, sv[s], acc[i * NSRC + s]);
    const double nx = rec_step(t, pc, pa);
    t += d2;
    pa = pc;
    pc = nx;
  }
}

// One slot of pass 2 over the block [top-B+1, top], descending: outputs p0
// (= j_l) and advances (p1, p0) = (j_{l+1}, j_l).  With MASK only l > m
// contributes (rel = top - m); with ACC false the block is only advanced.
template <int NSRC, int B, bool ACC, bool MASK>
__device__ __forceinline__ void desc_slot(double (&acc)[B * NSRC], double &p1, double &p0,
                                          double ix, const double (&sv)[NSRC], int top, int rel) {
  double t = (double)(2 * top + 1) * ix;
  const double d2 = ix + ix;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    if (ACC) {
      const int q = (B - 1 - i) * NSRC;
      const double o = MASK ? (i < rel ? p0 : 0.0) : p0;
#pragma unroll
      for (int s = 0; s < NSRC; ++s) acc[q + s] = fma(o, sv[s], acc[q + s]);
    }
    const double nx = rec_step(t, p0, p1);
    t -= d2;
    p1 = p0;
    p0 = nx;
  }
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
  double *jms = lds + npad;                // [npad]  w j_m, later the Miller seed
  uint32_t *mps = (uint32_t *)(lds + 2 * npad);  // [npad]  (m + 1) | (sblk + 1) << 16
  double *const lds2 = lds + 2 * npad + (npad + 1) / 2;
  double *stage = lds2 + w * fp64::stage_doubles(NV);      // per wave [16][NV+1]
  double *cross0 = lds2 + W * fp64::stage_doubles(NV);     // [2][W][NV]
  int *bnd = (int *)(cross0 + 2 * W * NV);       // [3]

  const double kk = a.k[ki];
  const double *srow[NSRC];  // uniform row pointers of this k
#pragma unroll
  for (int s = 0; s < NSRC; ++s) srow[s] = a.S + ((int64_t)s * a.nk + ki) * a.ntau;

  // ---------------- per-node setup ----------------
  // m = last row of the upward part, sblk = block of the Miller start, per node in mps
  double Ja[T], Jb[T];
#if LOS_IX_REG
  double Ix[T];  // 1/x per slot, kept in registers (read in every block)
#define IXV(j, n) Ix[j]
#else
#define IXV(j, n) ixs[n]
#endif
  // Per-slot block thresholds (wave-uniform), held by lane j for slot j:
  //   pass 1: slot runs unmasked in blocks bi <= thF, at all in blocks bi <= thA;
  //   pass 2: slot is live in blocks thL <= bi <= thU, unmasked for bi >= thG.
  int thF = -1, thA = -1, thL = INT_MAX, thU = -1, thG = INT_MAX;
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
        // The recurrence is linear, so the state carries w_n j_l: the weight
        // of the tau quadrature is applied once here instead of per block.
        const double wn = a.w[n];
        pa = wn * (cs * ix);  // w j_{-1}
        pc = wn * (sn * ix);  // w j_0
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
#if LOS_IX_REG
    Ix[j] = ix;
#endif
    jms[(w + W * j) * 64 + lane] = jm;
    mps[(w + W * j) * 64 + lane] = (uint32_t)(m + 1) | ((uint32_t)(sblk + 1) << 16);
    Ja[j] = pa;
    Jb[j] = pc;
    // wave-uniform bounds of this slot, so that per-block slot tests are scalar
    {
      const bool dsc = sblk >= 0;
      const int mmax = wave_max(m), mmin = wave_min(m);
      const int smax = wave_max(sblk);
      const int dmin = wave_min(dsc ? m : INT_MAX), dmax = wave_max(dsc ? m : -1);
      // unmasked in pass 1 while every lane has m >= b + B
      const int f = mmin - lmin - B >= 0 ? (mmin - lmin - B) / B : -1;
      const int ab = mmax >= lmin ? (mmax - lmin) / B : -1;
      // live in pass 2 from the block holding row dmin + 1 up to the highest start block
      const int lo = smax < 0 ? INT_MAX : (dmin + 1 <= lmin ? 0 : (dmin + 1 - lmin) / B);
      // unmasked in pass 2 once b > dmax
      const int g = smax < 0 ? INT_MAX : (dmax + 1 <= lmin ? 0 : (dmax + 1 - lmin + B - 1) / B);
      if (lane == j) {
        thF = f;
        thA = ab;
        thL = lo;
        thU = smax;
        thG = g;
      }
    }
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
    const uint64_t fm = slot_mask(thF >= bi);               // unmasked slots
    const uint64_t pm = slot_mask(thA >= bi) & ~fm;         // partially active slots
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    // Slots whose lanes all run through the whole block, then the partial ones:
    // two single-sided branches keep acc in place (an if/else per slot makes the
    // register allocator copy acc around every slot).
    {
      // sources of slot j+1 are loaded while slot j computes (L2 latency)
      double sv[NSRC], svn[NSRC];
      load_s<NSRC>(sv, srow, w * 64 + lane, ntau);
#pragma unroll
      for (int j = 0; j < T; ++j) {
        const int nb = (w + W * j) * 64;
        if (nb >= ntau) break;
        int n = nb + lane;
        asm volatile("" : "+v"(n));
        if (j + 1 < T) load_s<NSRC>(svn, srow, n + W * 64, ntau);
        // fully upward through the block, and j_m (if needed) lies beyond it
        if (has(fm, j)) asc_slot<NSRC, B, false>(acc, Ja[j], Jb[j], IXV(j, n), sv, b, 0, nullptr);
#pragma unroll
        for (int s = 0; s < NSRC; ++s) sv[s] = svn[s];
      }
    }
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const int nb = (w + W * j) * 64;
      if (nb >= ntau) break;
      int n = nb + lane;
      asm volatile("" : "+v"(n));
      const uint32_t mpj = mps[n];
      if (has(pm, j)) {
        const int m = (int)(mpj & 0xFFFFu) - 1;
        double sv[NSRC];
        load_s<NSRC>(sv, srow, n, ntau);
        int rel = m - b;  // opaque, so the compiler does not precompute m - i per slot
        asm volatile("" : "+v"(rel));
        asc_slot<NSRC, B, true>(acc, Ja[j], Jb[j], IXV(j, n), sv, b, rel, &jms[n]);
      }
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
  // Miller seed: the recurrence started from (0, 1) at the top of block sblk is
  // run down to l = m (whole blocks, then single steps) and scaled to meet the
  // upward value stored there.
#pragma unroll
  for (int j = 0; j < T; ++j) {
    Ja[j] = 0.0;
    Jb[j] = 0.0;
    const int nb = (w + W * j) * 64;
    if (nb >= ntau) break;
    const int n = nb + lane;
    const uint32_t mpj = mps[n];
    const int m = (int)(mpj & 0xFFFFu) - 1;
    const int sb = (int)(mpj >> 16) - 1;
    if (sb >= 0) {
      const double ix = IXV(j, n);
      const double d2 = ix + ix;
      const int mt = m;
      int l = lmin + sb * B + B - 1;
      double jp = 0.0, jc = 1.0;
      while (l - B >= mt) {  // whole blocks
        double t = (double)(2 * l + 1) * ix;
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const double nx = rec_step(t, jc, jp);
          t -= d2;
          jp = jc;
          jc = nx;
        }
        l -= B;
      }
      while (l > mt) {
        const double nx = rec_step((double)(2 * l + 1) * ix, jc, jp);
        jp = jc;
        jc = nx;
        --l;
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
    // the stored pass-1 sum of this block is read now and added after the reduction
    const bool mine = store && w == 0 && lane < NV && b + lane / NSRC <= lmax;
    double old = 0.0;
    if (mine) old = drow[(int64_t)(b - lmin) * NSRC + lane];
    const uint64_t live = slot_mask(thL <= bi && bi <= thU);
    const uint64_t gm0 = live & slot_mask(thG <= bi), gm1 = live & ~gm0;
    const bool act = live != 0;  // wave-uniform: this wave has a live slot in the block
    if (store) {
      // pass over slots in two single-sided groups (see pass 1)
#pragma unroll
      for (int g = 0; g < 2; ++g) {
#pragma unroll
        for (int j = 0; j < T; ++j) {
          const int nb = (w + W * j) * 64;
          if (nb >= ntau) break;
          int n = nb + lane;
          asm volatile("" : "+v"(n));
          const uint32_t mpj = mps[n];
          // live: some lane has started its Miller part and reaches above its m;
          // group 0: every Miller lane's upward range ends below the block
          if (!has(g == 0 ? gm0 : gm1, j)) continue;
          const int m = (int)(mpj & 0xFFFFu) - 1;
          const int sb = (int)(mpj >> 16) - 1;
          if (sb == bi) {  // Miller start of this lane
            Ja[j] = 0.0;
            Jb[j] = jms[n];
          }
          double sv[NSRC];
          load_s<NSRC>(sv, srow, n, ntau);
          if (g == 0) {
            desc_slot<NSRC, B, true, false>(acc, Ja[j], Jb[j], IXV(j, n), sv, top, 0);
          } else {
            int rel = top - m;  // opaque, see pass 1
            asm volatile("" : "+v"(rel));
            desc_slot<NSRC, B, true, true>(acc, Ja[j], Jb[j], IXV(j, n), sv, top, rel);
          }
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < T; ++j) {
        const int nb = (w + W * j) * 64;
        if (nb >= ntau) break;
        int n = nb + lane;
        asm volatile("" : "+v"(n));
        const uint32_t mpj = mps[n];
        if (!has(live, j)) continue;
        const int sb = (int)(mpj >> 16) - 1;
        if (sb == bi) {
          Ja[j] = 0.0;
          Jb[j] = jms[n];
        }
        double sv[NSRC];
        desc_slot<NSRC, B, false, false>(acc, Ja[j], Jb[j], IXV(j, n), sv, top, 0);
      }
    }
    if (store) {
      const double tot = wg_reduce<NV>(acc, stage, cross0 + parity * W * NV, W, w, lane, act);
      parity ^= 1;
      if (mine) drow[(int64_t)(b - lmin) * NSRC + lane] = old + tot;
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
    case 24: return launch_t<NSRC, 24>(a, sh, s);
    case 32: return launch_t<NSRC, 32>(a, sh, s);
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
  if (T > 16) T = T <= 24 ? 24 : 32;
  if (T > 32 || (int64_t)64 * W * T < ntau) return sh;  // waves == 0: unsupported
  sh.waves = W;
  sh.slots = T;
  const int NV = kB * nsrc;
  const int npad = W * 64 * T;
  sh.lds = sizeof(double) * ((size_t)2 * npad + (size_t)(npad + 1) / 2 + (size_t)W * fp64::stage_doubles(NV) +
                            2 * (size_t)W * NV) +
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
