// FP64 line-of-sight projection, single descending sweep (gCAMB paper
// Sec. 2.1 Eq. 2-3; Sec. 3.2 / Algorithm 1 for the k / l / tau loops):
//
//   delta[k][l][s] = sum_n w_n S[s][k][n] j_l(k (tau0 - tau_n))
//
// Same workgroup / wave / slot mapping and per-block reduction as
// project_fp64.hip, but every lane walks its l range once, from the top down:
//   * setup: each node finds w (j_R, j_{R+1}) at its top row R, the top row
//     of the B-row block that holds min(ltop(x), lmax).  For x >= lmax + 1
//     the upward recurrence from j_{-1} = cos x / x, j_0 = sin x / x runs to
//     R + 1 (stable on the oscillatory side; R is at most B - 1 rows past
//     lmax, and those rows are never stored).  Otherwise, for x >= kXDebye,
//     Debye's expansion gives the pair at Ls = max(ltop(x), R) and the
//     recurrence runs down to R; for smaller x the upward run goes to
//     m = floor(x) for j_m, and Miller's recurrence with seeds (0, 1) from Ls
//     runs down to m and is scaled there to j_m (j_m is near the last maximum
//     in l, never near a zero), giving the pair at R.  Rows between ltop(x)
//     and R carry values below the band cut.
//   * the sweep: blocks of B = 16 rows (8 selectable) from the highest top of
//     the workgroup down to lmin; each lane runs j_{l-1} = (2l+1)/x j_l -
//     j_{l+1} for its slots from its R down.  R being a block top, a lane is
//     live either throughout a block or not at all, so a slot whose lanes
//     start in different blocks runs the same code under an exec mask.
//     Downward is the stable direction above the turning point and neutrally
//     stable below it, so one sweep covers the whole band with no second pass
//     and no read-modify-write of delta.
// E-mode sources (bit s of emask; Sec. 2.1, Eq. 3: eps_l(x) =
// sqrt((l+2)!/(l-2)!) j_l(x) / x^2): their values are scaled by 1/x^2 per node
// as they are loaded and their output rows by sqrt((l-1) l (l+1) (l+2)); a node
// with x below kXTiny adds its limit w S sqrt(24)/15 to l = 2 only.
// Columns of x1mask / x2mask are scaled by 1/x / 1/x^2 per node with no row
// factor (the tensor-mode projection combines them afterwards); their x -> 0
// limits go to l = 1 (w S / 3) and l = 2 (w S / 15).  Column s reads source
// plane splane[s], so one source can feed several columns.
#pragma once

#include "bessel_dev.hpp"
#include "fp64_common.hpp"
#include "los_internal.hpp"

#include <climits>

namespace los {
namespace desc {

using fp64::has;
using fp64::load_s;
using fp64::slot_mask;
using fp64::wave_max;
using fp64::wave_min;
using fp64::wave_reduce;

// One slot over the block of rows top .. top-B+1, descending.  (p1, p0) =
// (w j_{l+1}, w j_l) at l = top on entry, at l = top - B on return.
template <int NSRC, int B>
__device__ __forceinline__ void sweep_slot(double (&acc)[B * NSRC], double &p1, double &p0,
                                           double ix, const double (&sv)[NSRC], int top) {
  double t = 0.0;
  const double d2 = ix + ix;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    // the coefficient (2l+1)/x is formed exactly every 8 rows and stepped by
    // -2/x in between (at most 7 rounding steps, whatever the block size)
    if (i % 8 == 0) t = (double)(2 * (top - i) + 1) * ix;
    const int q = (B - 1 - i) * NSRC;
#pragma unroll
    for (int s = 0; s < NSRC; ++s) acc[q + s] = fma(p0, sv[s], acc[q + s]);
    const double nx = rec_step(t, p0, p1);
    p1 = p0;
    p0 = nx;
    t -= d2;
  }
}

// SC: the kernel variant with per-column scalings (E-mode, 1/x, 1/x^2) and
// source planes; without it every column s reads plane s unscaled.
template <int NSRC, int T, int B, bool SMP, bool SC>
__global__ void __launch_bounds__(512) project_fp64_desc_kernel(ProjectArgs a) {
  constexpr int NV = B * NSRC;
  const int nblk = (a.nl + B - 1) / B;
  extern __shared__ double lds[];

  const int W = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ki = a.nk - 1 - (int64_t)blockIdx.x;  // large k (most work) first
  const int lmin = a.lmin, lmax = a.lmax;
  const int ntau = (int)a.ntau;
  const int npad = W * 64 * T;

  double *ixs = lds;                                  // [npad] 1/x per node
  int *rs = (int *)(lds + npad);                      // [npad] top row R per node (-1: none)
  double *const lds2 = lds + npad + (npad + 1) / 2;
  double *stage = lds2 + w * fp64::stage_doubles(NV);                 // per wave [16][NV+1]
  const int nring = a.ring, half = nring >> 1;         // 8 or 2 blocks of partials
  double *cross = lds2 + W * fp64::stage_doubles(NV);  // [nring][W][NV] block partials
  int *bnd = (int *)(cross + nring * W * NV);          // [1]

  const double kk = a.k[ki];
  const double *srow[NSRC];
#pragma unroll
  for (int s = 0; s < NSRC; ++s)
    srow[s] = a.S + ((int64_t)(SC ? a.splane[s] : s) * a.nk + ki) * a.ntau;

  // ---------------- per-node setup: the pair at the top row ----------------
  double Jn[T], Jc[T];  // w j_{l+1}, w j_l of the current row, per slot
  // Every node's top row R is the top row of a block (the block holding its
  // band edge or lmax), so in any block a lane is either live throughout or
  // not at all.  Rows between the band edge and R hold values below the band
  // cut; rows above lmax are swept but never stored.
  const int top_all = lmin + (lmax - lmin) / B * B + (B - 1);
  // Per-slot block thresholds held by lane j for slot j (wave-uniform):
  // the slot runs unmasked in blocks bi <= thF and at all in blocks bi <= thA.
  int thF = -1, thA = -1, my_top = -1;
  // Setup of slot j once its upward run has reached l = up (x, weight wn,
  // (p, q) = wn (j_{up-1}, j_up)): the Debye or Miller part where needed, the
  // pair at R, the per-node LDS entries and the slot's thresholds.
  auto finish = [&](int j, bool live, double x, double ix, double p, double q, double wn) {
    const int n = (w + W * j) * 64 + lane;
    int R = -1;
    double cur = 0.0, nxt = 0.0;
    if (live) {
      if (floor(x) >= (double)(lmax + 1)) {
        R = top_all;
        cur = p;  // w j_R
        nxt = q;  // w j_{R+1}
      } else {
        const int m = (int)floor(x);
        const double jm = q;  // w j_m
        const int L0 = ltop_of(x);
        const int Rc = L0 < lmax ? L0 : lmax;  // last row kept (band edge or lmax)
        if (Rc >= lmin) {
          // top row of the block holding Rc; the seeds sit at or above it
          R = lmin + (Rc - lmin) / B * B + (B - 1);
          const int Ls = L0 > R ? L0 : R;
          if (x >= kXDebye) {  // Debye's expansion at the band edge (no upward run)
            double hc = debye_j(Ls, x), hn = debye_j(Ls + 1, x);
            run_down(hn, hc, Ls, R, ix);
            cur = wn * hc;
            nxt = wn * hn;
          } else {
            double hn = 0.0, hc = 1.0;  // Miller seeds (0, 1) at Ls
            run_down(hn, hc, Ls, R, ix);
            const double hR = hc, hR1 = hn;
            run_down(hn, hc, R, m, ix);
            const double sc = jm / hc;
            cur = sc * hR;
            nxt = sc * hR1;
          }
        }
      }
    }
    ixs[n] = live ? ix : 0.0;
    rs[n] = R;
    Jc[j] = cur;
    Jn[j] = nxt;
    // wave-uniform thresholds of this slot
    const int rmax = wave_max(R), rmin = wave_min(R >= 0 ? R : -1);
    // unmasked in block bi when every lane's R >= top of the block
    const int f = rmin - lmin - (B - 1) >= 0 ? (rmin - lmin - (B - 1)) / B : -1;
    const int ab = rmax >= lmin ? (rmax - lmin) / B : -1;
    if (lane == j) {
      thF = f;
      thA = ab;
    }
    my_top = ab > my_top ? ab : my_top;
  };
  // Slots go in pairs: the two upward runs share their common length, two
  // independent recurrence chains in flight; each then finishes on its own.
#pragma unroll
  for (int j = 0; j < T; j += 2) {
    bool live[2];
    double xs[2], ixv[2], pv[2], qv[2], wv[2];
    int up[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int n = (w + W * (j + h)) * 64 + lane;
      live[h] = false;
      xs[h] = 0.0;
      ixv[h] = 0.0;
      pv[h] = 0.0;
      qv[h] = 0.0;
      wv[h] = 0.0;
      up[h] = 0;
      if (n < ntau) {
        const double x = kk * (a.tau0 - a.tau[n]);
        const double wn = a.w[n];
        if (x >= kXTiny && wn != 0.0) {
          live[h] = true;
          xs[h] = x;
          ixv[h] = 1.0 / x;
          wv[h] = wn;
          const double fx = floor(x);
          if (fx >= (double)(lmax + 1) || x < kXDebye) {
            double sn, cs;
            sincos(x, &sn, &cs);
            pv[h] = wn * (cs * ixv[h]);  // w j_{-1}
            qv[h] = wn * (sn * ixv[h]);  // w j_0
            // upward to the top row's successor (x >= lmax + 1) or to floor(x)
            up[h] = fx >= (double)(lmax + 1) ? top_all + 1 : (int)fx;
          }  // else: Debye seeds in finish, no upward run
        }
      }
    }
    const int common = up[0] < up[1] ? up[0] : up[1];
    const int l = run_up2(pv[0], qv[0], pv[1], qv[1], common, ixv[0], ixv[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      run_up(pv[h], qv[h], l, up[h], ixv[h]);
      finish(j + h, live[h], xs[h], ixv[h], pv[h], qv[h], wv[h]);
    }
  }
  if (threadIdx.x == 0) bnd[0] = -1;
  __syncthreads();
  atomicMax(&bnd[0], my_top);
  __syncthreads();
  const int top_blk = bnd[0];

  // Limits at x -> 0 of the scaled columns (the nodes below kXTiny are not
  // swept): j_2(x)/x^2 -> 1/15 for E-mode and 1/x^2 columns at l = 2,
  // j_1(x)/x -> 1/3 for 1/x columns at l = 1; every other row -> 0.  A column
  // has at most one such row, so one sum per column (added in block 0).
  const uint32_t m2 = SC ? (a.emask | a.x2mask) : 0u;
  const uint32_t m1 = SC ? a.x1mask : 0u;
  const bool lim1 = m1 != 0 && lmin <= 1;
  const bool lim2 = m2 != 0 && lmin <= 2;
  double elim[NSRC];
#pragma unroll
  for (int s = 0; s < NSRC; ++s) elim[s] = 0.0;
  if (lim1 || lim2) {
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const int n = (w + W * j) * 64 + lane;
      if (n < ntau && ixs[n] == 0.0) {
        const double x = kk * (a.tau0 - a.tau[n]);
        if (x < kXTiny) {
          const double wn = a.w[n];
#pragma unroll
          for (int s = 0; s < NSRC; ++s) {
            if (lim2 && ((m2 >> s) & 1u)) elim[s] += wn * srow[s][n] * (1.0 / 15.0);
            else if (lim1 && ((m1 >> s) & 1u)) elim[s] += wn * srow[s][n] * (1.0 / 3.0);
          }
        }
      }
    }
  }

  double *drow = a.delta + ki * (int64_t)(SMP ? a.nls : a.nl) * NSRC;
  // output offset of row l = b + lane / NSRC, source lane % NSRC (-1: not stored)
  auto out_at = [&](int b) -> int64_t {
    const int l = b + lane / NSRC;
    if (l > lmax) return -1;
    if (!SMP) return (int64_t)(b - lmin) * NSRC + lane;
    const int r = a.lsel[l - lmin];
    return r < 0 ? -1 : (int64_t)r * NSRC + lane % NSRC;
  };
  // blocks above every lane's top row are zero
  if (w == 0 && lane < NV) {
    for (int bi = top_blk + 1; bi < nblk; ++bi) {
      const int64_t o = out_at(lmin + bi * B);
      if (o >= 0) drow[o] = 0.0;
    }
  }
  // with limit terms, block 0 is swept even when no node reaches it
  const int first = ((lim1 || lim2) && top_blk < 0) ? 0 : top_blk;
  // Sources of the fully-live slots come through a ring of 4 register sets:
  // slot j uses ring[j % 4] and is loaded 3 slots ahead.  S does not depend
  // on the row block, so the last slots of a block prefetch the first slots
  // of the next one (T is a multiple of 4, so slot j keeps its ring entry).
  double ring[4][NSRC];
  if (first >= 0) {
    const uint64_t fm0 = slot_mask(thF >= first);
#pragma unroll
    for (int j = 0; j < 3 && j < T; ++j)
      if (has(fm0, j)) load_s<NSRC>(ring[j], srow, (w + W * j) * 64 + lane, ntau);
  }
  for (int bi = first; bi >= 0; --bi) {
    const int b = lmin + bi * B;
    const int top = b + B - 1;
    const uint64_t fm = slot_mask(thF >= bi);        // all lanes live through the block
    const uint64_t pm = slot_mask(thA >= bi) & ~fm;  // some lanes start inside it
    const uint64_t fmn = bi > 0 ? slot_mask(thF >= bi - 1) : 0;  // the next block's
    const uint32_t sm = SMP ? a.bmask[bi] : 0u;  // sampled rows of this block (bit r: row b + r)
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
      {
        const int jp = j + 3;  // prefetch: this block's slot jp or the next block's jp - T
        const int js = jp < T ? jp : jp - T;
        if (has(jp < T ? fm : fmn, js))
          load_s<NSRC>(ring[js % 4], srow, (w + W * js) * 64 + lane, ntau);
      }
      const int nb = (w + W * j) * 64;
      if (nb >= ntau || !has(fm, j)) continue;
      int n = nb + lane;
      asm volatile("" : "+v"(n));
      double(&sv)[NSRC] = ring[j % 4];
      const double ix = ixs[n];
      if (SC && (m2 | m1) != 0) {  // uniform; the ring entry is reloaded before its next use
        const double i2 = ix * ix;
#pragma unroll
        for (int s = 0; s < NSRC; ++s) {
          if ((m2 >> s) & 1u) sv[s] *= i2;
          else if ((m1 >> s) & 1u) sv[s] *= ix;
        }
      }
      sweep_slot<NSRC, B>(acc, Jn[j], Jc[j], ix, sv, top);
    }
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const int nb = (w + W * j) * 64;
      if (nb >= ntau) break;
      int n = nb + lane;
      asm volatile("" : "+v"(n));
      if (!has(pm, j)) continue;
      double sv[NSRC];
      load_s<NSRC>(sv, srow, n, ntau);
      if (SC && (m2 | m1) != 0) {  // uniform
        const double i2 = ixs[n] * ixs[n];
#pragma unroll
        for (int s = 0; s < NSRC; ++s) {
          if ((m2 >> s) & 1u) sv[s] *= i2;
          else if ((m1 >> s) & 1u) sv[s] *= ixs[n];
        }
      }
      if (rs[n] >= top)  // this lane is live through the block (R is a block top)
        sweep_slot<NSRC, B>(acc, Jn[j], Jc[j], ixs[n], sv, top);
    }
    if (SC && bi == 0) {  // the x -> 0 limit terms (zero unless a scaled column reaches l = 1 or 2)
      if (lmin == 1) {
#pragma unroll
        for (int s = 0; s < NSRC; ++s) {
          const bool r1 = (m1 >> s) & 1u;
          acc[s] += r1 ? elim[s] : 0.0;         // row 1
          acc[NSRC + s] += r1 ? 0.0 : elim[s];  // row 2
        }
      } else if (lmin == 2) {
#pragma unroll
        for (int s = 0; s < NSRC; ++s) acc[s] += elim[s];
      }
    }
    // Each wave leaves its block total in slot bi % nring; every nring/2
    // blocks (bi % (nring/2) == 0) the workgroup synchronises once and wave 0
    // sums the waves in a fixed order and stores those blocks, while the
    // other waves go on into the other half of the ring.
    // With multipole sampling, blocks holding no sampled row skip all of this
    // except the (uniform) barrier.
    if (!SMP || sm != 0u) {
      const double part = wave_reduce<NV>(acc, stage, lane);
      if (lane < NV) cross[((bi & (nring - 1)) * W + w) * NV + lane] = part;
    }
    if ((bi & (half - 1)) == 0) {
      __syncthreads();
      if (w == 0 && lane < NV) {
        const int hi = bi + half - 1 < first ? bi + half - 1 : first;
        for (int bb = hi; bb >= bi; --bb) {
          if (SMP && a.bmask[bb] == 0u) continue;
          double tot = 0.0;
          for (int ww = 0; ww < W; ++ww) tot += cross[((bb & (nring - 1)) * W + ww) * NV + lane];
          const int l = lmin + bb * B + lane / NSRC;
          if (SC && ((a.emask >> (lane % NSRC)) & 1u))
            tot *= sqrt((double)(l - 1) * (double)l * (double)(l + 1) * (double)(l + 2));
          const int64_t o = out_at(lmin + bb * B);
          if (o >= 0) drow[o] = tot;
        }
      }
    }
  }
}

template <int NSRC, int T, int B, bool SMP, bool SC>
hipError_t launch_t(const ProjectArgs &a, const ProjectShape &sh, hipStream_t s) {
  auto kern = project_fp64_desc_kernel<NSRC, T, B, SMP, SC>;
  if (sh.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
    if (e != hipSuccess) return e;
  }
  ProjectArgs b = a;
  b.ring = sh.ring;
  hipLaunchKernelGGL(kern, dim3((unsigned)b.nk), dim3(64 * sh.waves), sh.lds, s, b);
  return hipGetLastError();
}

template <int NSRC, int B, bool SMP, bool SC>
hipError_t launch_b(const ProjectArgs &a, const ProjectShape &sh, hipStream_t s) {
  switch (sh.slots) {
    case 4: return launch_t<NSRC, 4, B, SMP, SC>(a, sh, s);
    case 8: return launch_t<NSRC, 8, B, SMP, SC>(a, sh, s);
    case 12: return launch_t<NSRC, 12, B, SMP, SC>(a, sh, s);
    case 16: return launch_t<NSRC, 16, B, SMP, SC>(a, sh, s);
    default: return hipErrorInvalidValue;
  }
}

// The variants without scaled columns (plain j_l, source s in column s).
template <int NSRC>
hipError_t launch_plain(const ProjectArgs &a, const ProjectShape &sh, hipStream_t s) {
  if (a.lsel) {  // multipole sampling: 16-row blocks only
    if (sh.block != 16 || !a.bmask) return hipErrorInvalidValue;
    return launch_b<NSRC, 16, true, false>(a, sh, s);
  }
  return sh.block == 16 ? launch_b<NSRC, 16, false, false>(a, sh, s)
                        : launch_b<NSRC, 8, false, false>(a, sh, s);
}

// The variants with scaled columns or remapped source planes (16-row blocks only).
template <int NSRC>
hipError_t launch_scaled(const ProjectArgs &a, const ProjectShape &sh, hipStream_t s) {
  if (sh.block != 16) return hipErrorInvalidValue;
  if (a.lsel) {
    if (!a.bmask) return hipErrorInvalidValue;
    return launch_b<NSRC, 16, true, true>(a, sh, s);
  }
  return launch_b<NSRC, 16, false, true>(a, sh, s);
}

}  // namespace desc
}  // namespace los
