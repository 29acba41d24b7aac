// Device-side helpers for the spherical Bessel kernels j_l(x) of the
// line-of-sight integrals (gCAMB paper, Sec. 2.1 Eq. 2-3: flat space, so the
// radial kernel is j_l).
//
// Per argument x the library uses:
//   * upward   j_{l+1} = (2l+1)/x j_l - j_{l-1} from j_{-1} = cos x / x and
//              j_0 = sin x / x, for l <= m = floor(x) (oscillatory side, where
//              the upward direction is stable);
//   * Debye    for x >= kXDebye, the pair at the band edge ltop(x) (or above)
//              from Debye's asymptotic expansion (debye_j), then the same
//              recurrence run downward (stable there);
//   * Miller   for x < kXDebye, the recurrence run downward from a start
//              above the turning point with arbitrary seeds, scaled so that it
//              passes through the upward value at l = m.
// Above ltop(x) the values are below ~1e-21 of their peak and are dropped.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "debye_coef.hpp"

namespace los {

// Below this x the first power-series terms are exact in FP64; the
// projection treats such nodes as contributing nothing for l >= 2
// (|j_2(x)| < 7e-20 there).
constexpr double kXTiny = 1e-9;

// Last l kept for argument x.  x + 14.2 x^(1/3) + 10 lies above the root in
// nu of the Debye exponent nu*acosh(nu/x) - sqrt(nu^2 - x^2) = 50 for every
// x >= 1e-3 (margin 5 to 12 in nu), so |j_l(x)| < ~1e-21 of its peak for
// l + 1/2 beyond it.
__host__ __device__ inline int ltop_of(double x) {
  return (int)floor(x + 14.2 * cbrt(x) + 9.5);
}

// Band cut of the MFMA (FP32 / split-BF16x3) projections: above
// x + 9 x^(1/3) + 4, |j_l(x)| stays below 1.2e-12 of its largest value over l
// (checked for x = 1 .. 14000), far below the FP32 rounding of the values
// kept; the seeds still start at ltop(x) and run down to the cut.
__host__ __device__ inline int ltop_mfma_of(double x) {
  return (int)floor(x + 9.0 * cbrt(x) + 4.0);
}

// From this x on, the pair at the band edge comes from debye_j; below it the
// upward and Miller runs are short.
constexpr double kXDebye = 64.0;

// j_l(x) for nu = l + 1/2 above the turning point by at least ltop's margin
// (nu - x >= 14.2 x^(1/3) + 9), from Debye's expansion (DLMF 10.19.3)
//   J_nu(nu sech a) ~ e^eta / sqrt(2 pi nu tanh a) sum_k u_k(coth a) / nu^k,
//   eta = nu (tanh a - a),
// and j_l(x) = sqrt(pi / (2 x)) J_nu(x).  With q = sqrt(nu^2 - x^2) = nu tanh a
// and s = q / nu this is
//   j_l(x) = e^eta S / (2 sqrt(x q)),  S = 1 + sum_{k=1..10} u_k(nu/q) / nu^k,
// eta = -nu (atanh s - s): for s <= 0.7 from the series s^3 sum_m s^(2m)/(2m+3)
// (no cancellation), above from q - nu log((nu + q) / x).  Along the band edge
// nu s^3 stays near 60..150, where the ten terms leave a relative truncation
// error below ~1e-16 for every x >= 20.
__host__ __device__ inline double debye_j(int l, double x) {
  const double nu = (double)l + 0.5;
  const double q = sqrt((nu - x) * (nu + x));
  const double s = q / nu;
  double eta;
  if (s <= 0.7) {
    const double s2 = s * s;
    double f = kEtaC[kEtaTerms - 1];
#pragma unroll 1
    for (int m = kEtaTerms - 2; m >= 0; --m) f = fma(f, s2, kEtaC[m]);
    eta = -nu * (s * s2 * f);
  } else {
    eta = q - nu * log((nu + q) / x);
  }
  // u_k(t) / nu^k = z^k P_k(t^2) with t = nu / q, z = t / nu = 1 / q
  const double z = 1.0 / q, t = nu * z, y = t * t;
  double S = 0.0;
#pragma unroll 1
  for (int k = kDebyeK; k >= 1; --k) {
    const double *c = kDebyeC + kDebyeOff[k];
    double p = c[k];
#pragma unroll 1
    for (int i = k - 1; i >= 0; --i) p = fma(p, y, c[i]);
    S = (S + p) * z;
  }
  return exp(eta) * (1.0 + S) / (2.0 * sqrt(x * q));
}

// One step of the three-term recurrence with coefficient t = (2l+1)/x:
// returns t*c - p.
__host__ __device__ inline double rec_step(double t, double c, double p) { return fma(t, c, -p); }

// Upward run from (p, q) = (f_{l0-1}, f_{l0}) to l1 >= l0: on return
// (p, q) = (f_{l1-1}, f_{l1}).  The coefficient (2l+1)/x is formed exactly at
// the start of every 8 steps and stepped by 2/x in between, with no per-step
// test (a test per step is if-converted into a convert, a multiply and
// selects on every step).
__host__ __device__ inline void run_up(double &p, double &q, int l0, int l1, double ix) {
  const double d2 = ix + ix;
  int l = l0;
  for (; l + 8 <= l1; l += 8) {
    double t = (double)(2 * l + 1) * ix;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double r = rec_step(t, q, p);
      t += d2;
      p = q;
      q = r;
    }
  }
  double t = (double)(2 * l + 1) * ix;
  for (; l < l1; ++l) {
    const double r = rec_step(t, q, p);
    t += d2;
    p = q;
    q = r;
  }
}

// Two upward runs from l = 0, interleaved chunk by chunk (two independent
// chains in flight), for as many whole chunks of 8 as fit below l1; returns
// the l reached, from which each run goes on with run_up (the coefficient
// cadence, and so every rounding, is that of run_up from 0).
__device__ inline int run_up2(double &pa, double &qa, double &pb, double &qb, int l1, double ixa,
                              double ixb) {
  const double da = ixa + ixa, db = ixb + ixb;
  int l = 0;
  for (; l + 8 <= l1; l += 8) {
    const double c = (double)(2 * l + 1);
    double ta = c * ixa, tb = c * ixb;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double ra = rec_step(ta, qa, pa);
      const double rb = rec_step(tb, qb, pb);
      ta += da;
      tb += db;
      pa = qa;
      qa = ra;
      pb = qb;
      qb = rb;
    }
  }
  return l;
}

// Downward run from (hn, hc) = (f_{l0+1}, f_{l0}) to l1 <= l0: on return
// (hn, hc) = (f_{l1+1}, f_{l1}).  Coefficients as in run_up, stepped by -2/x.
__host__ __device__ inline void run_down(double &hn, double &hc, int l0, int l1, double ix) {
  const double d2 = ix + ix;
  int l = l0;
  for (; l - 8 >= l1; l -= 8) {
    double t = (double)(2 * l + 1) * ix;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double h = rec_step(t, hc, hn);
      t -= d2;
      hn = hc;
      hc = h;
    }
  }
  double t = (double)(2 * l + 1) * ix;
  for (; l > l1; --l) {
    const double h = rec_step(t, hc, hn);
    t -= d2;
    hn = hc;
    hc = h;
  }
}

// Normalised pair at a node's top row, the start of a descending sweep over
// rows lmin..lmax in 16-row blocks (Bessel tables and the fused projection).
// For x = k chi (x >= kXTiny), weight wt and band cut lcut <= ltop(x) (rows
// above it are dropped): R is the top row of the 16-row block (counted from
// lmin) that holds min(lcut, lmax), and on return (cur, nxt) = wt (j_R, j_{R+1}):
//   * x >= lmax + 1: upward recurrence from j_0 = sin x / x, j_{-1} = cos x / x
//     (stable on the oscillatory side) up to l = R + 1 (R is at most 15 rows
//     past lmax; those rows are never stored);
//   * otherwise, x >= kXDebye: the pair at Ld = max(ltop(x), R) from Debye's
//     expansion, then the recurrence down to R;
//   * otherwise: upward to m = floor(x) for j_m, and Miller's downward
//     recurrence from max(ltop(x), R) with seeds (0, 1) down to m, scaled
//     there by j_m (near the last maximum in l, never near a zero).
// Returns R, or -1 when no row in [lmin, lmax] is inside the band.
__host__ __device__ inline int node_top_pair(double x, double ix, double wt, int lmin, int lmax,
                                             int lcut, double &cur, double &nxt) {
  cur = 0.0;
  nxt = 0.0;
  const int m = (int)x;
  const int L0 = ltop_of(x);
  if (m < lmax + 1 && x >= kXDebye) {
    const int Rc = min(lcut, lmax);
    if (Rc < lmin) return -1;
    const int R = lmin + (Rc - lmin) / 16 * 16 + 15;
    const int Ld = max(L0, R);
    double hc = debye_j(Ld, x), hn = debye_j(Ld + 1, x);
    run_down(hn, hc, Ld, R, ix);
    cur = wt * hc;
    nxt = wt * hn;
    return R;
  }
  const double s = sin(x), c = cos(x);
  double p = c * ix, q = s * ix;  // j_{l-1}, j_l at l = 0
  if (m >= lmax + 1) {
    const int R = lmin + (lmax - lmin) / 16 * 16 + 15;
    run_up(p, q, 0, R + 1, ix);
    cur = wt * p;
    nxt = wt * q;
    return R;
  }
  run_up(p, q, 0, m, ix);
  const double jm = q;
  const int Rc = min(lcut, lmax);
  if (Rc < lmin) return -1;
  const int R = lmin + (Rc - lmin) / 16 * 16 + 15;
  double hn = 0.0, hc = 1.0;  // J^_{l+1}, J^_l
  run_down(hn, hc, max(L0, R), R, ix);
  const double hR = hc, hR1 = hn;
  run_down(hn, hc, R, m, ix);
  const double sc = wt * jm / hc;
  cur = sc * hR;
  nxt = sc * hR1;
  return R;
}

}  // namespace los
