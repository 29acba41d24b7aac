// FP64 line-of-sight projection, single descending sweep: launch shape and
// dispatch over the source count.  The kernel and its description are in
// project_fp64_desc_kernel.hpp; project_fp64_desc_n{1..4}{,s}.hip instantiate it.
#include "fp64_common.hpp"
#include "los_internal.hpp"

namespace los {

hipError_t project_fp64_desc_launch_n1(const ProjectArgs &a, const ProjectShape &sh,
                                        hipStream_t s);
hipError_t project_fp64_desc_launch_n1_sc(const ProjectArgs &a, const ProjectShape &sh,
                                           hipStream_t s);
hipError_t project_fp64_desc_launch_n2(const ProjectArgs &a, const ProjectShape &sh,
                                        hipStream_t s);
hipError_t project_fp64_desc_launch_n2_sc(const ProjectArgs &a, const ProjectShape &sh,
                                           hipStream_t s);
hipError_t project_fp64_desc_launch_n3(const ProjectArgs &a, const ProjectShape &sh,
                                        hipStream_t s);
hipError_t project_fp64_desc_launch_n3_sc(const ProjectArgs &a, const ProjectShape &sh,
                                           hipStream_t s);
hipError_t project_fp64_desc_launch_n4(const ProjectArgs &a, const ProjectShape &sh,
                                        hipStream_t s);
hipError_t project_fp64_desc_launch_n4_sc(const ProjectArgs &a, const ProjectShape &sh,
                                           hipStream_t s);

static size_t desc_lds_bytes(int W, int T, int NV, int ring, size_t lds_extra) {
  const size_t npad = (size_t)W * 64 * T;
  return sizeof(double) * (npad + (npad + 1) / 2 + (size_t)W * fp64::stage_doubles(NV) +
                           (size_t)ring * W * NV) +
         4 * sizeof(int) + lds_extra;
}

// Launch shape: W waves per workgroup, T slots per lane (T a multiple of 4,
// 64 W T >= ntau) and the ring of block partials (8, else 2 where 8 does not
// fit).  The kernel needs more than 128 VGPRs for every T, so a SIMD holds at
// most 2 of its waves (8 per CU); LDS (160 KiB per CU) may allow fewer.
// Chosen: the most resident waves per CU, then the least padding (idle
// lanes), then fewer waves per workgroup (less reduction work), then the
// larger ring (fewer barriers).
ProjectShape project_fp64_desc_shape(int nsrc, int64_t ntau, int force_waves, int force_slots,
                                     int block, size_t lds_extra) {
  ProjectShape sh{};
  sh.block = block == 8 ? 8 : 16;  // 16 rows per reduction halves the source reloads
  const int NV = sh.block * nsrc;
  constexpr size_t kLdsPerCu = 160 * 1024;
  int bestW = 0, bestT = 0, bestR = 0, best_res = -1;
  double best_eff = -1.0;
  for (int W = 1; W <= 8; ++W) {
    if (force_waves > 0 && W != force_waves) continue;
    for (int T = 4; T <= 16; T += 4) {
      if (force_slots > 0 && T != (force_slots + 3) / 4 * 4) continue;
      if ((int64_t)64 * W * T < ntau) continue;
      for (int ring = 8; ring >= 2; ring -= 6) {
        const size_t lds = desc_lds_bytes(W, T, NV, ring, lds_extra);
        if (lds > kLdsPerCu) continue;
        const int fit = (int)(kLdsPerCu / lds);
        const int res = (fit < 8 / W ? fit : 8 / W) * W;
        const double eff = (double)ntau / (64.0 * W * T);
        if (res > best_res || (res == best_res && eff > best_eff + 1e-9)) {
          bestW = W;
          bestT = T;
          bestR = ring;
          best_res = res;
          best_eff = eff;
        }
      }
    }
  }
  if (bestW == 0) return sh;  // waves == 0: unsupported
  sh.waves = bestW;
  sh.slots = bestT;
  sh.ring = bestR;
  sh.lds = desc_lds_bytes(bestW, bestT, NV, bestR, lds_extra);
  return sh;
}

hipError_t project_fp64_desc_launch(const ProjectArgs &a, int nsrc, const ProjectShape &sh,
                                    hipStream_t s) {
  // scaled columns or remapped source planes take the scaled variants
  bool sc = (a.emask | a.x1mask | a.x2mask) != 0u;
  for (int q = 0; q < nsrc && q < 4; ++q) sc = sc || a.splane[q] != q;
  switch (nsrc) {
    case 1: return sc ? project_fp64_desc_launch_n1_sc(a, sh, s) : project_fp64_desc_launch_n1(a, sh, s);
    case 2: return sc ? project_fp64_desc_launch_n2_sc(a, sh, s) : project_fp64_desc_launch_n2(a, sh, s);
    case 3: return sc ? project_fp64_desc_launch_n3_sc(a, sh, s) : project_fp64_desc_launch_n3(a, sh, s);
    case 4: return sc ? project_fp64_desc_launch_n4_sc(a, sh, s) : project_fp64_desc_launch_n4(a, sh, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace los
