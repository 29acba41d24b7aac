// Internal declarations shared by the host API and the kernel translation
// units of liblos.so.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace los {

// l rows per block of the projection kernels (also the granularity of the
// Miller start alignment).
constexpr int kProjectBlock = 8;

struct ProjectArgs {
  int lmin, lmax, nl, nblk;
  int64_t nk, ntau;
  double tau0;
  const double *k, *tau, *w;
  const double *S;  // [nsrc][nk][ntau]
  double *delta;    // [nk][nl][nsrc]
};

// Launch shape chosen by the host for the FP64 projection.
struct ProjectShape {
  int waves;   // waves per workgroup (1..8)
  int slots;   // tau slots per lane (4, 8, 12, 16)
  size_t lds;  // dynamic LDS bytes
};

// FP64 projection: one workgroup per k.
// force_waves / force_slots > 0 override the default shape (tuning).
ProjectShape project_fp64_shape(int nsrc, int64_t ntau, int force_waves = 0, int force_slots = 0);
hipError_t project_fp64_launch(const ProjectArgs &a, int nsrc, const ProjectShape &sh,
                               hipStream_t s);

// Bessel table out[(l-lmin)*nx + i] = j_l(x[i]).
hipError_t bessel_table_launch(const double *x, int64_t nx, int lmin, int lmax, double *out,
                               hipStream_t s);

// C_l reduction over k (deterministic, two passes through a partial buffer).
struct ClArgs {
  const void *delta;
  bool delta_f32;
  int nsrc, nl, npairs;
  int64_t nk;
  const double *w, *P;
  int pa[16], pb[16];
  double *cl;
  double *partial;  // [nseg][npairs][nl]
  int nseg;
};
int cl_segments(int64_t nk, int nl);
hipError_t cl_launch(const ClArgs &a, hipStream_t s);

}  // namespace los
