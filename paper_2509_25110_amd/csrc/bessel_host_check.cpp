// Host build of the Bessel seed functions of bessel_dev.hpp (the same source
// the kernels compile), so CPU tests can check them against high-precision
// values before they run on the GPU.  Not part of the C ABI of liblos.so.
#include <stdint.h>

#include "bessel_dev.hpp"

extern "C" {

// out[i] = j_{l[i]}(x[i]) by Debye's expansion (valid above the band edge).
void los_hostcheck_debye_j(int64_t n, const int32_t *l, const double *x, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = los::debye_j(l[i], x[i]);
}

// The seed pair of a descending sweep over lmin..lmax for each x[i] (weight 1)
// with the FP64 band cut ltop (mfma = 0) or the MFMA paths' ltop_mfma (1):
// R[i] = its top row (-1: none), (cur[i], nxt[i]) = (j_R, j_{R+1}).
void los_hostcheck_node_top_pair(int64_t n, const double *x, int32_t lmin, int32_t lmax,
                                 int32_t mfma, double *cur, double *nxt, int32_t *R) {
  for (int64_t i = 0; i < n; ++i) {
    double c = 0.0, d = 0.0;
    const int cut = mfma ? los::ltop_mfma_of(x[i]) : los::ltop_of(x[i]);
    R[i] = los::node_top_pair(x[i], 1.0 / x[i], 1.0, lmin, lmax, cut, c, d);
    cur[i] = c;
    nxt[i] = d;
  }
}

}  // extern "C"
