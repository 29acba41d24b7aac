// Internal declarations of the C_l emulator kernels (emu_kernels.hip) used by
// its host code (emu_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace los {
namespace emu {

constexpr int kEpiStore = 0;       // C = A B
constexpr int kEpiAccumulate = 1;  // C += A B
constexpr int kEpiBias = 2;        // C = A B + bias[n]
constexpr int kEpiBiasGelu = 3;    // Z = A B + bias[n], C = GELU(Z)
constexpr int kMaxQ = 112;         // largest PCA subspace (ncomp + oversampling)

// A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn],
// C(m, n) = C[m * ldc + n] (and Z likewise).
struct GemmF32 {
  int64_t M, N, K;
  const float *A;
  int64_t sam, sak;
  const float *B;
  int64_t sbk, sbn;
  float *C;
  int64_t ldc;
  const float *bias;
  float *Z;
};
struct GemmF64 {
  int64_t M, N, K;
  const double *A;
  int64_t sam, sak;
  const double *B;
  int64_t sbk, sbn;
  double *C;
  int64_t ldc;
};

hipError_t gemm_f32(const GemmF32 &g, int epi, hipStream_t s);
hipError_t gemm_f64(const GemmF64 &g, hipStream_t s);
hipError_t gelu_backward(float *G, const float *Z, int64_t n, hipStream_t s);
hipError_t colsum_f32(const float *X, int64_t rows, int64_t cols, float *out, hipStream_t s);
hipError_t mse_grad(const float *out, const float *z, int64_t cnt, float *G, float *partial,
                    float *loss, int accumulate, hipStream_t s);
hipError_t adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, int64_t t,
                hipStream_t s);
hipError_t gather_rows(const float *src, const int64_t *idx, int64_t rows, int64_t cols,
                       float *dst, hipStream_t s);
hipError_t scale_params(const double *p, int64_t n, int np, const double *lo, const double *hi,
                        float *u, hipStream_t s);
hipError_t transform(const double *cl, int64_t n, int nl, const double *t, double *y,
                     hipStream_t s);
hipError_t te_median(const double *cl, int64_t n, int nl, double *t, hipStream_t s);
hipError_t center(double *X, int64_t rows, int64_t cols, int64_t ld, double *mean, hipStream_t s);
// R^T R = G + shift_rel * trace(G) * I; Rinv = R^{-1}.
hipError_t chol_inv(const double *G, int q, double shift_rel, double *Rinv, int *status,
                    hipStream_t s);
hipError_t jacobi_eig(const double *A, int q, int sweeps, double *V, double *evals, double *U,
                      hipStream_t s);
hipError_t whiten(const double *c, int64_t n, int ncomp, int s_idx, int nout, double *sigma,
                  float *z, hipStream_t s);
hipError_t unwhiten(const float *out, int64_t n, int ncomp, int s_idx, int nout,
                    const double *sigma, float *cz, hipStream_t s);
// Member mean into cl and the error estimates: per row (err, flag) and / or
// per (row, spectrum) (err4, flag4), any of them NULL; err_bits has 4 n words.
hipError_t ensemble(const float *y, int members, int64_t n, int nl, const double *t, double *cl,
                    unsigned int *err_bits, float thr, float *err, unsigned char *flag,
                    float *err4, unsigned char *flag4, hipStream_t s);
// cl[rows[i]][*] = src[i][*] (row_len values each), err[rows[i]] = 0, flag[rows[i]] = 0
// (err, flag may be NULL); rows in [0, n) and distinct (checked by the caller).
hipError_t merge_rows(const int64_t *rows, int64_t nf, const double *src, int64_t row_len,
                      double *cl, float *err, unsigned char *flag, hipStream_t s);
// cl[rows[i]][spec][*] = src[i][*] (nl values each), err4 / flag4 of (rows[i], spec) = 0.
hipError_t merge_spectrum(const int64_t *rows, int64_t nf, const double *src, int nl, int spec,
                          double *cl, float *err4, unsigned char *flag4, hipStream_t s);

}  // namespace emu
}  // namespace los
