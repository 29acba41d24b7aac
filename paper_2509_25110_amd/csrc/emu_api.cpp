// C_l emulator: the C ABI entry points emu_* (include/los.h).
//
// The paper motivates fast repeated solves (Sec. 1: parameter-space sampling
// needs many spectra) but defines no emulator; this one is the project's own:
//   * inputs   u = 2 (p - lo) / (hi - lo) - 1 (the 5 source parameters);
//   * targets  per spectrum (TT, EE, TE, PP) over l = 2..lmax:
//              y = log C (TT, EE, PP), asinh(C_TE / t_l) (TE), t_l = lower
//              median over the training set of |C_TE(l)| (1 where it is 0);
//   * PCA      per spectrum in FP64: mean, top ncomp eigenvectors of the
//              covariance (randomised subspace iteration: q = ncomp + 8
//              columns, orthonormalised after every product by CholeskyQR3
//              with a shifted first pass, Rayleigh-Ritz by Jacobi); targets
//              z = c / sigma_s (FP32) with one scale per spectrum, sigma_s =
//              sqrt(variance of the kept components), so the loss weighs each
//              component by the variance it carries;
//   * MLP      u -> [width] x depth GELU layers -> 4 ncomp outputs, FP32 on
//              the matrix cores; MSE loss; Adam (0.9, 0.999, 1e-8) with the
//              step size lr (0.01 + 0.99 (1 + cos(pi (t - 1) / T)) / 2) over
//              T steps; minibatches from a SplitMix64 Fisher-Yates shuffle
//              per epoch; Glorot-uniform initial weights from SplitMix64;
//   * ensemble of `members` independently initialised networks: prediction
//              = member mean of C_l, error estimate = max over spectra, l and
//              members of |C_e - C_mean| / scale (scale |C_mean|, TE:
//              sqrt(C_TT C_EE)); need_fallback = estimate > threshold.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "emu_internal.hpp"
#include "los.h"
#include "los_internal.hpp"

using los::fail;
using los::hip_fail;
using los::ok;
namespace E = los::emu;

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  int reserve(size_t b) {
    if (b <= bytes) return LOS_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, b ? b : 1);
    if (e != hipSuccess) return fail(LOS_ERR_OOM, "emulator: hipMalloc(%zu): %s", b, hipGetErrorString(e));
    bytes = b;
    return LOS_OK;
  }
  template <class T>
  T *as() const { return (T *)p; }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

uint64_t splitmix(uint64_t &s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double unit(uint64_t &s) { return (double)(splitmix(s) >> 11) * 0x1.0p-53; }

}  // namespace

struct los_emu {
  int device = 0;
  int np = 0, nl = 0, ncomp = 0, width = 0, depth = 0, members = 0, nout = 0;
  uint64_t seed = 0;
  std::vector<int> sizes;        // layer widths, input first
  std::vector<int64_t> woff;     // offset of W_i in a member's parameters (b_i follows)
  int64_t nparams = 0;
  bool has_pca = false;
  DevBuf theta, adam_m, adam_v, grad;                 // [members][nparams], grad [nparams]
  DevBuf lo, hi, mean, basis, basis_f, mean_f, sigma, tscale;
  DevBuf act, pre, gbuf, gbuf2, ub, zb, idx, part, loss;  // training / inference scratch
  DevBuf y, X, Om, Yq, Yt, G, Rinv, Zq, Bm, U, Vj, ev, cfs, zt, ut, st, yall, errb, cz;
  DevBuf rows;  // emu_merge: the merged row indices
};

namespace {

int64_t layer_in(const los_emu *m, int i) { return m->sizes[i]; }
int64_t layer_out(const los_emu *m, int i) { return m->sizes[i + 1]; }
int nlayers(const los_emu *m) { return (int)m->sizes.size() - 1; }

#define HIPCHK(expr, what)                     \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Forward pass of member e on u [n][np]: activations act[i] [n][sizes[i]],
// pre-activations pre[i]; the output goes to `out` [n][nout].
int forward(los_emu *m, int e, const float *u, int64_t n, float *out, hipStream_t s) {
  const int L = nlayers(m);
  const int64_t wmax = m->width > 0 ? m->width : 1;
  int rc = m->act.reserve(sizeof(float) * (size_t)n * wmax * (L + 1));
  if (rc == LOS_OK) rc = m->pre.reserve(sizeof(float) * (size_t)n * wmax * (L + 1));
  if (rc != LOS_OK) return rc;
  const float *th = m->theta.as<float>() + (int64_t)e * m->nparams;
  const float *h = u;
  for (int i = 0; i < L; ++i) {
    const int64_t in = layer_in(m, i), o = layer_out(m, i);
    E::GemmF32 g{};
    g.M = n;
    g.N = o;
    g.K = in;
    g.A = h;
    g.sam = in;
    g.sak = 1;
    g.B = th + m->woff[i];
    g.sbk = 1;
    g.sbn = in;
    g.bias = th + m->woff[i] + o * in;
    g.ldc = o;
    if (i < L - 1) {
      g.C = m->act.as<float>() + (int64_t)(i + 1) * n * wmax;
      g.Z = m->pre.as<float>() + (int64_t)i * n * wmax;
      HIPCHK(E::gemm_f32(g, E::kEpiBiasGelu, s), "emulator: layer GEMM");
      h = g.C;
    } else {
      g.C = out;
      HIPCHK(E::gemm_f32(g, E::kEpiBias, s), "emulator: output GEMM");
    }
  }
  return LOS_OK;
}

// Loss and gradient of member e (after forward on the same u): dloss/dout is
// in gbuf; gradient written to grad [nparams].
int backward(los_emu *m, int e, const float *u, int64_t n, hipStream_t s) {
  const int L = nlayers(m);
  const int64_t wmax = m->width > 0 ? m->width : 1;
  int rc = m->gbuf2.reserve(sizeof(float) * (size_t)n * std::max<int64_t>(wmax, m->nout));
  if (rc != LOS_OK) return rc;
  const float *th = m->theta.as<float>() + (int64_t)e * m->nparams;
  float *gr = m->grad.as<float>();
  float *G = m->gbuf.as<float>(), *G2 = m->gbuf2.as<float>();
  for (int i = L - 1; i >= 0; --i) {
    const int64_t in = layer_in(m, i), o = layer_out(m, i);
    const float *h = i == 0 ? u : m->act.as<float>() + (int64_t)i * n * wmax;
    E::GemmF32 g{};  // dW_i = G^T h
    g.M = o;
    g.N = in;
    g.K = n;
    g.A = G;
    g.sam = 1;
    g.sak = o;
    g.B = h;
    g.sbk = in;
    g.sbn = 1;
    g.C = gr + m->woff[i];
    g.ldc = in;
    HIPCHK(E::gemm_f32(g, E::kEpiStore, s), "emulator: weight gradient");
    HIPCHK(E::colsum_f32(G, n, o, gr + m->woff[i] + o * in, s), "emulator: bias gradient");
    if (i > 0) {
      E::GemmF32 d{};  // G_prev = G W_i, then * gelu'(pre_{i-1})
      d.M = n;
      d.N = in;
      d.K = o;
      d.A = G;
      d.sam = o;
      d.sak = 1;
      d.B = th + m->woff[i];
      d.sbk = in;
      d.sbn = 1;
      d.C = G2;
      d.ldc = in;
      HIPCHK(E::gemm_f32(d, E::kEpiStore, s), "emulator: input gradient");
      HIPCHK(E::gelu_backward(G2, m->pre.as<float>() + (int64_t)(i - 1) * n * wmax, n * in, s),
             "emulator: GELU backward");
      std::swap(G, G2);
    }
  }
  return LOS_OK;
}

int loss_grad(los_emu *m, int e, const float *u, const float *z, int64_t n, float *loss,
              int accumulate, hipStream_t s) {
  int rc = m->ub.reserve(sizeof(float) * (size_t)n * m->nout);
  if (rc == LOS_OK) rc = m->gbuf.reserve(sizeof(float) * (size_t)n * std::max(m->width, m->nout));
  if (rc == LOS_OK) rc = m->part.reserve(sizeof(float) * (size_t)((n * m->nout + 255) / 256 + 1));
  if (rc != LOS_OK) return rc;
  float *out = m->ub.as<float>();
  if ((rc = forward(m, e, u, n, out, s)) != LOS_OK) return rc;
  HIPCHK(E::mse_grad(out, z, n * m->nout, m->gbuf.as<float>(), m->part.as<float>(), loss,
                     accumulate, s),
         "emulator: loss");
  return backward(m, e, u, n, s);
}

// Glorot-uniform weights and zero biases of member e from SplitMix64.
int init_member(los_emu *m, int e) {
  std::vector<float> h(m->nparams, 0.f);
  uint64_t st = m->seed + 0x632BE59BD9B4E019ull * (uint64_t)(e + 1);
  for (int i = 0; i < nlayers(m); ++i) {
    const int64_t in = layer_in(m, i), o = layer_out(m, i);
    const double a = std::sqrt(6.0 / (double)(in + o));
    for (int64_t k = 0; k < in * o; ++k) h[m->woff[i] + k] = (float)(a * (2.0 * unit(st) - 1.0));
  }
  HIPCHK(hipMemcpy(m->theta.as<float>() + (int64_t)e * m->nparams, h.data(),
                   sizeof(float) * m->nparams, hipMemcpyHostToDevice),
         "emulator: init copy");
  return LOS_OK;
}

// Adam on member e over (u, z) [n rows], from its current weights.
int fit_member(los_emu *m, int e, const float *u, const float *z, int64_t n, int epochs,
               int batch, double lr, float *hist, hipStream_t s) {
  const int64_t B = std::min<int64_t>(batch, n);
  const int64_t nb = (n + B - 1) / B;
  const int64_t T = (int64_t)epochs * nb;
  int rc = m->ut.reserve(sizeof(float) * (size_t)B * m->np);
  if (rc == LOS_OK) rc = m->zt.reserve(sizeof(float) * (size_t)B * m->nout);
  if (rc == LOS_OK) rc = m->idx.reserve(sizeof(int64_t) * (size_t)n);
  if (rc == LOS_OK) rc = m->loss.reserve(sizeof(float) * 2);
  if (rc != LOS_OK) return rc;
  float *wm = m->adam_m.as<float>() + (int64_t)e * m->nparams;
  float *wv = m->adam_v.as<float>() + (int64_t)e * m->nparams;
  HIPCHK(hipMemsetAsync(wm, 0, sizeof(float) * m->nparams, s), "emulator: adam reset");
  HIPCHK(hipMemsetAsync(wv, 0, sizeof(float) * m->nparams, s), "emulator: adam reset");
  std::vector<int64_t> perm(n);
  uint64_t st = m->seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(e + 1));
  int64_t t = 0;
  float *th = m->theta.as<float>() + (int64_t)e * m->nparams;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    if (B < n)
      for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[splitmix(st) % (uint64_t)(i + 1)]);
    HIPCHK(hipMemcpyAsync(m->idx.p, perm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s),
           "emulator: order copy");
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t r0 = b * B, rows = std::min(B, n - r0);
      const int64_t *ix = m->idx.as<int64_t>() + r0;
      HIPCHK(E::gather_rows(u, ix, rows, m->np, m->ut.as<float>(), s), "emulator: gather");
      HIPCHK(E::gather_rows(z, ix, rows, m->nout, m->zt.as<float>(), s), "emulator: gather");
      rc = loss_grad(m, e, m->ut.as<float>(), m->zt.as<float>(), rows, m->loss.as<float>(),
                     b > 0, s);
      if (rc != LOS_OK) return rc;
      ++t;
      const double sched = 0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * (double)(t - 1) / (double)T));
      HIPCHK(E::adam(th, m->grad.as<float>(), wm, wv, m->nparams, (float)(lr * sched), t, s),
             "emulator: adam");
    }
    if (hist) {
      float l = 0.f;
      HIPCHK(hipMemcpyAsync(&l, m->loss.p, sizeof(float), hipMemcpyDeviceToHost, s),
             "emulator: loss copy");
      HIPCHK(hipStreamSynchronize(s), "emulator: sync");
      hist[ep] = l / (float)nb;
    }
  }
  return LOS_OK;
}

// Y <- orth(Y) for Y [rows][q]: three CholeskyQR passes, the first shifted.
int orth(los_emu *m, double *Y, int64_t rows, int q, double *tmp, hipStream_t s) {
  const double u = std::ldexp(1.0, -53);
  for (int pass = 0; pass < 3; ++pass) {
    E::GemmF64 g{q, q, rows, Y, 1, q, Y, q, 1, m->G.as<double>(), q};  // G = Y^T Y
    HIPCHK(E::gemm_f64(g, s), "emulator: Gram");
    const double shift = pass == 0 ? 11.0 * ((double)rows * q + (double)q * (q + 1)) * u : 0.0;
    HIPCHK(E::chol_inv(m->G.as<double>(), q, shift, m->Rinv.as<double>(), m->st.as<int>(), s),
           "emulator: Cholesky");
    E::GemmF64 r{rows, q, q, Y, q, 1, m->Rinv.as<double>(), q, 1, tmp, q};
    HIPCHK(E::gemm_f64(r, s), "emulator: Q = Y R^-1");
    HIPCHK(hipMemcpyAsync(Y, tmp, sizeof(double) * rows * q, hipMemcpyDeviceToDevice, s),
           "emulator: copy");
  }
  return LOS_OK;
}

// PCA of spectrum sp from y [n][4][nl] (centred in place), basis [nl][ncomp].
int pca_spectrum(los_emu *m, int sp, int64_t n, hipStream_t s) {
  const int nl = m->nl, q = std::min(m->ncomp + 8, E::kMaxQ);
  double *X = m->y.as<double>() + (int64_t)sp * nl;  // rows of stride 4 nl
  const int64_t ld = 4 * (int64_t)nl;
  HIPCHK(E::center(X, n, nl, ld, m->mean.as<double>() + (int64_t)sp * nl, s), "emulator: mean");
  // Yq = X^T Om
  E::GemmF64 a{nl, q, n, X, 1, ld, m->Om.as<double>(), q, 1, m->Yq.as<double>(), q};
  HIPCHK(E::gemm_f64(a, s), "emulator: X^T Om");
  int rc = LOS_OK;
  for (int it = 0; it < 4; ++it) {
    if ((rc = orth(m, m->Yq.as<double>(), nl, q, m->Yt.as<double>(), s)) != LOS_OK) return rc;
    E::GemmF64 b{n, q, nl, X, ld, 1, m->Yq.as<double>(), q, 1, m->Zq.as<double>(), q};
    HIPCHK(E::gemm_f64(b, s), "emulator: X Q");
    if ((rc = orth(m, m->Zq.as<double>(), n, q, m->Bm.as<double>(), s)) != LOS_OK) return rc;
    E::GemmF64 c{nl, q, n, X, 1, ld, m->Zq.as<double>(), q, 1, m->Yq.as<double>(), q};
    HIPCHK(E::gemm_f64(c, s), "emulator: X^T Z");
  }
  if ((rc = orth(m, m->Yq.as<double>(), nl, q, m->Yt.as<double>(), s)) != LOS_OK) return rc;
  // Rayleigh-Ritz: (X Q)^T (X Q) = U diag U^T
  E::GemmF64 d{n, q, nl, X, ld, 1, m->Yq.as<double>(), q, 1, m->Bm.as<double>(), q};
  HIPCHK(E::gemm_f64(d, s), "emulator: X Q");
  E::GemmF64 gm{q, q, n, m->Bm.as<double>(), 1, q, m->Bm.as<double>(), q, 1, m->G.as<double>(), q};
  HIPCHK(E::gemm_f64(gm, s), "emulator: Ritz Gram");
  HIPCHK(E::jacobi_eig(m->G.as<double>(), q, 12, m->Vj.as<double>(), m->ev.as<double>(),
                       m->U.as<double>(), s),
         "emulator: Jacobi");
  double *basis = m->basis.as<double>() + (int64_t)sp * nl * m->ncomp;
  E::GemmF64 bb{nl, m->ncomp, q, m->Yq.as<double>(), q, 1, m->U.as<double>(), q, 1, basis, m->ncomp};
  HIPCHK(E::gemm_f64(bb, s), "emulator: basis");
  // coefficients and whitened targets
  E::GemmF64 cf{n, m->ncomp, nl, X, ld, 1, basis, m->ncomp, 1, m->cfs.as<double>(), m->ncomp};
  HIPCHK(E::gemm_f64(cf, s), "emulator: coefficients");
  HIPCHK(E::whiten(m->cfs.as<double>(), n, m->ncomp, sp, m->nout, m->sigma.as<double>(),
                   m->zb.as<float>(), s),
         "emulator: whiten");
  return LOS_OK;
}

int refresh_float_pca(los_emu *m, hipStream_t s) {
  std::vector<double> b((size_t)4 * m->nl * m->ncomp), mu((size_t)4 * m->nl);
  HIPCHK(hipMemcpyAsync(b.data(), m->basis.p, sizeof(double) * b.size(), hipMemcpyDeviceToHost, s),
         "emulator: basis copy");
  HIPCHK(hipMemcpyAsync(mu.data(), m->mean.p, sizeof(double) * mu.size(), hipMemcpyDeviceToHost, s),
         "emulator: mean copy");
  HIPCHK(hipStreamSynchronize(s), "emulator: sync");
  std::vector<float> bf(b.begin(), b.end()), mf(mu.begin(), mu.end());
  HIPCHK(hipMemcpy(m->basis_f.p, bf.data(), sizeof(float) * bf.size(), hipMemcpyHostToDevice),
         "emulator: basis copy");
  HIPCHK(hipMemcpy(m->mean_f.p, mf.data(), sizeof(float) * mf.size(), hipMemcpyHostToDevice),
         "emulator: mean copy");
  return LOS_OK;
}

}  // namespace

extern "C" {

int emu_create(los_ctx *ctx, int32_t nparam, int32_t nl, int32_t ncomp, int32_t width,
               int32_t depth, int32_t members, uint64_t seed, los_emu **out) {
  if (!out) return fail(LOS_ERR_INVALID, "emu_create: out is NULL");
  *out = nullptr;
  if (!ctx) return fail(LOS_ERR_INVALID, "emu_create: ctx is NULL");
  if (nparam < 1 || nparam > 64) return fail(LOS_ERR_INVALID, "emu_create: nparam = %d", nparam);
  if (nl < 1 || nl > 20000) return fail(LOS_ERR_INVALID, "emu_create: nl = %d", nl);
  if (ncomp < 1 || ncomp + 8 > E::kMaxQ || ncomp > nl)
    return fail(LOS_ERR_INVALID, "emu_create: ncomp = %d out of [1, %d] or above nl", ncomp,
                E::kMaxQ - 8);
  if (width < 1 || width > 4096 || depth < 1 || depth > 16)
    return fail(LOS_ERR_INVALID, "emu_create: width %d / depth %d out of range", width, depth);
  if (members < 1 || members > 16) return fail(LOS_ERR_INVALID, "emu_create: members = %d", members);
  los_emu *m = new (std::nothrow) los_emu;
  if (!m) return fail(LOS_ERR_OOM, "emu_create: out of host memory");
  (void)hipGetDevice(&m->device);
  m->np = nparam;
  m->nl = nl;
  m->ncomp = ncomp;
  m->width = width;
  m->depth = depth;
  m->members = members;
  m->nout = 4 * ncomp;
  m->seed = seed;
  m->sizes.push_back(nparam);
  for (int i = 0; i < depth; ++i) m->sizes.push_back(width);
  m->sizes.push_back(m->nout);
  int64_t off = 0;
  for (int i = 0; i + 1 < (int)m->sizes.size(); ++i) {
    m->woff.push_back(off);
    off += (int64_t)m->sizes[i] * m->sizes[i + 1] + m->sizes[i + 1];
  }
  m->nparams = off;
  const size_t P = (size_t)m->nparams * members;
  int rc = m->theta.reserve(sizeof(float) * P);
  if (rc == LOS_OK) rc = m->adam_m.reserve(sizeof(float) * P);
  if (rc == LOS_OK) rc = m->adam_v.reserve(sizeof(float) * P);
  if (rc == LOS_OK) rc = m->grad.reserve(sizeof(float) * m->nparams);
  if (rc == LOS_OK) rc = m->lo.reserve(sizeof(double) * nparam);
  if (rc == LOS_OK) rc = m->hi.reserve(sizeof(double) * nparam);
  if (rc == LOS_OK) rc = m->mean.reserve(sizeof(double) * 4 * nl);
  if (rc == LOS_OK) rc = m->mean_f.reserve(sizeof(float) * 4 * nl);
  if (rc == LOS_OK) rc = m->basis.reserve(sizeof(double) * 4 * (size_t)nl * ncomp);
  if (rc == LOS_OK) rc = m->basis_f.reserve(sizeof(float) * 4 * (size_t)nl * ncomp);
  if (rc == LOS_OK) rc = m->sigma.reserve(sizeof(double) * 4 * ncomp);
  if (rc == LOS_OK) rc = m->tscale.reserve(sizeof(double) * nl);
  if (rc == LOS_OK) rc = m->st.reserve(sizeof(int) * 4);
  for (int e = 0; e < members && rc == LOS_OK; ++e) rc = init_member(m, e);
  if (rc != LOS_OK) {
    delete m;
    return rc;
  }
  *out = m;
  return ok();
}

void emu_destroy(los_emu *emu) { delete emu; }

int emu_nparams(const los_emu *emu, int64_t *count) {
  if (!emu || !count) return fail(LOS_ERR_INVALID, "emu_nparams: NULL argument");
  *count = emu->nparams;
  return ok();
}

int emu_get_params(const los_emu *emu, int32_t member, float *host) {
  if (!emu || !host || member < 0 || member >= emu->members)
    return fail(LOS_ERR_INVALID, "emu_get_params: bad argument");
  HIPCHK(hipMemcpy(host, emu->theta.as<float>() + (int64_t)member * emu->nparams,
                   sizeof(float) * emu->nparams, hipMemcpyDeviceToHost),
         "emu_get_params");
  return ok();
}

int emu_set_params(los_emu *emu, int32_t member, const float *host) {
  if (!emu || !host || member < 0 || member >= emu->members)
    return fail(LOS_ERR_INVALID, "emu_set_params: bad argument");
  HIPCHK(hipMemcpy(emu->theta.as<float>() + (int64_t)member * emu->nparams, host,
                   sizeof(float) * emu->nparams, hipMemcpyHostToDevice),
         "emu_set_params");
  return ok();
}

int emu_forward(los_emu *emu, int32_t member, const float *u, int64_t n, float *out,
                void *stream) {
  if (!emu || !u || !out || n < 1 || member < 0 || member >= emu->members)
    return fail(LOS_ERR_INVALID, "emu_forward: bad argument");
  int rc = forward(emu, member, u, n, out, (hipStream_t)stream);
  return rc == LOS_OK ? ok() : rc;
}

int emu_loss_grad(los_emu *emu, int32_t member, const float *u, const float *z, int64_t n,
                  float *loss, float *grad, void *stream) {
  if (!emu || !u || !z || !loss || !grad || n < 1 || member < 0 || member >= emu->members)
    return fail(LOS_ERR_INVALID, "emu_loss_grad: bad argument");
  hipStream_t s = (hipStream_t)stream;
  int rc = loss_grad(emu, member, u, z, n, loss, 0, s);
  if (rc != LOS_OK) return rc;
  HIPCHK(hipMemcpyAsync(grad, emu->grad.p, sizeof(float) * emu->nparams, hipMemcpyDeviceToDevice, s),
         "emu_loss_grad: copy");
  return ok();
}

int emu_fit(los_emu *emu, int32_t member, const float *u, const float *z, int64_t n,
            int32_t epochs, int32_t batch, double lr, float *loss_hist, void *stream) {
  if (!emu || !u || !z || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.0) || member < 0 ||
      member >= emu->members)
    return fail(LOS_ERR_INVALID, "emu_fit: bad argument");
  int rc = fit_member(emu, member, u, z, n, epochs, batch, lr, loss_hist, (hipStream_t)stream);
  return rc == LOS_OK ? ok() : rc;
}

int emu_set_pca(los_emu *emu, const double *lo, const double *hi, const double *mean,
                const double *basis, const double *sigma, const double *te_scale) {
  if (!emu || !lo || !hi || !mean || !basis || !sigma || !te_scale)
    return fail(LOS_ERR_INVALID, "emu_set_pca: NULL argument");
  const size_t nl = emu->nl, nc = emu->ncomp;
  HIPCHK(hipMemcpy(emu->lo.p, lo, sizeof(double) * emu->np, hipMemcpyHostToDevice), "emu_set_pca");
  HIPCHK(hipMemcpy(emu->hi.p, hi, sizeof(double) * emu->np, hipMemcpyHostToDevice), "emu_set_pca");
  HIPCHK(hipMemcpy(emu->mean.p, mean, sizeof(double) * 4 * nl, hipMemcpyHostToDevice), "emu_set_pca");
  HIPCHK(hipMemcpy(emu->basis.p, basis, sizeof(double) * 4 * nl * nc, hipMemcpyHostToDevice),
         "emu_set_pca");
  HIPCHK(hipMemcpy(emu->sigma.p, sigma, sizeof(double) * 4 * nc, hipMemcpyHostToDevice),
         "emu_set_pca");
  HIPCHK(hipMemcpy(emu->tscale.p, te_scale, sizeof(double) * nl, hipMemcpyHostToDevice),
         "emu_set_pca");
  int rc = refresh_float_pca(emu, nullptr);
  if (rc != LOS_OK) return rc;
  emu->has_pca = true;
  return ok();
}

int emu_get_pca(const los_emu *emu, double *lo, double *hi, double *mean, double *basis,
                double *sigma, double *te_scale) {
  if (!emu || !lo || !hi || !mean || !basis || !sigma || !te_scale)
    return fail(LOS_ERR_INVALID, "emu_get_pca: NULL argument");
  if (!emu->has_pca) return fail(LOS_ERR_INVALID, "emu_get_pca: emulator has no PCA yet");
  const size_t nl = emu->nl, nc = emu->ncomp;
  HIPCHK(hipMemcpy(lo, emu->lo.p, sizeof(double) * emu->np, hipMemcpyDeviceToHost), "emu_get_pca");
  HIPCHK(hipMemcpy(hi, emu->hi.p, sizeof(double) * emu->np, hipMemcpyDeviceToHost), "emu_get_pca");
  HIPCHK(hipMemcpy(mean, emu->mean.p, sizeof(double) * 4 * nl, hipMemcpyDeviceToHost), "emu_get_pca");
  HIPCHK(hipMemcpy(basis, emu->basis.p, sizeof(double) * 4 * nl * nc, hipMemcpyDeviceToHost),
         "emu_get_pca");
  HIPCHK(hipMemcpy(sigma, emu->sigma.p, sizeof(double) * 4 * nc, hipMemcpyDeviceToHost),
         "emu_get_pca");
  HIPCHK(hipMemcpy(te_scale, emu->tscale.p, sizeof(double) * nl, hipMemcpyDeviceToHost),
         "emu_get_pca");
  return ok();
}

int emu_train(los_emu *emu, const double *params, const double *lo, const double *hi,
              const double *cl, int64_t n, int32_t epochs, int32_t batch, double lr,
              float *loss_hist, void *stream) {
  if (!emu || !params || !lo || !hi || !cl) return fail(LOS_ERR_INVALID, "emu_train: NULL argument");
  if (n < emu->ncomp + 8 || epochs < 1 || batch < 1 || !(lr > 0.0))
    return fail(LOS_ERR_INVALID, "emu_train: need n >= ncomp + 8, epochs, batch >= 1, lr > 0");
  for (int j = 0; j < emu->np; ++j)
    if (!(hi[j] > lo[j])) return fail(LOS_ERR_INVALID, "emu_train: hi[%d] <= lo[%d]", j, j);
  hipStream_t s = (hipStream_t)stream;
  los_emu *m = emu;
  const int q = std::min(m->ncomp + 8, E::kMaxQ);
  const int64_t nl = m->nl;
  int rc = m->y.reserve(sizeof(double) * (size_t)n * 4 * nl);
  if (rc == LOS_OK) rc = m->Om.reserve(sizeof(double) * (size_t)n * q);
  if (rc == LOS_OK) rc = m->Yq.reserve(sizeof(double) * (size_t)nl * q);
  if (rc == LOS_OK) rc = m->Yt.reserve(sizeof(double) * (size_t)std::max<int64_t>(nl, n) * q);
  if (rc == LOS_OK) rc = m->Zq.reserve(sizeof(double) * (size_t)n * q);
  if (rc == LOS_OK) rc = m->Bm.reserve(sizeof(double) * (size_t)std::max<int64_t>(nl, n) * q);
  if (rc == LOS_OK) rc = m->G.reserve(sizeof(double) * q * q);
  if (rc == LOS_OK) rc = m->Rinv.reserve(sizeof(double) * q * q);
  if (rc == LOS_OK) rc = m->U.reserve(sizeof(double) * q * q);
  if (rc == LOS_OK) rc = m->Vj.reserve(sizeof(double) * q * q);
  if (rc == LOS_OK) rc = m->ev.reserve(sizeof(double) * q);
  if (rc == LOS_OK) rc = m->cfs.reserve(sizeof(double) * (size_t)n * m->ncomp);
  if (rc == LOS_OK) rc = m->zb.reserve(sizeof(float) * (size_t)n * m->nout);
  if (rc == LOS_OK) rc = m->cz.reserve(sizeof(float) * (size_t)n * m->np);
  if (rc != LOS_OK) return rc;
  HIPCHK(hipMemcpy(m->lo.p, lo, sizeof(double) * m->np, hipMemcpyHostToDevice), "emu_train: lo");
  HIPCHK(hipMemcpy(m->hi.p, hi, sizeof(double) * m->np, hipMemcpyHostToDevice), "emu_train: hi");
  // random test matrix for the range finder, uniform on [-1, 1) from SplitMix64
  {
    std::vector<double> om((size_t)n * q);
    uint64_t st = m->seed ^ 0x2545F4914F6CDD1Dull;
    for (auto &v : om) v = 2.0 * unit(st) - 1.0;
    HIPCHK(hipMemcpy(m->Om.p, om.data(), sizeof(double) * om.size(), hipMemcpyHostToDevice),
           "emu_train: test matrix");
  }
  HIPCHK(hipMemsetAsync(m->st.p, 0, sizeof(int) * 4, s), "emu_train: status");
  HIPCHK(E::te_median(cl, n, (int)nl, m->tscale.as<double>(), s), "emu_train: TE scale");
  HIPCHK(E::transform(cl, n, (int)nl, m->tscale.as<double>(), m->y.as<double>(), s),
         "emu_train: transform");
  for (int sp = 0; sp < 4; ++sp)
    if ((rc = pca_spectrum(m, sp, n, s)) != LOS_OK) return rc;
  if ((rc = refresh_float_pca(m, s)) != LOS_OK) return rc;
  m->has_pca = true;
  HIPCHK(E::scale_params(params, n, m->np, m->lo.as<double>(), m->hi.as<double>(),
                         m->cz.as<float>(), s),
         "emu_train: inputs");
  for (int e = 0; e < m->members; ++e) {
    if ((rc = init_member(m, e)) != LOS_OK) return rc;
    rc = fit_member(m, e, m->cz.as<float>(), m->zb.as<float>(), n, epochs, batch, lr,
                    loss_hist ? loss_hist + (int64_t)e * epochs : nullptr, s);
    if (rc != LOS_OK) return rc;
  }
  return ok();
}

// Inference shared by emu_infer (per-model estimates) and emu_infer_spectra
// (per-spectrum estimates): any of err, need, err4, need4 may be NULL.
static int infer(los_emu *emu, const char *who, const double *params, int64_t n, double *cl,
                 float *err, uint8_t *need, float *err4, uint8_t *need4, double threshold,
                 void *stream) {
  if (!emu->has_pca) return fail(LOS_ERR_INVALID, "%s: emulator is not trained", who);
  hipStream_t s = (hipStream_t)stream;
  los_emu *m = emu;
  const int64_t nl = m->nl;
  int rc = m->ut.reserve(sizeof(float) * (size_t)n * m->np);
  if (rc == LOS_OK) rc = m->zt.reserve(sizeof(float) * (size_t)n * m->nout);
  if (rc == LOS_OK) rc = m->yall.reserve(sizeof(float) * (size_t)m->members * n * 4 * nl);
  if (rc == LOS_OK) rc = m->cz.reserve(sizeof(float) * (size_t)n * std::max(m->ncomp, m->np));
  if (rc == LOS_OK) rc = m->errb.reserve(sizeof(unsigned int) * 4 * (size_t)n);
  if (rc != LOS_OK) return rc;
  HIPCHK(E::scale_params(params, n, m->np, m->lo.as<double>(), m->hi.as<double>(),
                         m->ut.as<float>(), s),
         "emu_infer: inputs");
  for (int e = 0; e < m->members; ++e) {
    if ((rc = forward(m, e, m->ut.as<float>(), n, m->zt.as<float>(), s)) != LOS_OK) return rc;
    for (int sp = 0; sp < 4; ++sp) {
      HIPCHK(E::unwhiten(m->zt.as<float>(), n, m->ncomp, sp, m->nout, m->sigma.as<double>(),
                         m->cz.as<float>(), s),
             "emu_infer: unwhiten");
      E::GemmF32 g{};  // y = mean + cz basis^T
      g.M = n;
      g.N = nl;
      g.K = m->ncomp;
      g.A = m->cz.as<float>();
      g.sam = m->ncomp;
      g.sak = 1;
      g.B = m->basis_f.as<float>() + (int64_t)sp * nl * m->ncomp;
      g.sbk = 1;
      g.sbn = m->ncomp;
      g.C = m->yall.as<float>() + ((int64_t)e * n * 4 + sp) * nl;
      g.ldc = 4 * nl;
      g.bias = m->mean_f.as<float>() + (int64_t)sp * nl;
      HIPCHK(E::gemm_f32(g, E::kEpiBias, s), "emu_infer: reconstruction");
    }
  }
  HIPCHK(E::ensemble(m->yall.as<float>(), m->members, n, (int)nl, m->tscale.as<double>(), cl,
                     m->errb.as<unsigned int>(), (float)threshold, err, need, err4, need4, s),
         "emu_infer: ensemble");
  rc = los::check_result(who, cl, n * 4 * nl, false, s);
  return rc == LOS_OK ? ok() : rc;
}

int emu_infer(los_emu *emu, const double *params, int64_t n, double *cl, float *err,
              uint8_t *need_fallback, double threshold, void *stream) {
  if (!emu || !params || !cl || !err || !need_fallback || n < 1)
    return fail(LOS_ERR_INVALID, "emu_infer: bad argument");
  return infer(emu, "emu_infer", params, n, cl, err, need_fallback, nullptr, nullptr, threshold,
               stream);
}

int emu_infer_spectra(los_emu *emu, const double *params, int64_t n, double *cl, float *err4,
                      uint8_t *need4, double threshold, void *stream) {
  if (!emu || !params || !cl || !err4 || !need4 || n < 1)
    return fail(LOS_ERR_INVALID, "emu_infer_spectra: bad argument");
  return infer(emu, "emu_infer_spectra", params, n, cl, nullptr, nullptr, err4, need4, threshold,
               stream);
}

}  // extern "C"

// ---------------------------------------------------------------- checkpoints
//
// File layout (host byte order), version 1:
//   char magic[8] = "LOSEMU01"; uint32 version; int32 np, nl, ncomp, width,
//   depth, members, 0; uint64 seed; int64 nparams; int32 has_pca; int32 0
//   (64 bytes);
//   float theta[members][nparams], adam_m[...], adam_v[...];
//   if has_pca: double lo[np], hi[np], mean[4][nl], basis[4][nl][ncomp],
//               sigma[4][ncomp], te_scale[nl];
//   uint64 FNV-1a hash of every byte before it.

namespace {

constexpr char kEmuMagic[8] = {'L', 'O', 'S', 'E', 'M', 'U', '0', '1'};
constexpr uint32_t kEmuVersion = 1;

struct EmuHeader {  // 64 bytes, no implicit padding
  char magic[8];
  uint32_t version;
  int32_t np, nl, ncomp, width, depth, members;
  int32_t pad0;
  uint64_t seed;
  int64_t nparams;
  int32_t has_pca, reserved;
};
static_assert(sizeof(EmuHeader) == 64, "checkpoint header layout");

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

// The device arrays of a checkpoint, in file order: (buffer, bytes).
std::vector<std::pair<void *, size_t>> emu_sections(const los_emu *m) {
  const size_t P = (size_t)m->nparams * m->members, nl = m->nl, nc = m->ncomp;
  std::vector<std::pair<void *, size_t>> v = {{m->theta.p, sizeof(float) * P},
                                              {m->adam_m.p, sizeof(float) * P},
                                              {m->adam_v.p, sizeof(float) * P}};
  if (m->has_pca) {
    v.push_back({m->lo.p, sizeof(double) * m->np});
    v.push_back({m->hi.p, sizeof(double) * m->np});
    v.push_back({m->mean.p, sizeof(double) * 4 * nl});
    v.push_back({m->basis.p, sizeof(double) * 4 * nl * nc});
    v.push_back({m->sigma.p, sizeof(double) * 4 * nc});
    v.push_back({m->tscale.p, sizeof(double) * nl});
  }
  return v;
}

}  // namespace

extern "C" {

int emu_save(const los_emu *emu, const char *path, void *stream) {
  if (!emu || !path) return fail(LOS_ERR_INVALID, "emu_save: NULL argument");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream), "emu_save: stream");
  EmuHeader h{};
  std::memcpy(h.magic, kEmuMagic, 8);
  h.version = kEmuVersion;
  h.np = emu->np;
  h.nl = emu->nl;
  h.ncomp = emu->ncomp;
  h.width = emu->width;
  h.depth = emu->depth;
  h.members = emu->members;
  h.seed = emu->seed;
  h.nparams = emu->nparams;
  h.has_pca = emu->has_pca ? 1 : 0;
  std::vector<char> buf(sizeof h);
  std::memcpy(buf.data(), &h, sizeof h);
  for (const auto &sec : emu_sections(emu)) {
    const size_t at = buf.size();
    buf.resize(at + sec.second);
    HIPCHK(hipMemcpy(buf.data() + at, sec.first, sec.second, hipMemcpyDeviceToHost),
           "emu_save: copy");
  }
  const uint64_t hash = fnv1a(0xCBF29CE484222325ull, buf.data(), buf.size());
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(LOS_ERR_INVALID, "emu_save: cannot open %s for writing", path);
  const bool okw = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size() &&
                   std::fwrite(&hash, sizeof hash, 1, f) == 1;
  const bool okc = std::fclose(f) == 0;
  if (!okw || !okc) return fail(LOS_ERR_INVALID, "emu_save: write to %s failed", path);
  return ok();
}

int emu_load(los_ctx *ctx, const char *path, los_emu **out) {
  if (!out) return fail(LOS_ERR_INVALID, "emu_load: out is NULL");
  *out = nullptr;
  if (!ctx || !path) return fail(LOS_ERR_INVALID, "emu_load: NULL argument");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(LOS_ERR_INVALID, "emu_load: cannot open %s", path);
  std::vector<char> buf;
  char tmp[1 << 16];
  size_t got;
  while ((got = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
  std::fclose(f);
  EmuHeader h{};
  if (buf.size() < sizeof h + sizeof(uint64_t))
    return fail(LOS_ERR_INVALID, "emu_load: %s is too short to be an emulator file", path);
  std::memcpy(&h, buf.data(), sizeof h);
  if (std::memcmp(h.magic, kEmuMagic, 8) != 0)
    return fail(LOS_ERR_INVALID, "emu_load: %s is not an emulator file", path);
  if (h.version != kEmuVersion)
    return fail(LOS_ERR_UNSUPPORTED, "emu_load: %s has version %u (this library reads %u)", path,
                h.version, kEmuVersion);
  uint64_t hash;
  std::memcpy(&hash, buf.data() + buf.size() - sizeof hash, sizeof hash);
  if (fnv1a(0xCBF29CE484222325ull, buf.data(), buf.size() - sizeof hash) != hash)
    return fail(LOS_ERR_INVALID, "emu_load: %s is corrupt (checksum mismatch)", path);
  los_emu *m = nullptr;
  int rc = emu_create(ctx, h.np, h.nl, h.ncomp, h.width, h.depth, h.members, h.seed, &m);
  if (rc != LOS_OK) return rc;
  if (m->nparams != h.nparams) {
    emu_destroy(m);
    return fail(LOS_ERR_INVALID, "emu_load: %s holds %lld parameters per member, the shape "
                "gives %lld", path, (long long)h.nparams, (long long)m->nparams);
  }
  m->has_pca = h.has_pca != 0;
  size_t at = sizeof h;
  const auto secs = emu_sections(m);
  size_t need = at + sizeof hash;
  for (const auto &sec : secs) need += sec.second;
  if (need != buf.size()) {
    emu_destroy(m);
    return fail(LOS_ERR_INVALID, "emu_load: %s has %zu bytes, its header implies %zu", path,
                buf.size(), need);
  }
  for (const auto &sec : secs) {
    hipError_t e = hipMemcpy(sec.first, buf.data() + at, sec.second, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      emu_destroy(m);
      return hip_fail(e, "emu_load: copy");
    }
    at += sec.second;
  }
  if (m->has_pca && (rc = refresh_float_pca(m, nullptr)) != LOS_OK) {
    emu_destroy(m);
    return rc;
  }
  *out = m;
  return ok();
}

int emu_merge(los_emu *emu, const int64_t *rows, int64_t nf, const double *cl_solved, double *cl,
              int64_t n, float *err, uint8_t *need_fallback, void *stream) {
  if (!emu || nf < 0 || n < 1) return fail(LOS_ERR_INVALID, "emu_merge: bad argument");
  if (nf == 0) return ok();
  if (!rows || !cl_solved || !cl) return fail(LOS_ERR_INVALID, "emu_merge: NULL array");
  if (nf > n) return fail(LOS_ERR_INVALID, "emu_merge: nf = %lld > n = %lld", (long long)nf,
                          (long long)n);
  std::vector<char> seen((size_t)n, 0);
  for (int64_t i = 0; i < nf; ++i) {
    if (rows[i] < 0 || rows[i] >= n)
      return fail(LOS_ERR_INVALID, "emu_merge: rows[%lld] = %lld out of [0, %lld)", (long long)i,
                  (long long)rows[i], (long long)n);
    if (seen[(size_t)rows[i]]++)
      return fail(LOS_ERR_INVALID, "emu_merge: row %lld given twice", (long long)rows[i]);
  }
  hipStream_t s = (hipStream_t)stream;
  int rc = emu->rows.reserve(sizeof(int64_t) * (size_t)nf);
  if (rc != LOS_OK) return rc;
  HIPCHK(hipMemcpyAsync(emu->rows.p, rows, sizeof(int64_t) * (size_t)nf, hipMemcpyHostToDevice, s),
         "emu_merge: rows");
  HIPCHK(E::merge_rows(emu->rows.as<int64_t>(), nf, cl_solved, 4 * (int64_t)emu->nl, cl, err,
                       need_fallback, s),
         "emu_merge: launch");
  return ok();
}

int emu_merge_spectrum(los_emu *emu, int32_t spectrum, const int64_t *rows, int64_t nf,
                       const double *cl_solved, double *cl, int64_t n, float *err4,
                       uint8_t *need4, void *stream) {
  if (!emu || nf < 0 || n < 1 || spectrum < 0 || spectrum > 3)
    return fail(LOS_ERR_INVALID, "emu_merge_spectrum: bad argument");
  if (nf == 0) return ok();
  if (!rows || !cl_solved || !cl) return fail(LOS_ERR_INVALID, "emu_merge_spectrum: NULL array");
  if (nf > n)
    return fail(LOS_ERR_INVALID, "emu_merge_spectrum: nf = %lld > n = %lld", (long long)nf,
                (long long)n);
  std::vector<char> seen((size_t)n, 0);
  for (int64_t i = 0; i < nf; ++i) {
    if (rows[i] < 0 || rows[i] >= n)
      return fail(LOS_ERR_INVALID, "emu_merge_spectrum: rows[%lld] = %lld out of [0, %lld)",
                  (long long)i, (long long)rows[i], (long long)n);
    if (seen[(size_t)rows[i]]++)
      return fail(LOS_ERR_INVALID, "emu_merge_spectrum: row %lld given twice",
                  (long long)rows[i]);
  }
  hipStream_t s = (hipStream_t)stream;
  int rc = emu->rows.reserve(sizeof(int64_t) * (size_t)nf);
  if (rc != LOS_OK) return rc;
  HIPCHK(hipMemcpyAsync(emu->rows.p, rows, sizeof(int64_t) * (size_t)nf, hipMemcpyHostToDevice, s),
         "emu_merge_spectrum: rows");
  HIPCHK(E::merge_spectrum(emu->rows.as<int64_t>(), nf, cl_solved, emu->nl, spectrum, cl, err4,
                           need4, s),
         "emu_merge_spectrum: launch");
  return ok();
}

}  // extern "C"
