// Host side of the C ABI declared in include/los.h: argument validation,
// error reporting, the per-context device workspace, and kernel launches on
// the caller's stream.
#include "los.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "los_internal.hpp"

struct los_ctx {
  int device = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return LOS_OK;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(LOS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Grow the context workspace to at least `bytes` (never shrinks).
int ws_reserve(los_ctx *ctx, size_t bytes, void **out) {
  if (bytes <= ctx->ws_bytes) {
    *out = ctx->ws;
    return LOS_OK;
  }
  if (ctx->ws) {
    hipError_t e = hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
  }
  size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
  hipError_t e = hipMalloc(&ctx->ws, want);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    return fail(LOS_ERR_OOM, "workspace allocation of %zu bytes failed: %s", want,
                hipGetErrorString(e));
  }
  ctx->ws_bytes = want;
  *out = ctx->ws;
  return LOS_OK;
}

int env_int(const char *name) {
  const char *v = std::getenv(name);
  return v ? std::atoi(v) : 0;
}

}  // namespace

extern "C" {

const char *los_last_error(void) { return g_err.c_str(); }

const char *los_version(void) { return "los-mi355x 0.1 (gfx950)"; }

int los_ctx_create(los_ctx **ctx) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_ctx_create: ctx is NULL");
  *ctx = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  los_ctx *c = new (std::nothrow) los_ctx;
  if (!c) return fail(LOS_ERR_OOM, "los_ctx_create: out of host memory");
  c->device = dev;
  *ctx = c;
  return ok();
}

void los_ctx_destroy(los_ctx *ctx) {
  if (!ctx) return;
  if (ctx->ws) (void)hipFree(ctx->ws);
  delete ctx;
}

int los_bessel_table(los_ctx *ctx, const double *x, int64_t nx, int32_t lmin, int32_t lmax,
                     double *out, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_bessel_table: ctx is NULL");
  if (nx < 0) return fail(LOS_ERR_INVALID, "los_bessel_table: nx = %lld < 0", (long long)nx);
  if (lmin < 0 || lmax < lmin || lmax > 30000)
    return fail(LOS_ERR_INVALID, "los_bessel_table: need 0 <= lmin <= lmax <= 30000 (got %d, %d)",
                lmin, lmax);
  if (nx == 0) return ok();
  if (!x || !out) return fail(LOS_ERR_INVALID, "los_bessel_table: NULL array");
  if (nx > (int64_t)1 << 40) return fail(LOS_ERR_INVALID, "los_bessel_table: nx too large");
  hipError_t e = los::bessel_table_launch(x, nx, lmin, lmax, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "los_bessel_table launch");
  return ok();
}

int los_project(los_ctx *ctx, int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                const double *k, const double *tau, const double *w_tau, const void *S,
                int32_t nsrc, int32_t prec, void *delta, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_project: ctx is NULL");
  if (lmin < 2 || lmax < lmin || lmax > 16000)
    return fail(LOS_ERR_INVALID, "los_project: need 2 <= lmin <= lmax <= 16000 (got %d, %d)",
                lmin, lmax);
  if (nk < 1 || nk > ((int64_t)1 << 31) - 1)
    return fail(LOS_ERR_INVALID, "los_project: nk = %lld out of range", (long long)nk);
  if (ntau < 1 || ntau > 8192)
    return fail(LOS_ERR_INVALID, "los_project: ntau = %lld out of [1, 8192]", (long long)ntau);
  if (nsrc < 1 || nsrc > 4)
    return fail(LOS_ERR_INVALID, "los_project: nsrc = %d out of [1, 4]", nsrc);
  if (!(tau0 == tau0)) return fail(LOS_ERR_INVALID, "los_project: tau0 is NaN");
  if (!k || !tau || !w_tau || !S || !delta)
    return fail(LOS_ERR_INVALID, "los_project: NULL array");
  if (prec != LOS_FP64 && prec != LOS_FP32 && prec != LOS_BF16X3)
    return fail(LOS_ERR_INVALID, "los_project: unknown precision %d", prec);
  if (prec != LOS_FP64)
    return fail(LOS_ERR_UNSUPPORTED, "los_project: precision %d is not implemented", prec);

  los::ProjectShape sh =
      los::project_fp64_shape(nsrc, ntau, env_int("LOS_PROJ_WAVES"), env_int("LOS_PROJ_SLOTS"));
  if (sh.waves == 0)
    return fail(LOS_ERR_UNSUPPORTED, "los_project: no launch shape for ntau = %lld",
                (long long)ntau);
  if (sh.lds > 160 * 1024)
    return fail(LOS_ERR_UNSUPPORTED, "los_project: needs %zu bytes of LDS", sh.lds);
  los::ProjectArgs a{};
  a.lmin = lmin;
  a.lmax = lmax;
  a.nl = lmax - lmin + 1;
  a.nblk = (a.nl + los::kProjectBlock - 1) / los::kProjectBlock;
  a.nk = nk;
  a.ntau = ntau;
  a.tau0 = tau0;
  a.k = k;
  a.tau = tau;
  a.w = w_tau;
  a.S = (const double *)S;
  a.delta = (double *)delta;
  hipError_t e = los::project_fp64_launch(a, nsrc, sh, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "los_project launch");
  return ok();
}

int cl_integrate(los_ctx *ctx, const void *delta, int32_t delta_prec, int32_t nsrc, int32_t nl,
                 int64_t nk, const double *w_lnk, const double *Pk, const int32_t *pairs,
                 int32_t npairs, double *cl, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "cl_integrate: ctx is NULL");
  if (nsrc < 1 || nsrc > 4) return fail(LOS_ERR_INVALID, "cl_integrate: nsrc = %d", nsrc);
  if (nl < 1) return fail(LOS_ERR_INVALID, "cl_integrate: nl = %d", nl);
  if (nk < 1) return fail(LOS_ERR_INVALID, "cl_integrate: nk = %lld", (long long)nk);
  if (npairs < 1 || npairs > 16)
    return fail(LOS_ERR_INVALID, "cl_integrate: npairs = %d out of [1, 16]", npairs);
  if (!delta || !w_lnk || !Pk || !pairs || !cl)
    return fail(LOS_ERR_INVALID, "cl_integrate: NULL array");
  if (delta_prec != LOS_FP64 && delta_prec != LOS_FP32)
    return fail(LOS_ERR_INVALID, "cl_integrate: delta_prec must be LOS_FP64 or LOS_FP32");
  los::ClArgs a{};
  for (int p = 0; p < npairs; ++p) {
    if (pairs[2 * p] < 0 || pairs[2 * p] >= nsrc || pairs[2 * p + 1] < 0 ||
        pairs[2 * p + 1] >= nsrc)
      return fail(LOS_ERR_INVALID, "cl_integrate: pair %d = (%d, %d) out of [0, %d)", p,
                  pairs[2 * p], pairs[2 * p + 1], nsrc);
    a.pa[p] = pairs[2 * p];
    a.pb[p] = pairs[2 * p + 1];
  }
  a.delta = delta;
  a.delta_f32 = delta_prec == LOS_FP32;
  a.nsrc = nsrc;
  a.nl = nl;
  a.npairs = npairs;
  a.nk = nk;
  a.w = w_lnk;
  a.P = Pk;
  a.cl = cl;
  a.nseg = los::cl_segments(nk, nl);
  void *ws = nullptr;
  int rc = ws_reserve(ctx, sizeof(double) * (size_t)a.nseg * npairs * nl, &ws);
  if (rc != LOS_OK) return rc;
  a.partial = (double *)ws;
  hipError_t e = los::cl_launch(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "cl_integrate launch");
  return ok();
}

}  // extern "C"
