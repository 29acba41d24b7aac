// Host side of the C ABI declared in include/los.h: argument validation,
// error reporting, the per-context device workspace, and kernel launches on
// the caller's stream.
#include "los.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "los_internal.hpp"

// Workspace slots of a context: the C_l partial sums and the Bessel tables
// of the MFMA projection live in separate buffers, so a C_l call queued
// behind a projection never reallocates memory the projection still reads.
enum { WS_CL = 0, WS_JTAB = 1, WS_SPLINE = 2, WS_LSEL = 3, WS_CLI = 4, WS_TENSOR = 5, WS_COUNT = 6 };

struct los_ctx {
  int device = 0;
  std::string tune_cache;   // batch autotune cache file ("" = none)
  void *scratch = nullptr;  // device address of `scratch` on this device (cl_integrate_noalloc)
  void *ws[WS_COUNT] = {};
  size_t ws_bytes[WS_COUNT] = {};
  // multipole list whose sample tables are in WS_LSEL ({lmin, lmax, ls...})
  std::vector<int32_t> lsel_key;
  // multipole list whose knots (as doubles) are in WS_CLI
  std::vector<int32_t> cli_key;
};

namespace {
thread_local std::string g_err;
}  // namespace

// Device memory of the entry point that allocates nothing (cl_integrate_noalloc):
// room for the partial sums of the C_l reduction.  Each GPU the library runs on
// holds its own copy until the process ends; every call on a GPU shares it.
// In host code `scratch` is only a stand-in for the symbol: its device address
// (per device) comes from hipGetSymbolAddress in scratch_setup.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace los {

const char *ctx_tune_cache(const los_ctx *ctx) {
  return ctx && !ctx->tune_cache.empty() ? ctx->tune_cache.c_str() : nullptr;
}

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

int check_result(const char *who, const void *p, int64_t n, bool f32, hipStream_t s) {
  if (!finite_check_enabled()) return LOS_OK;
  unsigned long long bad = 0;
  hipError_t e = count_nonfinite(p, n, f32, s, &bad);
  if (e != hipSuccess) return hip_fail(e, who);
  if (bad)
    return fail(LOS_ERR_NUMERIC, "%s: %llu of %lld results are not finite", who, bad, (long long)n);
  return LOS_OK;
}

}  // namespace los

namespace {

using los::fail;
using los::hip_fail;
using los::ok;

// Grow workspace slot `slot` of the context to at least `bytes` (never
// shrinks).  hipFree waits for the device, so queued work that still uses the
// old buffer finishes first.
int ws_reserve(los_ctx *ctx, int slot, size_t bytes, void **out) {
  if (bytes <= ctx->ws_bytes[slot]) {
    *out = ctx->ws[slot];
    return LOS_OK;
  }
  if (ctx->ws[slot]) {
    hipError_t e = hipFree(ctx->ws[slot]);
    ctx->ws[slot] = nullptr;
    ctx->ws_bytes[slot] = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
  }
  size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
  hipError_t e = hipMalloc(&ctx->ws[slot], want);
  if (e != hipSuccess) {
    ctx->ws[slot] = nullptr;
    return fail(LOS_ERR_OOM, "workspace allocation of %zu bytes failed: %s", want,
                hipGetErrorString(e));
  }
  ctx->ws_bytes[slot] = want;
  *out = ctx->ws[slot];
  return LOS_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device dev, which must be current; looked
// up once per device and kept.
int scratch_setup(int dev, void **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LOS_ERR_UNSUPPORTED, "device index %d is beyond %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(LOS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LOS_OK;
}

int env_int(const char *name) {
  const char *v = std::getenv(name);
  return v ? std::atoi(v) : 0;
}

// Bytes of Bessel table per k row for the MFMA projection.
size_t jtab_bytes_per_k(int64_t nlp, int64_t ntp, int ntb) {
  return sizeof(float) * (size_t)nlp * (size_t)ntp + sizeof(int) * (size_t)ntb;
}

// Number of k rows per Bessel-table chunk: LOS_JTAB_MIB (default 4096 MiB)
// bounds the table workspace.
int64_t jtab_chunk(int64_t nk, size_t per_k) {
  int64_t mib = env_int("LOS_JTAB_MIB");
  if (mib <= 0) mib = 4096;
  int64_t kc = (int64_t)((size_t)mib * (1u << 20) / per_k);
  if (kc < 1) kc = 1;
  if (kc > nk) kc = nk;
  if (kc > 65535) kc = 65535;
  return kc;
}

los::GemmTile gemm_tile_for(int max_ncol) {
  los::GemmTile t{env_int("LOS_GEMM_MB"), env_int("LOS_GEMM_NC")};
  if (t.mb > 0 && t.nc > 0 && los::gemm_tile_supported(t)) return t;  // (checked per precision at launch)
  if (max_ncol <= 16) return {4, 1};
  if (max_ncol <= 32) return {2, 2};
  return {2, 4};
}

// Mixed-precision projection, default pipeline: per chunk of k rows the FP64
// Bessel seeds (every 32 multipoles), then the product with the Bessel tiles
// regenerated in LDS (project_fused.hip); no table reaches device memory.
// The seed workspace is bounded by LOS_JTAB_MIB (default 4096 MiB);
// LOS_FUSED_SHAPE picks the tile shape (default 4: 256 l x 16 columns).
int project_mixed_fused(los_ctx *ctx, int lmin, int lmax, int64_t nk, int64_t ntau, double tau0,
                        const double *k, const double *tau, const double *w_tau, const float *S,
                        int nsrc, int prec, float *delta, hipStream_t stream) {
  los::FusedArgs fa{};
  fa.lmin = lmin;
  fa.lmax = lmax;
  fa.nl = lmax - lmin + 1;
  fa.nlb = (fa.nl + 15) / 16;
  fa.nseg = (fa.nlb + 1) / 2;
  fa.ntau = ntau;
  fa.ntp = (ntau + 63) / 64 * 64;
  fa.row_index = nullptr;
  fa.tau0 = tau0;
  fa.k = k;
  fa.tau = tau;
  fa.w = w_tau;
  fa.S = S;
  fa.s_kstride = ntau;
  fa.s_cstride = nk * ntau;
  fa.ncol = nsrc;
  fa.dtrans = 0;
  fa.delta = delta;
  const size_t per_k = los::fused_seed_bytes_per_row(fa.nseg, fa.ntp);
  const int64_t kc = jtab_chunk(nk, per_k);
  void *ws = nullptr;
  int rc = ws_reserve(ctx, WS_JTAB, per_k * (size_t)kc, &ws);
  if (rc != LOS_OK) return rc;
  const char *sv = std::getenv("LOS_FUSED_SHAPE");
  const int shape = sv ? std::atoi(sv) : 4;
  if (shape < 0 || shape >= los::kFusedShapeCount)
    return fail(LOS_ERR_INVALID, "los_project: fused shape %d is not compiled", shape);
  for (int64_t k0 = 0; k0 < nk; k0 += kc) {
    const int cnt = (int)(nk - k0 < kc ? nk - k0 : kc);
    fa.k0 = k0;
    los::fused_workspace_at(fa, ws, cnt);
    hipError_t e = los::jseed_launch(fa, cnt, stream);
    if (e != hipSuccess) return hip_fail(e, "los_project: Bessel seed launch");
    e = los::fused_gemm_launch(fa, prec, shape, cnt, nsrc, stream);
    if (e != hipSuccess) return hip_fail(e, "los_project: fused product launch");
  }
  return ok();
}

// Mixed-precision projection, table pipeline (LOS_MIXED_FUSED=0): FP64 Bessel
// tables (w folded in, rounded to FP32) in chunks of k rows, each followed by
// the MFMA product with S.
int project_mixed(los_ctx *ctx, int lmin, int lmax, int64_t nk, int64_t ntau, double tau0,
                  const double *k, const double *tau, const double *w_tau, const float *S,
                  int nsrc, int prec, float *delta, hipStream_t stream) {
  const int nl = lmax - lmin + 1;
  const int nlb = (nl + 15) / 16;
  const int ntb = (int)((ntau + 31) / 32);
  const int64_t nlp = 16 * (int64_t)nlb, ntp = 32 * (int64_t)ntb;
  const size_t per_k = jtab_bytes_per_k(nlp, ntp, ntb);
  const int64_t kc = jtab_chunk(nk, per_k);
  void *ws = nullptr;
  int rc = ws_reserve(ctx, WS_JTAB, per_k * (size_t)kc, &ws);
  if (rc != LOS_OK) return rc;
  float *J = (float *)ws;
  int *top = (int *)((char *)ws + sizeof(float) * (size_t)nlp * (size_t)ntp * (size_t)kc);

  los::JTableArgs ja{};
  ja.lmin = lmin;
  ja.lmax = lmax;
  ja.nlb = nlb;
  ja.ntb = ntb;
  ja.nlp = nlp;
  ja.ntp = ntp;
  ja.ntau = ntau;
  ja.tau0 = tau0;
  ja.k = k;
  ja.tau = tau;
  ja.w = w_tau;
  ja.J = J;
  ja.top = top;

  los::GemmArgs ga{};
  ga.lmin = lmin;
  ga.nl = nl;
  ga.nlb = nlb;
  ga.ntb = ntb;
  ga.nlp = nlp;
  ga.ntp = ntp;
  ga.ntau = ntau;
  ga.J = J;
  ga.top = top;
  ga.S = S;
  ga.s_kstride = ntau;
  ga.s_cstride = nk * ntau;
  ga.ncol = nsrc;
  ga.delta = delta;
  const los::GemmTile tile = gemm_tile_for(nsrc);

  for (int64_t k0 = 0; k0 < nk; k0 += kc) {
    const int cnt = (int)(nk - k0 < kc ? nk - k0 : kc);
    ja.k0 = k0;
    ga.k0 = k0;
    hipError_t e = los::jtable_launch(ja, cnt, stream);
    if (e != hipSuccess) return hip_fail(e, "los_project: Bessel table launch");
    e = los::mfma_gemm_launch(ga, prec, tile, cnt, nsrc, stream);
    if (e != hipSuccess) return hip_fail(e, "los_project: MFMA product launch");
  }
  return ok();
}

}  // namespace

extern "C" {

const char *los_last_error(void) { return g_err.c_str(); }

const char *los_version(void) { return "los-mi355x 0.1 (gfx950)"; }

int los_ctx_create(los_ctx **ctx, const char *tune_cache_path) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_ctx_create: ctx is NULL");
  *ctx = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  void *sp = nullptr;
  int rc = scratch_setup(dev, &sp);
  if (rc != LOS_OK) return rc;
  los_ctx *c = new (std::nothrow) los_ctx;
  if (!c) return fail(LOS_ERR_OOM, "los_ctx_create: out of host memory");
  c->device = dev;
  c->scratch = sp;
  if (tune_cache_path) c->tune_cache = tune_cache_path;
  *ctx = c;
  return ok();
}

void los_ctx_destroy(los_ctx *ctx) {
  if (!ctx) return;
  for (int i = 0; i < WS_COUNT; ++i)
    if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
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
  const int rc = los::check_result("los_bessel_table", out, nx * (int64_t)(lmax - lmin + 1), false,
                                   (hipStream_t)stream);
  return rc == LOS_OK ? ok() : rc;
}

int los_project_kernels(los_ctx *ctx, int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau,
                        double tau0, const double *k, const double *tau, const double *w_tau,
                        const void *S, int32_t nsrc, uint32_t kernel_mask, int32_t prec,
                        void *delta, void *stream) {
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
  if (nsrc < 32 && (kernel_mask >> nsrc) != 0)
    return fail(LOS_ERR_INVALID, "los_project: kernel mask 0x%x names a source >= nsrc = %d",
                kernel_mask, nsrc);
  if (prec != LOS_FP64) {
    if (kernel_mask != 0)
      return fail(LOS_ERR_UNSUPPORTED, "los_project: the E-mode kernel is FP64 only");
    const char *fz = std::getenv("LOS_MIXED_FUSED");
    const bool tables = fz && std::atoi(fz) == 0;
    int rc = tables ? project_mixed(ctx, lmin, lmax, nk, ntau, tau0, k, tau, w_tau,
                                    (const float *)S, nsrc, prec, (float *)delta,
                                    (hipStream_t)stream)
                    : project_mixed_fused(ctx, lmin, lmax, nk, ntau, tau0, k, tau, w_tau,
                                          (const float *)S, nsrc, prec, (float *)delta,
                                          (hipStream_t)stream);
    if (rc != LOS_OK) return rc;
    rc = los::check_result("los_project", delta, nk * (int64_t)(lmax - lmin + 1) * nsrc, true,
                           (hipStream_t)stream);
    return rc == LOS_OK ? ok() : rc;
  }

  // Default: the single descending sweep; LOS_PROJ_SCHEME=0 selects the
  // two-pass kernel (ascending upward, then descending Miller).
  const char *scheme = std::getenv("LOS_PROJ_SCHEME");
  const bool desc = !(scheme && std::atoi(scheme) == 0);
  if (!desc && kernel_mask != 0)
    return fail(LOS_ERR_UNSUPPORTED, "los_project: the E-mode kernel needs the sweep scheme");
  los::ProjectShape sh =
      desc ? los::project_fp64_desc_shape(nsrc, ntau, env_int("LOS_PROJ_WAVES"),
                                          env_int("LOS_PROJ_SLOTS"),
                                          kernel_mask ? 16 : env_int("LOS_PROJ_BLOCK"),
                                          (size_t)std::max(0, env_int("LOS_PROJ_LDS_EXTRA")))
           : los::project_fp64_shape(nsrc, ntau, env_int("LOS_PROJ_WAVES"),
                                     env_int("LOS_PROJ_SLOTS"));
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
  a.emask = kernel_mask;
  hipError_t e = desc ? los::project_fp64_desc_launch(a, nsrc, sh, (hipStream_t)stream)
                      : los::project_fp64_launch(a, nsrc, sh, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "los_project launch");
  const int rc = los::check_result("los_project", delta, nk * (int64_t)a.nl * nsrc, false,
                                   (hipStream_t)stream);
  return rc == LOS_OK ? ok() : rc;
}

int los_project(los_ctx *ctx, int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                const double *k, const double *tau, const double *w_tau, const void *S,
                int32_t nsrc, int32_t prec, void *delta, void *stream) {
  return los_project_kernels(ctx, lmin, lmax, nk, ntau, tau0, k, tau, w_tau, S, nsrc, 0u, prec,
                             delta, stream);
}

int los_project_tensor(los_ctx *ctx, int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau,
                       double tau0, const double *k, const double *tau, const double *w_tau,
                       const double *S, double *delta, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_project_tensor: ctx is NULL");
  if (lmin < 2 || lmax < lmin || lmax > 16000)
    return fail(LOS_ERR_INVALID, "los_project_tensor: need 2 <= lmin <= lmax <= 16000 (got %d, %d)",
                lmin, lmax);
  if (nk < 1 || nk > ((int64_t)1 << 31) - 1)
    return fail(LOS_ERR_INVALID, "los_project_tensor: nk = %lld out of range", (long long)nk);
  if (ntau < 1 || ntau > 8192)
    return fail(LOS_ERR_INVALID, "los_project_tensor: ntau = %lld out of [1, 8192]",
                (long long)ntau);
  if (!(tau0 == tau0)) return fail(LOS_ERR_INVALID, "los_project_tensor: tau0 is NaN");
  if (!k || !tau || !w_tau || !S || !delta)
    return fail(LOS_ERR_INVALID, "los_project_tensor: NULL array");
  const char *scheme = std::getenv("LOS_PROJ_SCHEME");
  if (scheme && std::atoi(scheme) == 0)
    return fail(LOS_ERR_UNSUPPORTED, "los_project_tensor: needs the sweep scheme");
  // the sweep: rows lmin-1 .. lmax, columns S_P, S_P/x, S_P/x^2, S_T/x^2
  los::ProjectShape sh = los::project_fp64_desc_shape(
      4, ntau, env_int("LOS_PROJ_WAVES"), env_int("LOS_PROJ_SLOTS"), 16,
      (size_t)std::max(0, env_int("LOS_PROJ_LDS_EXTRA")));
  if (sh.waves == 0 || sh.lds > 160 * 1024)
    return fail(LOS_ERR_UNSUPPORTED, "los_project_tensor: no launch shape for ntau = %lld",
                (long long)ntau);
  const int nl = lmax - lmin + 1;
  void *ws = nullptr;
  int rc = ws_reserve(ctx, WS_TENSOR, sizeof(double) * 4 * (size_t)(nl + 1) * (size_t)nk, &ws);
  if (rc != LOS_OK) return rc;
  los::ProjectArgs a{};
  a.lmin = lmin - 1;
  a.lmax = lmax;
  a.nl = nl + 1;
  a.nblk = (a.nl + los::kProjectBlock - 1) / los::kProjectBlock;
  a.nk = nk;
  a.ntau = ntau;
  a.tau0 = tau0;
  a.k = k;
  a.tau = tau;
  a.w = w_tau;
  a.S = S;
  a.delta = (double *)ws;
  a.emask = 0u;
  a.x1mask = 0x2u;  // column 1: S_P / x
  a.x2mask = 0xcu;  // columns 2, 3: S_P / x^2, S_T / x^2
  a.splane[0] = 1;
  a.splane[1] = 1;
  a.splane[2] = 1;
  a.splane[3] = 0;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = los::project_fp64_desc_launch(a, 4, sh, st);
  if (e != hipSuccess) return hip_fail(e, "los_project_tensor: sweep launch");
  e = los::tensor_combine_launch((const double *)ws, delta, lmin, nl, nk, st);
  if (e != hipSuccess) return hip_fail(e, "los_project_tensor: combine launch");
  rc = los::check_result("los_project_tensor", delta, nk * (int64_t)nl * 3, false, st);
  return rc == LOS_OK ? ok() : rc;
}

int los_project_lsample(los_ctx *ctx, int32_t lmin, int32_t lmax, const int32_t *ls,
                        int32_t nls, int64_t nk, int64_t ntau, double tau0, const double *k,
                        const double *tau, const double *w_tau, const double *S, int32_t nsrc,
                        uint32_t kernel_mask, double *delta, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_project_lsample: ctx is NULL");
  if (lmin < 2 || lmax < lmin || lmax > 16000)
    return fail(LOS_ERR_INVALID, "los_project_lsample: need 2 <= lmin <= lmax <= 16000");
  if (!ls || nls < 1 || nls > lmax - lmin + 1)
    return fail(LOS_ERR_INVALID, "los_project_lsample: need 1 <= nls <= lmax - lmin + 1 and ls");
  for (int32_t i = 0; i < nls; ++i) {
    if (ls[i] < lmin || ls[i] > lmax || (i > 0 && ls[i] <= ls[i - 1]))
      return fail(LOS_ERR_INVALID,
                  "los_project_lsample: ls must increase strictly within [lmin, lmax] (ls[%d] = %d)",
                  i, ls[i]);
  }
  if (nk < 1 || nk > ((int64_t)1 << 31) - 1)
    return fail(LOS_ERR_INVALID, "los_project_lsample: nk = %lld out of range", (long long)nk);
  if (ntau < 1 || ntau > 8192)
    return fail(LOS_ERR_INVALID, "los_project_lsample: ntau = %lld out of [1, 8192]",
                (long long)ntau);
  if (nsrc < 1 || nsrc > 4)
    return fail(LOS_ERR_INVALID, "los_project_lsample: nsrc = %d out of [1, 4]", nsrc);
  if (!(tau0 == tau0)) return fail(LOS_ERR_INVALID, "los_project_lsample: tau0 is NaN");
  if (!k || !tau || !w_tau || !S || !delta)
    return fail(LOS_ERR_INVALID, "los_project_lsample: NULL array");
  if (nsrc < 32 && (kernel_mask >> nsrc) != 0)
    return fail(LOS_ERR_INVALID, "los_project_lsample: kernel mask 0x%x names a source >= nsrc",
                kernel_mask);
  const char *scheme = std::getenv("LOS_PROJ_SCHEME");
  if (scheme && std::atoi(scheme) == 0)
    return fail(LOS_ERR_UNSUPPORTED, "los_project_lsample: needs the sweep scheme");
  los::ProjectShape sh = los::project_fp64_desc_shape(
      nsrc, ntau, env_int("LOS_PROJ_WAVES"), env_int("LOS_PROJ_SLOTS"), 16,
      (size_t)std::max(0, env_int("LOS_PROJ_LDS_EXTRA")));
  if (sh.waves == 0 || sh.lds > 160 * 1024)
    return fail(LOS_ERR_UNSUPPORTED, "los_project_lsample: no launch shape for ntau = %lld",
                (long long)ntau);
  // device tables (output row per multipole, sampled-row mask per 16-row
  // block), rebuilt only when the list changes
  const int nl = lmax - lmin + 1, nblk = (nl + 15) / 16;
  const size_t bytes = sizeof(int32_t) * (size_t)nl + sizeof(uint32_t) * (size_t)nblk;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int32_t> key;
  key.reserve((size_t)nls + 2);
  key.push_back(lmin);
  key.push_back(lmax);
  key.insert(key.end(), ls, ls + nls);
  void *ws = ctx->ws[WS_LSEL];
  if (key != ctx->lsel_key || ctx->ws_bytes[WS_LSEL] < bytes) {
    std::vector<int32_t> lsel((size_t)nl, -1);
    std::vector<uint32_t> bmask((size_t)nblk, 0u);
    for (int32_t i = 0; i < nls; ++i) {
      const int r = ls[i] - lmin;
      lsel[(size_t)r] = i;
      bmask[(size_t)(r / 16)] |= 1u << (r % 16);
    }
    // the previous tables may still be read by queued work on this stream
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "los_project_lsample: stream");
    ctx->lsel_key.clear();
    int rc = ws_reserve(ctx, WS_LSEL, bytes, &ws);
    if (rc != LOS_OK) return rc;
    e = hipMemcpy(ws, lsel.data(), sizeof(int32_t) * (size_t)nl, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy((char *)ws + sizeof(int32_t) * (size_t)nl, bmask.data(),
                    sizeof(uint32_t) * (size_t)nblk, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "los_project_lsample: copying the sample tables");
    ctx->lsel_key.swap(key);
  }
  los::ProjectArgs a{};
  a.lmin = lmin;
  a.lmax = lmax;
  a.nl = nl;
  a.nblk = (nl + los::kProjectBlock - 1) / los::kProjectBlock;
  a.nk = nk;
  a.ntau = ntau;
  a.tau0 = tau0;
  a.k = k;
  a.tau = tau;
  a.w = w_tau;
  a.S = S;
  a.delta = delta;
  a.emask = kernel_mask;
  a.lsel = (const int32_t *)ws;
  a.bmask = (const uint32_t *)((const char *)ws + sizeof(int32_t) * (size_t)nl);
  a.nls = nls;
  hipError_t e = los::project_fp64_desc_launch(a, nsrc, sh, st);
  if (e != hipSuccess) return hip_fail(e, "los_project_lsample launch");
  const int rc2 = los::check_result("los_project_lsample", delta, nk * (int64_t)nls * nsrc, false, st);
  return rc2 == LOS_OK ? ok() : rc2;
}

}  // extern "C"

namespace {

// Validation shared by cl_integrate and cl_integrate_noalloc; fills everything
// of `a` except the partial-sum buffer.
int cl_args(const char *who, los_ctx *ctx, const void *delta, int32_t delta_prec, int32_t nsrc,
            int32_t nl, int64_t nk, const double *w_lnk, const double *Pk, const int32_t *pairs,
            int32_t npairs, double *cl, los::ClArgs *a) {
  if (!ctx) return fail(LOS_ERR_INVALID, "%s: ctx is NULL", who);
  if (nsrc < 1 || nsrc > 4) return fail(LOS_ERR_INVALID, "%s: nsrc = %d", who, nsrc);
  if (nl < 1) return fail(LOS_ERR_INVALID, "%s: nl = %d", who, nl);
  if (nk < 1) return fail(LOS_ERR_INVALID, "%s: nk = %lld", who, (long long)nk);
  if (npairs < 1 || npairs > 16)
    return fail(LOS_ERR_INVALID, "%s: npairs = %d out of [1, 16]", who, npairs);
  if (!delta || !w_lnk || !Pk || !pairs || !cl)
    return fail(LOS_ERR_INVALID, "%s: NULL array", who);
  if (delta_prec != LOS_FP64 && delta_prec != LOS_FP32)
    return fail(LOS_ERR_INVALID, "%s: delta_prec must be LOS_FP64 or LOS_FP32", who);
  *a = los::ClArgs{};
  for (int p = 0; p < npairs; ++p) {
    if (pairs[2 * p] < 0 || pairs[2 * p] >= nsrc || pairs[2 * p + 1] < 0 ||
        pairs[2 * p + 1] >= nsrc)
      return fail(LOS_ERR_INVALID, "%s: pair %d = (%d, %d) out of [0, %d)", who, p,
                  pairs[2 * p], pairs[2 * p + 1], nsrc);
    a->pa[p] = pairs[2 * p];
    a->pb[p] = pairs[2 * p + 1];
  }
  a->delta = delta;
  a->delta_f32 = delta_prec == LOS_FP32;
  a->nsrc = nsrc;
  a->nl = nl;
  a->npairs = npairs;
  a->nk = nk;
  a->w = w_lnk;
  a->P = Pk;
  a->cl = cl;
  a->nseg = los::cl_segments(nk, nl);
  return LOS_OK;
}

}  // namespace

extern "C" {

int cl_integrate(los_ctx *ctx, const void *delta, int32_t delta_prec, int32_t nsrc, int32_t nl,
                 int64_t nk, const double *w_lnk, const double *Pk, const int32_t *pairs,
                 int32_t npairs, double *cl, void *stream) {
  los::ClArgs a;
  int rc = cl_args("cl_integrate", ctx, delta, delta_prec, nsrc, nl, nk, w_lnk, Pk, pairs, npairs,
                   cl, &a);
  if (rc != LOS_OK) return rc;
  void *ws = nullptr;
  rc = ws_reserve(ctx, WS_CL, sizeof(double) * (size_t)a.nseg * npairs * nl, &ws);
  if (rc != LOS_OK) return rc;
  a.partial = (double *)ws;
  hipError_t e = los::cl_launch(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "cl_integrate launch");
  rc = los::check_result("cl_integrate", cl, (int64_t)npairs * nl, false, (hipStream_t)stream);
  return rc == LOS_OK ? ok() : rc;
}

int cl_integrate_noalloc(los_ctx *ctx, const void *delta, int32_t delta_prec, int32_t nsrc,
                         int32_t nl, int64_t nk, const double *w_lnk, const double *Pk,
                         const int32_t *pairs, int32_t npairs, double *cl, void *stream) {
  los::ClArgs a;
  int rc = cl_args("cl_integrate_noalloc", ctx, delta, delta_prec, nsrc, nl, nk, w_lnk, Pk, pairs,
                   npairs, cl, &a);
  if (rc != LOS_OK) return rc;
  const size_t need = sizeof(double) * (size_t)a.nseg * npairs * nl;
  if (need > kScratchBytes)
    return fail(LOS_ERR_INVALID,
                "cl_integrate_noalloc: needs %zu bytes of scratch (%d segments x %d pairs x %d "
                "multipoles, FP64), more than its fixed %zu; use cl_integrate",
                need, a.nseg, npairs, nl, kScratchBytes);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "cl_integrate_noalloc: hipGetDevice");
  if (dev != ctx->device || !ctx->scratch)
    return fail(LOS_ERR_INVALID,
                "cl_integrate_noalloc: the current device (%d) is not the context's (%d)", dev,
                ctx->device);
  a.partial = (double *)ctx->scratch;
  e = los::cl_launch(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "cl_integrate_noalloc launch");
  return ok();
}

namespace {

int spline_check(const char *fn, int32_t nsrc, int64_t nkc, int64_t ntau, const double *q,
                 const double *Sc) {
  if (nsrc < 1 || nsrc > 64) return fail(LOS_ERR_INVALID, "%s: nsrc = %d out of [1, 64]", fn, nsrc);
  const int64_t nmax = 2 + 16 * los::kSplineMaxSegments;
  if (nkc < 2 || nkc > nmax)
    return fail(LOS_ERR_INVALID, "%s: nkc = %lld out of [2, %lld]", fn, (long long)nkc,
                (long long)nmax);
  if (ntau < 1 || ntau > ((int64_t)1 << 31) - 1 || (int64_t)nsrc * ntau > ((int64_t)1 << 31) - 1)
    return fail(LOS_ERR_INVALID, "%s: ntau = %lld out of range", fn, (long long)ntau);
  if (!q || !Sc) return fail(LOS_ERR_INVALID, "%s: NULL array", fn);
  return LOS_OK;
}

}  // namespace

int los_spline_sources(los_ctx *ctx, int32_t nsrc, int64_t nkc, int64_t ntau, const double *q,
                       const double *Sc, double *M, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_spline_sources: ctx is NULL");
  int rc = spline_check("los_spline_sources", nsrc, nkc, ntau, q, Sc);
  if (rc != LOS_OK) return rc;
  if (!M) return fail(LOS_ERR_INVALID, "los_spline_sources: NULL array");
  if ((const double *)M == Sc)
    return fail(LOS_ERR_INVALID, "los_spline_sources: M must not alias Sc");
  los::SplineTabs t{};
  if (los::spline_segments(nkc) > 0) {
    void *ws = nullptr;
    rc = ws_reserve(ctx, WS_SPLINE, sizeof(double) * los::spline_tab_doubles(nkc), &ws);
    if (rc != LOS_OK) return rc;
    t = los::spline_tabs_at((double *)ws, nkc);
  }
  hipError_t e = los::spline_solve_launch(q, Sc, M, nkc, (int64_t)nsrc * ntau, ntau, t,
                                          (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "los_spline_sources launch");
  return ok();
}

int los_interp_sources(los_ctx *ctx, int32_t nsrc, int64_t nkc, int64_t ntau, const double *q,
                       const double *Sc, const double *M, int64_t nk, const double *k,
                       int32_t out_prec, void *S, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_interp_sources: ctx is NULL");
  int rc = spline_check("los_interp_sources", nsrc, nkc, ntau, q, Sc);
  if (rc != LOS_OK) return rc;
  if (nk < 0 || nk > ((int64_t)1 << 31) - 1)
    return fail(LOS_ERR_INVALID, "los_interp_sources: nk = %lld out of range", (long long)nk);
  if (out_prec != LOS_FP64 && out_prec != LOS_FP32)
    return fail(LOS_ERR_INVALID, "los_interp_sources: out_prec must be LOS_FP64 or LOS_FP32");
  if (nk == 0) return ok();
  if (!M || !k || !S) return fail(LOS_ERR_INVALID, "los_interp_sources: NULL array");
  if ((const void *)S == (const void *)Sc || (const void *)S == (const void *)M)
    return fail(LOS_ERR_INVALID, "los_interp_sources: S must not alias Sc or M");
  hipError_t e = los::spline_eval_launch(q, nkc, Sc, M, k, nk, nsrc, ntau, out_prec, S,
                                         (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "los_interp_sources launch");
  return ok();
}

int los_cl_interp(los_ctx *ctx, int32_t npairs, const int32_t *ls, int32_t nls,
                  const double *cls, int32_t lmin, int32_t lmax, double *cl, void *stream) {
  if (!ctx) return fail(LOS_ERR_INVALID, "los_cl_interp: ctx is NULL");
  if (npairs < 1 || npairs > 65535)
    return fail(LOS_ERR_INVALID, "los_cl_interp: npairs = %d out of [1, 65535]", npairs);
  if (!ls || nls < 1 || nls > 2048)
    return fail(LOS_ERR_INVALID, "los_cl_interp: need 1 <= nls <= 2048 and ls");
  if (lmin < 2 || lmax < lmin || ls[0] != lmin || ls[nls - 1] != lmax)
    return fail(LOS_ERR_INVALID,
                "los_cl_interp: need 2 <= lmin <= lmax with ls[0] = lmin and ls[nls-1] = lmax");
  for (int32_t i = 1; i < nls; ++i)
    if (ls[i] <= ls[i - 1])
      return fail(LOS_ERR_INVALID, "los_cl_interp: ls must increase strictly (ls[%d] = %d)", i,
                  ls[i]);
  if (!cls || !cl) return fail(LOS_ERR_INVALID, "los_cl_interp: NULL array");
  if ((const void *)cls == (const void *)cl)
    return fail(LOS_ERR_INVALID, "los_cl_interp: cl must not alias cls");
  hipStream_t st = (hipStream_t)stream;
  if (nls == 1) {  // lmin == lmax: the single value
    hipError_t e = hipMemcpyAsync(cl, cls, sizeof(double) * (size_t)npairs,
                                  hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "los_cl_interp copy");
    return ok();
  }
  std::vector<int32_t> key(ls, ls + nls);
  void *ws = ctx->ws[WS_CLI];
  if (key != ctx->cli_key || ctx->ws_bytes[WS_CLI] < sizeof(double) * (size_t)nls) {
    std::vector<double> knots((size_t)nls);
    for (int32_t i = 0; i < nls; ++i) knots[(size_t)i] = (double)ls[i];
    // the previous knots may still be read by queued work on this stream
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "los_cl_interp: stream");
    ctx->cli_key.clear();
    int rc = ws_reserve(ctx, WS_CLI, sizeof(double) * (size_t)nls, &ws);
    if (rc != LOS_OK) return rc;
    e = hipMemcpy(ws, knots.data(), sizeof(double) * (size_t)nls, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "los_cl_interp: copying the knots");
    ctx->cli_key.swap(key);
  }
  hipError_t e = los::cl_interp_launch((const double *)ws, nls, cls, npairs, lmin, lmax, cl, st);
  if (e != hipSuccess) return hip_fail(e, "los_cl_interp launch");
  return ok();
}

}  // extern "C"
