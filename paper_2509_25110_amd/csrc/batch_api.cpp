// Batched solve: many models whose k grids are subsets of one shared master
// grid (gCAMB paper, Sec. 3.2 / Algorithm 1: the work is independent per k;
// Eq. 2-3 per k is then one matrix product J_k . S_k whose columns are the
// sources of every model that uses k, so the Bessel table of k is built once
// for all of them).
//
// Plan (host, once): master rows used by at least one model are compacted;
// each row's columns are the (model, source) pairs that use it, ordered by
// model l_max (largest first) so a 16-column block can stop at the l_max of
// its first column.  Rows are processed in chunks that fit a bounded device
// workspace.  Default pipeline per chunk: Bessel seeds (jseed_kernel) ->
// product with the Bessel tiles regenerated in LDS and transposed output
// (fused_gemm_kernel, project_fused.hip) -> per-model C_l accumulation
// (batch_cl.hip).  LOS_BATCH_FUSED=0 selects the table pipeline instead:
// whole FP32 Bessel tables in HBM (jtable.hip) -> MFMA product
// (project_mfma*.hip).  The first solve times every compiled tile shape of
// the pipeline on two representative chunks and keeps the fastest
// (autotuner); the whole launch sequence is then captured once into a HIP
// graph per set of argument pointers and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "los.h"
#include "los_internal.hpp"

using los::fail;
using los::hip_fail;
using los::ok;

struct los_batch {
  int device = 0;
  int nmodels = 0, nsrc = 0, npairs = 0, prec = 0;
  int lmin = 2, lmax_g = 0, nl = 0, nlb = 0, ntb = 0;
  int pa[16] = {}, pb[16] = {};
  int64_t ntau = 0, nlp = 0, ntp = 0, nk_master = 0, ncols = 0, nrows = 0, npos = 0;
  std::vector<int64_t> pos_col;      // host copy: packed column of (model, j)
  std::vector<int64_t> chunk_row0;   // [nchunks + 1]
  std::vector<int> chunk_maxcol;     // widest row in each chunk
  int64_t kc = 0;
  int nchunks = 0;
  // device
  int64_t *d_rows = nullptr, *d_col_off = nullptr, *d_pos_col = nullptr, *d_koff = nullptr,
          *d_jr = nullptr;
  int *d_col_cnt = nullptr, *d_col_lmax = nullptr, *d_lmax = nullptr, *d_order = nullptr;
  float *J = nullptr, *D = nullptr;
  int *top = nullptr;
  // fused pipeline: seeds workspace (J unused)
  bool fused = true;
  int nseg = 0;
  int64_t ntp64 = 0;
  void *seedws = nullptr;
  int fshape = 0;
  float ftune_ms[los::kFusedShapeCount] = {};
  std::vector<int64_t> chunk_col0;  // packed column at the start of each chunk
  // tuning and graph
  los::GemmTile tile{2, 4};
  bool tuned = false;
  float tune_ms[los::kGemmTileCount] = {};
  std::string cache_path, cache_key;  // autotune cache (empty: none)
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *key[9] = {};
  double key_tau0 = 0.0;
};

namespace {

int env_i(const char *name, int dflt) {
  const char *v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

template <class T>
int dev_copy(T **dst, const T *src, size_t n) {
  hipError_t e = hipMalloc((void **)dst, sizeof(T) * (n ? n : 1));
  if (e != hipSuccess) return fail(LOS_ERR_OOM, "batch plan: hipMalloc failed: %s", hipGetErrorString(e));
  if (n) {
    e = hipMemcpy(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch plan: hipMemcpy");
  }
  return LOS_OK;
}

void free_plan(los_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  // `top` lives inside the J allocation
  void *ptrs[] = {b->d_rows, b->d_col_off, b->d_pos_col, b->d_koff, b->d_jr, b->d_col_cnt,
                  b->d_col_lmax, b->d_lmax, b->d_order, b->J, b->D, b->seedws};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete b;
}

// Autotune cache: one line per tuning, "<key> <value>"; the last line with a
// plan's key wins.  Key: architecture, pipeline, precision and buckets of the
// shape (n_tau padded to 64, multipoles in 256s, widest row and row count in
// powers of two); value: the fused shape index or the table tile "mb x nc".
int pow2_bucket(int64_t v) {
  int b = 0;
  while (v > 1) {
    v = (v + 1) / 2;
    ++b;
  }
  return b;
}

std::string tune_key(const los_batch *b, int maxcol) {
  hipDeviceProp_t prop{};
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s %s prec=%d ntau=%lld nl=%d col=%d rows=%d", arch.c_str(),
                b->fused ? "fused" : "table", b->prec, (long long)((b->ntau + 63) / 64 * 64),
                (b->nl + 255) / 256 * 256, pow2_bucket(maxcol), pow2_bucket(b->nrows));
  return buf;
}

// The cached value for the plan's key, or "" when there is none.
std::string cache_lookup(const los_batch *b) {
  std::string found;
  FILE *f = std::fopen(b->cache_path.c_str(), "r");
  if (!f) return found;
  char line[512];
  const size_t kl = b->cache_key.size();
  while (std::fgets(line, sizeof line, f)) {
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    if (l.size() > kl + 1 && l.compare(0, kl, b->cache_key) == 0 && l[kl] == ' ')
      found = l.substr(kl + 1);
  }
  std::fclose(f);
  return found;
}

// Apply a cached value; false when it names nothing this build has compiled.
bool cache_apply(los_batch *b, const std::string &v) {
  if (b->fused) {
    int sh = -1;
    if (std::sscanf(v.c_str(), "shape=%d", &sh) != 1 || sh < 0 || sh >= los::kFusedShapeCount)
      return false;
    b->fshape = sh;
    return true;
  }
  los::GemmTile t{0, 0};
  if (std::sscanf(v.c_str(), "tile=%dx%d", &t.mb, &t.nc) != 2 || !los::gemm_tile_supported(t) ||
      (t.mb == los::kGemmTileLds.mb && t.nc == los::kGemmTileLds.nc && b->prec != LOS_BF16X3))
    return false;
  b->tile = t;
  return true;
}

void cache_store(const los_batch *b) {
  if (b->cache_path.empty()) return;
  char val[64];
  if (b->fused)
    std::snprintf(val, sizeof val, "shape=%d", b->fshape);
  else
    std::snprintf(val, sizeof val, "tile=%dx%d", b->tile.mb, b->tile.nc);
  const std::string line = b->cache_key + " " + val + "\n";
  FILE *f = std::fopen(b->cache_path.c_str(), "a");
  if (!f) return;  // a cache that cannot be written only costs the next plan a tuning
  std::fwrite(line.data(), 1, line.size(), f);
  std::fclose(f);
}

struct SolveArgs {
  double tau0;
  const double *k, *tau, *w;
  const float *S;
  const double *w_lnk, *Pk;
  double *cl;
};

los::JTableArgs jargs(const los_batch *b, const SolveArgs &s, int64_t r0) {
  los::JTableArgs a{};
  a.lmin = b->lmin;
  a.lmax = b->lmax_g;
  a.nlb = b->nlb;
  a.ntb = b->ntb;
  a.nlp = b->nlp;
  a.ntp = b->ntp;
  a.ntau = b->ntau;
  a.k0 = r0;
  a.row_index = b->d_rows;
  a.tau0 = s.tau0;
  a.k = s.k;
  a.tau = s.tau;
  a.w = s.w;
  a.J = b->J;
  a.top = b->top;
  return a;
}

los::GemmArgs gargs(const los_batch *b, const SolveArgs &s, int c) {
  los::GemmArgs a{};
  a.lmin = b->lmin;
  a.nl = b->nl;
  a.nlb = b->nlb;
  a.ntb = b->ntb;
  a.nlp = b->nlp;
  a.ntp = b->ntp;
  a.ntau = b->ntau;
  a.k0 = b->chunk_row0[c];
  a.J = b->J;
  a.top = b->top;
  a.S = s.S;
  a.s_cstride = b->ntau;
  a.col_cnt = b->d_col_cnt;
  a.col_off = b->d_col_off;
  a.col_base = b->chunk_col0[c];
  a.col_lmax = b->d_col_lmax;
  a.dtrans = 1;
  a.delta = b->D;
  return a;
}

los::FusedArgs fargs(const los_batch *b, const SolveArgs &s, int c) {
  los::FusedArgs a{};
  a.lmin = b->lmin;
  a.lmax = b->lmax_g;
  a.nl = b->nl;
  a.nlb = b->nlb;
  a.nseg = b->nseg;
  a.ntau = b->ntau;
  a.ntp = b->ntp64;
  a.k0 = b->chunk_row0[c];
  a.row_index = b->d_rows;
  a.tau0 = s.tau0;
  a.k = s.k;
  a.tau = s.tau;
  a.w = s.w;
  los::fused_workspace_at(a, b->seedws, (int)(b->chunk_row0[c + 1] - b->chunk_row0[c]));
  a.S = s.S;
  a.s_cstride = b->ntau;
  a.col_cnt = b->d_col_cnt;
  a.col_off = b->d_col_off;
  a.col_base = b->chunk_col0[c];
  a.col_lmax = b->d_col_lmax;
  a.dtrans = 1;
  a.delta = b->D;
  return a;
}

// The product of chunk c: J . S for the chunk's rows into D (either pipeline).
int enqueue_product(los_batch *b, const SolveArgs &s, int c, hipStream_t st) {
  const int64_t r0 = b->chunk_row0[c];
  const int cnt = (int)(b->chunk_row0[c + 1] - r0);
  hipError_t e;
  if (b->fused) {
    const los::FusedArgs fa = fargs(b, s, c);
    e = los::jseed_launch(fa, cnt, st);
    if (e != hipSuccess) return hip_fail(e, "los_batch_solve: Bessel seed launch");
    e = los::fused_gemm_launch(fa, b->prec, b->fshape, cnt, b->chunk_maxcol[c], st);
    if (e != hipSuccess) return hip_fail(e, "los_batch_solve: fused product launch");
    return LOS_OK;
  }
  e = los::jtable_launch(jargs(b, s, r0), cnt, st);
  if (e != hipSuccess) return hip_fail(e, "los_batch_solve: Bessel table launch");
  e = los::mfma_gemm_launch(gargs(b, s, c), b->prec, b->tile, cnt, b->chunk_maxcol[c], st);
  if (e != hipSuccess) return hip_fail(e, "los_batch_solve: MFMA product launch");
  return LOS_OK;
}

// Enqueue the whole solve on stream st.
int enqueue(los_batch *b, const SolveArgs &s, hipStream_t st) {
  hipError_t e = los::fill_zero_launch(s.cl, (int64_t)b->nmodels * b->npairs * b->nl, st);
  if (e != hipSuccess) return hip_fail(e, "los_batch_solve: fill launch");
  for (int c = 0; c < b->nchunks; ++c) {
    int rc = enqueue_product(b, s, c, st);
    if (rc != LOS_OK) return rc;
    los::BatchClArgs ca{};
    ca.nmodels = b->nmodels;
    ca.nsrc = b->nsrc;
    ca.npairs = b->npairs;
    ca.lmin = b->lmin;
    ca.nl = b->nl;
    ca.chunk = c;
    std::memcpy(ca.pa, b->pa, sizeof ca.pa);
    std::memcpy(ca.pb, b->pb, sizeof ca.pb);
    ca.lmax = b->d_lmax;
    ca.koff = b->d_koff;
    ca.jr = b->d_jr;
    ca.order = b->d_order + (size_t)c * b->nmodels;
    ca.pos_col = b->d_pos_col;
    ca.col_base = b->chunk_col0[c];
    ca.D = b->D;
    ca.w_lnk = s.w_lnk;
    ca.Pk = s.Pk;
    ca.cl = s.cl;
    e = los::batch_cl_launch(ca, st);
    if (e != hipSuccess) return hip_fail(e, "los_batch_solve: C_l launch");
  }
  return LOS_OK;
}

// Fused pipeline: time the wide fused shapes (0..3) on two representative
// chunks after building their seeds once; keep the fastest total.
// LOS_BATCH_SHAPE pins a shape; LOS_BATCH_TUNE=0 keeps shape 0.
int autotune_fused(los_batch *b, const SolveArgs &s, hipStream_t st) {
  const char *pin = std::getenv("LOS_BATCH_SHAPE");
  if (pin) {
    const int sh = std::atoi(pin);
    if (sh < 0 || sh >= los::kFusedShapeCount)
      return fail(LOS_ERR_INVALID, "los_batch_solve: fused shape %d is not compiled", sh);
    b->fshape = sh;
    b->tuned = true;
    return LOS_OK;
  }
  if (!env_i("LOS_BATCH_TUNE", 1)) {
    b->tuned = true;
    return LOS_OK;
  }
  if (!b->cache_path.empty() && cache_apply(b, cache_lookup(b))) {
    b->tuned = true;
    return LOS_OK;
  }
  int probe[2] = {b->nchunks / 2, b->nchunks - 1};
  if (b->nchunks > 1 && b->chunk_row0[b->nchunks] - b->chunk_row0[b->nchunks - 1] < b->kc)
    probe[1] = b->nchunks - 2;
  const int nprobe = probe[0] == probe[1] ? 1 : 2;
  hipEvent_t t0, t1;
  hipError_t e;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return hip_fail(e, "autotune: event");
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "autotune: event");
  }
  constexpr int kWide = 4;  // the shapes with at least 128 columns
  constexpr int wide[kWide] = {0, 1, 2, 3};
  float total[kWide] = {};
  int rc = LOS_OK;
  for (int pi = 0; pi < nprobe && rc == LOS_OK; ++pi) {
    const int c = probe[pi];
    const int cnt = (int)(b->chunk_row0[c + 1] - b->chunk_row0[c]);
    const los::FusedArgs fa = fargs(b, s, c);
    e = los::jseed_launch(fa, cnt, st);
    if (e != hipSuccess) {
      rc = hip_fail(e, "autotune: Bessel seed launch");
      break;
    }
    for (int i = 0; i < kWide && rc == LOS_OK; ++i) {
      float ms = 0.f;
      for (int rep = 0; rep < 2 && rc == LOS_OK; ++rep) {  // first run warms up
        e = hipEventRecord(t0, st);
        if (e == hipSuccess)
          e = los::fused_gemm_launch(fa, b->prec, wide[i], cnt, b->chunk_maxcol[c], st);
        if (e == hipSuccess) e = hipEventRecord(t1, st);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess) rc = hip_fail(e, "autotune");
      }
      total[i] += ms;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc != LOS_OK) return rc;
  float best = 1e30f;
  for (int i = 0; i < kWide; ++i) {
    b->ftune_ms[wide[i]] = total[i];
    if (total[i] < best) {
      best = total[i];
      b->fshape = wide[i];
    }
  }
  b->tuned = true;
  cache_store(b);
  return LOS_OK;
}

// Table pipeline: time every compiled tile shape on two representative chunks
// (the middle one and the last full one, where k and the Bessel band are
// largest), each after building its Bessel table once; keep the fastest total.
// LOS_BATCH_TILE_MB / _NC pin a shape instead; LOS_BATCH_TUNE=0 keeps {2, 4}.
int autotune(los_batch *b, const SolveArgs &s, hipStream_t st) {
  if (b->fused) return autotune_fused(b, s, st);
  const int mb = env_i("LOS_BATCH_TILE_MB", 0), nc = env_i("LOS_BATCH_TILE_NC", 0);
  if (mb > 0 && nc > 0) {
    los::GemmTile t{mb, nc};
    if (!los::gemm_tile_supported(t) ||
        (t.mb == los::kGemmTileLds.mb && t.nc == los::kGemmTileLds.nc && b->prec != LOS_BF16X3))
      return fail(LOS_ERR_INVALID, "los_batch_solve: tile %d x %d is not compiled", mb, nc);
    b->tile = t;
    b->tuned = true;
    return LOS_OK;
  }
  if (!env_i("LOS_BATCH_TUNE", 1)) {
    b->tuned = true;
    return LOS_OK;
  }
  if (!b->cache_path.empty() && cache_apply(b, cache_lookup(b))) {
    b->tuned = true;
    return LOS_OK;
  }
  int probe[2] = {b->nchunks / 2, b->nchunks - 1};
  if (b->nchunks > 1 && b->chunk_row0[b->nchunks] - b->chunk_row0[b->nchunks - 1] < b->kc)
    probe[1] = b->nchunks - 2;  // the last chunk is a short remainder
  const int nprobe = probe[0] == probe[1] ? 1 : 2;
  hipEvent_t t0, t1;
  hipError_t e;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return hip_fail(e, "autotune: event");
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "autotune: event");
  }
  float total[los::kGemmTileCount] = {};
  int rc = LOS_OK;
  for (int pi = 0; pi < nprobe && rc == LOS_OK; ++pi) {
    const int c = probe[pi];
    const int cnt = (int)(b->chunk_row0[c + 1] - b->chunk_row0[c]);
    e = los::jtable_launch(jargs(b, s, b->chunk_row0[c]), cnt, st);
    if (e != hipSuccess) {
      rc = hip_fail(e, "autotune: Bessel table launch");
      break;
    }
    for (int i = 0; i < los::kGemmTileCount && rc == LOS_OK; ++i) {
      const los::GemmTile t = los::gemm_tile_at(i);
      if (t.mb == los::kGemmTileLds.mb && t.nc == los::kGemmTileLds.nc && b->prec != LOS_BF16X3) {
        total[i] = -1.f;  // not available in this precision
        continue;
      }
      float ms = 0.f;
      for (int rep = 0; rep < 2 && rc == LOS_OK; ++rep) {  // first run warms up
        e = hipEventRecord(t0, st);
        if (e == hipSuccess)
          e = los::mfma_gemm_launch(gargs(b, s, c), b->prec, t, cnt, b->chunk_maxcol[c], st);
        if (e == hipSuccess) e = hipEventRecord(t1, st);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess) rc = hip_fail(e, "autotune");
      }
      total[i] += ms;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc != LOS_OK) return rc;
  float best = 1e30f;
  for (int i = 0; i < los::kGemmTileCount; ++i) {
    b->tune_ms[i] = total[i];
    if (total[i] >= 0.f && total[i] < best) {
      best = total[i];
      b->tile = los::gemm_tile_at(i);
    }
  }
  b->tuned = true;
  cache_store(b);
  return LOS_OK;
}

}  // namespace

extern "C" {

int los_batch_create(los_ctx *ctx, int32_t nmodels, int32_t nsrc, const int32_t *lmax,
                     const int64_t *koff, const int64_t *k_index, int64_t nk_master, int64_t ntau,
                     const int32_t *pairs, int32_t npairs, int32_t prec, los_batch **plan) {
  if (!plan) return fail(LOS_ERR_INVALID, "los_batch_create: plan is NULL");
  *plan = nullptr;
  if (!ctx) return fail(LOS_ERR_INVALID, "los_batch_create: ctx is NULL");
  if (nmodels < 1) return fail(LOS_ERR_INVALID, "los_batch_create: nmodels = %d", nmodels);
  if (nsrc < 1 || nsrc > 4) return fail(LOS_ERR_INVALID, "los_batch_create: nsrc = %d", nsrc);
  if (!lmax || !koff || !k_index || !pairs)
    return fail(LOS_ERR_INVALID, "los_batch_create: NULL array");
  if (npairs < 1 || npairs > 16)
    return fail(LOS_ERR_INVALID, "los_batch_create: npairs = %d out of [1, 16]", npairs);
  if (prec != LOS_FP32 && prec != LOS_BF16X3)
    return fail(LOS_ERR_INVALID, "los_batch_create: prec must be LOS_FP32 or LOS_BF16X3");
  if (nk_master < 1 || nk_master > ((int64_t)1 << 31) - 1)
    return fail(LOS_ERR_INVALID, "los_batch_create: nk_master = %lld", (long long)nk_master);
  if (ntau < 1 || ntau > 8192)
    return fail(LOS_ERR_INVALID, "los_batch_create: ntau = %lld out of [1, 8192]", (long long)ntau);
  for (int p = 0; p < npairs; ++p)
    if (pairs[2 * p] < 0 || pairs[2 * p] >= nsrc || pairs[2 * p + 1] < 0 ||
        pairs[2 * p + 1] >= nsrc)
      return fail(LOS_ERR_INVALID, "los_batch_create: pair %d out of range", p);
  if (koff[0] != 0) return fail(LOS_ERR_INVALID, "los_batch_create: koff[0] must be 0");
  int lmax_g = 2;
  for (int m = 0; m < nmodels; ++m) {
    if (lmax[m] < 2 || lmax[m] > 16000)
      return fail(LOS_ERR_INVALID, "los_batch_create: lmax[%d] = %d out of [2, 16000]", m, lmax[m]);
    if (koff[m + 1] <= koff[m])
      return fail(LOS_ERR_INVALID, "los_batch_create: model %d has no k", m);
    for (int64_t p = koff[m]; p < koff[m + 1]; ++p) {
      if (k_index[p] < 0 || k_index[p] >= nk_master)
        return fail(LOS_ERR_INVALID, "los_batch_create: k_index[%lld] out of range", (long long)p);
      if (p > koff[m] && k_index[p] <= k_index[p - 1])
        return fail(LOS_ERR_INVALID, "los_batch_create: model %d k_index not increasing", m);
    }
    lmax_g = std::max(lmax_g, (int)lmax[m]);
  }

  los_batch *b = new (std::nothrow) los_batch;
  if (!b) return fail(LOS_ERR_OOM, "los_batch_create: out of host memory");
  (void)hipGetDevice(&b->device);
  b->nmodels = nmodels;
  b->nsrc = nsrc;
  b->npairs = npairs;
  b->prec = prec;
  for (int p = 0; p < npairs; ++p) {
    b->pa[p] = pairs[2 * p];
    b->pb[p] = pairs[2 * p + 1];
  }
  b->lmax_g = lmax_g;
  b->nl = lmax_g - b->lmin + 1;
  b->nlb = (b->nl + 15) / 16;
  b->nlp = 16 * (int64_t)b->nlb;
  b->ntau = ntau;
  b->ntb = (int)((ntau + 31) / 32);
  b->ntp = 32 * (int64_t)b->ntb;
  b->nk_master = nk_master;
  b->npos = koff[nmodels];

  // models per master row, each row ordered by l_max (largest first), then model index
  std::vector<int> order(nmodels);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return lmax[x] > lmax[y]; });
  std::vector<int64_t> users(nk_master + 1, 0);
  for (int64_t p = 0; p < b->npos; ++p) users[k_index[p] + 1]++;
  for (int64_t K = 0; K < nk_master; ++K) users[K + 1] += users[K];
  std::vector<int> row_models(b->npos);
  std::vector<int64_t> row_pos(b->npos);
  {
    std::vector<int64_t> fillp(users.begin(), users.end() - 1);
    for (int oi = 0; oi < nmodels; ++oi) {
      const int m = order[oi];
      for (int64_t p = koff[m]; p < koff[m + 1]; ++p) {
        const int64_t slot = fillp[k_index[p]]++;
        row_models[slot] = m;
        row_pos[slot] = p;
      }
    }
  }
  std::vector<int64_t> rows, col_off;
  std::vector<int> col_cnt, col_lmax;
  std::vector<int64_t> row_of_master(nk_master, -1);
  b->pos_col.assign(b->npos, 0);
  int64_t col = 0;
  for (int64_t K = 0; K < nk_master; ++K) {
    const int64_t u0 = users[K], u1 = users[K + 1];
    if (u0 == u1) continue;
    row_of_master[K] = (int64_t)rows.size();
    rows.push_back(K);
    col_off.push_back(col);
    col_cnt.push_back((int)((u1 - u0) * nsrc));
    for (int64_t u = u0; u < u1; ++u) {
      b->pos_col[row_pos[u]] = col;
      for (int s = 0; s < nsrc; ++s) col_lmax.push_back(lmax[row_models[u]]);
      col += nsrc;
    }
  }
  col_off.push_back(col);
  b->ncols = col;
  b->nrows = (int64_t)rows.size();

  // chunks of rows.  Table pipeline: Bessel tables within LOS_JTAB_MIB
  // (default 4096 MiB).  Fused pipeline: seeds plus the chunk's products
  // within LOS_BATCH_MIB (default 8192 MiB; 32768 runs C4 in 4 chunks instead
  // of 16, 1.3 % faster per step, but allocating it adds about 0.6 s to every
  // plan).
  b->fused = env_i("LOS_BATCH_FUSED", 1) != 0;
  b->nseg = (b->nlb + 1) / 2;
  b->ntp64 = (ntau + 63) / 64 * 64;
  const size_t jrow = sizeof(float) * (size_t)b->nlp * b->ntp + sizeof(int) * b->ntb;
  const size_t srow = los::fused_seed_bytes_per_row(b->nseg, b->ntp64);
  size_t dmax = 0;
  if (b->fused) {
    int64_t mib = env_i("LOS_BATCH_MIB", 8192);
    if (mib < 1) mib = 1;
    const size_t budget = (size_t)mib << 20;
    int64_t r0 = 0;
    b->kc = 0;
    while (r0 < b->nrows) {
      int64_t r1 = r0;
      size_t used = 0;
      while (r1 < b->nrows && r1 - r0 < 65535) {
        const size_t add = srow + sizeof(float) * (size_t)col_cnt[r1] * b->nl;
        if (r1 > r0 && used + add > budget) break;
        used += add;
        ++r1;
      }
      b->chunk_row0.push_back(r0);
      b->chunk_col0.push_back(col_off[r0]);
      int mc = 0;
      for (int64_t r = r0; r < r1; ++r) mc = std::max(mc, col_cnt[r]);
      b->chunk_maxcol.push_back(mc);
      dmax = std::max(dmax, (size_t)(col_off[r1] - col_off[r0]) * b->nl);
      b->kc = std::max(b->kc, r1 - r0);
      r0 = r1;
    }
  } else {
    int64_t mib = env_i("LOS_JTAB_MIB", 4096);
    if (mib < 1) mib = 1;
    b->kc = std::max<int64_t>(1, std::min<int64_t>((int64_t)((size_t)mib * (1u << 20) / jrow), 65535));
    b->kc = std::min(b->kc, b->nrows);
    for (int64_t r0 = 0; r0 < b->nrows; r0 += b->kc) {
      const int64_t r1 = std::min(b->nrows, r0 + b->kc);
      b->chunk_row0.push_back(r0);
      b->chunk_col0.push_back(col_off[r0]);
      int mc = 0;
      for (int64_t r = r0; r < r1; ++r) mc = std::max(mc, col_cnt[r]);
      b->chunk_maxcol.push_back(mc);
      dmax = std::max(dmax, (size_t)(col_off[r1] - col_off[r0]) * b->nl);
    }
  }
  b->chunk_row0.push_back(b->nrows);
  b->nchunks = (int)b->chunk_row0.size() - 1;

  // j range of every model in every chunk
  std::vector<int64_t> jr((size_t)b->nchunks * nmodels * 2);
  for (int m = 0; m < nmodels; ++m) {
    int64_t j = 0;
    const int64_t nkm = koff[m + 1] - koff[m];
    for (int c = 0; c < b->nchunks; ++c) {
      const int64_t jlo = j;
      while (j < nkm && row_of_master[k_index[koff[m] + j]] < b->chunk_row0[c + 1]) ++j;
      jr[((size_t)c * nmodels + m) * 2] = jlo;
      jr[((size_t)c * nmodels + m) * 2 + 1] = j;
    }
  }

  // per chunk, the models with the most rows in it first: the C_l launch
  // starts its longest workgroups first
  std::vector<int> cl_order((size_t)b->nchunks * nmodels);
  for (int c = 0; c < b->nchunks; ++c) {
    int *o = cl_order.data() + (size_t)c * nmodels;
    for (int m = 0; m < nmodels; ++m) o[m] = m;
    const int64_t *jc = jr.data() + (size_t)c * nmodels * 2;
    std::stable_sort(o, o + nmodels, [jc](int x, int y) {
      return jc[2 * x + 1] - jc[2 * x] > jc[2 * y + 1] - jc[2 * y];
    });
  }

  std::vector<int> lmax_v(lmax, lmax + nmodels);
  std::vector<int64_t> koff_v(koff, koff + nmodels + 1);
  int rc = LOS_OK;
  if (rc == LOS_OK) rc = dev_copy(&b->d_rows, rows.data(), rows.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_col_off, col_off.data(), col_off.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_col_cnt, col_cnt.data(), col_cnt.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_col_lmax, col_lmax.data(), col_lmax.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_pos_col, b->pos_col.data(), b->pos_col.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_koff, koff_v.data(), koff_v.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_lmax, lmax_v.data(), lmax_v.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_jr, jr.data(), jr.size());
  if (rc == LOS_OK) rc = dev_copy(&b->d_order, cl_order.data(), cl_order.size());
  if (rc == LOS_OK) {
    hipError_t e = b->fused ? hipMalloc(&b->seedws, srow * (size_t)b->kc)
                            : hipMalloc((void **)&b->J, jrow * (size_t)b->kc);
    if (e == hipSuccess) e = hipMalloc((void **)&b->D, sizeof(float) * (dmax ? dmax : 1));
    if (e != hipSuccess) rc = fail(LOS_ERR_OOM, "los_batch_create: workspace: %s", hipGetErrorString(e));
    if (b->J)
      b->top = (int *)((char *)b->J + sizeof(float) * (size_t)b->nlp * b->ntp * (size_t)b->kc);
  }
  if (rc == LOS_OK) {
    hipError_t e = hipStreamCreate(&b->cap);
    if (e != hipSuccess) rc = hip_fail(e, "los_batch_create: stream");
  }
  if (rc == LOS_OK && los::ctx_tune_cache(ctx)) {
    b->cache_path = los::ctx_tune_cache(ctx);
    int mc = 0;
    for (int v : b->chunk_maxcol) mc = std::max(mc, v);
    b->cache_key = tune_key(b, mc);
  }
  if (rc != LOS_OK) {
    free_plan(b);
    return rc;
  }
  *plan = b;
  return ok();
}

int los_batch_columns(const los_batch *plan, int64_t *col, int64_t *ncols) {
  if (!plan || !col || !ncols) return fail(LOS_ERR_INVALID, "los_batch_columns: NULL argument");
  std::memcpy(col, plan->pos_col.data(), sizeof(int64_t) * plan->pos_col.size());
  *ncols = plan->ncols;
  return ok();
}

int los_batch_info(const los_batch *plan, int32_t *info) {
  if (!plan || !info) return fail(LOS_ERR_INVALID, "los_batch_info: NULL argument");
  info[0] = plan->tile.mb;
  info[1] = plan->tile.nc;
  info[2] = (int32_t)plan->kc;
  info[3] = plan->nchunks;
  info[4] = (int32_t)plan->nrows;
  info[5] = plan->lmax_g;
  info[6] = plan->tuned ? 1 : 0;
  info[7] = plan->exec ? 1 : 0;
  info[8] = plan->fused ? 1 : 0;
  info[9] = plan->fshape;
  return ok();
}

int los_batch_solve(los_batch *plan, double tau0, const double *k_master, const double *tau,
                    const double *w_tau, const float *S_packed, const double *w_lnk,
                    const double *Pk, double *cl, void *stream) {
  if (!plan) return fail(LOS_ERR_INVALID, "los_batch_solve: plan is NULL");
  if (!k_master || !tau || !w_tau || !S_packed || !w_lnk || !Pk || !cl)
    return fail(LOS_ERR_INVALID, "los_batch_solve: NULL array");
  if (!(tau0 == tau0)) return fail(LOS_ERR_INVALID, "los_batch_solve: tau0 is NaN");
  hipStream_t st = (hipStream_t)stream;
  SolveArgs s{tau0, k_master, tau, w_tau, S_packed, w_lnk, Pk, cl};
  if (!plan->tuned) {
    int rc = autotune(plan, s, st);
    if (rc != LOS_OK) return rc;
  }
  if (!env_i("LOS_BATCH_GRAPH", 1)) {
    int rc = enqueue(plan, s, st);
    if (rc == LOS_OK)
      rc = los::check_result("los_batch_solve", cl,
                             (int64_t)plan->nmodels * plan->npairs * plan->nl, false, st);
    return rc == LOS_OK ? ok() : rc;
  }
  const void *key[9] = {k_master, tau, w_tau, S_packed, w_lnk, Pk, cl, nullptr, nullptr};
  const bool same = plan->exec && plan->key_tau0 == tau0 &&
                    std::memcmp(key, plan->key, sizeof key) == 0;
  if (!same) {
    if (plan->exec) {
      (void)hipGraphExecDestroy(plan->exec);
      plan->exec = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "los_batch_solve: begin capture");
    int rc = enqueue(plan, s, plan->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(plan->cap, &g);
    if (rc != LOS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "los_batch_solve: end capture");
    e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      plan->exec = nullptr;
      return hip_fail(e, "los_batch_solve: graph instantiate");
    }
    std::memcpy(plan->key, key, sizeof key);
    plan->key_tau0 = tau0;
  }
  hipError_t e = hipGraphLaunch(plan->exec, st);
  if (e != hipSuccess) return hip_fail(e, "los_batch_solve: graph launch");
  const int rc = los::check_result("los_batch_solve", cl,
                                   (int64_t)plan->nmodels * plan->npairs * plan->nl, false, st);
  return rc == LOS_OK ? ok() : rc;
}

int los_batch_solve_timed(los_batch *plan, double tau0, const double *k_master,
                          const double *tau, const double *w_tau, const float *S_packed,
                          const double *w_lnk, const double *Pk, double *cl, double *ms,
                          int32_t *launches, void *stream) {
  if (!plan) return fail(LOS_ERR_INVALID, "los_batch_solve_timed: plan is NULL");
  if (!k_master || !tau || !w_tau || !S_packed || !w_lnk || !Pk || !cl || !ms || !launches)
    return fail(LOS_ERR_INVALID, "los_batch_solve_timed: NULL array");
  if (!(tau0 == tau0)) return fail(LOS_ERR_INVALID, "los_batch_solve_timed: tau0 is NaN");
  hipStream_t st = (hipStream_t)stream;
  SolveArgs s{tau0, k_master, tau, w_tau, S_packed, w_lnk, Pk, cl};
  if (!plan->tuned) {
    int rc = autotune(plan, s, st);
    if (rc != LOS_OK) return rc;
  }
  // events: ev[0] before the first chunk, then after the Bessel kernel, the
  // product and the C_l kernel of every chunk
  std::vector<hipEvent_t> ev(3 * (size_t)plan->nchunks + 1, nullptr);
  int rc = LOS_OK;
  hipError_t e = hipSuccess;
  for (auto &x : ev)
    if ((e = hipEventCreate(&x)) != hipSuccess) break;
  if (e == hipSuccess) e = los::fill_zero_launch(cl, (int64_t)plan->nmodels * plan->npairs * plan->nl, st);
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  for (int c = 0; c < plan->nchunks && e == hipSuccess && rc == LOS_OK; ++c) {
    const int64_t r0 = plan->chunk_row0[c];
    const int cnt = (int)(plan->chunk_row0[c + 1] - r0);
    if (plan->fused) {
      const los::FusedArgs fa = fargs(plan, s, c);
      e = los::jseed_launch(fa, cnt, st);
      if (e == hipSuccess) e = hipEventRecord(ev[3 * c + 1], st);
      if (e == hipSuccess)
        e = los::fused_gemm_launch(fa, plan->prec, plan->fshape, cnt, plan->chunk_maxcol[c], st);
    } else {
      e = los::jtable_launch(jargs(plan, s, r0), cnt, st);
      if (e == hipSuccess) e = hipEventRecord(ev[3 * c + 1], st);
      if (e == hipSuccess)
        e = los::mfma_gemm_launch(gargs(plan, s, c), plan->prec, plan->tile, cnt,
                                  plan->chunk_maxcol[c], st);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[3 * c + 2], st);
    if (e != hipSuccess) break;
    los::BatchClArgs ca{};
    ca.nmodels = plan->nmodels;
    ca.nsrc = plan->nsrc;
    ca.npairs = plan->npairs;
    ca.lmin = plan->lmin;
    ca.nl = plan->nl;
    ca.chunk = c;
    std::memcpy(ca.pa, plan->pa, sizeof ca.pa);
    std::memcpy(ca.pb, plan->pb, sizeof ca.pb);
    ca.lmax = plan->d_lmax;
    ca.koff = plan->d_koff;
    ca.jr = plan->d_jr;
    ca.order = plan->d_order + (size_t)c * plan->nmodels;
    ca.pos_col = plan->d_pos_col;
    ca.col_base = plan->chunk_col0[c];
    ca.D = plan->D;
    ca.w_lnk = w_lnk;
    ca.Pk = Pk;
    ca.cl = cl;
    e = los::batch_cl_launch(ca, st);
    if (e == hipSuccess) e = hipEventRecord(ev[3 * c + 3], st);
  }
  if (e == hipSuccess) e = hipEventSynchronize(ev.back());
  double acc[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < plan->nchunks && e == hipSuccess; ++c) {
    for (int q = 0; q < 3 && e == hipSuccess; ++q) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, ev[3 * c + q], ev[3 * c + q + 1]);
      acc[q] += t;
    }
  }
  for (auto &x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(e, "los_batch_solve_timed");
  for (int q = 0; q < 3; ++q) {
    ms[q] = acc[q];
    launches[q] = plan->nchunks;
  }
  return ok();
}

void los_batch_destroy(los_batch *plan) {
  if (plan) free_plan(plan);
}

}  // extern "C"
