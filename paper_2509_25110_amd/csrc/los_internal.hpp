// Internal declarations shared by the host API and the kernel translation
// units of liblos.so.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct los_ctx;

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
  uint32_t emask;   // bit s: source s uses the E-mode kernel eps_l (sweep kernel only)
  // Sweep kernel only: bit s of x1mask / x2mask scales column s by 1/x / 1/x^2
  // per node (no row factor); a node below kXTiny then adds its limit, w S / 3
  // to row 1 (1/x: j_1(x)/x -> 1/3) or w S / 15 to row 2 (1/x^2: j_2(x)/x^2 ->
  // 1/15).  Column s reads source plane splane[s] of S (default s).
  uint32_t x1mask = 0, x2mask = 0;
  int splane[4] = {0, 1, 2, 3};
  // Multipole sampling (sweep kernel, 16-row blocks): when lsel is set, only
  // rows l with lsel[l - lmin] >= 0 are accumulated and stored, at output
  // row lsel[l - lmin] of delta[k][nls][nsrc]; bmask[bi] has bit r set when
  // row lmin + 16 bi + r is sampled.
  const int32_t *lsel = nullptr;
  const uint32_t *bmask = nullptr;
  int nls = 0;
  // sweep kernel: blocks of partial sums kept in LDS (2 or 8; the workgroup
  // synchronises every ring/2 blocks).  Set from ProjectShape::ring.
  int ring = 8;
};

// Launch shape chosen by the host for the FP64 projection.
struct ProjectShape {
  int waves;      // waves per workgroup (1..8)
  int slots;      // tau slots per lane (4, 8, 12, 16)
  size_t lds;     // dynamic LDS bytes
  int block = 8;  // l rows per block (descending sweep: 8 or 16)
  int ring = 8;   // descending sweep: blocks of partials in LDS (2 or 8)
};

// FP64 projection: one workgroup per k.
// force_waves / force_slots > 0 override the default shape (tuning).
ProjectShape project_fp64_shape(int nsrc, int64_t ntau, int force_waves = 0, int force_slots = 0);
hipError_t project_fp64_launch(const ProjectArgs &a, int nsrc, const ProjectShape &sh,
                               hipStream_t s);
// Single descending sweep variant (project_fp64_desc.hip), same arguments.
// block: 8 or 16 (default, also for 0) rows per reduction; lds_extra:
// additional LDS per workgroup (bounds the workgroups per CU).
ProjectShape project_fp64_desc_shape(int nsrc, int64_t ntau, int force_waves = 0,
                                     int force_slots = 0, int block = 8, size_t lds_extra = 0);
hipError_t project_fp64_desc_launch(const ProjectArgs &a, int nsrc, const ProjectShape &sh,
                                    hipStream_t s);

// Weighted Bessel tables for the MFMA projection (see jtable.hip):
// J[(kc*nlp + l - lmin)*ntp + n] = w_n j_l(k[k0 + kc] (tau0 - tau_n)) in FP32,
// top[kc*ntb + tb] = highest 16-row block with a non-zero row in node block tb.
struct JTableArgs {
  int lmin, lmax, nlb, ntb;
  int64_t nlp, ntp, ntau;
  int64_t k0;                 // first row of the chunk
  const int64_t *row_index;   // rows -> index into k (device) or nullptr (identity)
  double tau0;
  const double *k, *tau, *w;
  float *J;
  int *top;
};
hipError_t jtable_launch(const JTableArgs &a, int kcount, hipStream_t s);

// Per-k matrix product Delta_k = J_k . S_k on the matrix cores (see
// project_mfma.hip).  With r = k0 + kc (kc = row within the chunk), column c
// of row r of S is the node vector
//   S + sbase + c * s_cstride,  sbase = col_off ? col_off[r] * s_cstride : r * s_kstride,
// and the result goes to
//   delta[dbase + row * ncol + c]   (dtrans == 0)  or  delta[dbase + c * nl + row] (dtrans),
//   dbase = col_off ? (col_off[r] - col_base) * nl : r * nl * ncol.
// col_lmax (optional, per packed column, absolute l, non-increasing within a
// row): blocks above the first column of a 16-column block are skipped.
struct GemmArgs {
  int lmin, nl, nlb, ntb;
  int64_t nlp, ntp, ntau;
  int64_t k0;
  const float *J;
  const int *top;
  const float *S;
  int64_t s_kstride, s_cstride;
  int ncol;                  // columns per k when col_cnt == nullptr
  const int *col_cnt;        // per row column counts (device) or nullptr
  const int64_t *col_off;    // per row first packed column (device) or nullptr
  int64_t col_base;          // packed column that maps to delta offset 0
  const int *col_lmax;       // per packed column l_max (device) or nullptr
  int dtrans;
  float *delta;
};
struct GemmTile {
  int mb;  // 16-row l blocks per wave
  int nc;  // 16-column blocks per wave
};
bool gemm_tile_supported(const GemmTile &t);
// Tile shapes the batch autotuner tries.  The last, {16, 8} (256 rows x 128
// columns per workgroup), is the LDS-staged kernel (project_mfma_lds.hip),
// split-BF16x3 only.
constexpr int kGemmTileCount = 8;
constexpr GemmTile kGemmTileLds{16, 8};
GemmTile gemm_tile_at(int i);
hipError_t mfma_gemm_lds_launch(const GemmArgs &a, int kcount, int max_ncol, hipStream_t s);
hipError_t mfma_gemm_launch(const GemmArgs &a, int prec, const GemmTile &t, int kcount,
                            int max_ncol, hipStream_t s);

// Projection product with the Bessel tiles regenerated in LDS from FP64 seeds
// (project_fused.hip).  Rows of a chunk as for GemmArgs (k0, row_index for
// the k value, col_cnt / col_off / s_* / dtrans / delta for S and the
// output).  Workspace per chunk row: seeds at every 32-row segment top,
// 1/x and the top row R of every node, the largest R of every 64 nodes
// (fused_workspace_at).
struct FusedArgs {
  int lmin, lmax, nl, nlb, nseg;   // nseg = segments of 32 rows covering 16 * nlb rows
  int64_t ntau, ntp;               // ntp: nodes padded to a multiple of 64
  int64_t k0;
  const int64_t *row_index;        // chunk row -> k index (device) or nullptr (k0 + kc)
  double tau0;
  const double *k, *tau, *w;
  double2 *seed;                   // [kcount][nseg][ntp]
  double *nix;                     // [kcount][ntp]
  int *rtop;                       // [kcount][ntp]
  int *cmax;                       // [kcount][ntp / 64] largest R of each chunk of 64 nodes
  const float *S;
  int64_t s_kstride, s_cstride;
  int ncol;
  const int *col_cnt;
  const int64_t *col_off;
  int64_t col_base;
  const int *col_lmax;
  int dtrans;
  float *delta;
};
struct FusedShape {
  int tm, tn;  // l rows x columns per workgroup
};
// Compiled shapes: 0 256x128 (waves 4x2), 1 128x128 (2x2), 2 256x128 (2x4),
// 3 256x256 (2x4), 4 256x16 (8x1), 5 128x16 (4x1).
constexpr int kFusedShapeCount = 6;
FusedShape fused_shape_at(int i);
size_t fused_seed_bytes_per_row(int nseg, int64_t ntp);
void fused_workspace_at(FusedArgs &a, void *ws, int kcount);
hipError_t jseed_launch(const FusedArgs &a, int kcount, hipStream_t s);
hipError_t fused_gemm_launch(const FusedArgs &a, int prec, int shape, int kcount, int max_ncol,
                             hipStream_t s);

// Per-model C_l of a batch, one chunk of master rows at a time (batch_cl.hip).
// D is the chunk's transposed product: D[(packed column - col_base) * nl + l - lmin].
struct BatchClArgs {
  int nmodels, nsrc, npairs, lmin, nl, chunk;
  int pa[16], pb[16];
  const int *lmax;         // [nmodels]
  const int64_t *koff;     // [nmodels + 1] first k position of each model
  const int64_t *jr;       // [nchunks][nmodels][2] j range of each model in each chunk
  const int *order;        // [nmodels] this chunk's models, the most rows first
  const int64_t *pos_col;  // [koff[nmodels]] packed column of (model, j), source 0
  int64_t col_base;
  const float *D;
  const double *w_lnk, *Pk;  // [koff[nmodels]]
  double *cl;                // [nmodels][npairs][nl]
};
hipError_t fill_zero_launch(double *p, int64_t n, hipStream_t s);
hipError_t batch_cl_launch(const BatchClArgs &a, hipStream_t s);

// Tensor-mode combination (tensor.hip): d4[k][l - lmin + 1][4] holds the
// sweep's columns (P0, P1, P2, T2) on rows lmin-1 .. lmax; out[k][l - lmin][3]
// receives (Delta^T, Delta^E, Delta^B) for l = lmin .. lmax.
hipError_t tensor_combine_launch(const double *d4, double *out, int lmin, int nl, int64_t nk,
                                 hipStream_t s);

// The batch autotune cache file of a context (los_api.cpp), or nullptr.
const char *ctx_tune_cache(const los_ctx *ctx);

// Optional result check (finite_check.hip): enabled by LOS_CHECK_FINITE=1;
// count_nonfinite scans n values (float or double) on stream s and waits.
bool finite_check_enabled();
// LOS_OK, or LOS_ERR_NUMERIC when the check is enabled and finds a non-finite
// value among the n results (los_api.cpp).
int check_result(const char *who, const void *p, int64_t n, bool f32, hipStream_t s);
hipError_t count_nonfinite(const void *p, int64_t n, bool f32, hipStream_t s,
                           unsigned long long *bad);

// Error reporting shared by the C entry points (los_api.cpp).
int fail(int code, const char *fmt, ...);
int ok();
int hip_fail(hipError_t e, const char *what);

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

// C_l at every l from sampled multipoles: natural spline of l (l+1) C_l
// (cl_interp.hip); knots[nls] (doubles) in device memory, 2 <= nls <= 2048.
hipError_t cl_interp_launch(const double *knots, int nls, const double *cls, int npairs, int lmin,
                            int lmax, double *cl, hipStream_t s);

// Natural cubic spline of the sources in k (spline.hip).  The tables depend
// on the knots only: per interior row (P * 16 rows, padded) the local Thomas
// factors and the two spikes, per knot interval 1/h, per segment the factors
// of the 2x2-block reduced system.
struct SplineTabs {
  double *sub, *iden, *cp, *v, *w;  // [P * 16]
  double *ih;                       // [N - 1]
  double *red;                      // [P][6]
};
constexpr int64_t kSplineMaxSegments = 1024;  // N <= 2 + 16 * 1024
int64_t spline_segments(int64_t N);
size_t spline_tab_doubles(int64_t N);
SplineTabs spline_tabs_at(double *ws, int64_t N);
// M[s][j][n] for the ncols = nsrc * ntau columns of Sc[s][j][n] on knots q[N].
hipError_t spline_solve_launch(const double *q, const double *Sc, double *M, int64_t N,
                               int64_t ncols, int64_t ntau, const SplineTabs &t, hipStream_t s);
// out[s][i][n] = the spline at k[i] (double or float by out_prec).
hipError_t spline_eval_launch(const double *q, int64_t N, const double *Sc, const double *M,
                              const double *k, int64_t nk, int nsrc, int64_t ntau, int out_prec,
                              void *out, hipStream_t s);

}  // namespace los
