/*
 * los.h -- C ABI of liblos.so, an MI355X (gfx950) implementation of the
 * line-of-sight (LOS) projection and angular power spectrum of a flat-space
 * Einstein-Boltzmann solver.
 *
 * The operations are the ones the gCAMB paper states (Storchi et al., arXiv
 * 2509.25110):
 *   Sec. 2.1, Eq. 2-3: Delta^X_l(k) = int dtau S_X(k, tau) j_l(k (tau0 - tau)),
 *                      discretised as sum_n w_n S_X(k, tau_n) j_l(k chi_n),
 *                      chi_n = tau0 - tau_n, with spherical Bessel kernels j_l
 *                      (flat space, text below Eq. 3);
 *   Sec. 2.1, Eq. 1:   C^XY_l = 4 pi int dk/k P(k) Delta^X_l Delta^Y_l,
 *                      discretised as 4 pi sum_i w_i P(k_i) Delta^X_l Delta^Y_l
 *                      with w_i the caller's ln k quadrature weights;
 *   Sec. 3.2 / Algorithm 1: the work is independent per k ("gang"), and per k
 *                      over l and over tau ("vector").
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer (hipMalloc / torch CUDA tensor)
 *     unless its comment says "host".  The caller owns all of them; the
 *     library never frees or retains them after the call returns.
 *   - Arrays are dense row-major; index formulas are given per argument.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on that stream and returns; results are ready when the
 *     stream is synchronised.
 *   - Return value: LOS_OK (0) or a los_status error code.  Argument errors
 *     are detected before anything is launched (LOS_ERR_INVALID, nothing is
 *     written).  los_last_error() returns a message for the calling thread's
 *     most recent failure (valid until that thread's next call).
 *   - A los_ctx owns the library's device workspace (grown on demand and
 *     reused).  A context is not thread-safe: use one per host thread, and do
 *     not run two calls of one context concurrently on different streams.
 *   - Result check: with the environment variable LOS_CHECK_FINITE=1, the
 *     entry points that write spectra, transfer functions or Bessel tables
 *     (all but cl_integrate_noalloc) scan their output on the device after
 *     enqueueing, wait for the stream, and return LOS_ERR_NUMERIC if any value
 *     is NaN or infinite (the output is still written).  Off by default.
 *   - Floating point: FP64 entry points compute in IEEE double; results agree
 *     with a plain FP64 evaluation of the formulas above to about 1e-12
 *     (normwise); entries smaller than ~1e-20 of the local peak of j_l are
 *     treated as zero (band cut), see los_bessel_table.
 */
#ifndef LOS_H
#define LOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LOS_OK = 0,
    LOS_ERR_INVALID = 1,     /* bad argument; nothing launched               */
    LOS_ERR_HIP = 2,         /* HIP runtime or launch failure                */
    LOS_ERR_OOM = 3,         /* device workspace allocation failed           */
    LOS_ERR_UNSUPPORTED = 4, /* valid request outside what is implemented    */
    LOS_ERR_NUMERIC = 5      /* non-finite result (only with LOS_CHECK_FINITE) */
} los_status;

typedef enum {
    LOS_FP64 = 0,   /* IEEE double throughout                                 */
    LOS_FP32 = 1,   /* FP64 j_l rounded to FP32; FP32 MFMA product, FP32 sum  */
    LOS_BF16X3 = 2  /* FP64 j_l rounded to FP32, split into bf16 hi + lo;
                       three bf16 MFMA products, FP32 sum                      */
} los_prec;

typedef struct los_ctx los_ctx;

/* Message for the calling thread's last failed call ("" if none). */
const char *los_last_error(void);

/* Library version string (host, static storage). */
const char *los_version(void);

/* Create a context bound to the current HIP device.  *ctx receives a handle
 * owned by the caller and released with los_ctx_destroy.
 * tune_cache_path (host string, may be NULL): a text file where batch plans
 * created with this context look up the tile shape their autotuner chose
 * before, under a key of the device architecture, the precision, the pipeline
 * and buckets of n_tau, the multipole count, the widest master row and the row
 * count, and append a line after they tune; a plan that finds its key skips
 * the tuning.  The file need not exist; unreadable lines are ignored; lines are
 * appended with one write each.  NULL: every plan tunes itself.
 * Errors: LOS_ERR_INVALID (ctx == NULL), LOS_ERR_HIP (no device). */
int los_ctx_create(los_ctx **ctx, const char *tune_cache_path);

/* Release a context and its device workspace.  Waits for nothing: the caller
 * must make sure no work that uses the context is still queued.  NULL is a
 * no-op. */
void los_ctx_destroy(los_ctx *ctx);

/*
 * Spherical Bessel table (the radial kernel of Eq. 2-3, flat space).
 *
 *   out[(l - lmin) * nx + i] = j_l(x[i]),   l = lmin..lmax, i = 0..nx-1
 *
 * x: device, nx doubles, each finite and >= 0.  out: device, (lmax-lmin+1)*nx
 * doubles.  0 <= lmin <= lmax <= 30000, nx >= 0 (nx == 0 is a no-op).
 * Method: upward recurrence from j_0 = sin x / x (and j_{-1} = cos x / x) up to
 * l = floor(x); above that, Miller's downward recurrence started above the
 * turning point and matched to the upward value at l = floor(x).  Values with
 * l above x + 14.2 x^(1/3) + 9.5 (where |j_l| < ~1e-21 of its peak) are
 * returned as 0; for x < 1e-9 the first three power-series terms are used.
 * Errors: LOS_ERR_INVALID for NULL pointers or bad ranges (values of x are
 * not inspected on the host; a negative or non-finite x yields NaN there).
 */
int los_bessel_table(los_ctx *ctx, const double *x, int64_t nx, int32_t lmin, int32_t lmax,
                     double *out, void *stream);

/*
 * LOS projection, Eq. 2-3 (Algorithm 1: one workgroup per k, lanes over tau,
 * an l recurrence per lane).
 *
 *   delta[(i * nl + (l - lmin)) * nsrc + s]
 *       = sum_n w_tau[n] * S[(s * nk + i) * ntau + n] * j_l(k[i] * (tau0 - tau[n]))
 *
 *   nl = lmax - lmin + 1, i = 0..nk-1, s = 0..nsrc-1.
 *
 * k: device, nk doubles (> 0).  tau, w_tau: device, ntau doubles, with
 * tau[n] <= tau0.  S: device, nsrc*nk*ntau values.  delta: device,
 * nk*nl*nsrc values.  For prec == LOS_FP64, S and delta are double; for
 * LOS_FP32 and LOS_BF16X3 they are float.
 * Limits: 2 <= lmin <= lmax <= 16000, 1 <= nsrc <= 4, 1 <= ntau <= 8192,
 * nk >= 1.
 *
 * LOS_FP64: the j_l are generated on the fly in registers (never stored) and
 * the band where |j_l| < ~1e-21 of its peak is skipped.
 * LOS_FP32 / LOS_BF16X3 (Sec. 2.1 Eq. 2-3 as the per-k matrix product
 * Delta_k[l][s] = sum_n J_k[l][n] S[s][k][n], J_k[l][n] = w_n j_l(k chi_n)):
 * J_k is computed in FP64 (downward recurrence from the band edge, upward
 * recurrence for the normalisation) and rounded to FP32 as it is used.  By
 * default a first kernel keeps only the FP64 recurrence state every 32
 * multipoles (a context workspace of at most LOS_JTAB_MIB MiB, environment,
 * default 4096, per chunk of k rows) and the product kernel regenerates each
 * tile of J_k from it in on-chip memory, multiplying on the matrix cores with
 * FP32 accumulation; LOS_MIXED_FUSED=0 selects whole FP32 tables in the
 * workspace instead.  Both give the same values.  Expected C_l error ~1e-6
 * relative (both precisions).
 * Errors: LOS_ERR_OOM if the workspace cannot be allocated.
 */
int los_project(los_ctx *ctx, int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                const double *k, const double *tau, const double *w_tau, const void *S,
                int32_t nsrc, int32_t prec, void *delta, void *stream);

/*
 * LOS projection with a choice of radial kernel per source (Sec. 2.1, Eq. 3
 * and the text below it): as los_project, except that every source s whose
 * bit is set in kernel_mask is projected on the E-mode kernel
 *
 *   eps_l(x) = sqrt((l+2)! / (l-2)!) j_l(x) / x^2
 *            = sqrt((l-1) l (l+1) (l+2)) j_l(x) / x^2,
 *
 * whose x -> 0 limit is sqrt(24)/15 at l = 2 and 0 above (a node at
 * tau = tau0 adds w S sqrt(24)/15 to l = 2), and the others on j_l.
 * los_project is the kernel_mask = 0 case.  Errors: LOS_ERR_INVALID for a
 * mask bit >= nsrc; LOS_ERR_UNSUPPORTED for a non-zero mask with
 * prec != LOS_FP64 or with the two-pass FP64 kernel (environment
 * LOS_PROJ_SCHEME=0).
 */
int los_project_kernels(los_ctx *ctx, int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau,
                        double tau0, const double *k, const double *tau, const double *w_tau,
                        const void *S, int32_t nsrc, uint32_t kernel_mask, int32_t prec,
                        void *delta, void *stream);

/*
 * Tensor-mode LOS projection (Sec. 2.1: tensor perturbations and B modes give
 * equations of the same kind as Eq. 2-3; the radial kernels are the published
 * tensor kernels of the line-of-sight method the paper builds on):
 *
 *   delta[(i * nl + (l - lmin)) * 3 + 0] = sum_n w_n S_T(k_i, tau_n) K^T_l(x)
 *   delta[(i * nl + (l - lmin)) * 3 + 1] = sum_n w_n S_P(k_i, tau_n) K^E_l(x)
 *   delta[(i * nl + (l - lmin)) * 3 + 2] = sum_n w_n S_P(k_i, tau_n) K^B_l(x)
 *
 *   K^T_l = sqrt((l+2)!/(l-2)!) j_l / x^2
 *   K^E_l = -j_l + j_l'' + 2 j_l / x^2 + 4 j_l' / x
 *   K^B_l = 2 j_l' + 4 j_l / x,        x = k_i (tau0 - tau_n),
 *
 * with the x -> 0 limits K^T_2 = sqrt(24)/15, K^E_2 = 4/5 and 0 otherwise.
 * S: device, 2*nk*ntau doubles, S[(0 * nk + i) * ntau + n] = S_T and
 * S[(1 * nk + i) * ntau + n] = S_P.  delta: device, nk*nl*3 doubles (T, E, B).
 * k, tau, w_tau, tau0 and the limits as for los_project (FP64 only).
 * Computed as one FP64 sweep of the rows lmin-1 .. lmax over the columns
 * S_P, S_P/x, S_P/x^2, S_T/x^2, then a combination of neighbouring rows
 * (j_l' and j_l'' written through j_{l-1}, j_l); the intermediate
 * nk*(nl+1)*4 doubles live in the context workspace.  The spectra follow from
 * cl_integrate on delta with nsrc = 3 (pairs over T, E, B).
 * Errors: LOS_ERR_INVALID for NULL pointers or bad sizes; LOS_ERR_OOM if the
 * workspace cannot be allocated; LOS_ERR_UNSUPPORTED with the two-pass FP64
 * scheme (LOS_PROJ_SCHEME=0).
 */
int los_project_tensor(los_ctx *ctx, int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau,
                       double tau0, const double *k, const double *tau, const double *w_tau,
                       const double *S, double *delta, void *stream);

/*
 * Angular power spectra, Eq. 1 with the ln k quadrature written out:
 *
 *   cl[p * nl + l'] = 4 pi sum_i w_lnk[i] * Pk[i]
 *                          * delta[(i * nl + l') * nsrc + a_p] * delta[(i * nl + l') * nsrc + b_p]
 *
 * delta: device, nk*nl*nsrc values, double if delta_prec == LOS_FP64 and
 * float if LOS_FP32.  w_lnk, Pk: device, nk doubles.  pairs: HOST, 2*npairs
 * int32 source indices {a_0, b_0, a_1, b_1, ...}, each in [0, nsrc).
 * cl: device, npairs*nl doubles.  Accumulation is FP64 in a fixed order (the
 * result is bitwise reproducible for a given shape).  1 <= nsrc <= 4,
 * 1 <= npairs <= 16, nl >= 1, nk >= 1.
 */
int cl_integrate(los_ctx *ctx, const void *delta, int32_t delta_prec, int32_t nsrc, int32_t nl,
                 int64_t nk, const double *w_lnk, const double *Pk, const int32_t *pairs,
                 int32_t npairs, double *cl, void *stream);

/*
 * cl_integrate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and result as cl_integrate (bitwise), but the
 * partial sums live in a fixed device array of the library (16 MiB per GPU,
 * held until the process ends) instead of the context workspace, and the call
 * makes no allocation of any kind.  The array's device address is looked up
 * once per device by los_ctx_create, so the context must have been created on
 * the current device.
 * Limit: the partial sums take 8 * nseg * npairs * nl bytes, nseg =
 * min(nk, 1024, ceil(4096 / ceil(nl / 64))) (about 2.2 MB per pair, e.g.
 * 8.9 MB for 4 pairs at nl = 16000); a larger request fails with
 * LOS_ERR_INVALID and a message naming the size (use cl_integrate).
 * Every call on a GPU shares that GPU's array, and nothing in it needs to be
 * cleared between calls: calls that overlap on one GPU (several streams or
 * host threads at once) race and give wrong results.
 * Errors: as cl_integrate, plus LOS_ERR_INVALID when the current device is
 * not the context's.
 */
int cl_integrate_noalloc(los_ctx *ctx, const void *delta, int32_t delta_prec, int32_t nsrc,
                         int32_t nl, int64_t nk, const double *w_lnk, const double *Pk,
                         const int32_t *pairs, int32_t npairs, double *cl, void *stream);

/*
 * Multipole sampling (Sec. 3.1: the output l-sampling density sets how many
 * multipoles are computed explicitly; the others are interpolated).
 *
 * los_project_lsample: the FP64 projection (as los_project_kernels with
 *   prec LOS_FP64) at the multipoles ls[0..nls-1] only:
 *     delta[(i * nls + j) * nsrc + s] = Delta^s_{ls[j]}(k_i).
 *   ls: HOST, nls int32 strictly increasing within [lmin, lmax],
 *   1 <= nls <= lmax - lmin + 1.  The Bessel recurrence still walks every
 *   multipole (it needs them all); the accumulation, the reduction and the
 *   stores happen at the sampled ones only.  Other arguments, limits and
 *   kernel_mask as for los_project_kernels.  The row tables built from ls are
 *   kept in the context; a call with a different list than the previous one
 *   waits for the work queued on `stream` before replacing them.
 *
 * los_cl_interp: C_l at every l in [lmin, lmax] from its values at ls:
 *     cl[p * (lmax - lmin + 1) + l - lmin] = D_p(l) / (l (l + 1)),
 *   D_p the natural cubic spline in l (zero second derivative at both ends)
 *   through the points (ls[j], ls[j] (ls[j] + 1) cls[p * nls + j]).
 *   ls: HOST, strictly increasing, ls[0] = lmin, ls[nls-1] = lmax,
 *   1 <= nls <= 2048; cls: device, npairs*nls doubles (cl_integrate's output
 *   for the sampled delta); cl: device, npairs*(lmax-lmin+1) doubles, distinct
 *   from cls.  1 <= npairs <= 65535.  The knots are kept in the context as for
 *   los_project_lsample.
 *
 * Errors: LOS_ERR_INVALID for NULL pointers, bad lists or sizes;
 * LOS_ERR_UNSUPPORTED when the two-pass FP64 scheme is selected
 * (LOS_PROJ_SCHEME=0) or no launch shape fits ntau.
 */
int los_project_lsample(los_ctx *ctx, int32_t lmin, int32_t lmax, const int32_t *ls,
                        int32_t nls, int64_t nk, int64_t ntau, double tau0, const double *k,
                        const double *tau, const double *w_tau, const double *S, int32_t nsrc,
                        uint32_t kernel_mask, double *delta, void *stream);
int los_cl_interp(los_ctx *ctx, int32_t npairs, const int32_t *ls, int32_t nls,
                  const double *cls, int32_t lmin, int32_t lmax, double *cl, void *stream);

/*
 * Source preparation (Sec. 3.2: before the integrals, InterpolateSources
 * brings the source data onto the integration grid; the paper names the step
 * but not its scheme).  Here the sources are given on a coarse wavenumber
 * grid q_0 < ... < q_{nkc-1} at the projection's tau nodes, and each
 * (source, tau node) column is carried to the projection's k grid by the
 * natural cubic spline in k through its nkc values:
 *
 *   on [q_j, q_{j+1}], h = q_{j+1} - q_j, A = (q_{j+1} - k)/h, B = (k - q_j)/h:
 *   s(k) = A y_j + B y_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) h^2 / 6,
 *
 * M the second derivatives (continuous s'' at the knots, M_0 = M_{nkc-1} = 0).
 *
 * los_spline_sources: M[(s * nkc + j) * ntau + n] for the columns of
 *   Sc[(s * nkc + j) * ntau + n] (s < nsrc, j < nkc, n < ntau).  q: device,
 *   nkc doubles, strictly increasing (not checked: other grids give undefined
 *   values, never an access out of bounds).  Sc, M: device, nsrc*nkc*ntau
 *   doubles, M distinct from Sc.  1 <= nsrc <= 64, 2 <= nkc <= 16386,
 *   ntau >= 1, nsrc*ntau < 2^31.  The tridiagonal systems are solved in FP64
 *   (segments of 16 rows plus a reduced system for the segment ends; no
 *   pivoting is needed, the matrix being strictly diagonally dominant).
 *   Uses the context's workspace (about 40 doubles per 16 knots).
 *
 * los_interp_sources: S[(s * nk + i) * ntau + n] = s(k[i]) for the same
 *   columns, with M from los_spline_sources.  k: device, nk doubles; a k
 *   outside [q_0, q_{nkc-1}] takes the cubic of the end interval.  S: device,
 *   nsrc*nk*ntau values, double for out_prec == LOS_FP64, float (the FP64
 *   value rounded) for LOS_FP32; distinct from Sc and M.  The result is the
 *   S layout that los_project takes.  nk == 0 is a no-op.
 *
 * Errors: LOS_ERR_INVALID for NULL pointers, aliasing, out-of-range sizes or
 * an unknown out_prec.
 */
int los_spline_sources(los_ctx *ctx, int32_t nsrc, int64_t nkc, int64_t ntau, const double *q,
                       const double *Sc, double *M, void *stream);
int los_interp_sources(los_ctx *ctx, int32_t nsrc, int64_t nkc, int64_t ntau, const double *q,
                       const double *Sc, const double *M, int64_t nk, const double *k,
                       int32_t out_prec, void *S, void *stream);

/*
 * Batched solve (Sec. 3.2 / Algorithm 1: the projection is independent per k;
 * Eq. 2-3 and Eq. 1 per model).  nmodels models share one master k grid and
 * one tau grid; model m uses master rows k_index[koff[m] .. koff[m+1]-1]
 * (strictly increasing) and multipoles l = 2..lmax[m].  For every master row,
 * the sources of all models that use it form the columns of one matrix
 * product J_k . S_k (J_k generated once per l tile, FP64 then FP32),
 * computed on the matrix cores in `prec` (LOS_FP32 or LOS_BF16X3), and each
 * model's C_l are summed over its own k in FP64.  By default the Bessel
 * tiles are regenerated in LDS from FP64 recurrence seeds kept every 32
 * multipoles (no Bessel table in device memory); environment
 * LOS_BATCH_FUSED=0 at plan creation selects whole FP32 tables instead.
 *
 * los_batch_create (host arrays; allocates the plan's device tables and a
 * workspace of at most LOS_BATCH_MIB MiB (default 8192) of seeds plus
 * products -- with LOS_BATCH_FUSED=0, LOS_JTAB_MIB MiB (default 4096) of
 * Bessel tables plus one chunk of products): lmax[nmodels] in [2, 16000]; koff[nmodels+1] with koff[0] = 0
 * and koff[m+1] > koff[m]; k_index[koff[nmodels]] in [0, nk_master);
 * pairs[2*npairs] source indices (1 <= npairs <= 16, 1 <= nsrc <= 4);
 * 1 <= ntau <= 8192.  *plan receives a handle released by los_batch_destroy.
 *
 * los_batch_columns (host): col[koff[nmodels]] receives, for every (model m,
 * position j), the packed column p = col[koff[m] + j] of its source 0; source
 * s is column p + s.  *ncols receives the number of packed columns.  The
 * caller stores S_packed[p * ntau + n] = S_s of model m at (k_index[koff[m]+j],
 * tau_n), float.
 *
 * los_batch_solve (device arrays; enqueued on `stream`):
 *   k_master[nk_master], tau[ntau], w_tau[ntau] (double);
 *   S_packed[ncols * ntau] (float);
 *   w_lnk[koff[nmodels]], Pk[koff[nmodels]] (double): model m's ln k
 *     quadrature weights and primordial spectrum at its own k, position
 *     koff[m] + j;
 *   cl[nmodels * npairs * (L - 1)] (double, written), L = max lmax:
 *     cl[(m * npairs + p) * (L - 1) + l - 2] = 4 pi sum_j w P Delta^a Delta^b,
 *     zero for l > lmax[m].
 * The first call times every compiled tile shape of the pipeline (fused:
 * 256 x 128, 128 x 128 and 256 x 256 l x column tiles; tables: fragment
 * tiles and an LDS-staged 256 x 128 split-BF16x3 kernel) on two
 * representative chunks and keeps the fastest; each new set of argument
 * pointers is captured once into a HIP graph that later calls replay.  A
 * plan is not thread-safe.
 * los_batch_info (host): info[10] = {tile l blocks, tile column blocks
 * (table pipeline), rows per chunk, chunks, used master rows, max lmax,
 * tuned, graph captured, fused pipeline (1/0), fused shape index}.
 */
typedef struct los_batch los_batch;

int los_batch_create(los_ctx *ctx, int32_t nmodels, int32_t nsrc, const int32_t *lmax,
                     const int64_t *koff, const int64_t *k_index, int64_t nk_master, int64_t ntau,
                     const int32_t *pairs, int32_t npairs, int32_t prec, los_batch **plan);

int los_batch_columns(const los_batch *plan, int64_t *col, int64_t *ncols);

int los_batch_info(const los_batch *plan, int32_t *info);

int los_batch_solve(los_batch *plan, double tau0, const double *k_master, const double *tau,
                    const double *w_tau, const float *S_packed, const double *w_lnk,
                    const double *Pk, double *cl, void *stream);

/*
 * Instrumented solve (for measurement; not to be called under stream
 * capture): the same launches as los_batch_solve, enqueued directly on
 * `stream` (no graph) with HIP events around each kernel; returns after the
 * stream has reached the last event.  ms (host, 3 doubles) receives the
 * summed device time of the Bessel kernels (seeds or tables), the product
 * kernels and the C_l kernels; launches (host, 3 int32) their launch counts
 * (one each per chunk).  cl and the other arguments as for los_batch_solve.
 */
int los_batch_solve_timed(los_batch *plan, double tau0, const double *k_master,
                          const double *tau, const double *w_tau, const float *S_packed,
                          const double *w_lnk, const double *Pk, double *cl, double *ms,
                          int32_t *launches, void *stream);

void los_batch_destroy(los_batch *plan);

/*
 * C_l emulator.  The paper motivates fast repeated solves for parameter
 * sampling (Sec. 1) but defines no emulator; this one is specified here.
 * A network maps nparam source parameters p (scaled to u = 2 (p - lo) /
 * (hi - lo) - 1) to whitened PCA coefficients of the 4 transformed spectra
 * y = (log TT, log EE, asinh(TE / t_l), log PP) over nl multipoles:
 * `depth` GELU layers of `width` units, then a linear layer of 4 * ncomp
 * outputs, FP32 on the matrix cores.  `members` networks form an ensemble
 * whose spread is the error estimate.  Parameters of one member (nparams
 * floats): for each layer, W (out x in, row-major) then b (out).
 *
 * emu_create: 1 <= nparam <= 64, 1 <= nl <= 20000, 1 <= ncomp <= 104 and
 *   ncomp <= nl, 1 <= width <= 4096, 1 <= depth <= 16, 1 <= members <= 16;
 *   weights Glorot-uniform from SplitMix64(seed).
 * emu_train (device params[n][nparam], cl[n][4][nl] with TT, EE, PP > 0;
 *   host lo, hi [nparam]; host loss_hist[members * epochs] or NULL):
 *   t_l = lower median of |TE_l| (from at most 8192 evenly strided rows);
 *   per spectrum the mean and top ncomp covariance eigenvectors (FP64
 *   randomised subspace iteration, Rayleigh-Ritz) and one coefficient scale
 *   sigma_s = sqrt(variance of the kept components) (stored per component);
 *   targets z = coefficients / sigma_s; then every member is re-initialised
 *   and trained by emu_fit.  n >= ncomp + 8.
 * emu_fit (device u[n][nparam], z[n][4 ncomp], float): Adam (0.9, 0.999,
 *   1e-8) on the mean squared error, minibatches of `batch` rows from a
 *   SplitMix64 Fisher-Yates shuffle per epoch (no shuffle when batch >= n),
 *   step size lr (0.01 + 0.99 (1 + cos(pi (t-1) / T)) / 2) at step t of T;
 *   moments reset at the start.  loss_hist[epochs] (host, or NULL): mean
 *   minibatch loss per epoch.
 * emu_infer (device params[n][nparam] -> cl[n][4][nl] double, err[n] float,
 *   need_fallback[n] uint8): cl = member mean of the reconstructed spectra;
 *   err = max over spectra, l and members of |C_e - C_mean| / scale (scale
 *   |C_mean|, for TE sqrt(C_TT C_EE)); need_fallback = !(err <= threshold).
 * emu_infer_spectra: the same cl, with the estimate per spectrum instead:
 *   err4[n][4] (TT, EE, TE, PP: max over l and members), need4[n][4] =
 *   !(err4 <= threshold), so that a caller re-solves only the spectra that
 *   miss the threshold; max over the four of err4[r] is emu_infer's err[r].
 * emu_forward / emu_loss_grad (device, float): one member's network output
 *   out[n][4 ncomp], and the loss (device, 1 float) with its gradient
 *   (device, nparams floats).
 * emu_get_params / emu_set_params (host, nparams floats of one member);
 * emu_get_pca / emu_set_pca (host): lo, hi [nparam], mean [4][nl],
 *   basis [4][nl][ncomp], sigma [4][ncomp], te_scale [nl].
 * Calls are enqueued on `stream` except those with host outputs, which
 * return when the values are copied.  Not thread-safe per emulator.
 */
typedef struct los_emu los_emu;

int emu_create(los_ctx *ctx, int32_t nparam, int32_t nl, int32_t ncomp, int32_t width,
               int32_t depth, int32_t members, uint64_t seed, los_emu **emu);
void emu_destroy(los_emu *emu);
int emu_nparams(const los_emu *emu, int64_t *count);
int emu_get_params(const los_emu *emu, int32_t member, float *host);
int emu_set_params(los_emu *emu, int32_t member, const float *host);
int emu_get_pca(const los_emu *emu, double *lo, double *hi, double *mean, double *basis,
                double *sigma, double *te_scale);
int emu_set_pca(los_emu *emu, const double *lo, const double *hi, const double *mean,
                const double *basis, const double *sigma, const double *te_scale);
int emu_forward(los_emu *emu, int32_t member, const float *u, int64_t n, float *out,
                void *stream);
int emu_loss_grad(los_emu *emu, int32_t member, const float *u, const float *z, int64_t n,
                  float *loss, float *grad, void *stream);
int emu_fit(los_emu *emu, int32_t member, const float *u, const float *z, int64_t n,
            int32_t epochs, int32_t batch, double lr, float *loss_hist, void *stream);
int emu_train(los_emu *emu, const double *params, const double *lo, const double *hi,
              const double *cl, int64_t n, int32_t epochs, int32_t batch, double lr,
              float *loss_hist, void *stream);
int emu_infer(los_emu *emu, const double *params, int64_t n, double *cl, float *err,
              uint8_t *need_fallback, double threshold, void *stream);
int emu_infer_spectra(los_emu *emu, const double *params, int64_t n, double *cl, float *err4,
                      uint8_t *need4, double threshold, void *stream);

/*
 * Fallback merge: the rows of an emu_infer result that the caller re-solved
 * with the plain method (los_batch_solve on those models) replace the
 * emulator's values, on `stream`:
 *   cl[rows[i]][p][l] = cl_solved[i][p][l]   (p < 4, l < nl), i < nf,
 *   err[rows[i]] = 0, need_fallback[rows[i]] = 0   (err, need_fallback may be NULL).
 * rows: HOST, nf distinct indices in [0, n); cl_solved, cl: device doubles
 * [nf][4][nl] and [n][4][nl] (same layout as emu_infer's output).  nf == 0 is
 * a no-op.  Errors: LOS_ERR_INVALID for bad or repeated rows.
 */
int emu_merge(los_emu *emu, const int64_t *rows, int64_t nf, const double *cl_solved, double *cl,
              int64_t n, float *err, uint8_t *need_fallback, void *stream);

/*
 * One-spectrum fallback merge (after emu_infer_spectra): spectrum s of the
 * rows the caller re-solved replaces the emulator's, on `stream`:
 *   cl[rows[i]][s][l] = cl_solved[i][l]   (l < nl), i < nf,
 *   err4[rows[i]][s] = 0, need4[rows[i]][s] = 0   (err4, need4 may be NULL).
 * For example a solve of the temperature source alone (los_batch_create with
 * pairs {0, 0}) gives cl_solved[nf][1][nl] for s = 0 (TT).  rows: HOST, nf
 * distinct indices in [0, n); cl_solved device doubles [nf][nl]; cl as in
 * emu_infer.  nf == 0 is a no-op.  Errors: LOS_ERR_INVALID for s outside
 * 0..3 or bad or repeated rows.
 */
int emu_merge_spectrum(los_emu *emu, int32_t spectrum, const int64_t *rows, int64_t nf,
                       const double *cl_solved, double *cl, int64_t n, float *err4,
                       uint8_t *need4, void *stream);

/*
 * Checkpoints.  emu_save waits for `stream` (the stream of the emulator's last
 * calls), then writes to `path` a versioned file: a header with the shape
 * (nparam, nl, ncomp, width, depth, members) and seed, every member's
 * parameters and Adam moments (FP32), and, once trained, lo/hi, the PCA mean,
 * basis and sigma and the TE scale t_l (FP64), followed by a 64-bit FNV-1a
 * checksum.  emu_load creates an emulator on ctx's device from such a file;
 * *emu receives it (owned by the caller, released with emu_destroy); inference
 * from it is bitwise that of the emulator that was saved.  Errors:
 * LOS_ERR_INVALID for an unreadable, truncated, corrupt or foreign file,
 * LOS_ERR_UNSUPPORTED for another version, LOS_ERR_OOM / LOS_ERR_HIP from the
 * device.
 */
int emu_save(const los_emu *emu, const char *path, void *stream);
int emu_load(los_ctx *ctx, const char *path, los_emu **emu);

#ifdef __cplusplus
}
#endif

#endif /* LOS_H */
