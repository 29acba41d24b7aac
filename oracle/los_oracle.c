/*
 * Plain FP64 CPU oracle for the line-of-sight (LOS) projection and the
 * angular power spectrum of a flat-space Einstein-Boltzmann solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  The GPU library shares
 * no code, header or table with it.
 *
 * What it computes (gCAMB paper, Sec. 2.1 "Key equations", Eq. 1-3, and
 * Sec. 3.2 with Algorithm 1):
 *
 *   chi_n          = tau0 - tau_n                      (comoving distance)
 *   x_{i,n}        = k_i * chi_n
 *   Delta^X_l(k_i) = sum_n w_n S_X(k_i, tau_n) j_l(x_{i,n})       (Eq. 2-3)
 *   C^{XY}_l       = 4 pi sum_i w_i P(k_i) Delta^X_l(k_i) Delta^Y_l(k_i)
 *                                                                  (Eq. 1)
 *
 * The radial kernel is the spherical Bessel function j_l for every source
 * (flat space, Sec. 2.1 below Eq. 3).  w_n are the caller's tau-quadrature
 * weights and w_i the caller's ln k quadrature weights (Eq. 1 integrates
 * dk/k = d ln k).  No band cut: every tau contributes to every (l, k).
 *
 * j_l(x) is computed by one of two textbook methods, chosen by x:
 *   x >= lmax + 1 : upward three-term recurrence from the closed forms
 *                   j_0 = sin x / x, j_1 = sin x / x^2 - cos x / x
 *                   (stable while l < x);
 *   otherwise     : Miller's downward recurrence started far above the
 *                   turning point, normalised with the sum rule
 *                   sum_l (2l+1) j_l(x)^2 = 1;
 *   x < 1e-150    : leading power-series terms (exact in FP64 there).
 * All arithmetic is IEEE double, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#if defined(__SSE2__)
#include <xmmintrin.h>
#endif

#define OR_OK 0
#define OR_ERR_INVALID 1
#define OR_ERR_OOM 3

static const double OR_PI = 3.14159265358979323846264338327950288;

/* Subnormal results (|v| < 2.2e-308) are flushed to zero while oracle code
 * runs (FTZ and DAZ in the MXCSR of every thread that runs it): they cannot
 * move any comparison made at the tolerances used, and x86 subnormal
 * arithmetic is ~100x slower.  Everything else is plain IEEE.  Each entry
 * point restores the caller's mode on return, so code that runs after it in
 * the same thread (numpy, the other oracles) keeps IEEE subnormals. */
static unsigned fp_enter(void)
{
#if defined(__SSE2__)
    const unsigned saved = _mm_getcsr();
    _mm_setcsr(saved | 0x8040); /* FTZ | DAZ */
    return saved;
#else
    return 0u;
#endif
}

static void fp_leave(unsigned saved)
{
#if defined(__SSE2__)
    _mm_setcsr(saved);
#else
    (void)saved;
#endif
}

/* Upward recurrence j_{l+1} = (2l+1)/x j_l - j_{l-1}, valid for x >= lmax+1. */
static void jl_upward(int32_t lmax, double x, double *out)
{
    double s = sin(x), c = cos(x);
    out[0] = s / x;
    if (lmax == 0)
        return;
    out[1] = s / (x * x) - c / x;
    for (int32_t l = 1; l < lmax; ++l)
        out[l + 1] = (2.0 * l + 1.0) / x * out[l] - out[l - 1];
}

/* Miller downward recurrence j_{l-1} = (2l+1)/x j_l - j_{l+1} from a start
 * far above max(lmax, x), normalised by the sum rule.  The start value is
 * positive and j_l(x) > 0 for l > x, so the sequence carries the right sign.
 * Whenever the running value grows past 2^100 the two live values and the
 * running sum are brought back near 1 by an exact power-of-two scaling; each
 * stored value remembers the total scaling in force when it was stored
 * (ex[l]), and all stored values are brought to the final scaling at the end. */
static void jl_miller(int32_t lmax, double x, double *out, int *ex)
{
    double xm = x > 1.0 ? x : 1.0;
    int32_t top = lmax > (int32_t)ceil(x) ? lmax : (int32_t)ceil(x);
    int32_t ls = top + (int32_t)ceil(20.0 * cbrt(xm / 2.0)) + 20;
    double jp = 0.0;   /* j~_{l+1} */
    double jc = 1.0;   /* j~_l     */
    double sum = (2.0 * ls + 1.0) * jc * jc;
    int e_tot = 0;     /* values are currently multiplied by 2^-e_tot */
    for (int32_t l = ls; l >= 1; --l) {
        double jn = (2.0 * l + 1.0) / x * jc - jp; /* j~_{l-1} */
        jp = jc;
        jc = jn;
        sum += (2.0 * (l - 1) + 1.0) * jc * jc;
        if (l - 1 <= lmax) {
            out[l - 1] = jc;
            ex[l - 1] = e_tot;
        }
        if (fabs(jc) > 0x1p100) {
            int e = ilogb(jc);
            jc = ldexp(jc, -e);
            jp = ldexp(jp, -e);
            sum = ldexp(sum, -2 * e);
            e_tot += e;
        }
    }
    double norm = sqrt(sum);
    for (int32_t l = 0; l <= lmax; ++l)
        out[l] = ldexp(out[l], ex[l] - e_tot) / norm;
}

/* j_l(x) for l = 0..lmax, x >= 0, into out[0..lmax] (in the oracle's FP mode). */
static int sph_jl_body(int32_t lmax, double x, double *out)
{
    if (lmax < 0 || !(x >= 0.0) || !isfinite(x) || out == NULL)
        return OR_ERR_INVALID;
    if (x < 1e-150) {
        /* power series: j_l(x) = x^l / (2l+1)!! (1 - O(x^2)) */
        for (int32_t l = 0; l <= lmax; ++l)
            out[l] = 0.0;
        out[0] = 1.0;
        if (lmax >= 1)
            out[1] = x / 3.0;
        if (lmax >= 2)
            out[2] = x * x / 15.0;
        return OR_OK;
    }
    if (x >= (double)lmax + 1.0) {
        jl_upward(lmax, x, out);
        return OR_OK;
    }
    int *ex = (int *)malloc(sizeof(int) * (size_t)(lmax + 1));
    if (ex == NULL)
        return OR_ERR_OOM;
    jl_miller(lmax, x, out, ex);
    free(ex);
    return OR_OK;
}

int oracle_sph_jl(int32_t lmax, double x, double *out)
{
    const unsigned fpm = fp_enter();
    const int rc = sph_jl_body(lmax, x, out);
    fp_leave(fpm);
    return rc;
}

/* Table form: out[(l - lmin) * nx + i] = j_l(x[i]), l = lmin..lmax. */
int oracle_bessel_table(const double *x, int64_t nx, int32_t lmin, int32_t lmax, double *out)
{
    if (x == NULL || out == NULL || nx < 0 || lmin < 0 || lmax < lmin)
        return OR_ERR_INVALID;
    int bad = 0;
#pragma omp parallel
    {
        const unsigned fpm = fp_enter();
        double *jl = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        if (jl == NULL) {
#pragma omp atomic write
            bad = OR_ERR_OOM;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nx; ++i) {
            if (jl == NULL)
                continue;
            if (sph_jl_body(lmax, x[i], jl) != OR_OK) {
#pragma omp atomic write
                bad = OR_ERR_INVALID;
                continue;
            }
            for (int32_t l = lmin; l <= lmax; ++l)
                out[(int64_t)(l - lmin) * nx + i] = jl[l];
        }
        free(jl);
        fp_leave(fpm);
    }
    return bad;
}

/*
 * The E-mode radial kernel (Sec. 2.1, Eq. 3 and the text below it):
 *   eps_l(x) = sqrt((l+2)! / (l-2)!) j_l(x) / x^2 = sqrt((l-1) l (l+1) (l+2)) j_l(x) / x^2,
 * for l = 0..lmax into out[0..lmax] (0 for l < 2, where the factorial ratio
 * vanishes).  At x -> 0, j_l(x) / x^2 -> x^(l-2) / (2l+1)!!: 1/15 for l = 2 and
 * 0 above, used for x < 1e-150 (where x^2 would underflow).  jl is scratch
 * for j_l (lmax + 1 values, distinct from out).
 */
/* eps_l(x) from j_l(x), l = 0..lmax (jl and out must not overlap). */
static void eps_from_jl(int32_t lmax, double x, const double *jl, double *out)
{
    for (int32_t l = 0; l <= lmax; ++l)
        out[l] = 0.0;
    if (x < 1e-150) {
        if (lmax >= 2)
            out[2] = sqrt(24.0) / 15.0;
        return;
    }
    const double ix2 = 1.0 / (x * x);
    for (int32_t l = 2; l <= lmax; ++l) {
        const double f = (double)(l - 1) * (double)l * (double)(l + 1) * (double)(l + 2);
        out[l] = sqrt(f) * (jl[l] * ix2);
    }
}

int oracle_eps_l(int32_t lmax, double x, double *jl, double *out)
{
    if (lmax < 0 || !(x >= 0.0) || !isfinite(x) || jl == NULL || out == NULL || jl == out)
        return OR_ERR_INVALID;
    const unsigned fpm = fp_enter();
    int rc = sph_jl_body(lmax, x, jl);
    if (rc == OR_OK)
        eps_from_jl(lmax, x, jl, out);
    fp_leave(fpm);
    return rc;
}

/*
 * Eq. 2-3: delta[(i*nl + (l-lmin))*nsrc + s] = sum_n w_tau[n] S[s][i][n] K_s,l(k_i (tau0 - tau_n))
 * with K_s,l = eps_l for the sources whose bit is set in eps_mask and j_l for
 * the others.  S is [nsrc][nk][ntau] row-major.  If absdelta is not NULL it
 * receives sum_n |w_tau[n] S[s][i][n] K_s,l(x)| in the same layout (the scale
 * used for normwise comparisons).
 */
int oracle_project_kernels(int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                           const double *k, const double *tau, const double *w_tau,
                           const double *S, int32_t nsrc, uint32_t eps_mask, double *delta,
                           double *absdelta)
{
    if (lmin < 0 || lmax < lmin || nk < 0 || ntau < 0 || nsrc < 1 || k == NULL || tau == NULL ||
        w_tau == NULL || S == NULL || delta == NULL)
        return OR_ERR_INVALID;
    const int64_t nl = (int64_t)lmax - lmin + 1;
    int bad = 0;
#pragma omp parallel
    {
        const unsigned fpm = fp_enter();
        double *jl = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        double *el = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        if (jl == NULL || el == NULL) {
#pragma omp atomic write
            bad = OR_ERR_OOM;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nk; ++i) {
            if (jl == NULL || el == NULL)
                continue;
            double *d = delta + i * nl * nsrc;
            double *a = absdelta ? absdelta + i * nl * nsrc : NULL;
            for (int64_t q = 0; q < nl * nsrc; ++q) {
                d[q] = 0.0;
                if (a)
                    a[q] = 0.0;
            }
            for (int64_t n = 0; n < ntau; ++n) {
                double chi = tau0 - tau[n];
                double x = k[i] * chi;
                if (sph_jl_body(lmax, x, jl) != OR_OK) {
#pragma omp atomic write
                    bad = OR_ERR_INVALID;
                    continue;
                }
                if (eps_mask != 0)
                    eps_from_jl(lmax, x, jl, el);
                for (int32_t s = 0; s < nsrc; ++s) {
                    double ws = w_tau[n] * S[((int64_t)s * nk + i) * ntau + n];
                    if (ws == 0.0)
                        continue; /* adds exactly zero */
                    const double *K = ((eps_mask >> s) & 1u) ? el : jl;
                    for (int32_t l = lmin; l <= lmax; ++l) {
                        double term = ws * K[l];
                        d[(int64_t)(l - lmin) * nsrc + s] += term;
                        if (a)
                            a[(int64_t)(l - lmin) * nsrc + s] += fabs(term);
                    }
                }
            }
        }
        free(jl);
        free(el);
        fp_leave(fpm);
    }
    return bad;
}

/*
 * Tensor (gravitational-wave) radial kernels of the line-of-sight method in
 * flat space.  Sec. 2.1 of the gCAMB paper states that tensor perturbations
 * and B modes give equations of the same kind as Eq. 2-3 and cites Seljak &
 * Zaldarriaga (1996) for the method; the kernels are those published for it
 * (Seljak & Zaldarriaga 1996; Zaldarriaga & Seljak 1997, tensor modes):
 *
 *   K^T_l(x) = sqrt((l+2)!/(l-2)!) j_l(x) / x^2
 *   K^E_l(x) = -j_l(x) + j_l''(x) + 2 j_l(x) / x^2 + 4 j_l'(x) / x
 *   K^B_l(x) = 2 j_l'(x) + 4 j_l(x) / x
 *
 * with the derivatives written out from their textbook definitions
 * (DLMF 10.51.2 and the differential equation DLMF 10.47.1):
 *   j_l'  = j_{l-1} - (l+1) j_l / x
 *   j_l'' = -(2/x) j_l' - (1 - l(l+1)/x^2) j_l.
 * For l < 2 every kernel is set to 0 (the spin-2 projection starts at l = 2).
 * At x -> 0 (x < 1e-150, where 1/x^2 would overflow) the power series
 * j_l ~ x^l/(2l+1)!! gives K^T_2 -> sqrt(24)/15, K^E_2 -> 2/15 + 2/15 + 8/15
 * = 4/5, and 0 for K^B_2 and for every kernel at l >= 3.
 * jl is scratch for j_l (lmax + 1 values); kt, ke, kb receive l = 0..lmax.
 */
static void tensor_from_jl(int32_t lmax, double x, const double *jl, double *kt, double *ke,
                           double *kb)
{
    for (int32_t l = 0; l <= lmax; ++l) {
        kt[l] = 0.0;
        ke[l] = 0.0;
        kb[l] = 0.0;
    }
    if (x < 1e-150) {
        if (lmax >= 2) {
            kt[2] = sqrt(24.0) / 15.0;
            ke[2] = 4.0 / 5.0;
        }
        return;
    }
    const double ix = 1.0 / x;
    const double ix2 = ix * ix;
    for (int32_t l = 2; l <= lmax; ++l) {
        const double j = jl[l];
        const double jp = jl[l - 1] - (double)(l + 1) * j * ix;
        const double jpp = -2.0 * ix * jp - (1.0 - (double)l * (double)(l + 1) * ix2) * j;
        const double f = (double)(l - 1) * (double)l * (double)(l + 1) * (double)(l + 2);
        kt[l] = sqrt(f) * (j * ix2);
        ke[l] = -j + jpp + 2.0 * j * ix2 + 4.0 * jp * ix;
        kb[l] = 2.0 * jp + 4.0 * j * ix;
    }
}

/* The three tensor kernels at one x, l = 0..lmax (jl: scratch of lmax + 1). */
int oracle_tensor_kernels(int32_t lmax, double x, double *jl, double *kt, double *ke, double *kb)
{
    if (lmax < 0 || !(x >= 0.0) || !isfinite(x) || jl == NULL || kt == NULL || ke == NULL ||
        kb == NULL)
        return OR_ERR_INVALID;
    const unsigned fpm = fp_enter();
    int rc = sph_jl_body(lmax, x, jl);
    if (rc == OR_OK)
        tensor_from_jl(lmax, x, jl, kt, ke, kb);
    fp_leave(fpm);
    return rc;
}

/*
 * Tensor line-of-sight transfer functions (the tensor analogue of Eq. 2-3):
 *   delta[(i*nl + l-lmin)*3 + 0] = sum_n w_n S_T(k_i, tau_n) K^T_l(x)
 *   delta[(i*nl + l-lmin)*3 + 1] = sum_n w_n S_P(k_i, tau_n) K^E_l(x)
 *   delta[(i*nl + l-lmin)*3 + 2] = sum_n w_n S_P(k_i, tau_n) K^B_l(x)
 * x = k_i (tau0 - tau_n).  S is [2][nk][ntau] (S_T, then S_P), row-major.
 * absdelta (optional) receives the sums of |w S| times the sum of the
 * absolute values of each kernel's terms as written above (for E:
 * |j| + |j''| + |2j/x^2| + |4j'/x|; for B: |2j'| + |4j/x|; for T: |K^T|),
 * the scale of a normwise comparison that the cancellation between a
 * kernel's own terms does not shrink.
 */
int oracle_project_tensor(int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                          const double *k, const double *tau, const double *w_tau,
                          const double *S, double *delta, double *absdelta)
{
    if (lmin < 2 || lmax < lmin || nk < 0 || ntau < 0 || k == NULL || tau == NULL ||
        w_tau == NULL || S == NULL || delta == NULL)
        return OR_ERR_INVALID;
    const int64_t nl = (int64_t)lmax - lmin + 1;
    int bad = 0;
#pragma omp parallel
    {
        const unsigned fpm = fp_enter();
        double *buf = (double *)malloc(sizeof(double) * 7 * (size_t)(lmax + 1));
        if (buf == NULL) {
#pragma omp atomic write
            bad = OR_ERR_OOM;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nk; ++i) {
            if (buf == NULL)
                continue;
            double *jl = buf, *kt = buf + (lmax + 1), *ke = kt + (lmax + 1), *kb = ke + (lmax + 1);
            double *at = kb + (lmax + 1), *ae = at + (lmax + 1), *ab = ae + (lmax + 1);
            double *d = delta + i * nl * 3;
            double *a = absdelta ? absdelta + i * nl * 3 : NULL;
            for (int64_t q = 0; q < nl * 3; ++q) {
                d[q] = 0.0;
                if (a)
                    a[q] = 0.0;
            }
            for (int64_t n = 0; n < ntau; ++n) {
                const double chi = tau0 - tau[n];
                const double x = k[i] * chi;
                if (sph_jl_body(lmax, x, jl) != OR_OK) {
#pragma omp atomic write
                    bad = OR_ERR_INVALID;
                    continue;
                }
                tensor_from_jl(lmax, x, jl, kt, ke, kb);
                if (a) {
                    /* absolute term sums of each kernel (see above) */
                    for (int32_t l = 0; l <= lmax; ++l) {
                        at[l] = fabs(kt[l]);
                        ae[l] = fabs(ke[l]);
                        ab[l] = fabs(kb[l]);
                    }
                    if (x >= 1e-150) {
                        const double ix = 1.0 / x, ix2 = ix * ix;
                        for (int32_t l = 2; l <= lmax; ++l) {
                            const double j = jl[l];
                            const double jp = jl[l - 1] - (double)(l + 1) * j * ix;
                            const double jpp =
                                -2.0 * ix * jp - (1.0 - (double)l * (double)(l + 1) * ix2) * j;
                            ae[l] = fabs(j) + fabs(jpp) + fabs(2.0 * j * ix2) + fabs(4.0 * jp * ix);
                            ab[l] = fabs(2.0 * jp) + fabs(4.0 * j * ix);
                        }
                    }
                }
                const double wt = w_tau[n] * S[((int64_t)0 * nk + i) * ntau + n];
                const double wp = w_tau[n] * S[((int64_t)1 * nk + i) * ntau + n];
                for (int32_t l = lmin; l <= lmax; ++l) {
                    double *dl = d + (int64_t)(l - lmin) * 3;
                    dl[0] += wt * kt[l];
                    dl[1] += wp * ke[l];
                    dl[2] += wp * kb[l];
                    if (a) {
                        double *al = a + (int64_t)(l - lmin) * 3;
                        al[0] += fabs(wt) * at[l];
                        al[1] += fabs(wp) * ae[l];
                        al[2] += fabs(wp) * ab[l];
                    }
                }
            }
        }
        free(buf);
        fp_leave(fpm);
    }
    return bad;
}

/* Eq. 2-3 with the j_l kernel for every source. */
int oracle_project(int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                   const double *k, const double *tau, const double *w_tau, const double *S,
                   int32_t nsrc, double *delta, double *absdelta)
{
    return oracle_project_kernels(lmin, lmax, nk, ntau, tau0, k, tau, w_tau, S, nsrc, 0u, delta,
                                  absdelta);
}

/*
 * Eq. 1 with the ln k quadrature written out:
 *   cl[p*nl + l] = 4 pi sum_i w_lnk[i] Pk[i] delta[i][l][a_p] delta[i][l][b_p]
 * pairs = {a_0, b_0, a_1, b_1, ...} are source indices into delta's last axis.
 */
int oracle_cl(int32_t nl, int64_t nk, int32_t nsrc, const double *delta, const double *w_lnk,
              const double *Pk, const int32_t *pairs, int32_t npairs, double *cl)
{
    if (nl < 1 || nk < 0 || nsrc < 1 || delta == NULL || w_lnk == NULL || Pk == NULL ||
        pairs == NULL || npairs < 1 || cl == NULL)
        return OR_ERR_INVALID;
    for (int32_t p = 0; p < npairs; ++p)
        if (pairs[2 * p] < 0 || pairs[2 * p] >= nsrc || pairs[2 * p + 1] < 0 ||
            pairs[2 * p + 1] >= nsrc)
            return OR_ERR_INVALID;
#pragma omp parallel
    {
        const unsigned fpm = fp_enter();
#pragma omp for schedule(static) collapse(2)
        for (int32_t p = 0; p < npairs; ++p) {
            for (int32_t l = 0; l < nl; ++l) {
                int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
                double acc = 0.0;
                for (int64_t i = 0; i < nk; ++i) {
                    const double *d = delta + ((int64_t)i * nl + l) * nsrc;
                    acc += w_lnk[i] * Pk[i] * d[a] * d[b];
                }
                cl[(int64_t)p * nl + l] = 4.0 * OR_PI * acc;
            }
        }
        fp_leave(fpm);
    }
    return OR_OK;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
