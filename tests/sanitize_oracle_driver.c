/*
 * Driver for the sanitizer run of the oracle (tests/test_sanitize.py): every
 * entry point of oracle/los_oracle.c on small grids, edge arguments (x = 0,
 * x far beyond lmax, lmin = lmax, one node, one k) and rejected arguments, so
 * that AddressSanitizer and UndefinedBehaviorSanitizer see every code path.
 * Exit status 0 when every call returned what it should.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sph_jl(int32_t lmax, double x, double *out);
int oracle_bessel_table(const double *x, int64_t nx, int32_t lmin, int32_t lmax, double *out);
int oracle_eps_l(int32_t lmax, double x, double *jl, double *out);
int oracle_project_kernels(int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                           const double *k, const double *tau, const double *w_tau,
                           const double *S, int32_t nsrc, uint32_t emask, double *delta,
                           double *absdelta);
int oracle_project(int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                   const double *k, const double *tau, const double *w_tau, const double *S,
                   int32_t nsrc, double *delta, double *absdelta);
int oracle_cl(int32_t nl, int64_t nk, int32_t nsrc, const double *delta, const double *w_lnk,
              const double *Pk, const int32_t *pairs, int32_t npairs, double *cl);
int oracle_tensor_kernels(int32_t lmax, double x, double *jl, double *kt, double *ke, double *kb);
int oracle_project_tensor(int32_t lmin, int32_t lmax, int64_t nk, int64_t ntau, double tau0,
                          const double *k, const double *tau, const double *w_tau,
                          const double *S, double *delta, double *absdelta);

static int failures = 0;

static void expect(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

int main(void)
{
    enum { LMAX = 60, NK = 5, NT = 37, NSRC = 3 };
    double jl[LMAX + 1], e[LMAX + 1], kt[LMAX + 1], ke[LMAX + 1], kb[LMAX + 1];
    const double xs[] = {0.0, 1e-200, 1e-9, 0.5, 7.25, 59.0, 61.5, 300.0, 14000.0};
    for (size_t i = 0; i < sizeof xs / sizeof xs[0]; ++i) {
        expect(oracle_sph_jl(LMAX, xs[i], jl) == 0, "sph_jl");
        expect(isfinite(jl[0]) && isfinite(jl[LMAX]), "sph_jl finite");
        expect(oracle_eps_l(LMAX, xs[i], jl, e) == 0, "eps_l");
        expect(oracle_tensor_kernels(LMAX, xs[i], jl, kt, ke, kb) == 0, "tensor_kernels");
        expect(isfinite(ke[2]) && isfinite(kb[LMAX]), "tensor kernels finite");
    }
    expect(oracle_sph_jl(0, 3.0, jl) == 0, "sph_jl lmax 0");
    expect(oracle_sph_jl(-1, 3.0, jl) != 0, "sph_jl rejects lmax < 0");
    expect(oracle_sph_jl(5, -1.0, jl) != 0, "sph_jl rejects x < 0");
    expect(oracle_sph_jl(5, NAN, jl) != 0, "sph_jl rejects NaN");
    expect(oracle_tensor_kernels(5, INFINITY, jl, kt, ke, kb) != 0, "tensor rejects inf");

    double table[3 * 9];
    expect(oracle_bessel_table(xs, 9, 4, 6, table) == 0, "bessel_table");
    expect(oracle_bessel_table(xs, 0, 4, 6, table) == 0, "bessel_table nx = 0");
    expect(oracle_bessel_table(xs, 9, 6, 4, table) != 0, "bessel_table rejects lmax < lmin");
    expect(oracle_bessel_table(NULL, 9, 4, 6, table) != 0, "bessel_table rejects NULL");

    double k[NK], tau[NT], w[NT], S[NSRC * NK * NT], S2[2 * NK * NT];
    for (int i = 0; i < NK; ++i) k[i] = 1e-3 * pow(10.0, 1.5 * i / (NK - 1));
    for (int n = 0; n < NT; ++n) {
        tau[n] = 14000.0 * n / (NT - 1);
        w[n] = (n == 0 || n == NT - 1) ? 0.5 * 14000.0 / (NT - 1) : 14000.0 / (NT - 1);
    }
    for (int q = 0; q < NSRC * NK * NT; ++q) S[q] = sin(0.37 * q) + 0.1;
    for (int q = 0; q < 2 * NK * NT; ++q) S2[q] = cos(0.11 * q);
    const int nl = LMAX - 2 + 1;
    double *d = malloc(sizeof(double) * NK * nl * NSRC), *A = malloc(sizeof(double) * NK * nl * NSRC);
    double *dt = malloc(sizeof(double) * NK * nl * 3), *At = malloc(sizeof(double) * NK * nl * 3);
    double cl[4 * LMAX];
    if (!d || !A || !dt || !At)
        return 2;
    expect(oracle_project(2, LMAX, NK, NT, 14000.0, k, tau, w, S, NSRC, d, A) == 0, "project");
    expect(oracle_project(2, LMAX, NK, NT, 14000.0, k, tau, w, S, NSRC, d, NULL) == 0,
           "project without A");
    expect(oracle_project_kernels(2, LMAX, NK, NT, 14000.0, k, tau, w, S, NSRC, 0x2u, d, A) == 0,
           "project_kernels E-mode");
    expect(oracle_project(LMAX, LMAX, NK, 1, 14000.0, k, tau, w, S, 1, d, NULL) == 0,
           "project one node, one multipole");
    expect(oracle_project(2, LMAX, 0, NT, 14000.0, k, tau, w, S, NSRC, d, NULL) == 0,
           "project nk = 0");
    expect(oracle_project(2, LMAX, NK, NT, 14000.0, NULL, tau, w, S, NSRC, d, NULL) != 0,
           "project rejects NULL");
    const int32_t pairs[8] = {0, 0, 1, 1, 0, 1, 2, 2};
    double wl[NK], pk[NK];
    for (int i = 0; i < NK; ++i) {
        wl[i] = 0.3;
        pk[i] = 2e-9;
    }
    expect(oracle_project(2, LMAX, NK, NT, 14000.0, k, tau, w, S, NSRC, d, NULL) == 0, "project");
    expect(oracle_cl(nl, NK, NSRC, d, wl, pk, pairs, 4, cl) == 0, "cl");
    const int32_t badpairs[2] = {0, 3};
    expect(oracle_cl(nl, NK, NSRC, d, wl, pk, badpairs, 1, cl) != 0, "cl rejects a bad pair");
    expect(oracle_project_tensor(2, LMAX, NK, NT, 14000.0, k, tau, w, S2, dt, At) == 0,
           "project_tensor");
    for (int q = 0; q < NK * nl * 3; ++q)
        expect(isfinite(dt[q]) && isfinite(At[q]), "tensor delta finite");
    expect(oracle_project_tensor(7, 9, NK, NT, 14000.0, k, tau, w, S2, dt, NULL) == 0,
           "project_tensor lmin 7");
    expect(oracle_project_tensor(1, LMAX, NK, NT, 14000.0, k, tau, w, S2, dt, NULL) != 0,
           "project_tensor rejects lmin < 2");
    free(d);
    free(A);
    free(dt);
    free(At);
    if (failures)
        fprintf(stderr, "%d failures\n", failures);
    else
        printf("sanitized oracle run: every call returned as expected\n");
    return failures ? 1 : 0;
}
