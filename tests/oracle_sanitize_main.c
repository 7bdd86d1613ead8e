/* Standalone driver for the CPU oracle (test infrastructure): calls every
 * entry point of hqr_oracle.h on small seeded inputs so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer sees each code path (AED
 * and sweeps, the small solver, swaps of every block size, rejected swaps,
 * the three deflation conditions, the eigenvalue backward, the QZ variant
 * with infinite eigenvalues).  Exits non-zero on a failed return code or a
 * non-finite result; the sanitizers report memory and arithmetic errors. */
#include "../oracle/hqr_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

/* splitmix64 step, then a uniform double in (-1, 1) */
static double urand(void)
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return ((double)(z >> 11) / 9007199254740992.0) * 2.0 - 1.0;
}

static double *hessenberg(int n)
{
    double *H = calloc((size_t)(n > 0 ? n : 1) * (n > 0 ? n : 1), sizeof(double));
    for (int c = 0; c < n; ++c)
        for (int r = 0; r <= c + 1 && r < n; ++r) H[r + (size_t)c * n] = urand();
    return H;
}

static double *identity(int n)
{
    double *Q = calloc((size_t)(n > 0 ? n : 1) * (n > 0 ? n : 1), sizeof(double));
    for (int i = 0; i < n; ++i) Q[i + (size_t)i * n] = 1.0;
    return Q;
}

static int finite_all(const double *a, size_t len)
{
    for (size_t i = 0; i < len; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int failures = 0;

static void expect(int ok, const char *what, int n)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s (n=%d)\n", what, n);
        ++failures;
    }
}

static void schur_cases(void)
{
    const int sizes[] = {0, 1, 2, 3, 7, 40, 130};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s) {
        const int n = sizes[s], ld = n > 0 ? n : 1;
        double *H = hessenberg(n), *Q = identity(n);
        double *wr = calloc(ld, sizeof(double)), *wi = calloc(ld, sizeof(double));
        const int info = hqr_oracle_schur(H, Q, n, ld, wr, wi);
        expect(info == 0, "schur", n);
        expect(finite_all(H, (size_t)n * n) && finite_all(Q, (size_t)n * n), "schur finite", n);
        free(H), free(Q), free(wr), free(wi);
    }
    /* small windows: AED steps, sweeps and small-block solves all run */
    for (int mode = 0; mode <= 2; ++mode) {
        const int n = 150;
        double *H = hessenberg(n), *Q = identity(n);
        double *wr = calloc(n, sizeof(double)), *wi = calloc(n, sizeof(double));
        int64_t st[6];
        const int info = hqr_oracle_schur_defl(H, Q, n, n, wr, wi, 8, 24, 12, 0, st, mode,
                                               mode == 2 ? 1e-12 : 0.0);
        expect(info == 0, "schur_defl", n);
        expect(st[0] > 0 && st[1] > 0, "schur_defl AED steps and sweeps", n);
        free(H), free(Q), free(wr), free(wi);
    }
    /* iteration limit reached */
    {
        const int n = 120;
        double *H = hessenberg(n), *Q = identity(n);
        double *wr = calloc(n, sizeof(double)), *wi = calloc(n, sizeof(double));
        const int info = hqr_oracle_schur_ex(H, Q, n, n, wr, wi, 0, 0, 0, 1, NULL);
        expect(info > 0, "schur iteration limit", n);
        free(H), free(Q), free(wr), free(wi);
    }
}

static void sweep_aed_cases(void)
{
    const int n = 80;
    double *H = hessenberg(n), *Q = identity(n);
    double sr[8], si[8];
    for (int i = 0; i < 8; i += 2) {
        sr[i] = sr[i + 1] = urand();
        si[i] = fabs(urand());
        si[i + 1] = -si[i];
    }
    expect(hqr_oracle_sweep(H, Q, n, n, 3, n - 5, 8, sr, si, 1) == 0, "sweep", n);
    double cr[80], ci[80];
    int ncand = 0;
    const int nd = hqr_oracle_aed(H, Q, n, n, 0, n - 1, 30, cr, ci, &ncand);
    expect(nd >= 0 && ncand >= 0 && ncand <= 30, "aed", n);
    const int nd2 = hqr_oracle_aed_ex(H, Q, n, n, 0, n - 1 - nd, 24, cr, ci, &ncand, 1, 0.0);
    expect(nd2 >= 0, "aed_ex", n);
    expect(finite_all(H, (size_t)n * n) && finite_all(Q, (size_t)n * n), "sweep/aed finite", n);
    free(H), free(Q);
}

static void swap_cases(void)
{
    /* every block-size combination, on a quasi-triangular matrix with a
       standardized 2x2 block wherever a size is 2 */
    for (int p = 1; p <= 2; ++p)
        for (int q = 1; q <= 2; ++q) {
            const int n = 8, j = 2;
            double T[64], Q[64];
            memset(T, 0, sizeof T);
            for (int c = 0; c < n; ++c)
                for (int r = 0; r <= c; ++r) T[r + c * n] = urand();
            if (p == 2) {
                T[j + j * n] = T[(j + 1) + (j + 1) * n] = 0.5;
                T[j + (j + 1) * n] = 2.0;
                T[(j + 1) + j * n] = -1.5;
            }
            if (q == 2) {
                const int k = j + p;
                T[k + k * n] = T[(k + 1) + (k + 1) * n] = -0.7;
                T[k + (k + 1) * n] = 1.1;
                T[(k + 1) + k * n] = -0.9;
            }
            for (int i = 0; i < 64; ++i) Q[i] = (i % 9 == 0) ? 1.0 : 0.0;
            expect(hqr_oracle_swap(T, Q, n, n, j, p, q) == 0, "swap", 10 * p + q);
            hqr_oracle_force_swap_failure(1);
            expect(hqr_oracle_swap(T, Q, n, n, j, q, p) == 1, "forced swap rejection", 10 * q + p);
            hqr_oracle_force_swap_failure(0);
            double a = 1.0, b = 2.0, c = -3.0, d = 0.5, cs, sn;
            hqr_oracle_std2x2(&a, &b, &c, &d, &cs, &sn);
            expect(isfinite(a) && isfinite(cs), "std2x2", 2);
        }
    hqr_oracle_swap_rejections(1);
}

static void backward_cases(void)
{
    const int n = 30;
    double *H = hessenberg(n), *Q = identity(n), *dH = calloc((size_t)n * n, sizeof(double));
    double wr[30], wi[30], gr[30], gi[30];
    expect(hqr_oracle_schur(H, Q, n, n, wr, wi) == 0, "schur for backward", n);
    for (int i = 0; i < n; ++i) {
        gr[i] = urand();
        gi[i] = (wi[i] != 0.0) ? urand() : 0.0;
    }
    expect(hqr_oracle_eig_backward(H, Q, n, n, wr, wi, gr, gi, dH, 1) == 0, "eig_backward", n);
    expect(finite_all(dH, (size_t)n * n), "eig_backward finite", n);
    free(H), free(Q), free(dH);
}

static void qz_cases(void)
{
    const int sizes[] = {0, 1, 2, 3, 9, 40};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s) {
        const int n = sizes[s], ld = n > 0 ? n : 1;
        double *H = hessenberg(n), *T = calloc((size_t)ld * ld, sizeof(double));
        double *Q = identity(n), *Z = identity(n);
        for (int c = 0; c < n; ++c)
            for (int r = 0; r <= c; ++r) T[r + (size_t)c * n] = urand();
        if (n >= 3) T[1 + (size_t)1 * n] = 0.0; /* an infinite eigenvalue */
        double *ar = calloc(ld, sizeof(double)), *ai = calloc(ld, sizeof(double)), *be = calloc(ld, sizeof(double));
        expect(hqr_oracle_qz(H, T, Q, Z, n, ld, ar, ai, be, 0) == 0, "qz", n);
        expect(finite_all(H, (size_t)n * n) && finite_all(T, (size_t)n * n), "qz finite", n);
        free(H), free(T), free(Q), free(Z), free(ar), free(ai), free(be);
    }
}

int main(void)
{
    schur_cases();
    sweep_aed_cases();
    swap_cases();
    backward_cases();
    qz_cases();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("all oracle entry points ran\n");
    return 0;
}
