/* The oracle on small problems under AddressSanitizer, LeakSanitizer and
 * UndefinedBehaviorSanitizer (built and run by test_oracle_sanitizers.py):
 * every kernel family, calibrated and given r1, r2, the three DataReduct
 * methods, the swap pass, duplicate points and a single point.  Exits 0 when
 * every product is finite and within 100 tol of the dense product. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct h2o h2o;
h2o *h2o_build_ex(const double *pts, int n, int d, int kid, const double *prm, double tol, int q, double tau,
                  int r1, int r2, uint64_t seed, int nthreads, int dr, double srrqr_f);
void h2o_free(h2o *h);
void h2o_matvec(const h2o *h, const double *x, double *y, int nrhs);
void h2o_dense_rows(const double *pts, int n, int d, int kid, const double *prm, const double *x, int nrhs,
                    const int *rows, int nrows, double *out, int nthreads);

static uint64_t state = 12345;
static double u01(void)
{
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) * 0x1.0p-53;
}

static int run(const char *name, int n, int d, int kid, double prm, double tol, int q, int r, int dr, double f,
               int ndup)
{
    double *P = malloc(sizeof(double) * n * d), *x = malloc(sizeof(double) * 2 * n);
    double *y = malloc(sizeof(double) * 2 * n), *yd = malloc(sizeof(double) * 2 * n);
    int *rows = malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) {
        rows[i] = i;
        for (int a = 0; a < d; ++a) P[i * d + a] = i < ndup ? 0.5 : u01();
    }
    for (int i = 0; i < 2 * n; ++i) x[i] = 2.0 * u01() - 1.0;
    h2o *h = h2o_build_ex(P, n, d, kid, &prm, tol, q, 0.7, r, 2 * r, 0x5EED, 2, dr, f);
    int ok = h != NULL;
    double num = 0.0, den = 0.0;
    if (ok) {
        h2o_matvec(h, x, y, 2);
        h2o_dense_rows(P, n, d, kid, &prm, x, 2, rows, n, yd, 2);
        for (int i = 0; i < 2 * n; ++i) {
            ok = ok && isfinite(y[i]);
            num += (y[i] - yd[i]) * (y[i] - yd[i]);
            den += yd[i] * yd[i];
        }
        const double e = den > 0.0 ? sqrt(num / den) : sqrt(num);
        ok = ok && e <= 100.0 * tol;
        printf("%s: n %d error %.2e %s\n", name, n, e, ok ? "ok" : "FAILED");
        h2o_free(h);
    } else {
        printf("%s: build returned NULL\n", name);
    }
    free(P);
    free(x);
    free(y);
    free(yd);
    free(rows);
    return ok;
}

int main(void)
{
    int ok = 1;
    ok &= run("coulomb-3d-calibrated", 1500, 3, 0, 1.0, 1e-4, 32, 0, 0, 0.0, 0);
    ok &= run("gaussian-2d-fps", 1200, 2, 1, 0.1, 1e-5, 24, 64, 1, 0.0, 0);
    ok &= run("matern-3d-surface-swaps", 1000, 3, 3, 0.2, 1e-5, 24, 50, 2, 1.2, 0);
    ok &= run("exponential-1d-duplicates", 600, 1, 2, 0.3, 1e-6, 16, 20, 0, 0.0, 150);
    ok &= run("bump-3d", 900, 3, 4, 0.1, 1e-5, 24, 40, 0, 0.0, 0);
    ok &= run("cosine-3d", 800, 3, 5, 1.0, 1e-5, 24, 40, 0, 0.0, 0);
    ok &= run("advection-3d", 800, 3, 6, 2.0, 1e-5, 24, 60, 0, 0.0, 0);
    ok &= run("single-point", 1, 3, 0, 1.0, 1e-6, 8, 0, 0, 0.0, 0);
    return ok ? 0 : 1;
}
