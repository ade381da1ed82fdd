/* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer:
 * whole steps on small grids of every boundary combination (uniform and
 * stretched z), the bordered dense solve, the 1-D pieces over a range of
 * lengths, and the sampled evaluators including rejected indices. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int g_fail = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                       \
        }                                                                   \
    } while (0)

static double urand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return ((*s >> 8) + 0.5) / 16777216.0;
}

int main(void)
{
    unsigned seed = 12345u;
    const int dims[][3] = {{2, 2, 2}, {4, 6, 5}, {6, 3, 4}, {8, 8, 3}, {12, 10, 7}, {16, 9, 6}};
    for (size_t t = 0; t < sizeof dims / sizeof dims[0]; ++t)
        for (int bc = 0; bc < 8; ++bc)
            for (int str = 0; str < 2; ++str) {
                int nx = dims[t][0], ny = dims[t][1], nz = dims[t][2];
                if ((bc & 2) == 0 && ny % 2) continue; /* odd ny needs a wall in y */
                size_t n = (size_t)nx * ny * nz;
                double *zf = malloc((nz + 1) * sizeof(double));
                for (int k = 0; k <= nz; ++k) zf[k] = (double)k / nz + (str && k > 0 && k < nz ? 0.2 / nz * sin(k) : 0.0);
                or_grid g = {nx, ny, nz, 1.0, 1.5, zf, (bc >> 2) & 1, (bc >> 1) & 1, bc & 1};
                double *a[9];
                for (int q = 0; q < 9; ++q) a[q] = malloc(n * sizeof(double));
                for (size_t c = 0; c < n; ++c) {
                    a[0][c] = 1.0 + 999.0 * urand(&seed);
                    for (int q = 1; q < 5; ++q) a[q][c] = urand(&seed) - 0.5;
                }
                or_diag dg;
                CHECK(oracle_step(&g, 1e-3, 1.0, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8], &dg) == 0);
                CHECK(isfinite(dg.max_div_rel) && dg.max_div_rel < 1e-10);
                if (n <= 1024) {
                    double *p = malloc(n * sizeof(double));
                    CHECK(oracle_dense_poisson(&g, a[1], p) == 0);
                    free(p);
                }
                int64_t cells[3] = {0, (int64_t)n - 1, (int64_t)n}; /* the last is out of range */
                int32_t dirs[3] = {0, 2, 1};
                double out[3];
                CHECK(oracle_rhs_at(&g, 1e-3, 1.0, a[0], a[1], a[2], a[3], a[4], 2, cells, out) == 0);
                CHECK(oracle_rhs_at(&g, 1e-3, 1.0, a[0], a[1], a[2], a[3], a[4], 3, cells, out) == 1);
                CHECK(oracle_correct_at(&g, 1e-3, 1.0, a[0], a[1], a[2], a[3], a[4], a[8], 2, dirs, cells, out) == 0);
                CHECK(oracle_correct_at(&g, 1e-3, 1.0, a[0], a[1], a[2], a[3], a[4], a[8], 3, dirs, cells, out) == 1);
                for (int q = 0; q < 9; ++q) free(a[q]);
                free(zf);
            }
    for (int n = 1; n <= 97; ++n) {
        double *re = malloc(n * sizeof(double)), *im = malloc(n * sizeof(double));
        double *x = malloc(n * sizeof(double)), *X = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double));
        for (int i = 0; i < n; ++i) { re[i] = urand(&seed); im[i] = urand(&seed); x[i] = urand(&seed); }
        CHECK(oracle_fft(n, re, im, -1) == 0);
        CHECK(oracle_fft(n, re, im, 1) == 0);
        CHECK(oracle_dct2(n, x, X) == 0);
        CHECK(oracle_dct3(n, X, y) == 0);
        for (int i = 0; i < n; ++i) CHECK(fabs(y[i] - x[i]) < 1e-12);
        double *aa = malloc(n * sizeof(double)), *bb = malloc(n * sizeof(double)), *cc = malloc(n * sizeof(double));
        for (int i = 0; i < n; ++i) { aa[i] = 1.0; cc[i] = 1.0; bb[i] = -4.0; }
        if (n >= 2) CHECK(oracle_thomas(n, aa, bb, cc, x) == 0);
        if (n >= 3) CHECK(oracle_cyclic(n, aa, bb, cc, y) == 0);
        free(re); free(im); free(x); free(X); free(y); free(aa); free(bb); free(cc);
    }
    printf("oracle checks: %d failures\n", g_fail);
    return g_fail ? 1 : 0;
}
