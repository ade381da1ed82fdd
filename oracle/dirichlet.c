/*
 * dirichlet.c -- plain FP64 reference for the constant-coefficient Poisson
 * solve with any mix of periodic, Neumann (wall) and homogeneous Dirichlet
 * directions: the fast direct solver of CaNS that the paper's splitting
 * relies on ("Methods and Implementation strategy"), in its Dirichlet (sine
 * transform) variants as well as the periodic and cosine ones.
 *
 * TEST INFRASTRUCTURE ONLY: the product library never links or calls this
 * file.  Deliberately simple: every x and y transform is an explicit O(n^2)
 * sum over the direction's eigenvectors (complex exponentials, cosines or
 * sines), no FFT; the z direction is a tridiagonal solve per mode.
 *
 * Discretization: cell-centred unknowns, the 7-point operator with variable
 * z spacing.  Across a Dirichlet boundary the ghost value is -p (p = 0 on
 * the boundary face), across a Neumann boundary +p; in z the ghost centre is
 * the mirror image, one cell width away.  Eigenvalues of the second
 * difference (mode l of n cells, spacing h):
 *   periodic  -(4/h^2) sin^2(pi l / n)            vector exp(2 pi i l n' / n)
 *   Neumann   -(4/h^2) sin^2(pi l / (2n))         vector cos(pi l (n' + 1/2) / n)
 *   Dirichlet -(4/h^2) sin^2(pi (l + 1) / (2n))   vector sin(pi (l + 1)(n' + 1/2) / n)
 */
#include "dirichlet.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef struct {
    double re, im;
} zc;

static int check(const or_grid *g)
{
    if (!g || !g->zf || g->nx < 2 || g->ny < 2 || g->nz < 2) return 1;
    if (!(g->lx > 0.0) || !(g->ly > 0.0)) return 1;
    const int bc[3] = {g->bcx, g->bcy, g->bcz};
    for (int d = 0; d < 3; ++d)
        if (bc[d] < 0 || bc[d] > 2) return 1;
    for (int k = 0; k < g->nz; ++k)
        if (!(g->zf[k + 1] > g->zf[k])) return 1;
    return 0;
}

int oracle_has_dirichlet(const or_grid *g) { return g->bcx == 2 || g->bcy == 2 || g->bcz == 2; }

/* eigenvector entry and squared norm of mode l of a direction */
static double basis(int bc, int n, int l, int x, double *im)
{
    *im = 0.0;
    if (bc == 0) {
        const double a = 2.0 * M_PI * (double)l * (double)x / (double)n;
        *im = sin(a);
        return cos(a);
    }
    if (bc == 1) return cos(M_PI * (double)l * ((double)x + 0.5) / (double)n);
    return sin(M_PI * (double)(l + 1) * ((double)x + 0.5) / (double)n);
}

static double norm2(int bc, int n, int l)
{
    if (bc == 0) return (double)n;
    if (bc == 1) return l == 0 ? (double)n : 0.5 * (double)n;
    return l == n - 1 ? (double)n : 0.5 * (double)n;
}

double oracle_eig_bc(int n, double h, int bc, int l)
{
    double s;
    if (bc == 0) {
        const int ll = l <= n - l ? l : n - l;
        s = sin(M_PI * (double)ll / (double)n);
    } else if (bc == 1) {
        s = sin(M_PI * (double)l / (2.0 * (double)n));
    } else {
        s = sin(M_PI * (double)(l + 1) / (2.0 * (double)n));
    }
    return -4.0 / (h * h) * s * s;
}

/* Transform of the lines of a complex array along one direction: out[l] =
 * sum_x in[x] conj(v_l(x)) (forward) or in[l] v_l(x) / |v_l|^2 summed over l
 * (inverse).  stride/count describe the lines. */
static void transform(zc *a, int n, int bc, size_t stride, size_t nlines, size_t lstride, int inverse)
{
    zc *t = malloc(sizeof(zc) * (size_t)n);
    for (size_t q = 0; q < nlines; ++q) {
        zc *line = a + q * lstride;
        for (int o = 0; o < n; ++o) {
            double sr = 0.0, si = 0.0;
            for (int x = 0; x < n; ++x) {
                double vi;
                const int l = inverse ? x : o, pos = inverse ? o : x;
                const double vr = basis(bc, n, l, pos, &vi);
                const zc u = line[(size_t)x * stride];
                if (!inverse) { /* u conj(v) */
                    sr += u.re * vr + u.im * vi;
                    si += u.im * vr - u.re * vi;
                } else { /* u v / |v|^2 */
                    const double w = 1.0 / norm2(bc, n, l);
                    sr += (u.re * vr - u.im * vi) * w;
                    si += (u.im * vr + u.re * vi) * w;
                }
            }
            t[o].re = sr;
            t[o].im = si;
        }
        for (int o = 0; o < n; ++o) line[(size_t)o * stride] = t[o];
    }
    free(t);
}

/* z operator rows for shift s (the x and y eigenvalues): a p_{k-1} + b p_k
 * + c p_{k+1}, cyclic when z is periodic */
static void zrows(const or_grid *g, const double *dzf, const double *dzc, double s, double *a, double *b, double *c)
{
    const int nz = g->nz, bc = g->bcz;
    for (int k = 0; k < nz; ++k) {
        const int per = bc == 0;
        const double dlo = k > 0 ? dzc[k - 1] : (per ? dzc[nz - 1] : dzf[0]);
        const double dhi = k < nz - 1 ? dzc[k] : (per ? dzc[nz - 1] : dzf[nz - 1]);
        a[k] = 1.0 / (dzf[k] * dlo);
        c[k] = 1.0 / (dzf[k] * dhi);
        b[k] = -(a[k] + c[k]) + s;
        if (!per && k == 0) {
            if (bc == 1) b[k] += a[k]; /* Neumann: ghost = p_0 */
            else b[k] -= a[k];         /* Dirichlet: ghost = -p_0 */
            a[k] = 0.0;
        }
        if (!per && k == nz - 1) {
            if (bc == 1) b[k] += c[k];
            else b[k] -= c[k];
            c[k] = 0.0;
        }
    }
}

int oracle_poisson_bc(const or_grid *g, const double *f, double *p)
{
    if (check(g) || !f || !p) return 1;
    if (!oracle_has_dirichlet(g)) return 2; /* singular: oracle_poisson */
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t n = (size_t)nx * ny * nz;
    double *dzf = malloc(sizeof(double) * nz), *dzc = malloc(sizeof(double) * nz);
    for (int k = 0; k < nz; ++k) dzf[k] = g->zf[k + 1] - g->zf[k];
    for (int k = 0; k < nz - 1; ++k) dzc[k] = 0.5 * (dzf[k] + dzf[k + 1]);
    dzc[nz - 1] = 0.5 * (dzf[nz - 1] + dzf[0]);
    zc *a = malloc(sizeof(zc) * n);
    for (size_t q = 0; q < n; ++q) { a[q].re = f[q]; a[q].im = 0.0; }
    /* forward in x (lines of stride 1), then y (stride nx) */
    transform(a, nx, g->bcx, 1, (size_t)ny * nz, (size_t)nx, 0);
    for (int k = 0; k < nz; ++k)
        transform(a + (size_t)k * nx * ny, ny, g->bcy, (size_t)nx, (size_t)nx, 1, 0);
    /* z solve per mode, real and imaginary parts separately */
    double *za = malloc(sizeof(double) * nz), *zb = malloc(sizeof(double) * nz), *zcc = malloc(sizeof(double) * nz);
    double *re = malloc(sizeof(double) * nz), *im = malloc(sizeof(double) * nz);
    const double hx = g->lx / nx, hy = g->ly / ny;
    for (int m = 0; m < ny; ++m)
        for (int l = 0; l < nx; ++l) {
            const double s = oracle_eig_bc(nx, hx, g->bcx, l) + oracle_eig_bc(ny, hy, g->bcy, m);
            zrows(g, dzf, dzc, s, za, zb, zcc);
            for (int k = 0; k < nz; ++k) {
                const zc v = a[((size_t)k * ny + m) * nx + l];
                re[k] = v.re;
                im[k] = v.im;
            }
            int rc;
            if (g->bcz == 0) rc = oracle_cyclic(nz, za, zb, zcc, re) | oracle_cyclic(nz, za, zb, zcc, im);
            else rc = oracle_thomas(nz, za, zb, zcc, re) | oracle_thomas(nz, za, zb, zcc, im);
            if (rc) { free(a); free(za); free(zb); free(zcc); free(re); free(im); free(dzf); free(dzc); return 1; }
            for (int k = 0; k < nz; ++k) {
                zc *v = &a[((size_t)k * ny + m) * nx + l];
                v->re = re[k];
                v->im = im[k];
            }
        }
    for (int k = 0; k < nz; ++k)
        transform(a + (size_t)k * nx * ny, ny, g->bcy, (size_t)nx, (size_t)nx, 1, 1);
    transform(a, nx, g->bcx, 1, (size_t)ny * nz, (size_t)nx, 1);
    for (size_t q = 0; q < n; ++q) p[q] = a[q].re;
    free(a); free(za); free(zb); free(zcc); free(re); free(im); free(dzf); free(dzc);
    return 0;
}

int oracle_apply_L_bc(const or_grid *g, const double *p, double *out)
{
    if (check(g) || !p || !out) return 1;
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const double hx = g->lx / nx, hy = g->ly / ny;
    double *dzf = malloc(sizeof(double) * nz), *dzc = malloc(sizeof(double) * nz);
    for (int k = 0; k < nz; ++k) dzf[k] = g->zf[k + 1] - g->zf[k];
    for (int k = 0; k < nz - 1; ++k) dzc[k] = 0.5 * (dzf[k] + dzf[k + 1]);
    dzc[nz - 1] = 0.5 * (dzf[nz - 1] + dzf[0]);
#define P(i, j, k) p[(((size_t)(k)) * ny + (j)) * nx + (i)]
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double c = P(i, j, k);
                /* neighbour values with the boundary ghosts */
                double e, w, nn, s, t, b;
                if (i < nx - 1) e = P(i + 1, j, k);
                else e = g->bcx == 0 ? P(0, j, k) : (g->bcx == 1 ? c : -c);
                if (i > 0) w = P(i - 1, j, k);
                else w = g->bcx == 0 ? P(nx - 1, j, k) : (g->bcx == 1 ? c : -c);
                if (j < ny - 1) nn = P(i, j + 1, k);
                else nn = g->bcy == 0 ? P(i, 0, k) : (g->bcy == 1 ? c : -c);
                if (j > 0) s = P(i, j - 1, k);
                else s = g->bcy == 0 ? P(i, ny - 1, k) : (g->bcy == 1 ? c : -c);
                if (k < nz - 1) t = P(i, j, k + 1);
                else t = g->bcz == 0 ? P(i, j, 0) : (g->bcz == 1 ? c : -c);
                if (k > 0) b = P(i, j, k - 1);
                else b = g->bcz == 0 ? P(i, j, nz - 1) : (g->bcz == 1 ? c : -c);
                const int per = g->bcz == 0;
                const double dlo = k > 0 ? dzc[k - 1] : (per ? dzc[nz - 1] : dzf[0]);
                const double dhi = k < nz - 1 ? dzc[k] : (per ? dzc[nz - 1] : dzf[nz - 1]);
                out[(((size_t)k) * ny + j) * nx + i] = (e - 2.0 * c + w) / (hx * hx) + (nn - 2.0 * c + s) / (hy * hy) +
                                                       ((t - c) / dhi - (c - b) / dlo) / dzf[k];
            }
#undef P
    free(dzf);
    free(dzc);
    return 0;
}
