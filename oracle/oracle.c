/*
 * oracle.c -- plain FP64 single-threaded reference for the pressure-correction
 * step of a one-fluid two-phase solver (CaNS-Fizzy, "Methods and
 * Implementation strategy": staggered second-order finite differences,
 * pressure-correction projection, a splitting that makes the Poisson equation
 * constant-coefficient, and a fast direct solver with FFTs in x and y and a
 * tridiagonal solve in z).
 *
 * TEST INFRASTRUCTURE ONLY: the product library never links or calls this
 * file.  It is written for clarity, not speed, and deliberately uses different
 * algorithms from the GPU path: a full complex DFT of real rows (no
 * half-length packing), a DCT through the even extension of length 2N, plain
 * Thomas and Sherman-Morrison solves per (l, m) mode, one mode at a time.
 *
 * The definition this reaches (up to rounding):
 *   f     = (rho0/dt) D u* + D[(1 - rho0/rho_face) G p*]
 *   L p   = f - <f>,   <p> = 0,   L = D G           (<.> volume-weighted mean)
 *   u_out = u* - dt [ (1/rho0) G p + (1/rho_face - 1/rho0) G p* ]
 * on every non-wall face, 0 on wall faces.  rho_face is the arithmetic mean
 * of the two neighbouring cells in x and y and the linear interpolation to
 * the face in z; 1/rho_face is the reciprocal of that interpolated density.
 * Build with -ffp-contract=off and without fast-math.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double re, im;
} cx;

typedef struct {
    int nx, ny, nz, bcx, bcy, bcz;
    double dx, dy, lz;
    double *dzf, *zc, *dzc;
} geo;

#define IDX(i, j, k) ((((size_t)(k)) * (size_t)ny + (size_t)(j)) * (size_t)nx + (size_t)(i))

static int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

int oracle_check_grid(const or_grid *g)
{
    if (!g || !g->zf) return 1;
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return 1;
    if (!(g->lx > 0.0) || !(g->ly > 0.0)) return 1;
    if (g->bcx < 0 || g->bcx > 1 || g->bcy < 0 || g->bcy > 1 || g->bcz < 0 || g->bcz > 1) return 1;
    for (int k = 0; k < g->nz; ++k)
        if (!(g->zf[k + 1] > g->zf[k])) return 1;
    return 0;
}

static void geo_free(geo *m)
{
    free(m->dzf);
    free(m->zc);
    free(m->dzc);
}

/* Grid metrics of the staggered grid (uniform x, y; possibly stretched z). */
static int geo_init(const or_grid *g, geo *m)
{
    if (oracle_check_grid(g)) return 1;
    int nz = g->nz;
    m->nx = g->nx; m->ny = g->ny; m->nz = nz;
    m->bcx = g->bcx; m->bcy = g->bcy; m->bcz = g->bcz;
    m->dx = g->lx / g->nx;
    m->dy = g->ly / g->ny;
    m->lz = g->zf[nz] - g->zf[0];
    m->dzf = malloc(sizeof(double) * nz);
    m->zc = malloc(sizeof(double) * nz);
    m->dzc = malloc(sizeof(double) * nz);
    if (!m->dzf || !m->zc || !m->dzc) { geo_free(m); return 1; }
    for (int k = 0; k < nz; ++k) {
        m->dzf[k] = g->zf[k + 1] - g->zf[k];
        m->zc[k] = 0.5 * (g->zf[k] + g->zf[k + 1]);
    }
    for (int k = 0; k < nz - 1; ++k) m->dzc[k] = m->zc[k + 1] - m->zc[k];
    /* periodic wrap distance between the last and the first centre */
    m->dzc[nz - 1] = 0.5 * (m->dzf[nz - 1] + m->dzf[0]);
    return 0;
}

/* ---------------------------------------------------------------- stencils */

/* Face value of a staggered component along a direction of n cells with the
 * given bc, at face index s in [-1, n-1] (face s sits above cell s). */
static double face_val(const double *a, size_t base, size_t stride, int s, int n, int bc)
{
    if (bc == 1) {
        if (s < 0 || s == n - 1) return 0.0; /* wall faces */
        return a[base + (size_t)s * stride];
    }
    return a[base + (size_t)wrapi(s, n) * stride];
}

/* G q on the +dir face of cell (i, j, k); 0 on a wall face. */
static double face_grad(const geo *m, const double *q, int dir, int i, int j, int k)
{
    int nx = m->nx, ny = m->ny, nz = m->nz;
    size_t c = IDX(i, j, k);
    if (dir == 0) {
        if (m->bcx == 1 && i == nx - 1) return 0.0;
        return (q[IDX(wrapi(i + 1, nx), j, k)] - q[c]) / m->dx;
    }
    if (dir == 1) {
        if (m->bcy == 1 && j == ny - 1) return 0.0;
        return (q[IDX(i, wrapi(j + 1, ny), k)] - q[c]) / m->dy;
    }
    if (m->bcz == 1 && k == nz - 1) return 0.0;
    return (q[IDX(i, j, wrapi(k + 1, nz))] - q[c]) / m->dzc[k];
}

/* G: cell centres -> faces.  gx on the +x face of each cell, 0 on wall faces. */
static void grad_impl(const geo *m, const double *q, double *gx, double *gy, double *gz)
{
    int nx = m->nx, ny = m->ny, nz = m->nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IDX(i, j, k);
                if (gx) gx[c] = face_grad(m, q, 0, i, j, k);
                if (gy) gy[c] = face_grad(m, q, 1, i, j, k);
                if (gz) gz[c] = face_grad(m, q, 2, i, j, k);
            }
}

/* D: faces -> cell centres, with wall faces read as 0. */
static void div_impl(const geo *m, const double *u, const double *v, const double *w, double *out)
{
    int nx = m->nx, ny = m->ny, nz = m->nz;
    size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * ny;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IDX(i, j, k);
                size_t bx = IDX(0, j, k), by = IDX(i, 0, k), bz = IDX(i, j, 0);
                double ddx = (face_val(u, bx, sx, i, nx, m->bcx) - face_val(u, bx, sx, i - 1, nx, m->bcx)) / m->dx;
                double ddy = (face_val(v, by, sy, j, ny, m->bcy) - face_val(v, by, sy, j - 1, ny, m->bcy)) / m->dy;
                double ddz = (face_val(w, bz, sz, k, nz, m->bcz) - face_val(w, bz, sz, k - 1, nz, m->bcz)) / m->dzf[k];
                out[c] = ddx + ddy + ddz;
            }
}

/* Density interpolated to the +x/+y/+z face of cell (i,j,k): arithmetic mean
 * in x and y, linear interpolation between the two centres in z. */
static double rho_face(const geo *m, const double *rho, int dir, int i, int j, int k)
{
    int nx = m->nx, ny = m->ny, nz = m->nz;
    double r0 = rho[IDX(i, j, k)];
    if (dir == 0) return 0.5 * (r0 + rho[IDX(wrapi(i + 1, nx), j, k)]);
    if (dir == 1) return 0.5 * (r0 + rho[IDX(i, wrapi(j + 1, ny), k)]);
    int kp = wrapi(k + 1, nz);
    double r1 = rho[IDX(i, j, kp)];
    return (r0 * m->dzf[kp] + r1 * m->dzf[k]) / (2.0 * m->dzc[k]);
}

static int face_is_wall(const geo *m, int dir, int i, int j, int k)
{
    if (dir == 0) return m->bcx == 1 && i == m->nx - 1;
    if (dir == 1) return m->bcy == 1 && j == m->ny - 1;
    return m->bcz == 1 && k == m->nz - 1;
}

/* --------------------------------------------------------------------- FFT */

typedef struct {
    int n;
    cx *w;   /* w[e] = exp(-2 pi i e / n), e in [0, n) */
    cx *tmp; /* scratch, n */
    cx *buf; /* line buffer, n */
    cx *out; /* transform output, n */
} fft_plan;

static int fft_plan_init(fft_plan *p, int n)
{
    p->n = n;
    p->w = malloc(sizeof(cx) * n);
    p->tmp = malloc(sizeof(cx) * n);
    p->buf = malloc(sizeof(cx) * n);
    p->out = malloc(sizeof(cx) * n);
    if (!p->w || !p->tmp || !p->buf || !p->out) return 1;
    for (int e = 0; e < n; ++e) {
        /* exact integer reduction: e is already in [0, n) */
        double ang = 2.0 * M_PI * (double)e / (double)n;
        p->w[e].re = cos(ang);
        p->w[e].im = -sin(ang);
    }
    return 0;
}

static void fft_plan_free(fft_plan *p)
{
    free(p->w);
    free(p->tmp);
    free(p->buf);
    free(p->out);
}

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* y[0..n) = DFT_n of x[0], x[xs], ..., x[(n-1) xs], by recursive
 * decimation in time over the smallest prime factor p of n: n = p m, split
 * into p interleaved subsequences, transform each, then combine with the
 * definition  Y[k + q m] = sum_r W_n^{r (k + q m)} Y_r[k].
 * W is the root table of length N (n divides N); sign -1 forward, +1 inverse. */
static void fft_rec(int n, const cx *x, size_t xs, cx *y, cx *tmp, const cx *W, int N, int sign)
{
    if (n == 1) {
        y[0] = x[0];
        return;
    }
    int p = smallest_factor(n);
    int m = n / p;
    for (int r = 0; r < p; ++r) fft_rec(m, x + (size_t)r * xs, xs * (size_t)p, y + (size_t)r * m, tmp + (size_t)r * m, W, N, sign);
    int step = N / n;
    for (int q = 0; q < p; ++q)
        for (int k = 0; k < m; ++k) {
            int kk = k + q * m;
            double are = 0.0, aim = 0.0;
            for (int r = 0; r < p; ++r) {
                long e = ((long)r * kk) % n;
                cx wv = W[e * step];
                double wim = sign < 0 ? wv.im : -wv.im;
                cx v = y[(size_t)r * m + k];
                are += wv.re * v.re - wim * v.im;
                aim += wv.re * v.im + wim * v.re;
            }
            tmp[kk].re = are;
            tmp[kk].im = aim;
        }
    memcpy(y, tmp, sizeof(cx) * n);
}

/* In-place DFT of the line a[0], a[s], ... (n = plan length). */
static void fft_line(fft_plan *p, cx *a, size_t s, int sign)
{
    int n = p->n;
    for (int i = 0; i < n; ++i) p->buf[i] = a[(size_t)i * s];
    fft_rec(n, p->buf, 1, p->out, p->tmp, p->w, n, sign);
    for (int i = 0; i < n; ++i) a[(size_t)i * s] = p->out[i];
}

int oracle_fft(int n, double *re, double *im, int sign)
{
    if (n < 1 || !re || !im) return 1;
    fft_plan p;
    if (fft_plan_init(&p, n)) { fft_plan_free(&p); return 1; }
    cx *a = malloc(sizeof(cx) * n);
    for (int i = 0; i < n; ++i) { a[i].re = re[i]; a[i].im = im[i]; }
    fft_line(&p, a, 1, sign);
    for (int i = 0; i < n; ++i) { re[i] = a[i].re; im[i] = a[i].im; }
    free(a);
    fft_plan_free(&p);
    return 0;
}

/* DCT-II, X_l = sum_i x_i cos(pi l (i + 1/2) / N), through the DFT of the even
 * extension y = [x_0 .. x_{N-1}, x_{N-1} .. x_0] of length 2N:
 * Y_l = 2 exp(+i pi l / (2N)) X_l.  p2 is a plan of length 2N. */
static void dct2_line(fft_plan *p2, const double *x, size_t xs, double *X, size_t Xs)
{
    int N = p2->n / 2;
    cx *y = malloc(sizeof(cx) * 2 * N);
    for (int i = 0; i < N; ++i) {
        y[i].re = x[(size_t)i * xs]; y[i].im = 0.0;
        y[2 * N - 1 - i].re = x[(size_t)i * xs]; y[2 * N - 1 - i].im = 0.0;
    }
    fft_line(p2, y, 1, -1);
    for (int l = 0; l < N; ++l) {
        double th = M_PI * (double)l / (2.0 * N);
        /* Re(exp(-i th) Y_l) / 2 */
        X[(size_t)l * Xs] = 0.5 * (cos(th) * y[l].re + sin(th) * y[l].im);
    }
    free(y);
}

/* DCT-III inverse of dct2: x_i = (1/N)[X_0 + 2 sum_{l>=1} X_l cos(pi l (i+1/2)/N)],
 * through the inverse DFT of length 2N of Y_l = 2 exp(i pi l/(2N)) X_l,
 * Y_N = 0, Y_{2N-l} = conj(Y_l). */
static void dct3_line(fft_plan *p2, const double *X, size_t Xs, double *x, size_t xs)
{
    int N = p2->n / 2;
    cx *y = malloc(sizeof(cx) * 2 * N);
    for (int l = 0; l < N; ++l) {
        double th = M_PI * (double)l / (2.0 * N);
        double v = 2.0 * X[(size_t)l * Xs];
        y[l].re = v * cos(th);
        y[l].im = v * sin(th);
    }
    y[N].re = 0.0; y[N].im = 0.0;
    for (int l = 1; l < N; ++l) { y[2 * N - l].re = y[l].re; y[2 * N - l].im = -y[l].im; }
    fft_line(p2, y, 1, +1);
    for (int i = 0; i < N; ++i) x[(size_t)i * xs] = y[i].re / (2.0 * N);
    free(y);
}

int oracle_dct2(int n, const double *x, double *X)
{
    if (n < 1 || !x || !X) return 1;
    fft_plan p;
    if (fft_plan_init(&p, 2 * n)) { fft_plan_free(&p); return 1; }
    dct2_line(&p, x, 1, X, 1);
    fft_plan_free(&p);
    return 0;
}

int oracle_dct3(int n, const double *X, double *x)
{
    if (n < 1 || !x || !X) return 1;
    fft_plan p;
    if (fft_plan_init(&p, 2 * n)) { fft_plan_free(&p); return 1; }
    dct3_line(&p, X, 1, x, 1);
    fft_plan_free(&p);
    return 0;
}

/* -------------------------------------------------------------- tridiagonal */

int oracle_thomas(int n, const double *a, const double *b, const double *c, double *d)
{
    if (n < 1) return 1;
    double *cp = malloc(sizeof(double) * n);
    double piv = b[0];
    if (piv == 0.0) { free(cp); return 1; }
    cp[0] = c[0] / piv;
    d[0] = d[0] / piv;
    for (int k = 1; k < n; ++k) {
        piv = b[k] - a[k] * cp[k - 1];
        if (piv == 0.0) { free(cp); return 1; }
        cp[k] = c[k] / piv;
        d[k] = (d[k] - a[k] * d[k - 1]) / piv;
    }
    for (int k = n - 2; k >= 0; --k) d[k] -= cp[k] * d[k + 1];
    free(cp);
    return 0;
}

/* Cyclic tridiagonal by Sherman-Morrison: A = A' + u v^T with
 * u = [gamma, 0, .., 0, c[n-1]], v = [1, 0, .., 0, a[0]/gamma], gamma = -b[0]. */
int oracle_cyclic(int n, const double *a, const double *b, const double *c, double *d)
{
    if (n < 2) return 1;
    double alpha = c[n - 1]; /* A[n-1][0] */
    double beta = a[0];      /* A[0][n-1] */
    double gamma = -b[0];
    double *aa = malloc(sizeof(double) * n), *bb = malloc(sizeof(double) * n);
    double *cc = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    for (int k = 0; k < n; ++k) { aa[k] = a[k]; bb[k] = b[k]; cc[k] = c[k]; z[k] = 0.0; }
    aa[0] = 0.0;
    cc[n - 1] = 0.0;
    bb[0] = b[0] - gamma;
    bb[n - 1] = b[n - 1] - alpha * beta / gamma;
    int rc = oracle_thomas(n, aa, bb, cc, d);
    z[0] = gamma;
    z[n - 1] = alpha;
    rc |= oracle_thomas(n, aa, bb, cc, z);
    if (!rc) {
        double fact = (d[0] + beta * d[n - 1] / gamma) / (1.0 + z[0] + beta * z[n - 1] / gamma);
        for (int k = 0; k < n; ++k) d[k] -= fact * z[k];
    }
    free(aa); free(bb); free(cc); free(z);
    return rc;
}

/* Eigenvalue of the 1-D second difference for mode l: periodic
 * -(4/h^2) sin^2(pi l / n) (l folded to min(l, n-l) so that l and n-l agree
 * bit for bit); cell-centred Neumann (DCT-II basis) -(4/h^2) sin^2(pi l/(2n)). */
double oracle_eig(int n, double h, int bc, int l)
{
    double s;
    if (bc == 0) {
        int ll = l <= n - l ? l : n - l;
        s = sin(M_PI * (double)ll / (double)n);
    } else {
        s = sin(M_PI * (double)l / (2.0 * (double)n));
    }
    return -4.0 / (h * h) * s * s;
}

/* ------------------------------------------------------------------ public */

double oracle_volume_mean(const or_grid *g, const double *q)
{
    geo m;
    if (geo_init(g, &m)) return NAN;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    double num = 0.0, den = 0.0;
    for (int k = 0; k < nz; ++k) {
        double s = 0.0;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) s += q[IDX(i, j, k)];
        num += s * m.dzf[k];
        den += m.dzf[k] * (double)nx * (double)ny;
    }
    geo_free(&m);
    return num / den;
}

int oracle_grad(const or_grid *g, const double *q, double *gx, double *gy, double *gz)
{
    geo m;
    if (geo_init(g, &m)) return 1;
    grad_impl(&m, q, gx, gy, gz);
    geo_free(&m);
    return 0;
}

int oracle_div(const or_grid *g, const double *u, const double *v, const double *w, double *out)
{
    geo m;
    if (geo_init(g, &m)) return 1;
    div_impl(&m, u, v, w, out);
    geo_free(&m);
    return 0;
}

int oracle_apply_L(const or_grid *g, const double *p, double *out)
{
    geo m;
    if (geo_init(g, &m)) return 1;
    size_t n = (size_t)m.nx * m.ny * m.nz;
    double *gx = malloc(sizeof(double) * n), *gy = malloc(sizeof(double) * n), *gz = malloc(sizeof(double) * n);
    grad_impl(&m, p, gx, gy, gz);
    div_impl(&m, gx, gy, gz, out);
    free(gx); free(gy); free(gz);
    geo_free(&m);
    return 0;
}

/* f = (rho0/dt) D u* + D[(1 - rho0/rho_face) G p*]  (splitting right-hand side) */
int oracle_rhs(const or_grid *g, double dt, double rho0, const double *rho, const double *pstar,
               const double *u, const double *v, const double *w, double *f)
{
    if (!(dt > 0.0) || !(rho0 > 0.0)) return 1;
    geo m;
    if (geo_init(g, &m)) return 1;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    size_t n = (size_t)nx * ny * nz;
    double *gx = malloc(sizeof(double) * n), *gy = malloc(sizeof(double) * n), *gz = malloc(sizeof(double) * n);
    double *dv = malloc(sizeof(double) * n);
    grad_impl(&m, pstar, gx, gy, gz);
    double *gg[3] = {gx, gy, gz};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                for (int d = 0; d < 3; ++d) {
                    size_t c = IDX(i, j, k);
                    if (face_is_wall(&m, d, i, j, k)) gg[d][c] = 0.0;
                    else gg[d][c] = (1.0 - rho0 / rho_face(&m, rho, d, i, j, k)) * gg[d][c];
                }
    div_impl(&m, gx, gy, gz, f);
    div_impl(&m, u, v, w, dv);
    for (size_t c = 0; c < n; ++c) f[c] = (rho0 / dt) * dv[c] + f[c];
    free(gx); free(gy); free(gz); free(dv);
    geo_free(&m);
    return 0;
}

/* u_out = u* - dt [ (1/rho0) G p + (1/rho_face - 1/rho0) G p* ], wall faces 0. */
int oracle_correct(const or_grid *g, double dt, double rho0, const double *rho, const double *pstar,
                   const double *u, const double *v, const double *w, const double *p,
                   double *uo, double *vo, double *wo)
{
    if (!(dt > 0.0) || !(rho0 > 0.0)) return 1;
    geo m;
    if (geo_init(g, &m)) return 1;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    size_t n = (size_t)nx * ny * nz;
    double *gp[3], *gs[3];
    for (int d = 0; d < 3; ++d) { gp[d] = malloc(sizeof(double) * n); gs[d] = malloc(sizeof(double) * n); }
    grad_impl(&m, p, gp[0], gp[1], gp[2]);
    grad_impl(&m, pstar, gs[0], gs[1], gs[2]);
    const double *in[3] = {u, v, w};
    double *out[3] = {uo, vo, wo};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                for (int d = 0; d < 3; ++d) {
                    size_t c = IDX(i, j, k);
                    if (face_is_wall(&m, d, i, j, k)) { out[d][c] = 0.0; continue; }
                    double rf = rho_face(&m, rho, d, i, j, k);
                    out[d][c] = in[d][c] - dt * ((1.0 / rho0) * gp[d][c] + (1.0 / rf - 1.0 / rho0) * gs[d][c]);
                }
    for (int d = 0; d < 3; ++d) { free(gp[d]); free(gs[d]); }
    geo_free(&m);
    return 0;
}

/* ------------------------------------------------------ sampled outputs */
/* Point evaluations of the RHS and of the corrected velocity, for checking
 * grids whose full oracle step would not fit a test's time.  Same
 * expressions, in the same order, as oracle_rhs and oracle_correct. */

/* (1 - rho0/rho_face) G p* on the +dir face of cell (i, j, k); 0 on walls. */
static double split_flux(const geo *m, double rho0, const double *rho, const double *pstar, int dir, int i, int j,
                         int k)
{
    if (face_is_wall(m, dir, i, j, k)) return 0.0;
    return (1.0 - rho0 / rho_face(m, rho, dir, i, j, k)) * face_grad(m, pstar, dir, i, j, k);
}

/* flux on the -dir face of cell (i, j, k): the +dir face of the cell below,
 * wrapped when periodic, 0 below the first cell of a wall direction */
static double split_flux_lo(const geo *m, double rho0, const double *rho, const double *pstar, int dir, int i,
                            int j, int k)
{
    int bc = dir == 0 ? m->bcx : (dir == 1 ? m->bcy : m->bcz);
    int s = dir == 0 ? i : (dir == 1 ? j : k);
    int n = dir == 0 ? m->nx : (dir == 1 ? m->ny : m->nz);
    if (s == 0 && bc == 1) return 0.0;
    s = wrapi(s - 1, n);
    return split_flux(m, rho0, rho, pstar, dir, dir == 0 ? s : i, dir == 1 ? s : j, dir == 2 ? s : k);
}

int oracle_rhs_at(const or_grid *g, double dt, double rho0, const double *rho, const double *pstar,
                  const double *u, const double *v, const double *w, int64_t n, const int64_t *cells, double *out)
{
    if (!(dt > 0.0) || !(rho0 > 0.0) || n < 0) return 1;
    geo m;
    if (geo_init(g, &m)) return 1;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * ny;
    for (int64_t s = 0; s < n; ++s) {
        int64_t c = cells[s];
        if (c < 0 || c >= (int64_t)nx * ny * nz) { geo_free(&m); return 1; }
        int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((int64_t)nx * ny));
        size_t bx = IDX(0, j, k), by = IDX(i, 0, k), bz = IDX(i, j, 0);
        double ddx = (face_val(u, bx, sx, i, nx, m.bcx) - face_val(u, bx, sx, i - 1, nx, m.bcx)) / m.dx;
        double ddy = (face_val(v, by, sy, j, ny, m.bcy) - face_val(v, by, sy, j - 1, ny, m.bcy)) / m.dy;
        double ddz = (face_val(w, bz, sz, k, nz, m.bcz) - face_val(w, bz, sz, k - 1, nz, m.bcz)) / m.dzf[k];
        double dv = ddx + ddy + ddz;
        double fx = (split_flux(&m, rho0, rho, pstar, 0, i, j, k) - split_flux_lo(&m, rho0, rho, pstar, 0, i, j, k)) / m.dx;
        double fy = (split_flux(&m, rho0, rho, pstar, 1, i, j, k) - split_flux_lo(&m, rho0, rho, pstar, 1, i, j, k)) / m.dy;
        double fz = (split_flux(&m, rho0, rho, pstar, 2, i, j, k) - split_flux_lo(&m, rho0, rho, pstar, 2, i, j, k)) / m.dzf[k];
        out[s] = (rho0 / dt) * dv + (fx + fy + fz);
    }
    geo_free(&m);
    return 0;
}

int oracle_correct_at(const or_grid *g, double dt, double rho0, const double *rho, const double *pstar,
                      const double *u, const double *v, const double *w, const double *p, int64_t n,
                      const int32_t *dirs, const int64_t *cells, double *out)
{
    if (!(dt > 0.0) || !(rho0 > 0.0) || n < 0) return 1;
    geo m;
    if (geo_init(g, &m)) return 1;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    const double *in[3] = {u, v, w};
    for (int64_t s = 0; s < n; ++s) {
        int64_t c = cells[s];
        int d = dirs[s];
        if (c < 0 || c >= (int64_t)nx * ny * nz || d < 0 || d > 2) { geo_free(&m); return 1; }
        int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((int64_t)nx * ny));
        if (face_is_wall(&m, d, i, j, k)) { out[s] = 0.0; continue; }
        double rf = rho_face(&m, rho, d, i, j, k);
        out[s] = in[d][c] - dt * ((1.0 / rho0) * face_grad(&m, p, d, i, j, k) +
                                  (1.0 / rf - 1.0 / rho0) * face_grad(&m, pstar, d, i, j, k));
    }
    geo_free(&m);
    return 0;
}

/* Solve the z system of mode (l, m) with shift s = lambda_x + lambda_y, for
 * one real right-hand side d (overwritten).  Rows:
 *   a_k p_{k-1} + (s + b_k) p_k + c_k p_{k+1} = d_k,
 *   a_k = 1/(dzf_k dzc_{k-1}), c_k = 1/(dzf_k dzc_k), b_k = -(a_k + c_k),
 * with a_0 = c_{nz-1} = 0 at walls and cyclic corners when periodic.
 * The singular mode (zero shift) is solved with p_{nz-1} pinned to 0 on the
 * first nz-1 rows, then shifted to zero dzf-weighted mean. */
static int zsolve(const geo *m, double s, int singular, double *d, double *a, double *b, double *c)
{
    int nz = m->nz;
    for (int k = 0; k < nz; ++k) {
        int has_lo = (k > 0) || (m->bcz == 0);
        int has_hi = (k < nz - 1) || (m->bcz == 0);
        a[k] = has_lo ? 1.0 / (m->dzf[k] * m->dzc[wrapi(k - 1, nz)]) : 0.0;
        c[k] = has_hi ? 1.0 / (m->dzf[k] * m->dzc[k]) : 0.0;
        b[k] = s - (a[k] + c[k]);
    }
    int rc;
    if (singular) {
        int n1 = nz - 1;
        double a0 = a[0], cl = c[n1 - 1];
        a[0] = 0.0;      /* coupling to the pinned p_{nz-1} = 0 */
        c[n1 - 1] = 0.0; /* likewise */
        rc = oracle_thomas(n1, a, b, c, d);
        a[0] = a0; c[n1 - 1] = cl;
        d[n1] = 0.0;
        double num = 0.0;
        for (int k = 0; k < nz; ++k) num += m->dzf[k] * d[k];
        double mean = num / m->lz;
        for (int k = 0; k < nz; ++k) d[k] -= mean;
    } else if (m->bcz == 0) {
        rc = oracle_cyclic(nz, a, b, c, d);
    } else {
        rc = oracle_thomas(nz, a, b, c, d);
    }
    return rc;
}

/* p with L p = f - <f>, <p> = 0, by transforms in x and y and a tridiagonal
 * solve in z per mode pair. */
int oracle_poisson(const or_grid *g, const double *f, double *p)
{
    geo m;
    if (geo_init(g, &m)) return 1;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    size_t n = (size_t)nx * ny * nz;
    int rc = 0;
    cx *F = malloc(sizeof(cx) * n);
    if (!F) { geo_free(&m); return 1; }

    /* O4: compatibility, f - <f> */
    double fm = oracle_volume_mean(g, f);
    for (size_t c = 0; c < n; ++c) { F[c].re = f[c] - fm; F[c].im = 0.0; }

    fft_plan px, py;
    int lx_len = m.bcx == 0 ? nx : 2 * nx;
    int ly_len = m.bcy == 0 ? ny : 2 * ny;
    int nmax = nx > ny ? nx : ny;
    double *tre = malloc(sizeof(double) * nmax);
    double *tim = malloc(sizeof(double) * nmax);
    double *tout = malloc(sizeof(double) * nmax);
    if (fft_plan_init(&px, lx_len) | fft_plan_init(&py, ly_len)) { rc = 1; goto done; }

    /* O5: forward x (rows), then forward y (columns) */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            cx *row = F + IDX(0, j, k);
            if (m.bcx == 0) {
                fft_line(&px, row, 1, -1);
            } else {
                for (int i = 0; i < nx; ++i) { tre[i] = row[i].re; tim[i] = row[i].im; }
                dct2_line(&px, tre, 1, tout, 1);
                for (int i = 0; i < nx; ++i) row[i].re = tout[i];
                dct2_line(&px, tim, 1, tout, 1);
                for (int i = 0; i < nx; ++i) row[i].im = tout[i];
            }
        }
    for (int k = 0; k < nz; ++k)
        for (int l = 0; l < nx; ++l) {
            cx *col = F + IDX(l, 0, k);
            if (m.bcy == 0) {
                fft_line(&py, col, (size_t)nx, -1);
            } else {
                for (int j = 0; j < ny; ++j) { tre[j] = col[(size_t)j * nx].re; tim[j] = col[(size_t)j * nx].im; }
                dct2_line(&py, tre, 1, tout, 1);
                for (int j = 0; j < ny; ++j) col[(size_t)j * nx].re = tout[j];
                dct2_line(&py, tim, 1, tout, 1);
                for (int j = 0; j < ny; ++j) col[(size_t)j * nx].im = tout[j];
            }
        }

    /* O6: z solve per (l, m) */
    {
        double *za = malloc(sizeof(double) * nz), *zb = malloc(sizeof(double) * nz), *zc = malloc(sizeof(double) * nz);
        double *dre = malloc(sizeof(double) * nz), *dim = malloc(sizeof(double) * nz);
        for (int mm = 0; mm < ny && !rc; ++mm)
            for (int l = 0; l < nx && !rc; ++l) {
                double s = oracle_eig(nx, m.dx, m.bcx, l) + oracle_eig(ny, m.dy, m.bcy, mm);
                int singular = (l == 0 && mm == 0);
                for (int k = 0; k < nz; ++k) { dre[k] = F[IDX(l, mm, k)].re; dim[k] = F[IDX(l, mm, k)].im; }
                rc |= zsolve(&m, s, singular, dre, za, zb, zc);
                rc |= zsolve(&m, s, singular, dim, za, zb, zc);
                for (int k = 0; k < nz; ++k) { F[IDX(l, mm, k)].re = dre[k]; F[IDX(l, mm, k)].im = dim[k]; }
            }
        free(za); free(zb); free(zc); free(dre); free(dim);
    }

    /* O7: inverse y, then inverse x, with 1/N each */
    for (int k = 0; k < nz; ++k)
        for (int l = 0; l < nx; ++l) {
            cx *col = F + IDX(l, 0, k);
            if (m.bcy == 0) {
                fft_line(&py, col, (size_t)nx, +1);
                for (int j = 0; j < ny; ++j) { col[(size_t)j * nx].re /= ny; col[(size_t)j * nx].im /= ny; }
            } else {
                for (int j = 0; j < ny; ++j) { tre[j] = col[(size_t)j * nx].re; tim[j] = col[(size_t)j * nx].im; }
                dct3_line(&py, tre, 1, tout, 1);
                for (int j = 0; j < ny; ++j) col[(size_t)j * nx].re = tout[j];
                dct3_line(&py, tim, 1, tout, 1);
                for (int j = 0; j < ny; ++j) col[(size_t)j * nx].im = tout[j];
            }
        }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            cx *row = F + IDX(0, j, k);
            if (m.bcx == 0) {
                fft_line(&px, row, 1, +1);
                for (int i = 0; i < nx; ++i) p[IDX(i, j, k)] = row[i].re / nx;
            } else {
                for (int i = 0; i < nx; ++i) tre[i] = row[i].re;
                dct3_line(&px, tre, 1, tout, 1);
                for (int i = 0; i < nx; ++i) p[IDX(i, j, k)] = tout[i];
            }
        }
    /* O8: gauge, <p> = 0 */
    {
        double pm = oracle_volume_mean(g, p);
        for (size_t c = 0; c < n; ++c) p[c] -= pm;
    }
done:
    free(tre); free(tim); free(tout);
    fft_plan_free(&px);
    fft_plan_free(&py);
    free(F);
    geo_free(&m);
    return rc;
}

static double max_abs(const double *a, size_t n)
{
    double mx = 0.0;
    for (size_t c = 0; c < n; ++c) {
        double v = fabs(a[c]);
        if (v > mx || v != v) mx = v;
    }
    return mx;
}

int oracle_step(const or_grid *g, double dt, double rho0, const double *rho, const double *pstar,
                const double *u, const double *v, const double *w,
                double *uo, double *vo, double *wo, double *po, or_diag *diag)
{
    if (oracle_check_grid(g) || !(dt > 0.0) || !(rho0 > 0.0)) return 1;
    if (!rho || !pstar || !u || !v || !w || !uo || !vo || !wo || !po) return 1;
    size_t n = (size_t)g->nx * g->ny * g->nz;
    double *f = malloc(sizeof(double) * n);
    if (!f) return 1;
    int rc = oracle_rhs(g, dt, rho0, rho, pstar, u, v, w, f);
    if (!rc) rc = oracle_poisson(g, f, po);
    if (!rc) rc = oracle_correct(g, dt, rho0, rho, pstar, u, v, w, po, uo, vo, wo);
    if (!rc && diag) {
        double *t = malloc(sizeof(double) * n);
        oracle_apply_L(g, po, t);
        for (size_t c = 0; c < n; ++c) t[c] = f[c] - t[c];
        diag->f_inf = max_abs(f, n);
        diag->rel_residual = max_abs(t, n) / diag->f_inf;
        oracle_div(g, uo, vo, wo, t);
        diag->max_div_abs = max_abs(t, n);
        diag->max_div_rel = diag->max_div_abs / ((dt / rho0) * diag->f_inf);
        diag->mean_p = oracle_volume_mean(g, po);
        free(t);
    }
    free(f);
    return rc;
}

/* Bordered dense system [[L, 1], [vol^T, 0]] [p; s] = [f; 0], solved by
 * Gaussian elimination with partial pivoting.  The columns of L are L applied
 * to unit vectors.  Brute force for grids of at most 1024 cells. */
int oracle_dense_poisson(const or_grid *g, const double *f, double *p)
{
    geo m;
    if (geo_init(g, &m)) return 1;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    int n = nx * ny * nz;
    if (n > 1024) { geo_free(&m); return 1; }
    int N = n + 1;
    double *A = calloc((size_t)N * N, sizeof(double));
    double *rhs = calloc(N, sizeof(double));
    double *e = calloc(n, sizeof(double)), *col = calloc(n, sizeof(double));
    for (int jc = 0; jc < n; ++jc) {
        e[jc] = 1.0;
        oracle_apply_L(g, e, col);
        e[jc] = 0.0;
        for (int r = 0; r < n; ++r) A[(size_t)r * N + jc] = col[r];
    }
    for (int r = 0; r < n; ++r) { A[(size_t)r * N + n] = 1.0; rhs[r] = f[r]; }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) A[(size_t)n * N + IDX(i, j, k)] = m.dx * m.dy * m.dzf[k];
    int rc = 0;
    for (int c = 0; c < N && !rc; ++c) {
        int piv = c;
        for (int r = c + 1; r < N; ++r)
            if (fabs(A[(size_t)r * N + c]) > fabs(A[(size_t)piv * N + c])) piv = r;
        if (A[(size_t)piv * N + c] == 0.0) { rc = 1; break; }
        if (piv != c) {
            for (int q = 0; q < N; ++q) {
                double t = A[(size_t)c * N + q]; A[(size_t)c * N + q] = A[(size_t)piv * N + q]; A[(size_t)piv * N + q] = t;
            }
            double t = rhs[c]; rhs[c] = rhs[piv]; rhs[piv] = t;
        }
        for (int r = c + 1; r < N; ++r) {
            double fac = A[(size_t)r * N + c] / A[(size_t)c * N + c];
            if (fac == 0.0) continue;
            for (int q = c; q < N; ++q) A[(size_t)r * N + q] -= fac * A[(size_t)c * N + q];
            rhs[r] -= fac * rhs[c];
        }
    }
    if (!rc) {
        for (int r = N - 1; r >= 0; --r) {
            double s = rhs[r];
            for (int q = r + 1; q < N; ++q) s -= A[(size_t)r * N + q] * rhs[q];
            rhs[r] = s / A[(size_t)r * N + r];
        }
        for (int r = 0; r < n; ++r) p[r] = rhs[r];
    }
    free(A); free(rhs); free(e); free(col);
    geo_free(&m);
    return rc;
}
