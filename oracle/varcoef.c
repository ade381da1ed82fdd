/*
 * varcoef.c -- plain FP64 reference of the variable-coefficient projection
 * that the splitting replaces ("Methods and Implementation strategy": the
 * conventional variable-coefficient pressure equation, which the paper's
 * code also solves, by multigrid):
 *   D((1/rho_f) G p) = D u* / dt,   <p> = 0,
 *   u = u* - dt (1/rho_f) G p          (0 on wall faces)
 * with rho_f the face density of the projection (mean in x, y, linear
 * interpolation in z).  Its result against the split step's is the
 * splitting error.
 *
 * TEST INFRASTRUCTURE ONLY.  Solved by conjugate gradients in the
 * volume-weighted inner product (the operator is symmetric there),
 * preconditioned by rho0 times the constant-coefficient solve of oracle.c;
 * the singular mode is kept out by removing the volume-weighted mean of
 * the residual.
 */
#include "varcoef.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, nz, bc[3];
    double dx, dy;
    double *dzf, *dzc;
} vgeo;

#define VI(i, j, k) ((((size_t)(k)) * m->ny + (size_t)(j)) * m->nx + (size_t)(i))

static int vgeo_init(const or_grid *g, vgeo *m)
{
    if (oracle_check_grid(g)) return 1;
    m->nx = g->nx; m->ny = g->ny; m->nz = g->nz;
    m->bc[0] = g->bcx; m->bc[1] = g->bcy; m->bc[2] = g->bcz;
    m->dx = g->lx / g->nx;
    m->dy = g->ly / g->ny;
    m->dzf = malloc(sizeof(double) * g->nz);
    m->dzc = malloc(sizeof(double) * g->nz);
    for (int k = 0; k < g->nz; ++k) m->dzf[k] = g->zf[k + 1] - g->zf[k];
    for (int k = 0; k < g->nz - 1; ++k) m->dzc[k] = 0.5 * (m->dzf[k] + m->dzf[k + 1]);
    m->dzc[g->nz - 1] = 0.5 * (m->dzf[g->nz - 1] + m->dzf[0]);
    return 0;
}

static void vgeo_free(vgeo *m)
{
    free(m->dzf);
    free(m->dzc);
}

/* (1/rho_f) (G p) on the +d face of cell (i, j, k); 0 on a wall face */
static double bgrad(const vgeo *m, const double *rho, const double *p, int d, int i, int j, int k)
{
    const int n[3] = {m->nx, m->ny, m->nz};
    int q[3] = {i, j, k};
    const int s = q[d];
    if (m->bc[d] == 1 && s == n[d] - 1) return 0.0;
    q[d] = s == n[d] - 1 ? 0 : s + 1;
    const size_t c = VI(i, j, k), c1 = VI(q[0], q[1], q[2]);
    double rf, h;
    if (d < 2) {
        rf = 0.5 * (rho[c] + rho[c1]);
        h = d == 0 ? m->dx : m->dy;
    } else {
        const int kp = q[2];
        rf = (rho[c] * m->dzf[kp] + rho[c1] * m->dzf[k]) / (2.0 * m->dzc[k]);
        h = m->dzc[k];
    }
    return (p[c1] - p[c]) / h / rf;
}

/* D of the face field computed by bgrad at every cell */
static void apply_impl(const vgeo *m, const double *rho, const double *p, double *out)
{
    const int n[3] = {m->nx, m->ny, m->nz};
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                double s = 0.0;
                const int ix[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    const double up = bgrad(m, rho, p, d, i, j, k);
                    double lo = 0.0;
                    if (!(m->bc[d] == 1 && ix[d] == 0)) {
                        int q[3] = {i, j, k};
                        q[d] = ix[d] == 0 ? n[d] - 1 : ix[d] - 1;
                        lo = bgrad(m, rho, p, d, q[0], q[1], q[2]);
                    }
                    const double h = d == 0 ? m->dx : (d == 1 ? m->dy : m->dzf[k]);
                    s += (up - lo) / h;
                }
                out[VI(i, j, k)] = s;
            }
}

int oracle_varcoef_apply(const or_grid *g, const double *rho, const double *p, double *out)
{
    vgeo m;
    if (!rho || !p || !out || vgeo_init(g, &m)) return 1;
    apply_impl(&m, rho, p, out);
    vgeo_free(&m);
    return 0;
}

static double vdot(const vgeo *m, const double *a, const double *b)
{
    double s = 0.0;
    for (int k = 0; k < m->nz; ++k) {
        double t = 0.0;
        for (size_t c = (size_t)k * m->nx * m->ny; c < (size_t)(k + 1) * m->nx * m->ny; ++c) t += a[c] * b[c];
        s += t * m->dzf[k];
    }
    return s;
}

static void remove_mean(const vgeo *m, double *a)
{
    double num = 0.0, den = 0.0;
    for (int k = 0; k < m->nz; ++k) {
        double t = 0.0;
        for (size_t c = (size_t)k * m->nx * m->ny; c < (size_t)(k + 1) * m->nx * m->ny; ++c) t += a[c];
        num += t * m->dzf[k];
        den += m->dzf[k] * (double)m->nx * (double)m->ny;
    }
    const double mean = num / den;
    const size_t n = (size_t)m->nx * m->ny * m->nz;
    for (size_t c = 0; c < n; ++c) a[c] -= mean;
}

int oracle_varcoef_solve(const or_grid *g, const double *rho, double rho0, const double *rhs, double *p, double tol,
                         int maxit, int *iters, double *relres)
{
    vgeo mm;
    if (!rho || !rhs || !p || !(rho0 > 0.0) || vgeo_init(g, &mm)) return 1;
    const vgeo *m = &mm;
    const size_t n = (size_t)m->nx * m->ny * m->nz;
    /* minus the operator is positive semidefinite in the volume product */
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double)), *d = malloc(n * sizeof(double)),
           *q = malloc(n * sizeof(double));
    memset(p, 0, n * sizeof(double));
    for (size_t c = 0; c < n; ++c) r[c] = -rhs[c];
    remove_mean(m, r);
    const double bnorm = sqrt(vdot(m, r, r));
    int it = 0, rc = 0;
    double res = bnorm > 0.0 ? 1.0 : 0.0;
    if (bnorm > 0.0) {
        /* z = M^-1 r with M = -L / rho0 */
        if (oracle_poisson(g, r, z)) rc = 1;
        for (size_t c = 0; c < n; ++c) z[c] *= -rho0;
        memcpy(d, z, n * sizeof(double));
        double rz = vdot(m, r, z);
        while (!rc && it < maxit) {
            apply_impl(m, rho, d, q);
            for (size_t c = 0; c < n; ++c) q[c] = -q[c];
            const double alpha = rz / vdot(m, d, q);
            for (size_t c = 0; c < n; ++c) {
                p[c] += alpha * d[c];
                r[c] -= alpha * q[c];
            }
            remove_mean(m, r);
            ++it;
            res = sqrt(vdot(m, r, r)) / bnorm;
            if (res <= tol) break;
            if (oracle_poisson(g, r, z)) { rc = 1; break; }
            for (size_t c = 0; c < n; ++c) z[c] *= -rho0;
            const double rz1 = vdot(m, r, z);
            const double beta = rz1 / rz;
            rz = rz1;
            for (size_t c = 0; c < n; ++c) d[c] = z[c] + beta * d[c];
        }
    }
    remove_mean(m, p);
    if (iters) *iters = it;
    if (relres) *relres = res;
    free(r); free(z); free(d); free(q);
    vgeo_free(&mm);
    return rc ? 1 : (res <= tol ? 0 : 3);
}

int oracle_varcoef_project(const or_grid *g, double dt, const double *rho, double rho0, const double *u,
                           const double *v, const double *w, double *uo, double *vo, double *wo, double *p,
                           double tol, int maxit, int *iters, double *relres)
{
    vgeo mm;
    if (!(dt > 0.0) || !u || !v || !w || !uo || !vo || !wo || vgeo_init(g, &mm)) return 1;
    const vgeo *m = &mm;
    const size_t n = (size_t)m->nx * m->ny * m->nz;
    double *rhs = malloc(n * sizeof(double));
    if (oracle_div(g, u, v, w, rhs)) { free(rhs); vgeo_free(&mm); return 1; }
    for (size_t c = 0; c < n; ++c) rhs[c] /= dt;
    const int st = oracle_varcoef_solve(g, rho, rho0, rhs, p, tol, maxit, iters, relres);
    const double *vin[3] = {u, v, w};
    double *vout[3] = {uo, vo, wo};
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i)
                for (int d = 0; d < 3; ++d) {
                    const size_t c = VI(i, j, k);
                    const int s = d == 0 ? i : (d == 1 ? j : k);
                    const int nn = d == 0 ? m->nx : (d == 1 ? m->ny : m->nz);
                    if (m->bc[d] == 1 && s == nn - 1) vout[d][c] = 0.0;
                    else vout[d][c] = vin[d][c] - dt * bgrad(m, rho, p, d, i, j, k);
                }
    free(rhs);
    vgeo_free(&mm);
    return st;
}
