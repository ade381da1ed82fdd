/*
 * oracle.h -- plain, single-threaded FP64 CPU reference for the
 * pressure-correction step of one Runge-Kutta substep of a one-fluid
 * two-phase solver (CaNS-Fizzy, "Methods and Implementation strategy").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this code; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no source with the GPU path.
 *
 * Conventions (all arrays C-contiguous [k][j][i], i fastest, FP64):
 *   cells i in [0,nx), j in [0,ny), k in [0,nz); dx = lx/nx, dy = ly/ny;
 *   z faces zf[0..nz] (possibly stretched), dzf[k] = zf[k+1]-zf[k],
 *   zc[k] = (zf[k]+zf[k+1])/2, dzc[k] = zc[k+1]-zc[k] (periodic wrap at
 *   k = nz-1: (dzf[nz-1]+dzf[0])/2).
 *   u[k][j][i] lives on the +x face of cell i (likewise v on +y, w on +z).
 *   In a wall direction the last stored face (index n-1) is the wall: it is
 *   ignored on input and written 0; the face below cell 0 is an implicit 0.
 *   bc: 0 = periodic, 1 = wall (zero normal velocity, zero normal gradient).
 */
#ifndef PCX_ORACLE_H
#define PCX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny, nz;
    double lx, ly;
    const double *zf; /* nz+1 face coordinates, strictly increasing */
    int bcx, bcy, bcz;
} or_grid;

typedef struct {
    double f_inf;        /* ||f||inf of the assembled right-hand side        */
    double rel_residual; /* ||f - L p||inf / ||f||inf                         */
    double max_div_abs;  /* max |D u_out|                                     */
    double max_div_rel;  /* max |D u_out| / ((dt/rho0) ||f||inf)              */
    double mean_p;       /* volume-weighted mean of p                         */
} or_diag;

/* 0 on success, 1 for an invalid descriptor or argument. */
int oracle_check_grid(const or_grid *g);

/* Whole step: RHS, Poisson solve with gauge, velocity correction, diagnostics.
 * diag may be NULL. */
int oracle_step(const or_grid *g, double dt, double rho0, const double *rho,
                const double *pstar, const double *u, const double *v,
                const double *w, double *uo, double *vo, double *wo,
                double *po, or_diag *diag);

/* Building blocks, exposed for the pins. */
int oracle_rhs(const or_grid *g, double dt, double rho0, const double *rho,
               const double *pstar, const double *u, const double *v,
               const double *w, double *f);
int oracle_poisson(const or_grid *g, const double *f, double *p);

/* Sampled outputs: f at n flat cell indices; corrected face velocity at n
 * (dir, flat cell index) faces (dir 0/1/2 = u/v/w, +dir face of the cell)
 * given a pressure p.  1 on an invalid argument or index. */
int oracle_rhs_at(const or_grid *g, double dt, double rho0, const double *rho,
                  const double *pstar, const double *u, const double *v,
                  const double *w, int64_t n, const int64_t *cells, double *out);
int oracle_correct_at(const or_grid *g, double dt, double rho0, const double *rho,
                      const double *pstar, const double *u, const double *v,
                      const double *w, const double *p, int64_t n,
                      const int32_t *dirs, const int64_t *cells, double *out);
int oracle_correct(const or_grid *g, double dt, double rho0, const double *rho,
                   const double *pstar, const double *u, const double *v,
                   const double *w, const double *p, double *uo, double *vo,
                   double *wo);
int oracle_grad(const or_grid *g, const double *q, double *gx, double *gy,
                double *gz);
int oracle_div(const or_grid *g, const double *u, const double *v,
               const double *w, double *out);
int oracle_apply_L(const or_grid *g, const double *p, double *out);
double oracle_volume_mean(const or_grid *g, const double *q);
/* Bordered dense LU: [[L, 1],[vol^T, 0]] [p; s] = [f; 0].  At most 1024 cells. */
int oracle_dense_poisson(const or_grid *g, const double *f, double *p);

/* 1-D pieces. fft: in-place complex DFT, unnormalised, sign -1 forward. */
int oracle_fft(int n, double *re, double *im, int sign);
int oracle_dct2(int n, const double *x, double *X);
int oracle_dct3(int n, const double *X, double *x);
/* Tridiagonal a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k]; d is overwritten
 * by x.  cyclic: a[0] couples to x[n-1] and c[n-1] to x[0]. */
int oracle_thomas(int n, const double *a, const double *b, const double *c,
                  double *d);
int oracle_cyclic(int n, const double *a, const double *b, const double *c,
                  double *d);
/* Eigenvalue of the 1-D second-difference operator for mode l (bc 0/1). */
double oracle_eig(int n, double h, int bc, int l);

#ifdef __cplusplus
}
#endif
#endif
