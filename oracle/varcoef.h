/*
 * varcoef.h -- plain FP64 reference of the variable-coefficient projection
 * D((1/rho_f) G p) = (D u*) / dt, u = u* - dt (1/rho_f) G p (see varcoef.c).
 * TEST INFRASTRUCTURE ONLY.  Grid conventions and boundary codes (0
 * periodic, 1 wall) as in oracle.h.
 */
#ifndef PCX_ORACLE_VARCOEF_H
#define PCX_ORACLE_VARCOEF_H

#include "oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out = D((1/rho_f) G p) */
int oracle_varcoef_apply(const or_grid *g, const double *rho, const double *p, double *out);
/* D((1/rho_f) G p) = rhs - <rhs>, <p> = 0, by preconditioned conjugate
 * gradients to ||r||/||rhs|| <= tol (volume-weighted 2-norms).  Returns 0
 * when converged, 3 when maxit was reached (p holds the last iterate). */
int oracle_varcoef_solve(const or_grid *g, const double *rho, double rho0, const double *rhs, double *p, double tol,
                         int maxit, int *iters, double *relres);
/* the whole variable-coefficient projection of (u, v, w) */
int oracle_varcoef_project(const or_grid *g, double dt, const double *rho, double rho0, const double *u,
                           const double *v, const double *w, double *uo, double *vo, double *wo, double *p,
                           double tol, int maxit, int *iters, double *relres);

#ifdef __cplusplus
}
#endif
#endif
