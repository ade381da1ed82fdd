/*
 * pcx_varcoef.h -- C ABI of the variable-coefficient projection that the
 * constant-coefficient splitting replaces (CaNS-Fizzy, "Methods and
 * Implementation strategy": the conventional pressure equation with the
 * density inside the divergence, which needs an iterative solver):
 *   D((1/rho_f) G p) = (D u*) / dt,   <p> = 0 (volume-weighted mean),
 *   u = u* - dt (1/rho_f) G p          (0 on wall faces),
 * with rho_f the face density of pcx_step (mean in x, y, linear
 * interpolation in z).  It is the comparator for the splitting: the
 * difference between its velocity and pcx_step's is the splitting error,
 * and its cost is what the splitting saves.  pcx_step with p_star equal to
 * this p reproduces it exactly.
 *
 * Solved by conjugate gradients in the volume-weighted inner product (the
 * operator is symmetric there), preconditioned by rho0 times the inverse of
 * the constant-coefficient Laplacian: every iteration runs one FP64
 * transform + tridiagonal solve of pcx_poisson_solve.  The residual mean is
 * removed every iteration (the singular mode).  Grid and field conventions
 * of pcx.h (FP64 device fields [nz][ny][nx], face components on the +face);
 * periodic and wall directions only.
 */
#ifndef PCX_VARCOEF_H
#define PCX_VARCOEF_H

#include "pcx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcx_varcoef_s *pcx_varcoef;

/* Validates the grid (a Dirichlet direction: UNSUPPORTED), creates the FP64
 * constant-coefficient plan of the preconditioner (opts as for
 * pcx_plan_create; a precision other than PCX_FP64 is UNSUPPORTED) and
 * allocates four fields of workspace plus reduction slots on the current
 * device.  Errors: INVALID, UNSUPPORTED, NOMEM, HIP; on error *out is NULL. */
pcx_status pcx_varcoef_create(const pcx_grid *grid, const pcx_options *opts, pcx_varcoef *out);
pcx_status pcx_varcoef_destroy(pcx_varcoef vc);

/* out = D((1/rho_f) G p) at every cell (walls: zero flux).  out must not
 * alias rho or p.  Enqueues on `stream`. */
pcx_status pcx_varcoef_apply(pcx_varcoef vc, const double *rho, const double *p, double *out, void *stream);

/* The projection of (u, v, w) with density rho (> 0 everywhere; not
 * checked) and time step dt > 0.  rho0 > 0 scales the preconditioner
 * (normally min rho).  Iterates until the volume-weighted 2-norm of the
 * residual, relative to that of the mean-free right-hand side, is <= tol,
 * or maxit iterations (>= 1).  Outputs u_out, v_out, w_out, p_out must not
 * alias any input or each other.  Synchronizes `stream` once per
 * iteration (the stop test reads the residual norm).  *iters and *relres
 * (either may be NULL) receive the iterations run and the last relative
 * residual.  Returns OK when converged, NOT_CONVERGED (outputs from the
 * last iterate) when maxit was reached, NONFINITE when the residual norm is
 * not finite (outputs undefined). */
pcx_status pcx_varcoef_project(pcx_varcoef vc, double dt, double rho0, const double *rho, const double *u,
                               const double *v, const double *w, double tol, int32_t maxit, double *u_out,
                               double *v_out, double *w_out, double *p_out, void *stream, int32_t *iters,
                               double *relres);

#ifdef __cplusplus
}
#endif
#endif
