/*
 * dirichlet.h -- plain FP64 reference of the constant-coefficient Poisson
 * solve with periodic (0), Neumann / wall (1) or homogeneous Dirichlet (2)
 * directions.  TEST INFRASTRUCTURE ONLY (see dirichlet.c).
 */
#ifndef PCX_ORACLE_DIRICHLET_H
#define PCX_ORACLE_DIRICHLET_H

#include "oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

/* nonzero when some direction of g is Dirichlet (the operator is then
 * non-singular) */
int oracle_has_dirichlet(const or_grid *g);
/* eigenvalue of mode l of the second difference on n cells of spacing h */
double oracle_eig_bc(int n, double h, int bc, int l);
/* L p with the boundary ghosts of each direction's condition */
int oracle_apply_L_bc(const or_grid *g, const double *p, double *out);
/* L p = f for grids with at least one Dirichlet direction; returns 2 (and
 * does nothing) when there is none (the singular case: oracle_poisson). */
int oracle_poisson_bc(const or_grid *g, const double *f, double *p);

#ifdef __cplusplus
}
#endif
#endif
