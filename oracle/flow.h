/*
 * flow.h -- plain, single-threaded FP64 CPU reference for the parts of one
 * Runge-Kutta substep of a one-fluid two-phase solver (CaNS-Fizzy,
 * "Mathematical model" and "Methods and Implementation strategy") that
 * surround the pressure-correction step: the ACDI phase-field transport, the
 * momentum predictor, the linear property maps, the extrapolated pressure
 * and the low-storage three-step Runge-Kutta update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this code; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no source with the GPU path.
 *
 * Layout and grid conventions as in oracle.h.  phi is the phase indicator
 * (1 in phase 1, 0 in phase 2) at cell centres.  In a wall direction the
 * walls are no-slip for the tangential velocity (ghost value -u across the
 * wall) and zero-gradient for cell-centred scalars (ghost = the cell itself).
 */
#ifndef PCX_ORACLE_FLOW_H
#define PCX_ORACLE_FLOW_H

#include "oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ACDI parameters: velocity scale Gamma, interface thickness eps, and the
 * small shift eps_s inside the logarithm of psi. */
typedef struct {
    double gamma, eps, eps_s;
} or_acdi;

/* Two-phase parameters: densities and viscosities of phase 1 (phi = 1) and
 * phase 2 (phi = 0), surface tension sigma, body acceleration g, and the
 * ACDI parameters (also used by the regularization term of the momentum). */
typedef struct {
    double rho1, rho2, mu1, mu2, sigma, gx, gy, gz;
    or_acdi acdi;
} or_flow;

/* psi = eps ln((phi + eps_s) / (1 - phi + eps_s)) and the unit normal
 * n = grad psi / |grad psi| (0 where grad psi = 0) at every cell centre. */
int oracle_acdi_normals(const or_grid *g, const or_acdi *a, const double *phi, double *psi, double *nx,
                        double *ny, double *nz);
/* Regularization flux a = Gamma [eps grad phi - 1/4 (1 - tanh^2(psi/(2 eps))) n]
 * on the +x, +y, +z face of every cell (0 on wall faces). */
int oracle_acdi_flux(const or_grid *g, const or_acdi *a, const double *phi, double *ax, double *ay, double *az);
/* Right-hand side of d phi/dt + div(u phi) = div a at every cell centre. */
int oracle_acdi_rhs(const or_grid *g, const or_acdi *a, const double *phi, const double *u, const double *v,
                    const double *w, double *rhs);
/* Curvature kappa = -div n at every cell centre (n from psi, face values
 * by interpolation, 0 on wall faces). */
int oracle_curvature(const or_grid *g, const or_acdi *a, const double *phi, double *kappa);
/* Momentum predictor right-hand side per unit mass on every face (0 on wall
 * faces): -div(u u) + [div(mu (grad u + grad u^T)) + sigma kappa grad phi
 * + (rho1 - rho2)(a . grad) u] / rho_face + g, with rho and mu linear in phi. */
int oracle_momentum_rhs(const or_grid *g, const or_flow *f, const double *phi, const double *u, const double *v,
                        const double *w, double *ru, double *rv, double *rw);
/* Coefficients of substep s (1..3) of the low-storage scheme
 * q_s = q_{s-1} + Dt (gamma_s R_{s-1} + zeta_s R_{s-2}), alpha_s = gamma_s + zeta_s. */
int oracle_rk3_coeffs(int s, double *gamma, double *zeta, double *alpha);
/* One whole substep: phase field, momentum predictor, density of the new
 * phase field, p* = (1 + r) p1 - r p2, pressure-correction step with
 * dt = alpha_s Dt and rho0 = min(rho).  hphi, hu, hv, hw hold the previous
 * substep's right-hand sides on entry (ignored for s = 1) and this
 * substep's on return. */
int oracle_flow_substep(const or_grid *g, const or_flow *f, int s, double Dt, const double *phi, const double *u,
                        const double *v, const double *w, const double *p1, const double *p2, double r,
                        double *hphi, double *hu, double *hv, double *hw, double *phi_out, double *u_out,
                        double *v_out, double *w_out, double *p_out, or_diag *diag);

#ifdef __cplusplus
}
#endif
#endif
