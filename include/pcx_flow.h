/*
 * pcx_flow.h -- C ABI of the Runge-Kutta substep around the pressure
 * correction (CaNS-Fizzy, "Mathematical model" and "Methods and
 * Implementation strategy"): ACDI transport of the phase indicator with its
 * interface-regularization flux, properties linear in the phase indicator,
 * the momentum predictor (centred advection, variable-viscosity stress, CSF
 * surface force, the regularization term of the mass-consistent momentum,
 * body force), the extrapolated pressure, and the low-storage three-step
 * Runge-Kutta update with the pressure-correction step of pcx.h at the end
 * of each substep.
 *
 * Discretization (second order, staggered, the grid and field conventions
 * of pcx.h): psi = eps ln((q + eps_s)/(1 - q + eps_s)) with q = phi clamped
 * to [0, 1]; n = grad psi /
 * |grad psi| at cell centres (central differences); on faces
 * a = gamma [eps grad phi - 1/4 (1 - tanh^2(psi_f/(2 eps))) n_f] with face
 * values by the mean in x, y and linear interpolation in z;
 * d phi/dt = -div(u phi_f) + div a; kappa = -div n_f; momentum per unit
 * mass -div(u u) + [div(mu (grad u + grad u^T)) + sigma kappa_f grad phi +
 * (rho1 - rho2)(a . grad) u] / rho_f + g; rho, mu = phase-2 value +
 * (phase-1 - phase-2 value) phi.  Walls: zero flux, zero normal velocity,
 * no-slip tangential velocity, zero-gradient cell scalars.  Substep s
 * (1..3): q_s = q_{s-1} + Dt (gamma_s R_{s-1} + zeta_s R_{s-2}) with
 * gamma = 8/15, 5/12, 3/4 and zeta = 0, -17/60, -5/12, both right-hand sides
 * from the state at the start of the substep; then the correction with
 * dt = (gamma_s + zeta_s) Dt, the density of the new phase field,
 * rho0 = its minimum and p* = (1 + r) p1 - r p2.
 *
 * Every field is FP64 device memory [nz][ny][nx] of the flow's device.
 * Errors as in pcx.h (return codes, pcx_last_error).
 */
#ifndef PCX_FLOW_H
#define PCX_FLOW_H

#include "pcx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    /* every field finite (INVALID otherwise) */
    double rho1, rho2;   /* densities of phase 1 (phi = 1) and phase 2, > 0 */
    double mu1, mu2;     /* dynamic viscosities, >= 0 */
    double sigma;        /* surface tension, >= 0 */
    double gx, gy, gz;   /* body acceleration */
    double gamma;        /* ACDI velocity scale, >= 0 */
    double eps;          /* ACDI interface thickness, > 0 */
    double eps_s;        /* shift inside the logarithm of psi, >= 0 (1e-100) */
} pcx_flow_params;

typedef struct pcx_flow_s *pcx_flow;

/* Validates grid and parameters, creates the pressure-correction plan
 * (opts as for pcx_plan_create, NULL = FP64) and allocates the substep's
 * workspace (13 fields).  Errors: INVALID, UNSUPPORTED, NOMEM, HIP. */
pcx_status pcx_flow_create(const pcx_grid *grid, const pcx_flow_params *params, const pcx_options *opts,
                           pcx_flow *out);
pcx_status pcx_flow_destroy(pcx_flow flow);

/* Right-hand side of the phase-field transport at every cell centre
 * (rhs must not alias an input).  Enqueues on stream. */
pcx_status pcx_flow_phase_rhs(pcx_flow flow, const double *phi, const double *u, const double *v, const double *w,
                              double *rhs, void *stream);
/* Momentum predictor right-hand side per unit mass on every face (0 on wall
 * faces; outputs must not alias inputs).  Enqueues on stream. */
pcx_status pcx_flow_momentum_rhs(pcx_flow flow, const double *phi, const double *u, const double *v,
                                 const double *w, double *ru, double *rv, double *rw, void *stream);
/* One substep s (1..3) of step Dt > 0 from (phi, u, v, w) with the
 * pressures p1, p2 of the two previous substeps and their ratio r.
 * hphi, hu, hv, hw: the previous substep's right-hand sides on entry
 * (ignored for s = 1), this substep's on return.  These and the outputs
 * phi_out, u_out, v_out, w_out, p_out must not alias any input or each
 * other (INVALID).  The call
 * reads back the minimum density (one 8-byte copy: it synchronizes the
 * stream once) and then enqueues the correction; report as for pcx_step. */
pcx_status pcx_flow_substep(pcx_flow flow, int32_t s, double Dt, const double *phi, const double *u,
                            const double *v, const double *w, const double *p1, const double *p2, double r,
                            double *hphi, double *hu, double *hv, double *hw, double *phi_out, double *u_out,
                            double *v_out, double *w_out, double *p_out, void *stream, pcx_report *report);

/* The same substep up to, not including, the pressure correction: the
 * inputs, hphi .. hw and phi_out as in pcx_flow_substep; returns the
 * predicted velocity u_star, v_star, w_star (0 on wall faces), the density
 * of the updated phase field (rho), the extrapolated pressure p_star, and
 * on the host *rho0 = min rho and *dt = (gamma_s + zeta_s) Dt: the inputs of
 * the correction pcx_flow_substep applies (pcx_step with these gives its
 * outputs bit for bit), for callers that correct otherwise, e.g. with the
 * variable-coefficient projection of pcx_varcoef.h.  Outputs must not alias
 * any input or each other; synchronizes the stream once (rho0). */
pcx_status pcx_flow_predict(pcx_flow flow, int32_t s, double Dt, const double *phi, const double *u,
                            const double *v, const double *w, const double *p1, const double *p2, double r,
                            double *hphi, double *hu, double *hv, double *hw, double *phi_out, double *u_star,
                            double *v_star, double *w_star, double *rho, double *p_star, double *rho0, double *dt,
                            void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PCX_FLOW_H */
