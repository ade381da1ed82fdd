// varcoef_host.cpp -- C ABI of the variable-coefficient projection:
// validation, workspace, and the conjugate-gradient loop (kernels in
// varcoef_kernels.hip, preconditioner = the plan's FP64 constant-coefficient
// solve, pcx_poisson_solve).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "pcx.h"
#include "pcx_plan.hpp"
#include "pcx_varcoef.h"
#include "varcoef_launch.hpp"

using namespace pcx;
using namespace pcx::vc;

struct pcx_varcoef_s {
    std::vector<double> zf;
    flow::FGrid G;
    flow::TilePlan tp;
    pcx_plan plan = nullptr;
    double *tab = nullptr; // z metric tables (metric_tables)
    double *ws = nullptr;  // r, z, d, q
    double *red = nullptr; // partials, first level, scalars
    size_t ncell = 0;
    double *r, *z, *d, *q;
    VRed R;
};

static void vc_free(pcx_varcoef V)
{
    if (!V) return;
    if (V->plan) pcx_plan_destroy(V->plan);
    if (V->tab) (void)hipFree(V->tab);
    if (V->ws) (void)hipFree(V->ws);
    if (V->red) (void)hipFree(V->red);
    delete V;
}

#define VCHK(x)                                                                                          \
    do {                                                                                                 \
        hipError_t e_ = (x);                                                                             \
        if (e_ != hipSuccess) return fail(PCX_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" pcx_status pcx_varcoef_create(const pcx_grid *grid, const pcx_options *opts, pcx_varcoef *out)
{
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    pcx_status st = validate_grid(grid);
    if (st != PCX_OK) return st;
    if (grid->bc_x == PCX_BC_DIRICHLET || grid->bc_y == PCX_BC_DIRICHLET || grid->bc_z == PCX_BC_DIRICHLET)
        return fail(PCX_ERR_UNSUPPORTED, "the projection takes periodic and wall boundaries only");
    if (opts && opts->precision != PCX_FP64)
        return fail(PCX_ERR_UNSUPPORTED, "the preconditioner runs FP64 solves only");
    pcx_varcoef V = new pcx_varcoef_s();
    const int nx = grid->nx, ny = grid->ny, nz = grid->nz;
    V->zf.assign(grid->zf, grid->zf + nz + 1);
    pcx_grid g = *grid;
    g.zf = V->zf.data();
    st = pcx_plan_create(&g, opts, &V->plan);
    if (st != PCX_OK) {
        V->plan = nullptr;
        vc_free(V);
        return st;
    }
    const std::vector<double> t = flow::metric_tables(V->zf.data(), nz, grid->bc_z == PCX_BC_PERIODIC);
    double zsum = 0.0;
    for (int k = 0; k < nz; ++k) zsum += t[k];
    flow::FGrid &G = V->G;
    G.n[0] = nx; G.n[1] = ny; G.n[2] = nz;
    G.per[0] = grid->bc_x == PCX_BC_PERIODIC;
    G.per[1] = grid->bc_y == PCX_BC_PERIODIC;
    G.per[2] = grid->bc_z == PCX_BC_PERIODIC;
    G.h[0] = grid->lx / nx;
    G.h[1] = grid->ly / ny;
    G.ih[0] = 1.0 / G.h[0];
    G.ih[1] = 1.0 / G.h[1];
    V->ncell = (size_t)nx * ny * nz;
    V->tp = flow::tile_plan(G);
    const int nb = V->tp.nslots;
    // the vector kernels run nb workgroups of one cell per thread
    if ((size_t)nb * flow::FT < V->ncell) {
        vc_free(V);
        return fail(PCX_ERR_INVALID, "reduction slots do not cover the grid");
    }
    const size_t nred = 2 * (size_t)nb + 2 * RED_WG + NSC;
    if (hipMalloc(&V->tab, t.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&V->ws, 4 * V->ncell * sizeof(double)) != hipSuccess ||
        hipMalloc(&V->red, nred * sizeof(double)) != hipSuccess) {
        vc_free(V);
        return fail(PCX_ERR_NOMEM, "projection workspace allocation failed");
    }
    G.dzf = V->tab;
    G.dzc = V->tab + nz;
    G.rz = V->tab + 2 * nz;
    V->r = V->ws;
    V->z = V->ws + V->ncell;
    V->d = V->ws + 2 * V->ncell;
    V->q = V->ws + 3 * V->ncell;
    V->R.part = V->red;
    V->R.lvl = V->red + 2 * (size_t)nb;
    V->R.sc = V->R.lvl + 2 * RED_WG;
    V->R.nb = nb;
    // the scalar slots start at zero but for the total weight nx ny sum(dzf)
    std::vector<double> sc(NSC, 0.0);
    sc[S_WTOT] = (double)nx * (double)ny * zsum;
    if (hipMemcpy(V->tab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(V->R.sc, sc.data(), NSC * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        vc_free(V);
        return fail(PCX_ERR_HIP, "projection table copy failed");
    }
    *out = V;
    return PCX_OK;
}

extern "C" pcx_status pcx_varcoef_destroy(pcx_varcoef V)
{
    vc_free(V);
    return PCX_OK;
}

extern "C" pcx_status pcx_varcoef_apply(pcx_varcoef V, const double *rho, const double *p, double *out,
                                        void *stream)
{
    if (!V || !rho || !p || !out) return fail(PCX_ERR_INVALID, "NULL argument");
    if (out == rho || out == p) return fail(PCX_ERR_INVALID, "out aliases an input");
    VCHK(launch_apply(V->G, V->tp, rho, p, out, 1.0, nullptr, (hipStream_t)stream));
    return PCX_OK;
}

// reads one scalar slot (synchronizes the stream)
static pcx_status read_sc(pcx_varcoef V, int slot, hipStream_t s, double *out)
{
    VCHK(hipMemcpyAsync(out, V->R.sc + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    VCHK(hipStreamSynchronize(s));
    return PCX_OK;
}

extern "C" pcx_status pcx_varcoef_project(pcx_varcoef V, double dt, double rho0, const double *rho,
                                          const double *u, const double *v, const double *w, double tol,
                                          int32_t maxit, double *u_out, double *v_out, double *w_out, double *p_out,
                                          void *stream, int32_t *iters, double *relres)
{
    if (!V) return fail(PCX_ERR_INVALID, "projection is NULL");
    if (!rho || !u || !v || !w || !u_out || !v_out || !w_out || !p_out)
        return fail(PCX_ERR_INVALID, "NULL field pointer");
    if (!(dt > 0.0) || !std::isfinite(dt) || !(rho0 > 0.0) || !std::isfinite(rho0))
        return fail(PCX_ERR_INVALID, "dt and rho0 must be finite and > 0");
    if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 1) return fail(PCX_ERR_INVALID, "tol >= 0 and maxit >= 1");
    const void *ins[] = {rho, u, v, w};
    const void *outs[] = {u_out, v_out, w_out, p_out};
    for (int a = 0; a < 4; ++a) {
        for (const void *in : ins)
            if (outs[a] == in) return fail(PCX_ERR_INVALID, "an output aliases an input");
        for (int b = 0; b < a; ++b)
            if (outs[a] == outs[b]) return fail(PCX_ERR_INVALID, "outputs alias each other");
    }
    hipStream_t s = (hipStream_t)stream;
    const flow::FGrid &G = V->G;
    const VRed &R = V->R;
    double *p = p_out;
    // r = -(D u*)/dt minus its mean; bnorm = its norm
    VCHK(launch_rhs(G, V->tp, u, v, w, 1.0 / dt, V->r, R, s));
    VCHK(red_scal(R, MODE_MEAN, s));
    VCHK(launch_center(G, V->tp, V->r, R, s));
    VCHK(red_scal(R, MODE_BNORM, s));
    VCHK(hipMemsetAsync(p, 0, V->ncell * sizeof(double), s));
    double res = 0.0;
    pcx_status st = read_sc(V, S_RES, s, &res);
    if (st != PCX_OK) return st;
    int it = 0;
    if (res > 0.0) {
        // z = -rho0 L^-1 r (the solve; the factor is folded into the kernels)
        st = pcx_poisson_solve(V->plan, V->r, V->z, stream);
        if (st != PCX_OK) return st;
        VCHK(launch_dinit(G, V->tp, V->r, V->z, V->d, rho0, R, s));
        VCHK(red_scal(R, MODE_RZ, s));
        while (it < maxit) {
            VCHK(launch_apply(G, V->tp, rho, V->d, V->q, -1.0, &R, s));
            VCHK(red_scal(R, MODE_ALPHA, s));
            VCHK(launch_update(G, V->tp, p, V->d, V->r, V->q, R, s));
            VCHK(red_scal(R, MODE_RES, s));
            ++it;
            st = read_sc(V, S_RES, s, &res);
            if (st != PCX_OK) return st;
            if (!std::isfinite(res)) {
                if (iters) *iters = it;
                if (relres) *relres = res;
                return fail(PCX_ERR_NONFINITE, "residual norm is not finite");
            }
            if (res <= tol) break;
            // the solve ignores the residual's mean (it removes the singular
            // mode); the dot pass removes it from r itself
            st = pcx_poisson_solve(V->plan, V->r, V->z, stream);
            if (st != PCX_OK) return st;
            VCHK(launch_dot(G, V->tp, V->r, V->z, rho0, R, s));
            VCHK(red_scal(R, MODE_BETA, s));
            VCHK(launch_dupd(G, V->tp, V->z, V->d, rho0, R, s));
        }
    }
    // correction with p (its gradient does not see the mean), then the gauge
    VCHK(launch_pmean(G, V->tp, p, R, s));
    VCHK(red_scal(R, MODE_PMEAN, s));
    VCHK(launch_correct(G, V->tp, rho, p, u, v, w, dt, u_out, v_out, w_out, s));
    VCHK(launch_pshift(G, V->tp, p, R, s));
    if (iters) *iters = it;
    if (relres) *relres = res;
    if (res > tol) return fail(PCX_ERR_NOT_CONVERGED, "maxit reached before tol");
    return PCX_OK;
}
