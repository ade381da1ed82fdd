// flow_host.cpp -- C ABI of the Runge-Kutta substep around the pressure
// correction: validation, device tables and workspace, pass sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "flow_launch.hpp"
#include "pcx.h"
#include "pcx_flow.h"
#include "pcx_plan.hpp"

using namespace pcx;
using namespace pcx::flow;

// workspace fields: psi, n (3), a (3), kappa, new density, p*, u* (3)
constexpr int NWS = 13;

struct pcx_flow_s {
    pcx_grid grid;
    std::vector<double> zf;
    FGrid G;
    TilePlan tp;  // phase and momentum kernels
    TilePlan tpn; // normals and flux (interior planes from 2 on with walls in z)
    FParams P;
    pcx_plan plan = nullptr;
    double *tab = nullptr;           // z metric tables (metric_tables)
    double *ws = nullptr;            // NWS fields
    unsigned long long *key = nullptr;
    unsigned long long *part = nullptr; // per-workgroup minimum keys
    size_t ncell = 0;
    double *psi, *n[3], *a[3], *kap, *rho_new, *pstar, *us[3];
};

static void flow_free(pcx_flow F)
{
    if (!F) return;
    if (F->plan) pcx_plan_destroy(F->plan);
    if (F->tab) (void)hipFree(F->tab);
    if (F->ws) (void)hipFree(F->ws);
    if (F->key) (void)hipFree(F->key);
    if (F->part) (void)hipFree(F->part);
    delete F;
}

static bool fin(double x) { return std::isfinite(x); }

extern "C" pcx_status pcx_flow_create(const pcx_grid *grid, const pcx_flow_params *prm, const pcx_options *opts,
                                      pcx_flow *out)
{
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!prm) return fail(PCX_ERR_INVALID, "params is NULL");
    pcx_status st = validate_grid(grid);
    if (st != PCX_OK) return st;
    if (grid->bc_x == PCX_BC_DIRICHLET || grid->bc_y == PCX_BC_DIRICHLET || grid->bc_z == PCX_BC_DIRICHLET)
        return fail(PCX_ERR_UNSUPPORTED, "the substep takes periodic and wall boundaries only");
    const pcx_flow_params &q = *prm;
    if (!(q.rho1 > 0.0) || !(q.rho2 > 0.0) || !(q.mu1 >= 0.0) || !(q.mu2 >= 0.0) || !(q.sigma >= 0.0) ||
        !(q.gamma >= 0.0) || !(q.eps > 0.0) || !(q.eps_s >= 0.0) || !fin(q.rho1) || !fin(q.rho2) || !fin(q.mu1) ||
        !fin(q.mu2) || !fin(q.sigma) || !fin(q.gamma) || !fin(q.eps) || !fin(q.eps_s) || !fin(q.gx) || !fin(q.gy) ||
        !fin(q.gz))
        return fail(PCX_ERR_INVALID, "flow parameters out of range");
    pcx_flow F = new pcx_flow_s();
    F->grid = *grid;
    F->zf.assign(grid->zf, grid->zf + grid->nz + 1);
    F->grid.zf = F->zf.data();
    st = pcx_plan_create(&F->grid, opts, &F->plan);
    if (st != PCX_OK) {
        F->plan = nullptr;
        flow_free(F);
        return st;
    }
    const int nx = grid->nx, ny = grid->ny, nz = grid->nz;
    const std::vector<double> t = metric_tables(F->zf.data(), nz, grid->bc_z == PCX_BC_PERIODIC);
    F->ncell = (size_t)nx * ny * nz;
    if (hipMalloc(&F->tab, t.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&F->ws, NWS * F->ncell * sizeof(double)) != hipSuccess ||
        hipMalloc(&F->key, sizeof(unsigned long long)) != hipSuccess) {
        flow_free(F);
        return fail(PCX_ERR_NOMEM, "flow workspace allocation failed");
    }
    if (hipMemcpy(F->tab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        flow_free(F);
        return fail(PCX_ERR_HIP, "flow table copy failed");
    }
    FGrid &G = F->G;
    G.n[0] = nx; G.n[1] = ny; G.n[2] = nz;
    G.per[0] = grid->bc_x == PCX_BC_PERIODIC;
    G.per[1] = grid->bc_y == PCX_BC_PERIODIC;
    G.per[2] = grid->bc_z == PCX_BC_PERIODIC;
    G.h[0] = grid->lx / nx;
    G.h[1] = grid->ly / ny;
    G.ih[0] = 1.0 / G.h[0];
    G.ih[1] = 1.0 / G.h[1];
    G.dzf = F->tab;
    G.dzc = F->tab + nz;
    G.rz = F->tab + 2 * nz;
    F->P = FParams{q.rho1, q.rho2, q.mu1, q.mu2, q.sigma, {q.gx, q.gy, q.gz}, q.gamma, q.eps, q.eps_s, 0.5 / q.eps};
    F->tp = tile_plan(G);
    F->tpn = tile_plan(G, 2);
    if (hipMalloc(&F->part, (size_t)F->tp.nslots * sizeof(unsigned long long)) != hipSuccess) {
        flow_free(F);
        return fail(PCX_ERR_NOMEM, "flow workspace allocation failed");
    }
    double *w = F->ws;
    auto take = [&]() { double *p = w; w += F->ncell; return p; };
    F->psi = take();
    for (auto &p : F->n) p = take();
    for (auto &p : F->a) p = take();
    F->kap = take();
    F->rho_new = take();
    F->pstar = take();
    for (auto &p : F->us) p = take();
    if (w != F->ws + NWS * F->ncell) {
        flow_free(F);
        return fail(PCX_ERR_INVALID, "flow workspace layout does not match its allocation");
    }
    *out = F;
    return PCX_OK;
}

extern "C" pcx_status pcx_flow_destroy(pcx_flow F)
{
    flow_free(F);
    return PCX_OK;
}

static FArgs base_args(pcx_flow F, const double *phi, const double *u, const double *v, const double *w)
{
    FArgs A;
    std::memset(&A, 0, sizeof(A));
    A.G = F->G;
    A.P = F->P;
    A.phi = phi; A.u = u; A.v = v; A.w = w;
    A.psi = F->psi;
    for (int d = 0; d < 3; ++d) {
        A.n[d] = F->n[d];
        A.a[d] = F->a[d];
    }
    A.kap = F->kap;
    A.first = 1;
    A.rho_min_key = F->key;
    A.rho_part = F->part;
    return A;
}

#define FCHK(x)                                                                                   \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) return fail(PCX_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static bool aliases(const void *o, std::initializer_list<const void *> ins)
{
    for (const void *p : ins)
        if (p == o) return true;
    return false;
}

extern "C" pcx_status pcx_flow_phase_rhs(pcx_flow F, const double *phi, const double *u, const double *v,
                                         const double *w, double *rhs, void *stream)
{
    if (!F || !phi || !u || !v || !w || !rhs) return fail(PCX_ERR_INVALID, "NULL argument");
    if (aliases(rhs, {phi, u, v, w})) return fail(PCX_ERR_INVALID, "rhs aliases an input");
    hipStream_t s = (hipStream_t)stream;
    FArgs A = base_args(F, phi, u, v, w);
    A.hphi = rhs;
    FCHK(launch_normals(A, F->tpn, s));
    FCHK(launch_flux(A, F->tpn, s));
    FCHK(launch_phase(A, F->tp, s));
    return PCX_OK;
}

extern "C" pcx_status pcx_flow_momentum_rhs(pcx_flow F, const double *phi, const double *u, const double *v,
                                            const double *w, double *ru, double *rv, double *rw, void *stream)
{
    if (!F || !phi || !u || !v || !w || !ru || !rv || !rw) return fail(PCX_ERR_INVALID, "NULL argument");
    for (const double *o : {ru, rv, rw})
        if (aliases(o, {phi, u, v, w})) return fail(PCX_ERR_INVALID, "an output aliases an input");
    if (ru == rv || ru == rw || rv == rw) return fail(PCX_ERR_INVALID, "outputs alias each other");
    hipStream_t s = (hipStream_t)stream;
    FArgs A = base_args(F, phi, u, v, w);
    A.hu = ru; A.hv = rv; A.hw = rw;
    FCHK(launch_normals(A, F->tpn, s));
    FCHK(launch_flux(A, F->tpn, s));
    FCHK(launch_momentum(A, F->tp, s));
    return PCX_OK;
}

// The substep up to the correction: normals, flux and curvature, momentum
// predictor, phase update; u*, the new density and p* into the given
// buffers; rho0 read back (one 8-byte copy: synchronizes the stream).
static pcx_status predictor(pcx_flow F, int32_t sub, double Dt, const double *phi, const double *u, const double *v,
                            const double *w, const double *p1, const double *p2, double r, double *hphi, double *hu,
                            double *hv, double *hw, double *phi_out, double *const us[3], double *rho_new,
                            double *pstar, hipStream_t s, double *rho0, double *dt)
{
    static const double GA[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
    static const double ZE[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
    FArgs A = base_args(F, phi, u, v, w);
    A.Dt = Dt;
    A.ga = GA[sub - 1];
    A.ze = ZE[sub - 1];
    A.first = sub == 1;
    A.hphi = hphi; A.hu = hu; A.hv = hv; A.hw = hw;
    A.phi_out = phi_out;
    for (int d = 0; d < 3; ++d) A.us[d] = us[d];
    A.rho_new = rho_new;
    A.p1 = p1; A.p2 = p2; A.r = r;
    A.pstar = pstar;
    FCHK(launch_normals(A, F->tpn, s));
    FCHK(launch_flux(A, F->tpn, s));
    // one pass: the momentum predictor and the phase update read the state at
    // the start of the substep only
    FCHK(launch_momentum_phase(A, F->tp, s));
    unsigned long long key = 0;
    FCHK(hipMemcpyAsync(&key, F->key, sizeof(key), hipMemcpyDeviceToHost, s));
    FCHK(hipStreamSynchronize(s));
    *rho0 = key_to_double(key);
    if (!(*rho0 > 0.0) || !std::isfinite(*rho0)) return fail(PCX_ERR_NONFINITE, "minimum density is not positive and finite");
    *dt = (GA[sub - 1] + ZE[sub - 1]) * Dt;
    return PCX_OK;
}

// ins: read-only inputs; hs: the right-hand sides read and rewritten in
// place (each only at its own cell); outs: written.  hs and outs must each
// be distinct from everything else (other threads read the inputs'
// neighbours while a cell is written).
static pcx_status check_substep_args(pcx_flow F, int32_t sub, double Dt, double r,
                                     std::initializer_list<const void *> ins, std::initializer_list<const void *> hs,
                                     std::initializer_list<const void *> outs)
{
    if (!F) return fail(PCX_ERR_INVALID, "flow is NULL");
    if (sub < 1 || sub > 3) return fail(PCX_ERR_INVALID, "substep must be 1, 2 or 3");
    if (!(Dt > 0.0) || !std::isfinite(Dt) || !std::isfinite(r)) return fail(PCX_ERR_INVALID, "Dt must be > 0, r finite");
    for (auto l : {ins, hs, outs})
        for (const void *p : l)
            if (!p) return fail(PCX_ERR_INVALID, "NULL field pointer");
    for (auto l : {hs, outs})
        for (const void *o : l) {
            if (aliases(o, ins)) return fail(PCX_ERR_INVALID, "an output aliases an input");
            int same = 0;
            for (auto m : {hs, outs})
                for (const void *o2 : m) same += o2 == o;
            if (same > 1) return fail(PCX_ERR_INVALID, "outputs alias each other");
        }
    return PCX_OK;
}

extern "C" pcx_status pcx_flow_substep(pcx_flow F, int32_t sub, double Dt, const double *phi, const double *u,
                                       const double *v, const double *w, const double *p1, const double *p2,
                                       double r, double *hphi, double *hu, double *hv, double *hw, double *phi_out,
                                       double *u_out, double *v_out, double *w_out, double *p_out, void *stream,
                                       pcx_report *report)
{
    pcx_status st = check_substep_args(F, sub, Dt, r, {phi, u, v, w, p1, p2}, {hphi, hu, hv, hw},
                                       {phi_out, u_out, v_out, w_out, p_out});
    if (st != PCX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    double rho0 = 0.0, dt = 0.0;
    st = predictor(F, sub, Dt, phi, u, v, w, p1, p2, r, hphi, hu, hv, hw, phi_out, F->us, F->rho_new, F->pstar, s,
                   &rho0, &dt);
    if (st != PCX_OK) return st;
    return pcx_step(F->plan, dt, rho0, F->rho_new, F->pstar, F->us[0], F->us[1], F->us[2], u_out, v_out, w_out, p_out,
                    stream, report);
}

extern "C" pcx_status pcx_flow_predict(pcx_flow F, int32_t sub, double Dt, const double *phi, const double *u,
                                       const double *v, const double *w, const double *p1, const double *p2,
                                       double r, double *hphi, double *hu, double *hv, double *hw, double *phi_out,
                                       double *u_star, double *v_star, double *w_star, double *rho, double *p_star,
                                       double *rho0, double *dt, void *stream)
{
    pcx_status st = check_substep_args(F, sub, Dt, r, {phi, u, v, w, p1, p2}, {hphi, hu, hv, hw},
                                       {phi_out, u_star, v_star, w_star, rho, p_star});
    if (st != PCX_OK) return st;
    if (!rho0 || !dt) return fail(PCX_ERR_INVALID, "rho0 and dt must not be NULL");
    double *const us[3] = {u_star, v_star, w_star};
    return predictor(F, sub, Dt, phi, u, v, w, p1, p2, r, hphi, hu, hv, hw, phi_out, us, rho, p_star,
                     (hipStream_t)stream, rho0, dt);
}
