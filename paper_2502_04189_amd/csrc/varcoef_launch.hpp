// varcoef_launch.hpp -- host launchers of the variable-coefficient
// projection kernels (varcoef_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "flow_tile.hpp"

namespace pcx {
namespace vc {

// device scalar slots of the conjugate-gradient iteration
enum { S_RZ, S_DQ, S_ALPHA, S_BETA, S_M, S_RES, S_BNORM, S_WTOT, S_PMEAN, NSC };

// what the scalar kernel makes of the two reduced sums (S0, S1)
enum {
    MODE_MEAN,  // m = S0 / wtot
    MODE_BNORM, // bnorm = sqrt(S0); res = 1 (0 when S0 = 0)
    MODE_RZ,    // rz = S0
    MODE_ALPHA, // dq = S0; alpha = rz / dq
    MODE_RES,   // m = S0 / wtot; res = sqrt(S1 - m S0) / bnorm
    MODE_BETA,  // beta = S0 / rz; rz = S0
    MODE_PMEAN  // pmean = S0 / wtot
};

// workgroups of the first reduction level (partials -> lvl)
constexpr int RED_WG = 256;

// Reductions: every partial-writing kernel stores the two sums of its
// workgroup b (numbered over the launches of the tile plan) at part[b] and
// part[nb + b] (nb = TilePlan::nslots); red_scal sums them in a fixed order
// into the scalar slots.
struct VRed {
    double *part; // 2 nb
    double *lvl;  // 2 RED_WG
    double *sc;   // NSC
    int nb;
};

using flow::FGrid;

using flow::TilePlan;

hipError_t launch_apply(const FGrid &G, const TilePlan &tp, const double *rho, const double *p, double *out,
                        double sign, const VRed *R, hipStream_t s);
hipError_t launch_rhs(const FGrid &G, const TilePlan &tp, const double *u, const double *v, const double *w,
                      double idt, double *r, const VRed &R, hipStream_t s);
hipError_t launch_center(const FGrid &G, const TilePlan &tp, double *r, const VRed &R, hipStream_t s);
hipError_t launch_dinit(const FGrid &G, const TilePlan &tp, const double *r, const double *z, double *d, double rho0,
                        const VRed &R, hipStream_t s);
hipError_t launch_update(const FGrid &G, const TilePlan &tp, double *p, const double *d, double *r, const double *q,
                         const VRed &R, hipStream_t s);
hipError_t launch_dot(const FGrid &G, const TilePlan &tp, double *r, const double *z, double rho0, const VRed &R,
                      hipStream_t s);
hipError_t launch_dupd(const FGrid &G, const TilePlan &tp, const double *z, double *d, double rho0, const VRed &R,
                       hipStream_t s);
hipError_t launch_pmean(const FGrid &G, const TilePlan &tp, const double *p, const VRed &R, hipStream_t s);
hipError_t launch_correct(const FGrid &G, const TilePlan &tp, const double *rho, const double *p, const double *u,
                          const double *v, const double *w, double dt, double *uo, double *vo, double *wo,
                          hipStream_t s);
hipError_t launch_pshift(const FGrid &G, const TilePlan &tp, double *p, const VRed &R, hipStream_t s);
// the two-level reduction of the partials and the scalar step `mode`
hipError_t red_scal(const VRed &R, int mode, hipStream_t s);

} // namespace vc
} // namespace pcx
