// flow_launch.hpp -- launch arguments and host launchers of the substep
// kernels (flow_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "flow_tile.hpp"

namespace pcx {
namespace flow {

struct FArgs {
    FGrid G;
    FParams P;
    const double *phi, *u, *v, *w;   // state at the start of the substep
    double *psi, *n[3], *a[3], *kap; // normals, regularization flux (faces), curvature
    double Dt, ga, ze;               // step and the substep's coefficients
    int first;                       // first substep: no previous right-hand side
    double *hphi, *hu, *hv, *hw;     // previous right-hand sides in, this substep's out
    double *phi_out, *us[3], *rho_new; // NULL: right-hand sides only
    unsigned long long *rho_min_key;
    unsigned long long *rho_part;    // one key per workgroup of the phase pass (TilePlan::nslots)
    const double *p1, *p2;           // pressures of the two previous substeps
    double r;
    double *pstar;                   // NULL: no extrapolation
};

hipError_t launch_normals(const FArgs &A, const TilePlan &tp, hipStream_t s);
hipError_t launch_flux(const FArgs &A, const TilePlan &tp, hipStream_t s);
hipError_t launch_phase(const FArgs &A, const TilePlan &tp, hipStream_t s);
hipError_t launch_momentum(const FArgs &A, const TilePlan &tp, hipStream_t s);
// the substep's momentum predictor and phase update in one pass (phi_out,
// hphi and rho_new set), then the density minimum
hipError_t launch_momentum_phase(const FArgs &A, const TilePlan &tp, hipStream_t s);
double key_to_double(unsigned long long k);

} // namespace flow
} // namespace pcx
