// flow_kernels.hip -- kernels of the Runge-Kutta substep around the pressure
// correction: normals, regularization flux and curvature, phase-field
// update, momentum predictor.  One thread per cell, 256-thread workgroups
// of 64 x 4 cells of one plane; consecutive workgroups go to different XCDs,
// so the launch hands XCD x a contiguous range of tiles (its planes), and a
// tile's y and z neighbours are mostly in that XCD's L2.
#include "flow_dev.hpp"
#include "flow_launch.hpp"

namespace pcx {
namespace flow {

constexpr int FT = 256, FTI = 64, FTJ = FT / FTI;

struct FTile {
    int i, j, k;
    bool act;
};

__device__ __forceinline__ FTile ftile(const FGrid &G)
{
    const int ti = (G.n[0] + FTI - 1) / FTI, tj = (G.n[1] + FTJ - 1) / FTJ;
    const long nt = (long)ti * tj * G.n[2];
    const long per = (nt + 7) >> 3;
    const long t = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    FTile c;
    c.act = false;
    c.i = c.j = c.k = 0;
    if (t >= nt) return c;
    const int k = (int)(t / ((long)ti * tj));
    const int r = (int)(t - (long)k * ti * tj);
    const int jt = r / ti, it = r - jt * ti;
    c.i = it * FTI + (threadIdx.x % FTI);
    c.j = jt * FTJ + (threadIdx.x / FTI);
    c.k = k;
    c.act = c.i < G.n[0] && c.j < G.n[1];
    return c;
}

__global__ __launch_bounds__(FT) void k_flow_normals(FArgs A)
{
    const FTile t = ftile(A.G);
    if (!t.act) return;
    double psi, nx, ny, nz;
    normal_cell(A.G, A.P, A.phi, t.i, t.j, t.k, psi, nx, ny, nz);
    const size_t c = at(A.G, t.i, t.j, t.k);
    A.psi[c] = psi;
    A.n[0][c] = nx;
    A.n[1][c] = ny;
    A.n[2][c] = nz;
}

__global__ __launch_bounds__(FT) void k_flow_flux(FArgs A)
{
    const FTile t = ftile(A.G);
    if (!t.act) return;
    const size_t c = at(A.G, t.i, t.j, t.k);
    A.a[0][c] = flux_face<0>(A.G, A.P, A.phi, A.psi, A.n[0], t.i, t.j, t.k);
    A.a[1][c] = flux_face<1>(A.G, A.P, A.phi, A.psi, A.n[1], t.i, t.j, t.k);
    A.a[2][c] = flux_face<2>(A.G, A.P, A.phi, A.psi, A.n[2], t.i, t.j, t.k);
    A.kap[c] = curvature_cell(A.G, A.n, t.i, t.j, t.k);
}

// order-preserving key of a double for atomicMin
__device__ __forceinline__ unsigned long long fkey(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Phase-field right-hand side; with phi_out, the substep's update, the new
// density and its minimum (one atomicMin per workgroup).
__global__ __launch_bounds__(FT) void k_flow_phase(FArgs A)
{
    __shared__ unsigned long long red[FT / 64];
    const FTile t = ftile(A.G);
    unsigned long long key = ~0ull;
    if (t.act) {
        const size_t c = at(A.G, t.i, t.j, t.k);
        const double *vel[3] = {A.u, A.v, A.w};
        const double r = acdi_cell(A.G, A.phi, vel, A.a, t.i, t.j, t.k);
        if (A.phi_out) {
            const double old = A.first ? 0.0 : A.hphi[c];
            const double q = A.phi[c] + A.Dt * (A.ga * r + A.ze * old);
            A.phi_out[c] = q;
            const double rho = A.P.rho2 + (A.P.rho1 - A.P.rho2) * q;
            A.rho_new[c] = rho;
            key = fkey(rho);
        }
        A.hphi[c] = r;
    }
    if (!A.phi_out) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long x = __shfl_xor(key, o, 64);
        key = x < key ? x : key;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < FT / 64; ++i) key = red[i] < key ? red[i] : key;
        key = red[0] < key ? red[0] : key;
        atomicMin(A.rho_min_key, key);
    }
}

template <int C>
__device__ __forceinline__ void mom_one(const FArgs &A, const FTile &t, size_t c, double *hc, const double *qc,
                                        double *qs)
{
    const int s = C == 0 ? t.i : (C == 1 ? t.j : t.k);
    const double *vel[3] = {A.u, A.v, A.w};
    double m = 0.0;
    if (!wallf(A.G, C, s)) m = mom_face<C>(A.G, A.P, A.phi, A.kap, vel, A.a, t.i, t.j, t.k);
    if (qs) {
        const double old = A.first ? 0.0 : hc[c];
        // the wall face of u* is written 0 (the correction ignores it)
        qs[c] = wallf(A.G, C, s) ? 0.0 : qc[c] + A.Dt * (A.ga * m + A.ze * old);
    }
    hc[c] = m;
}

// Momentum right-hand side of the three components; with u*, the
// substep's predictor; with p*, the extrapolated pressure.
__global__ __launch_bounds__(FT) void k_flow_momentum(FArgs A)
{
    const FTile t = ftile(A.G);
    if (!t.act) return;
    const size_t c = at(A.G, t.i, t.j, t.k);
    mom_one<0>(A, t, c, A.hu, A.u, A.us[0]);
    mom_one<1>(A, t, c, A.hv, A.v, A.us[1]);
    mom_one<2>(A, t, c, A.hw, A.w, A.us[2]);
    if (A.pstar) A.pstar[c] = (1.0 + A.r) * A.p1[c] - A.r * A.p2[c];
}

__global__ void k_flow_key_reset(unsigned long long *k) { *k = ~0ull; }

static int ngrid(const FGrid &G)
{
    const long nt = (long)((G.n[0] + FTI - 1) / FTI) * ((G.n[1] + FTJ - 1) / FTJ) * G.n[2];
    return (int)(((nt + 7) >> 3) << 3);
}

#define FLAUNCH(fn, A, s)                                                            \
    do {                                                                             \
        hipLaunchKernelGGL(fn, dim3(ngrid((A).G)), dim3(FT), 0, (s), (A));           \
        return hipGetLastError();                                                    \
    } while (0)

hipError_t launch_normals(const FArgs &A, hipStream_t s) { FLAUNCH(k_flow_normals, A, s); }
hipError_t launch_flux(const FArgs &A, hipStream_t s) { FLAUNCH(k_flow_flux, A, s); }
hipError_t launch_phase(const FArgs &A, hipStream_t s)
{
    if (A.phi_out) {
        hipLaunchKernelGGL(k_flow_key_reset, dim3(1), dim3(1), 0, s, A.rho_min_key);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    FLAUNCH(k_flow_phase, A, s);
}
hipError_t launch_momentum(const FArgs &A, hipStream_t s) { FLAUNCH(k_flow_momentum, A, s); }

double key_to_double(unsigned long long k)
{
    const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double v;
    __builtin_memcpy(&v, &u, 8);
    return v;
}

} // namespace flow
} // namespace pcx
