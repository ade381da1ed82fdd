// varcoef_kernels.hip -- kernels of the variable-coefficient projection
// D((1/rho_f) G p) = (D u*) / dt solved by preconditioned conjugate gradients
// (the preconditioner is the constant-coefficient solve of the plan, run by
// the host between these kernels).  Stencil and vector kernels run one
// thread per cell on the plane tiles of flow_tile.hpp (the stencils with the
// interior accessor on the interior box, the general one elsewhere); the inner
// products are volume-weighted (the dzf factor; dx dy is common to all cells
// and cancels in every ratio the iteration takes) and are reduced in a fixed
// order, so a run is deterministic.  The iteration's scalars stay in device
// memory: no kernel waits for the host.
#include "varcoef_launch.hpp"

namespace pcx {
namespace vc {

using namespace pcx::flow;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sums a and b over the workgroup (fixed order); thread 0 holds the sums
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    __shared__ double red[2][FT / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = red[0][0];
        b = red[1][0];
        for (int i = 1; i < FT / 64; ++i) {
            a += red[0][i];
            b += red[1][i];
        }
    }
}

__device__ __forceinline__ void put2(const VRed &R, int slot0, double a, double b)
{
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        R.part[slot0 + blockIdx.x] = a;
        R.part[R.nb + slot0 + blockIdx.x] = b;
    }
}

// (1/rho_f) G p on the +D face of the cell s steps along D; 0 on a wall face
template <int D, class X, class R, class P> __device__ __forceinline__ double bflux(const X &x, R rho, P p, int s)
{
    if (x.template wall<D>(s)) return 0.0;
    return cgrad<D>(x, p, s) / cface<D>(x, rho, s);
}

// D((1/rho_f) G p) at the cell
template <class X, class R, class P> __device__ __forceinline__ double vdiv_cell(const X &x, R rho, P p)
{
    return (bflux<0>(x, rho, p, 0) - bflux<0>(x, rho, p, -1)) * x.ih(0) +
           (bflux<1>(x, rho, p, 0) - bflux<1>(x, rho, p, -1)) * x.ih(1) +
           (bflux<2>(x, rho, p, 0) - bflux<2>(x, rho, p, -1)) * x.izf(0);
}

// D u at the cell (wall faces carry no flux)
template <class X>
__device__ __forceinline__ double div_cell(const X &x, const double *u, const double *v, const double *w)
{
    return (x.template fv<0>(u, 0, 0, 0) - x.template fv<0>(u, -1, 0, 0)) * x.ih(0) +
           (x.template fv<1>(v, 0, 0, 0) - x.template fv<1>(v, 0, -1, 0)) * x.ih(1) +
           (x.template fv<2>(w, 0, 0, 0) - x.template fv<2>(w, 0, 0, -1)) * x.izf(0);
}

// out = sign D((1/rho_f) G p); with R, partial sums of dzf p out
template <bool FAST>
__global__ __launch_bounds__(FT) void k_vc_apply(TileBox bx, int slot0, FGrid G, const double *rho, const double *p, double *out,
                                                 double sign, VRed R, int want)
{
    const FTile t = btile(G, bx);
    double a = 0.0;
    if (t.act) {
        double q = 0.0;
        if constexpr (FAST) {
            // rho and p from registers, loaded up front
            double rg[2][27];
            const double *const src[2] = {rho, p};
            stage_regs<2>(G, t, src, rg);
            q = sign * vdiv_cell(StageAcc<0>(G, t.i, t.j, t.k, nullptr, 0, rg), SField<0>{}, SField<1>{});
        } else {
            with_acc<false>(G, t, [&](const auto &x) { q = sign * vdiv_cell(x, rho, p); });
        }
        const size_t c = at(G, t.i, t.j, t.k);
        out[c] = q;
        a = G.dzf[t.k] * p[c] * q;
    }
    if (want) put2(R, slot0, a, 0.0);
}

// r = -(D u) / dt; partial sum of dzf r
template <bool FAST>
__global__ __launch_bounds__(FT) void k_vc_rhs(TileBox bx, int slot0, FGrid G, const double *u, const double *v, const double *w,
                                               double idt, double *r, VRed R)
{
    const FTile t = btile(G, bx);
    double a = 0.0;
    if (t.act) {
        double q = 0.0;
        with_acc<FAST>(G, t, [&](const auto &x) { q = -div_cell(x, u, v, w) * idt; });
        r[at(G, t.i, t.j, t.k)] = q;
        a = G.dzf[t.k] * q;
    }
    put2(R, slot0, a, 0.0);
}

// The vector kernels take the cells in memory order, one per thread, so a
// workgroup streams 2 KB contiguous per field; workgroup b owns slot b of
// the partials (the launch has nb workgroups, at least one per 256 cells;
// the ones past the grid add zeros).
struct LCell {
    size_t c;
    int k;
    bool act;
};
__device__ __forceinline__ LCell lcell(const FGrid &G)
{
    const unsigned plane = (unsigned)G.n[0] * (unsigned)G.n[1];
    const unsigned n = plane * (unsigned)G.n[2]; // below 2^31 (grid validation)
    const unsigned c = blockIdx.x * FT + threadIdx.x;
    LCell l;
    l.act = c < n;
    l.c = c;
    l.k = l.act ? (int)(c / plane) : 0;
    return l;
}

// r -= m; partial sum of dzf r^2
__global__ __launch_bounds__(FT) void k_vc_center(FGrid G, double *r, VRed R)
{
    const LCell l = lcell(G);
    double a = 0.0;
    if (l.act) {
        const double q = r[l.c] - R.sc[S_M];
        r[l.c] = q;
        a = G.dzf[l.k] * q * q;
    }
    put2(R, 0, a, 0.0);
}

// d = -rho0 z (z: the constant-coefficient solve of r); partial dzf r d
__global__ __launch_bounds__(FT) void k_vc_dinit(FGrid G, const double *r, const double *z, double *d, double rho0,
                                                 VRed R)
{
    const LCell l = lcell(G);
    double a = 0.0;
    if (l.act) {
        const double q = -rho0 * z[l.c];
        d[l.c] = q;
        a = G.dzf[l.k] * r[l.c] * q;
    }
    put2(R, 0, a, 0.0);
}

// p += alpha d; r -= alpha q; partial sums of dzf r and dzf r^2
__global__ __launch_bounds__(FT) void k_vc_update(FGrid G, double *p, const double *d, double *r, const double *q,
                                                  VRed R)
{
    const LCell l = lcell(G);
    double a = 0.0, b = 0.0;
    if (l.act) {
        const double al = R.sc[S_ALPHA];
        p[l.c] += al * d[l.c];
        const double rr = r[l.c] - al * q[l.c];
        r[l.c] = rr;
        const double wz = G.dzf[l.k];
        a = wz * rr;
        b = wz * rr * rr;
    }
    put2(R, 0, a, b);
}

// r -= m (the mean the residual drifted by); partial dzf r (-rho0 z)
__global__ __launch_bounds__(FT) void k_vc_dot(FGrid G, double *r, const double *z, double rho0, VRed R)
{
    const LCell l = lcell(G);
    double a = 0.0;
    if (l.act) {
        const double rr = r[l.c] - R.sc[S_M];
        r[l.c] = rr;
        a = G.dzf[l.k] * rr * (-rho0 * z[l.c]);
    }
    put2(R, 0, a, 0.0);
}

// d = -rho0 z + beta d
__global__ __launch_bounds__(FT) void k_vc_dupd(FGrid G, const double *z, double *d, double rho0, VRed R)
{
    const LCell l = lcell(G);
    if (l.act) d[l.c] = -rho0 * z[l.c] + R.sc[S_BETA] * d[l.c];
}

__global__ __launch_bounds__(FT) void k_vc_pmean(FGrid G, const double *p, VRed R)
{
    const LCell l = lcell(G);
    put2(R, 0, l.act ? G.dzf[l.k] * p[l.c] : 0.0, 0.0);
}

__global__ __launch_bounds__(FT) void k_vc_pshift(FGrid G, double *p, VRed R)
{
    const LCell l = lcell(G);
    if (l.act) p[l.c] -= R.sc[S_PMEAN];
}

// u_out = u - dt (1/rho_f) G p on the +face of each direction, 0 on a wall face
template <bool FAST>
__global__ __launch_bounds__(FT) void k_vc_correct(TileBox bx, int slot0, FGrid G, const double *rho, const double *p, const double *u,
                                                   const double *v, const double *w, double dt, double *uo,
                                                   double *vo, double *wo)
{
    const FTile t = btile(G, bx);
    if (!t.act) return;
    const size_t c = at(G, t.i, t.j, t.k);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    with_acc<FAST>(G, t, [&](const auto &x) {
        gx = bflux<0>(x, rho, p, 0);
        gy = bflux<1>(x, rho, p, 0);
        gz = bflux<2>(x, rho, p, 0);
    });
    uo[c] = wallf(G, 0, t.i) ? 0.0 : u[c] - dt * gx;
    vo[c] = wallf(G, 1, t.j) ? 0.0 : v[c] - dt * gy;
    wo[c] = wallf(G, 2, t.k) ? 0.0 : w[c] - dt * gz;
}

// first level: workgroup g sums a contiguous chunk of the partials
__global__ __launch_bounds__(FT) void k_vc_red(VRed R)
{
    const int chunk = (R.nb + RED_WG - 1) / RED_WG;
    const int b0 = blockIdx.x * chunk;
    const int b1 = b0 + chunk < R.nb ? b0 + chunk : R.nb;
    double a = 0.0, b = 0.0;
    for (int i = b0 + (int)threadIdx.x; i < b1; i += FT) {
        a += R.part[i];
        b += R.part[R.nb + i];
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        R.lvl[blockIdx.x] = a;
        R.lvl[RED_WG + blockIdx.x] = b;
    }
}

// second level and the scalar step of the iteration
__global__ __launch_bounds__(FT) void k_vc_scal(VRed R, int mode)
{
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < RED_WG; i += FT) {
        a += R.lvl[i];
        b += R.lvl[RED_WG + i];
    }
    block_sum2(a, b);
    if (threadIdx.x != 0) return;
    double *sc = R.sc;
    switch (mode) {
    case MODE_MEAN: sc[S_M] = a / sc[S_WTOT]; break;
    case MODE_BNORM:
        sc[S_BNORM] = sqrt(a);
        sc[S_RES] = a > 0.0 ? 1.0 : 0.0;
        break;
    case MODE_RZ: sc[S_RZ] = a; break;
    case MODE_ALPHA:
        sc[S_DQ] = a;
        sc[S_ALPHA] = sc[S_RZ] / a;
        break;
    case MODE_RES: {
        const double m = a / sc[S_WTOT];
        sc[S_M] = m;
        // sum dzf (r - m)^2 = sum dzf r^2 - m sum dzf r
        sc[S_RES] = sqrt(fmax(b - m * a, 0.0)) / sc[S_BNORM];
        break;
    }
    case MODE_BETA:
        sc[S_BETA] = a / sc[S_RZ];
        sc[S_RZ] = a;
        break;
    case MODE_PMEAN: sc[S_PMEAN] = a / sc[S_WTOT]; break;
    default: break;
    }
}

hipError_t launch_apply(const FGrid &G, const TilePlan &tp, const double *rho, const double *p, double *out,
                        double sign, const VRed *R, hipStream_t s)
{
    const VRed r0{};
    return FLOW_LAUNCH_PLAN(tp, k_vc_apply, s, G, rho, p, out, sign, R ? *R : r0, R ? 1 : 0);
}
hipError_t launch_rhs(const FGrid &G, const TilePlan &tp, const double *u, const double *v, const double *w,
                      double idt, double *r, const VRed &R, hipStream_t s)
{
    return FLOW_LAUNCH_PLAN(tp, k_vc_rhs, s, G, u, v, w, idt, r, R);
}
hipError_t launch_center(const FGrid &G, const TilePlan &tp, double *r, const VRed &R, hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_center, dim3((unsigned)R.nb), dim3(FT), 0, s, G, r, R);
    return hipGetLastError();
}
hipError_t launch_dinit(const FGrid &G, const TilePlan &tp, const double *r, const double *z, double *d, double rho0,
                        const VRed &R, hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_dinit, dim3((unsigned)R.nb), dim3(FT), 0, s, G, r, z, d, rho0, R);
    return hipGetLastError();
}
hipError_t launch_update(const FGrid &G, const TilePlan &tp, double *p, const double *d, double *r, const double *q,
                         const VRed &R, hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_update, dim3((unsigned)R.nb), dim3(FT), 0, s, G, p, d, r, q, R);
    return hipGetLastError();
}
hipError_t launch_dot(const FGrid &G, const TilePlan &tp, double *r, const double *z, double rho0, const VRed &R,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_dot, dim3((unsigned)R.nb), dim3(FT), 0, s, G, r, z, rho0, R);
    return hipGetLastError();
}
hipError_t launch_dupd(const FGrid &G, const TilePlan &tp, const double *z, double *d, double rho0, const VRed &R,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_dupd, dim3((unsigned)R.nb), dim3(FT), 0, s, G, z, d, rho0, R);
    return hipGetLastError();
}
hipError_t launch_pmean(const FGrid &G, const TilePlan &tp, const double *p, const VRed &R, hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_pmean, dim3((unsigned)R.nb), dim3(FT), 0, s, G, p, R);
    return hipGetLastError();
}
hipError_t launch_correct(const FGrid &G, const TilePlan &tp, const double *rho, const double *p, const double *u,
                          const double *v, const double *w, double dt, double *uo, double *vo, double *wo,
                          hipStream_t s)
{
    return FLOW_LAUNCH_PLAN(tp, k_vc_correct, s, G, rho, p, u, v, w, dt, uo, vo, wo);
}
hipError_t launch_pshift(const FGrid &G, const TilePlan &tp, double *p, const VRed &R, hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_pshift, dim3((unsigned)R.nb), dim3(FT), 0, s, G, p, R);
    return hipGetLastError();
}
hipError_t red_scal(const VRed &R, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_vc_red, dim3(RED_WG), dim3(FT), 0, s, R);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vc_scal, dim3(1), dim3(FT), 0, s, R, mode);
    return hipGetLastError();
}

} // namespace vc
} // namespace pcx
