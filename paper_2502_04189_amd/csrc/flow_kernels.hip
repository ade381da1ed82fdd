// flow_kernels.hip -- kernels of the Runge-Kutta substep around the pressure
// correction: normals, regularization flux and curvature, phase-field
// update, momentum predictor.  One thread per cell on the plane tiles of
// flow_tile.hpp: each stencil kernel is instantiated with the interior
// accessor (FAST) for the interior box and with the general one for the
// boxes along the walls.
#include "flow_launch.hpp"
#include "flow_tile.hpp"

namespace pcx {
namespace flow {

// every output of these kernels is streamed: written once, read by a later
// kernel only, so it is stored non-temporally (it does not evict the
// neighbour values other workgroups of the same kernel still read)
__device__ __forceinline__ void put(double *p, double v) { __builtin_nontemporal_store(v, p); }
// inputs read at their own cell only (previous right-hand sides, pressures)
__device__ __forceinline__ double own(const double *p) { return __builtin_nontemporal_load(p); }

// psi of every cell (one logarithm per cell), then the normals from it
__global__ __launch_bounds__(FT) void k_flow_psi(FArgs A)
{
    const size_t n = (size_t)A.G.n[0] * A.G.n[1] * A.G.n[2];
    const size_t c = (size_t)blockIdx.x * FT + threadIdx.x;
    if (c < n) put(A.psi + c, psi_of(A.P, A.phi[c]));
}

// the normals on the tiles along the walls (the interior tiles' flux kernel
// evaluates its own)
__global__ __launch_bounds__(FT) void k_flow_normals(TileBox b, int, FArgs A)
{
    const FTile t = btile(A.G, b);
    if (!t.act) return;
    double nx, ny, nz;
    with_acc<false>(A.G, t, [&](const auto &x) { normal_cell(x, A.psi, nx, ny, nz); });
    const size_t c = at(A.G, t.i, t.j, t.k);
    put(A.n[0] + c, nx);
    put(A.n[1] + c, ny);
    put(A.n[2] + c, nz);
}

// Regularization flux and curvature.  On the interior box (planes from 2 on
// with walls in z) the normals of the cell and its six neighbours are
// evaluated here from psi (the cells up to two steps along one axis or one
// step along two) instead of being stored by a normals pass and read back:
// 6 GiB less HBM traffic per substep at 512^3.  The box's cells next to a
// wall box store their own normal, which the wall tiles read.
template <bool FAST> __global__ __launch_bounds__(FT) void k_flow_flux(TileBox b, int, FArgs A)
{
    const FTile t = btile(A.G, b);
    if (!t.act) return;
    const size_t c = at(A.G, t.i, t.j, t.k);
    if constexpr (FAST) {
        const FGrid &G = A.G;
        const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
        const size_t sz = (size_t)nx * ny;
        // offsets of the cells -2 .. 2 steps along each axis (wrapped once
        // across a periodic direction; a wall is at least two cells away)
        size_t ox[5], oy[5], oz[5];
        int kw[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            int v = t.i + d - 2;
            ox[d] = (size_t)(v < 0 ? v + nx : (v >= nx ? v - nx : v));
            v = t.j + d - 2;
            oy[d] = (size_t)(v < 0 ? v + ny : (v >= ny ? v - ny : v)) * nx;
            v = t.k + d - 2;
            kw[d] = v < 0 ? v + nz : (v >= nz ? v - nz : v);
            oz[d] = (size_t)kw[d] * sz;
        }
        // psi [c][b][a] at offset (a, b, c) - 2 and phi over the 3 x 3 x 3
        // neighbourhood, all loaded up front (loads no stencil reads are
        // removed by the compiler)
        double ps[5][5][5];
#pragma unroll
        for (int cc = 0; cc < 5; ++cc)
#pragma unroll
            for (int bb = 0; bb < 5; ++bb)
#pragma unroll
                for (int aa = 0; aa < 5; ++aa) ps[cc][bb][aa] = A.psi[oz[cc] + oy[bb] + ox[aa]];
        double rg[5][27];
#pragma unroll
        for (int n = 0; n < 27; ++n) {
            const int aa = n % 3 + 1, bb = (n / 3) % 3 + 1, cc = n / 9 + 1;
            rg[0][n] = A.phi[oz[cc] + oy[bb] + ox[aa]];
            rg[1][n] = ps[cc][bb][aa];
            rg[2][n] = rg[3][n] = rg[4][n] = 0.0;
        }
        // the normal at offset (a, b, c) as the normals pass computes it
        const double hx = 0.5 * G.ih[0], hy = 0.5 * G.ih[1];
        auto normal_at = [&](int a, int bo, int co) {
            const double iz = G.rz[6 * (size_t)kw[co + 2] + 4];
            const double gx = (ps[co + 2][bo + 2][a + 3] - ps[co + 2][bo + 2][a + 1]) * hx;
            const double gy = (ps[co + 2][bo + 3][a + 2] - ps[co + 2][bo + 1][a + 2]) * hy;
            const double gz = (ps[co + 3][bo + 2][a + 2] - ps[co + 1][bo + 2][a + 2]) * iz;
            const int n = 9 * (co + 1) + 3 * (bo + 1) + a + 1;
            unit_normal(gx, gy, gz, rg[2][n], rg[3][n], rg[4][n]);
        };
        normal_at(0, 0, 0);
        normal_at(-1, 0, 0);
        normal_at(1, 0, 0);
        normal_at(0, -1, 0);
        normal_at(0, 1, 0);
        normal_at(0, 0, -1);
        normal_at(0, 0, 1);
        const StageAcc<0> x(G, t.i, t.j, t.k, nullptr, 0, rg);
        const SVec<2> n;
        put(A.a[0] + c, flux_face<0>(x, A.P, SField<0>{}, SField<1>{}, SField<2>{}));
        put(A.a[1] + c, flux_face<1>(x, A.P, SField<0>{}, SField<1>{}, SField<3>{}));
        put(A.a[2] + c, flux_face<2>(x, A.P, SField<0>{}, SField<1>{}, SField<4>{}));
        put(A.kap + c, curvature_cell(x, n));
        const bool edge = (!G.per[0] && (t.i == b.it0 * FTI || t.i == (b.it0 + b.nit) * FTI - 1)) ||
                          (!G.per[1] && (t.j == b.jt0 * FTJ || t.j == (b.jt0 + b.njt) * FTJ - 1)) ||
                          (!G.per[2] && (t.k == b.k0 || t.k == b.k0 + b.nk - 1));
        if (edge) {
            put(A.n[0] + c, rg[2][13]);
            put(A.n[1] + c, rg[3][13]);
            put(A.n[2] + c, rg[4][13]);
        }
    } else {
        const PVec n{A.n[0], A.n[1], A.n[2]};
        with_acc<false>(A.G, t, [&](const auto &x) {
            put(A.a[0] + c, flux_face<0>(x, A.P, A.phi, A.psi, A.n[0]));
            put(A.a[1] + c, flux_face<1>(x, A.P, A.phi, A.psi, A.n[1]));
            put(A.a[2] + c, flux_face<2>(x, A.P, A.phi, A.psi, A.n[2]));
            put(A.kap + c, curvature_cell(x, n));
        });
    }
}

// order-preserving key of a double for atomicMin
__device__ __forceinline__ unsigned long long fkey(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// the substep's phase update of cell c from its right-hand side r: the new
// phi and density, this substep's right-hand side; key: the density's
// minimum key
__device__ __forceinline__ void phase_put(const FArgs &A, size_t c, double r, double phi_c, double old,
                                          unsigned long long &key)
{
    const double q = phi_c + A.Dt * (A.ga * r + A.ze * old);
    put(A.phi_out + c, q);
    const double rho = A.P.rho2 + (A.P.rho1 - A.P.rho2) * q;
    put(A.rho_new + c, rho);
    key = fkey(rho);
    put(A.hphi + c, r);
}

// the workgroup's minimum key into its slot (every thread of the workgroup
// takes part; one slot per workgroup, reduced by k_flow_min: an atomic per
// workgroup on one address would serialize half a million workgroups)
__device__ __forceinline__ void key_to_slot(unsigned long long key, unsigned long long *slot)
{
    __shared__ unsigned long long red[FT / 64];
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
        *slot = key;
    }
}

// Phase-field right-hand side only (the phase right-hand side entry point;
// the substep's update runs in the momentum pass)
template <bool FAST> __global__ __launch_bounds__(FT) void k_flow_phase(TileBox b, int, FArgs A)
{
    const FTile t = btile(A.G, b);
    if (!t.act) return;
    double r = 0.0;
    if constexpr (FAST) {
        // phi, u, v, w, a_x, a_y, a_z from registers, loaded up front
        double rg[7][27];
        const double *const src[7] = {A.phi, A.u, A.v, A.w, A.a[0], A.a[1], A.a[2]};
        stage_regs<7>(A.G, t, src, rg);
        r = acdi_cell(StageAcc<0>(A.G, t.i, t.j, t.k, nullptr, 0, rg), SField<0>{}, SVec<1>{}, SVec<4>{});
    } else {
        const PVel vel{A.u, A.v, A.w};
        const PVec av{A.a[0], A.a[1], A.a[2]};
        with_acc<false>(A.G, t, [&](const auto &x) { r = acdi_cell(x, A.phi, vel, av); });
    }
    put(A.hphi + at(A.G, t.i, t.j, t.k), r);
}

// minimum of the n workgroup keys into *rho_min_key (a few workgroups, one
// atomic each)
__global__ __launch_bounds__(FT) void k_flow_min(const unsigned long long *part, int n, unsigned long long *key_out)
{
    __shared__ unsigned long long red[FT / 64];
    unsigned long long key = ~0ull;
    for (int i = blockIdx.x * FT + threadIdx.x; i < n; i += gridDim.x * FT) key = part[i] < key ? part[i] : key;
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
        atomicMin(key_out, key);
    }
}

template <int C, class X, class V, class PH, class KP, class AV>
__device__ __forceinline__ double mom_rhs(const FArgs &A, const X &x, const FTile &t, const V &vel, PH phi, KP kap,
                                          const AV &a)
{
    const int s = C == 0 ? t.i : (C == 1 ? t.j : t.k);
    return wallf(A.G, C, s) ? 0.0 : mom_face<C>(x, A.P, phi, kap, vel, a);
}

// this substep's right-hand side m into hc (the previous one read first)
// and, with u*, the predictor (0 on a wall face: the correction ignores it)
// (old: the previous right-hand side, qv: the velocity component at c)
template <int C>
__device__ __forceinline__ void mom_put(const FArgs &A, const FTile &t, size_t c, double m, double old, double qv,
                                        double *hc, double *qs)
{
    const int s = C == 0 ? t.i : (C == 1 ? t.j : t.k);
    if (qs) put(qs + c, wallf(A.G, C, s) ? 0.0 : qv + A.Dt * (A.ga * m + A.ze * old));
    put(hc + c, m);
}
template <int C>
__device__ __forceinline__ void mom_store(const FArgs &A, const FTile &t, size_t c, double m, double *hc,
                                          const double *qc, double *qs)
{
    const double old = qs && !A.first ? hc[c] : 0.0;
    mom_put<C>(A, t, c, m, old, qs ? qc[c] : 0.0, hc, qs);
}

static_assert(SLX == FTI + 2 && SLY == FTJ + 2, "stage shape follows the tile shape");

// Copies u, v, w and phi over the tile of (i0, j0, k) and its one-cell halo
// into the stage: every load of a thread is issued before its first LDS
// store.  Interior tiles only: a halo index leaves the grid only across a
// periodic direction, where it wraps (by one period: the tile plan has no
// interior box when a periodic direction is shorter than the tile and halo).
__device__ __forceinline__ void stage_fields(const FArgs &A, int i0, int j0, int k, double *st)
{
    constexpr int NR = (SFLD + FT - 1) / FT;
    const int nx = A.G.n[0], ny = A.G.n[1], nz = A.G.n[2];
    const double *src[SNF] = {A.u, A.v, A.w, A.phi};
    size_t g[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        int e = threadIdx.x + q * FT;
        e = e < SFLD ? e : SFLD - 1;
        const int kk = e / SPL, r = e - kk * SPL;
        const int jj = r / SLX, ii = r - jj * SLX;
        int gi = i0 - 1 + ii, gj = j0 - 1 + jj, gk = k - 1 + kk;
        gi = gi < 0 ? gi + nx : (gi >= nx ? gi - nx : gi);
        gj = gj < 0 ? gj + ny : (gj >= ny ? gj - ny : gj);
        gk = gk < 0 ? gk + nz : (gk >= nz ? gk - nz : gk);
        g[q] = ((size_t)gk * ny + gj) * nx + gi;
    }
    double v[SNF][NR];
#pragma unroll
    for (int f = 0; f < SNF; ++f)
#pragma unroll
        for (int q = 0; q < NR; ++q) v[f][q] = src[f][g[q]];
#pragma unroll
    for (int f = 0; f < SNF; ++f)
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int e = threadIdx.x + q * FT;
            if (e < SFLD) st[f * SFLD + e] = v[f][q];
        }
}

// Momentum right-hand side of the three components (all loads before any
// store); with u*, the substep's predictor; with p*, the extrapolated
// pressure.  Interior tiles read u, v, w and phi (about two thirds of the
// stencil's neighbour values) from a stage in LDS that the workgroup fills
// with one round of loads: read from memory one by one, in the rounds the
// compiler's schedule allowed, they left the kernel waiting on memory
// latency.  (One kernel per component took 13 % longer in all.)  With PH
// the kernel also takes the phase field's right-hand side and update (the
// substep), whose stencil reads only values the momentum stages already
// hold: a separate phase pass read phi, u, v, w and a again.
template <bool FAST, bool PH> __device__ __forceinline__ void momentum_body(const TileBox &b, int slot0, const FArgs &A)
{
    const FTile t = btile(A.G, b);
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    unsigned long long key = ~0ull;
    if constexpr (FAST) {
        // hu, hv, hw (and hphi) are read and written in place: each thread
        // reads and writes only its own cell
        __shared__ double st[SNF * SFLD];
        if (t.valid) { // uniform over the workgroup
            const int tx = threadIdx.x % FTI, ty = threadIdx.x / FTI;
            stage_fields(A, t.i - tx, t.j - ty, t.k, st);
            // register stage: issued with the LDS stage's loads, before the
            // barrier (threads past the grid read their clamped cell)
            double rg[SNR][27];
            const double *const rsrc[SNR] = {A.a[0], A.a[1], A.a[2], A.kap};
            stage_regs<SNR>(A.G, t, rsrc, rg);
            // the cell's previous right-hand sides and pressures, loaded with
            // the stages
            const size_t cc = at(A.G, t.act ? t.i : A.G.n[0] - 1, t.act ? t.j : A.G.n[1] - 1, t.k);
            double old[3] = {0.0, 0.0, 0.0}, pp1 = 0.0, pp2 = 0.0, oldp = 0.0;
            if (!A.first) {
                if (A.us[0]) old[0] = own(A.hu + cc);
                if (A.us[1]) old[1] = own(A.hv + cc);
                if (A.us[2]) old[2] = own(A.hw + cc);
                if (PH) oldp = own(A.hphi + cc);
            }
            if (A.pstar) {
                pp1 = own(A.p1 + cc);
                pp2 = own(A.p2 + cc);
            }
            __syncthreads();
            if (t.act) {
                const StageAcc<SNF> x(A.G, t.i, t.j, t.k, st, SPL + (ty + 1) * SLX + tx + 1, rg);
                const SVel vel;
                const SVec<4> av;
                m0 = mom_rhs<0>(A, x, t, vel, SField<3>{}, SField<7>{}, av);
                m1 = mom_rhs<1>(A, x, t, vel, SField<3>{}, SField<7>{}, av);
                m2 = mom_rhs<2>(A, x, t, vel, SField<3>{}, SField<7>{}, av);
                mom_put<0>(A, t, cc, m0, old[0], x.cv(SField<0>{}, 0, 0, 0), A.hu, A.us[0]);
                mom_put<1>(A, t, cc, m1, old[1], x.cv(SField<1>{}, 0, 0, 0), A.hv, A.us[1]);
                mom_put<2>(A, t, cc, m2, old[2], x.cv(SField<2>{}, 0, 0, 0), A.hw, A.us[2]);
                if (A.pstar) put(A.pstar + cc, (1.0 + A.r) * pp1 - A.r * pp2);
                if constexpr (PH)
                    phase_put(A, cc, acdi_cell(x, SField<3>{}, vel, av), x.cv(SField<3>{}, 0, 0, 0), oldp, key);
            }
        }
    } else if (t.act) {
        const PVel vel{A.u, A.v, A.w};
        const PVec av{A.a[0], A.a[1], A.a[2]};
        double r = 0.0;
        with_acc<false>(A.G, t, [&](const auto &x) {
            m0 = mom_rhs<0>(A, x, t, vel, A.phi, A.kap, av);
            m1 = mom_rhs<1>(A, x, t, vel, A.phi, A.kap, av);
            m2 = mom_rhs<2>(A, x, t, vel, A.phi, A.kap, av);
            if constexpr (PH) r = acdi_cell(x, A.phi, vel, av);
        });
        const size_t c = at(A.G, t.i, t.j, t.k);
        mom_store<0>(A, t, c, m0, A.hu, A.u, A.us[0]);
        mom_store<1>(A, t, c, m1, A.hv, A.v, A.us[1]);
        mom_store<2>(A, t, c, m2, A.hw, A.w, A.us[2]);
        if (A.pstar) put(A.pstar + c, (1.0 + A.r) * A.p1[c] - A.r * A.p2[c]);
        if constexpr (PH) phase_put(A, c, r, A.phi[c], A.first ? 0.0 : own(A.hphi + c), key);
    }
    if constexpr (PH) key_to_slot(key, A.rho_part + slot0 + blockIdx.x);
}

template <bool FAST> __global__ __launch_bounds__(FT) void k_flow_momentum(TileBox b, int slot0, FArgs A)
{
    momentum_body<FAST, false>(b, slot0, A);
}
// the substep's momentum predictor with the phase update
template <bool FAST> __global__ __launch_bounds__(FT) void k_flow_mom_phase(TileBox b, int slot0, FArgs A)
{
    momentum_body<FAST, true>(b, slot0, A);
}

__global__ void k_flow_key_reset(unsigned long long *k) { *k = ~0ull; }

// The normals and the flux take a plan made with zlow = 2 (the flux kernel's
// interior form reads psi two cells away).
hipError_t launch_normals(const FArgs &A, const TilePlan &tp, hipStream_t s)
{
    if (tp.zlow < 2) return hipErrorInvalidValue;
    const size_t n = (size_t)A.G.n[0] * A.G.n[1] * A.G.n[2];
    hipLaunchKernelGGL(k_flow_psi, dim3((unsigned)((n + FT - 1) / FT)), dim3(FT), 0, s, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the tiles along the walls only: the interior box's flux kernel
    // evaluates its normals itself
    for (int b = 0; b < tp.n; ++b) {
        if (tp.fast[b]) continue;
        hipLaunchKernelGGL(k_flow_normals, dim3(box_grid(tp.box[b])), dim3(FT), 0, s, tp.box[b], tp.slot0[b], A);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
hipError_t launch_flux(const FArgs &A, const TilePlan &tp, hipStream_t s)
{
    if (tp.zlow < 2) return hipErrorInvalidValue;
    return FLOW_LAUNCH_PLAN(tp, k_flow_flux, s, A);
}
hipError_t launch_phase(const FArgs &A, const TilePlan &tp, hipStream_t s)
{
    return FLOW_LAUNCH_PLAN(tp, k_flow_phase, s, A);
}
hipError_t launch_momentum(const FArgs &A, const TilePlan &tp, hipStream_t s)
{
    return FLOW_LAUNCH_PLAN(tp, k_flow_momentum, s, A);
}
hipError_t launch_momentum_phase(const FArgs &A, const TilePlan &tp, hipStream_t s)
{
    if (!A.phi_out || !A.hphi || !A.rho_new) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flow_key_reset, dim3(1), dim3(1), 0, s, A.rho_min_key);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = FLOW_LAUNCH_PLAN(tp, k_flow_mom_phase, s, A);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_flow_min, dim3(64), dim3(FT), 0, s, (const unsigned long long *)A.rho_part, tp.nslots,
                       A.rho_min_key);
    return hipGetLastError();
}

double key_to_double(unsigned long long k)
{
    const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double v;
    __builtin_memcpy(&v, &u, 8);
    return v;
}

} // namespace flow
} // namespace pcx
