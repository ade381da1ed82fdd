// flow_dev.hpp -- device stencils of the Runge-Kutta substep around the
// pressure correction (CaNS-Fizzy, "Mathematical model", "Methods and
// Implementation strategy"): the ACDI phase-field transport with its
// interface-regularization flux, the interface curvature, and the momentum
// predictor (centred advection, variable-viscosity stress, CSF surface
// force, the regularization term that keeps mass and momentum consistent,
// body force), all second-order on the staggered grid.
//
// One thread per cell; neighbours are read from memory (the cells of a
// workgroup's neighbours are mostly in the XCD's L2).  Index rules:
//   cell scalars one cell outside: periodic wrap, or the cell itself across
//   a wall (zero normal gradient);
//   face component c in its own direction: faces -1 and n-1 of a wall
//   direction are the walls (0); one cell outside in another direction:
//   periodic wrap, or minus the adjacent value (no-slip ghost).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcx {
namespace flow {

struct FGrid {
    int n[3];          // nx, ny, nz
    int per[3];        // 1 periodic, 0 wall
    double h[2];       // dx, dy
    const double *dzf; // nz cell widths
    const double *dzc; // centre k -> k+1 (periodic wrap at nz-1)
};

struct FParams {
    double rho1, rho2, mu1, mu2, sigma, g[3], gamma, eps, eps_s;
};

__device__ __forceinline__ size_t at(const FGrid &G, int i, int j, int k)
{
    return ((size_t)k * G.n[1] + j) * G.n[0] + i;
}

// index one outside [0, n): periodic wrap or clamp
__device__ __forceinline__ int cwrap(const FGrid &G, int d, int s)
{
    const int n = G.n[d];
    if (s < 0) return G.per[d] ? s + n : 0;
    if (s >= n) return G.per[d] ? s - n : n - 1;
    return s;
}

__device__ __forceinline__ double cv(const FGrid &G, const double *q, int i, int j, int k)
{
    return q[at(G, cwrap(G, 0, i), cwrap(G, 1, j), cwrap(G, 2, k))];
}

// Is the +d face of index s a wall (s in [-1, n-1])?
__device__ __forceinline__ bool wallf(const FGrid &G, int d, int s) { return !G.per[d] && (s < 0 || s >= G.n[d] - 1); }

// face component c of the field q at (i, j, k), see the rules above
template <int C>
__device__ __forceinline__ double fv(const FGrid &G, const double *q, int i, int j, int k)
{
    int ix[3] = {i, j, k};
    double sg = 1.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int n = G.n[d];
        if (d == C) {
            if (G.per[d]) ix[d] = ix[d] < 0 ? ix[d] + n : (ix[d] >= n ? ix[d] - n : ix[d]);
            else if (ix[d] < 0 || ix[d] >= n - 1) return 0.0;
        } else if (ix[d] < 0 || ix[d] >= n) {
            if (G.per[d]) ix[d] = ix[d] < 0 ? ix[d] + n : ix[d] - n;
            else { ix[d] = ix[d] < 0 ? 0 : n - 1; sg = -sg; }
        }
    }
    return sg * q[at(G, ix[0], ix[1], ix[2])];
}

__device__ __forceinline__ double dzf_at(const FGrid &G, int k)
{
    const int nz = G.n[2];
    if (k < 0) return G.dzf[G.per[2] ? nz - 1 : 0];
    if (k >= nz) return G.dzf[G.per[2] ? 0 : nz - 1];
    return G.dzf[k];
}
// centre k to centre k+1; across a wall the mirror ghost is one width away
__device__ __forceinline__ double dzc_at(const FGrid &G, int k)
{
    const int nz = G.n[2];
    if (k < 0) return G.per[2] ? G.dzc[nz - 1] : G.dzf[0];
    if (k >= nz - 1) return G.per[2] ? G.dzc[nz - 1] : G.dzf[nz - 1];
    return G.dzc[k];
}
// cell width in direction d at plane k; centre spacing s -> s+1 in d
__device__ __forceinline__ double hcell(const FGrid &G, int d, int k) { return d < 2 ? G.h[d] : G.dzf[k]; }
__device__ __forceinline__ double hcen(const FGrid &G, int d, int s) { return d < 2 ? G.h[d] : dzc_at(G, s); }

// cell quantity on the +d face of (i, j, k): mean in x, y; linear in z
template <int D>
__device__ __forceinline__ double cface(const FGrid &G, const double *q, int i, int j, int k)
{
    const double q0 = cv(G, q, i, j, k);
    if constexpr (D == 0) return 0.5 * (q0 + cv(G, q, i + 1, j, k));
    else if constexpr (D == 1) return 0.5 * (q0 + cv(G, q, i, j + 1, k));
    else {
        const double q1 = cv(G, q, i, j, k + 1);
        return (q0 * dzf_at(G, k + 1) + q1 * dzf_at(G, k)) / (2.0 * dzc_at(G, k));
    }
}

// the same for the linear map b0 + b1 q of the cell values (density or
// viscosity of the phase indicator q), mapped cell by cell
template <int D>
__device__ __forceinline__ double cface_map(const FGrid &G, const double *q, double b0, double b1, int i, int j, int k)
{
    const double q0 = b0 + b1 * cv(G, q, i, j, k);
    if constexpr (D == 0) return 0.5 * (q0 + (b0 + b1 * cv(G, q, i + 1, j, k)));
    else if constexpr (D == 1) return 0.5 * (q0 + (b0 + b1 * cv(G, q, i, j + 1, k)));
    else {
        const double q1 = b0 + b1 * cv(G, q, i, j, k + 1);
        return (q0 * dzf_at(G, k + 1) + q1 * dzf_at(G, k)) / (2.0 * dzc_at(G, k));
    }
}

template <int D>
__device__ __forceinline__ double cgrad(const FGrid &G, const double *q, int i, int j, int k)
{
    constexpr int oi = D == 0, oj = D == 1, ok = D == 2;
    return (cv(G, q, i + oi, j + oj, k + ok) - cv(G, q, i, j, k)) / hcen(G, D, k);
}

__device__ __forceinline__ double psi_of(const FParams &P, double phi)
{
    return P.eps * log((phi + P.eps_s) / (1.0 - phi + P.eps_s));
}

// ---------------------------------------------------------------- passes

// psi and the unit normal grad psi / |grad psi| at cell (i, j, k)
__device__ __forceinline__ void normal_cell(const FGrid &G, const FParams &P, const double *phi, int i, int j, int k,
                                            double &psi, double &nx, double &ny, double &nz)
{
    psi = psi_of(P, cv(G, phi, i, j, k));
    const double gx = (psi_of(P, cv(G, phi, i + 1, j, k)) - psi_of(P, cv(G, phi, i - 1, j, k))) / (2.0 * G.h[0]);
    const double gy = (psi_of(P, cv(G, phi, i, j + 1, k)) - psi_of(P, cv(G, phi, i, j - 1, k))) / (2.0 * G.h[1]);
    const double gz = (psi_of(P, cv(G, phi, i, j, k + 1)) - psi_of(P, cv(G, phi, i, j, k - 1))) /
                      (dzc_at(G, k) + dzc_at(G, k - 1));
    const double m = sqrt(gx * gx + gy * gy + gz * gz);
    if (m > 0.0) {
        nx = gx / m;
        ny = gy / m;
        nz = gz / m;
    } else {
        nx = ny = nz = 0.0;
    }
}

// regularization flux on the +D face of (i, j, k) (0 on a wall face)
template <int D>
__device__ __forceinline__ double flux_face(const FGrid &G, const FParams &P, const double *phi, const double *psi,
                                            const double *nd, int i, int j, int k)
{
    const int s = D == 0 ? i : (D == 1 ? j : k);
    if (wallf(G, D, s)) return 0.0;
    const double t = tanh(cface<D>(G, psi, i, j, k) / (2.0 * P.eps));
    return P.gamma * (P.eps * cgrad<D>(G, phi, i, j, k) - 0.25 * (1.0 - t * t) * cface<D>(G, nd, i, j, k));
}

// face normal component D on the +D face (0 on a wall face)
template <int D>
__device__ __forceinline__ double nface(const FGrid &G, const double *nd, int i, int j, int k)
{
    const int s = D == 0 ? i : (D == 1 ? j : k);
    return wallf(G, D, s) ? 0.0 : cface<D>(G, nd, i, j, k);
}

// curvature -div n_f at the cell
__device__ __forceinline__ double curvature_cell(const FGrid &G, const double *const n[3], int i, int j, int k)
{
    const double sx = nface<0>(G, n[0], i, j, k) - (wallf(G, 0, i - 1) ? 0.0 : nface<0>(G, n[0], cwrap(G, 0, i - 1), j, k));
    const double sy = nface<1>(G, n[1], i, j, k) - (wallf(G, 1, j - 1) ? 0.0 : nface<1>(G, n[1], i, cwrap(G, 1, j - 1), k));
    const double sz = nface<2>(G, n[2], i, j, k) - (wallf(G, 2, k - 1) ? 0.0 : nface<2>(G, n[2], i, j, cwrap(G, 2, k - 1)));
    return -(sx / G.h[0] + sy / G.h[1] + sz / G.dzf[k]);
}

// net phase flux u phi_f - a through the +D face of (i, j, k), 0 on walls
template <int D>
__device__ __forceinline__ double jface(const FGrid &G, const double *phi, const double *vel, const double *ad, int i,
                                        int j, int k)
{
    const int s = D == 0 ? i : (D == 1 ? j : k);
    if (wallf(G, D, s)) return 0.0;
    return fv<D>(G, vel, i, j, k) * cface<D>(G, phi, i, j, k) - ad[at(G, i, j, k)];
}

// -div(u phi_f - a) at the cell
__device__ __forceinline__ double acdi_cell(const FGrid &G, const double *phi, const double *const vel[3],
                                            const double *const a[3], int i, int j, int k)
{
    double r = 0.0;
    {
        const double jp = jface<0>(G, phi, vel[0], a[0], i, j, k);
        const double jm = wallf(G, 0, i - 1) ? 0.0 : jface<0>(G, phi, vel[0], a[0], cwrap(G, 0, i - 1), j, k);
        r -= (jp - jm) / G.h[0];
    }
    {
        const double jp = jface<1>(G, phi, vel[1], a[1], i, j, k);
        const double jm = wallf(G, 1, j - 1) ? 0.0 : jface<1>(G, phi, vel[1], a[1], i, cwrap(G, 1, j - 1), k);
        r -= (jp - jm) / G.h[1];
    }
    {
        const double jp = jface<2>(G, phi, vel[2], a[2], i, j, k);
        const double jm = wallf(G, 2, k - 1) ? 0.0 : jface<2>(G, phi, vel[2], a[2], i, j, cwrap(G, 2, k - 1));
        r -= (jp - jm) / G.dzf[k];
    }
    return r;
}

// mean of a cell quantity over the four cells around the edge touching the
// +A and +B faces of (i, j, k)
template <int A, int B>
__device__ __forceinline__ double edge_mean(const FGrid &G, const double *q, double b0, double b1, int i, int j, int k)
{
    constexpr int ai = A == 0, aj = A == 1, ak = A == 2, bi = B == 0, bj = B == 1, bk = B == 2;
    return 0.25 * ((b0 + b1 * cv(G, q, i, j, k)) + (b0 + b1 * cv(G, q, i + ai, j + aj, k + ak)) +
                   (b0 + b1 * cv(G, q, i + bi, j + bj, k + bk)) +
                   (b0 + b1 * cv(G, q, i + ai + bi, j + aj + bj, k + ak + bk)));
}

// component D of the regularization flux at the position of the +C face:
// its own value when D == C, else the mean of the four D faces around
template <int C, int D>
__device__ __forceinline__ double a_at(const FGrid &G, const double *ad, int i, int j, int k)
{
    if constexpr (C == D) {
        return ad[at(G, i, j, k)];
    } else {
        constexpr int ci = C == 0, cj = C == 1, ck = C == 2, di = D == 0, dj = D == 1, dk = D == 2;
        const int ix[4][3] = {{i, j, k}, {i + ci, j + cj, k + ck}, {i - di, j - dj, k - dk},
                              {i + ci - di, j + cj - dj, k + ck - dk}};
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int q[3] = {ix[t][0], ix[t][1], ix[t][2]};
            if (wallf(G, D, q[D])) continue;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                if (q[e] < 0) q[e] += G.n[e];
                else if (q[e] >= G.n[e]) q[e] -= G.n[e];
            }
            s += ad[at(G, q[0], q[1], q[2])];
        }
        return 0.25 * s;
    }
}

// Transverse (D != C) contribution to the advection, viscous stress and
// regularization terms of component C on its +C face.
template <int C, int D>
__device__ __forceinline__ void mom_transverse(const FGrid &G, const FParams &P, const double *const vel[3],
                                               const double *phi, int i, int j, int k, double q0, double hc,
                                               double &adv, double &visc)
{
    constexpr int ci = C == 0, cj = C == 1, ck = C == 2, di = D == 0, dj = D == 1, dk = D == 2;
    const double *q = vel[C], *p = vel[D];
    const int sd = D == 0 ? i : (D == 1 ? j : k);
    const double pu0 = fv<D>(G, p, i, j, k), pu1 = fv<D>(G, p, i + ci, j + cj, k + ck);
    const double pd0 = fv<D>(G, p, i - di, j - dj, k - dk), pd1 = fv<D>(G, p, i + ci - di, j + cj - dj, k + ck - dk);
    const double qu = fv<C>(G, q, i + di, j + dj, k + dk), qd = fv<C>(G, q, i - di, j - dj, k - dk);
    const double hd = hcell(G, D, k);
    adv += (0.5 * (pu0 + pu1) * 0.5 * (q0 + qu) - 0.5 * (pd0 + pd1) * 0.5 * (qd + q0)) / hd;
    const double m0 = P.mu2, m1 = P.mu1 - P.mu2;
    const double muu = edge_mean<C, D>(G, phi, m0, m1, i, j, k);
    const double mud = edge_mean<C, D>(G, phi, m0, m1, i - di, j - dj, k - dk);
    const double tu = muu * ((qu - q0) / hcen(G, D, sd) + (pu1 - pu0) / hc);
    const double td = mud * ((q0 - qd) / hcen(G, D, sd - 1) + (pd1 - pd0) / hc);
    visc += (tu - td) / hd;
}

template <int C, int D>
__device__ __forceinline__ double mom_reg(const FGrid &G, const double *const vel[3], const double *const a[3], int i,
                                          int j, int k)
{
    constexpr int di = D == 0, dj = D == 1, dk = D == 2;
    const double *q = vel[C];
    const int sd = D == 0 ? i : (D == 1 ? j : k);
    const double qp = fv<C>(G, q, i + di, j + dj, k + dk), qm = fv<C>(G, q, i - di, j - dj, k - dk);
    double h;
    if constexpr (C == D) h = (D < 2 ? 2.0 * G.h[D] : dzf_at(G, k) + dzf_at(G, k + 1));
    else h = hcen(G, D, sd) + hcen(G, D, sd - 1);
    return a_at<C, D>(G, a[D], i, j, k) * (qp - qm) / h;
}

// Momentum right-hand side per unit mass of component C on the +C face of
// (i, j, k), which is not a wall face.
template <int C>
__device__ __forceinline__ double mom_face(const FGrid &G, const FParams &P, const double *phi, const double *kap,
                                           const double *const vel[3], const double *const a[3], int i, int j, int k)
{
    constexpr int ci = C == 0, cj = C == 1, ck = C == 2;
    const double *q = vel[C];
    const int sc = C == 0 ? i : (C == 1 ? j : k);
    const double q0 = fv<C>(G, q, i, j, k);
    const double hc = hcen(G, C, sc);
    double adv, visc;
    {
        const double qm = fv<C>(G, q, i - ci, j - cj, k - ck), qp = fv<C>(G, q, i + ci, j + cj, k + ck);
        const double cm = 0.5 * (qm + q0), cp = 0.5 * (q0 + qp);
        adv = (cp * cp - cm * cm) / hc;
        const double h1 = C < 2 ? G.h[C] : dzf_at(G, k + 1), h0 = C < 2 ? G.h[C] : G.dzf[k];
        const double mu1 = P.mu2 + (P.mu1 - P.mu2) * cv(G, phi, i + ci, j + cj, k + ck);
        const double mu0 = P.mu2 + (P.mu1 - P.mu2) * cv(G, phi, i, j, k);
        const double tp = 2.0 * mu1 * (qp - q0) / h1;
        const double tm = 2.0 * mu0 * (q0 - qm) / h0;
        visc = (tp - tm) / hc;
    }
    if constexpr (C != 0) mom_transverse<C, 0>(G, P, vel, phi, i, j, k, q0, hc, adv, visc);
    if constexpr (C != 1) mom_transverse<C, 1>(G, P, vel, phi, i, j, k, q0, hc, adv, visc);
    if constexpr (C != 2) mom_transverse<C, 2>(G, P, vel, phi, i, j, k, q0, hc, adv, visc);
    const double reg = mom_reg<C, 0>(G, vel, a, i, j, k) + mom_reg<C, 1>(G, vel, a, i, j, k) +
                       mom_reg<C, 2>(G, vel, a, i, j, k);
    const double st = P.sigma * cface<C>(G, kap, i, j, k) * cgrad<C>(G, phi, i, j, k);
    const double rf = cface_map<C>(G, phi, P.rho2, P.rho1 - P.rho2, i, j, k);
    return -adv + (visc + st + (P.rho1 - P.rho2) * reg) / rf + P.g[C];
}

} // namespace flow
} // namespace pcx
