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
    double ih[2];      // 1/dx, 1/dy
    const double *dzf; // nz cell widths
    const double *dzc; // centre k -> k+1 (periodic wrap at nz-1)
    // per plane k, 6 reciprocals (the z metrics the interior accessor uses):
    // 1/dzf(k), 1/dzf(k+1), 1/dzc(k-1), 1/dzc(k), 1/(dzc(k) + dzc(k-1)),
    // 1/(dzf(k) + dzf(k+1)), with dzf(.), dzc(.) as dzf_at, dzc_at below
    const double *rz;
};

struct FParams {
    double rho1, rho2, mu1, mu2, sigma, g[3], gamma, eps, eps_s;
    double ihe; // 1 / (2 eps)
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

// ------------------------------------------------------------ accessors
// The stencils below are written once against an accessor X that reads a
// field at a small constant offset (a, b, c), each in {-1, 0, +1}, from the
// thread's cell:
//   Gen  applies the wrap / wall / ghost rules above to every access;
//   Fast is for tiles whose stencils reach no wall: offsets precomputed per
//        thread (periodic wrap folded in), z metrics of planes k-1..k+1 in
//        registers, no branch per access.
struct Gen {
    const FGrid &G;
    int i, j, k;
    __device__ __forceinline__ double cv(const double *q, int a, int b, int c) const
    {
        return flow::cv(G, q, i + a, j + b, k + c);
    }
    template <int C>
    __device__ __forceinline__ double fv(const double *q, int a, int b, int c) const
    {
        return flow::fv<C>(G, q, i + a, j + b, k + c);
    }
    // is the +D face of the cell s steps along D a wall?
    template <int D> __device__ __forceinline__ bool wall(int s) const
    {
        return wallf(G, D, (D == 0 ? i : (D == 1 ? j : k)) + s);
    }
    __device__ __forceinline__ double dzf(int s) const { return dzf_at(G, k + s); }
    __device__ __forceinline__ double dzc(int s) const { return dzc_at(G, k + s); }
    __device__ __forceinline__ double h(int d) const { return G.h[d]; }
    // reciprocals: 1/h, 1/dzf(s), 1/dzc(s), 1/(dzc(0) + dzc(-1)), 1/(dzf(0) + dzf(1))
    __device__ __forceinline__ double ih(int d) const { return 1.0 / G.h[d]; }
    __device__ __forceinline__ double izf(int s) const { return 1.0 / dzf(s); }
    __device__ __forceinline__ double izc(int s) const { return 1.0 / dzc(s); }
    __device__ __forceinline__ double izc2() const { return 1.0 / (dzc(0) + dzc(-1)); }
    __device__ __forceinline__ double izf2() const { return 1.0 / (dzf(0) + dzf(1)); }
    __device__ __forceinline__ size_t idx(int a, int b, int c) const
    {
        return at(G, cwrap(G, 0, i + a), cwrap(G, 1, j + b), cwrap(G, 2, k + c));
    }
};

struct Fast {
    size_t c0;
    long xm, xp, ym, yp, zm, zp;
    double zf_m, zf_0, zf_p, zc_m, zc_0, hx, hy;
    double ihx, ihy, izf_0, izf_p, izc_m, izc_0, izc2_, izf2_;
    __device__ __forceinline__ Fast(const FGrid &G, int i, int j, int k)
    {
        const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
        const long sy = nx, sz = (long)nx * ny;
        c0 = at(G, i, j, k);
        xm = i == 0 ? nx - 1 : -1;
        xp = i == nx - 1 ? -(nx - 1) : 1;
        ym = j == 0 ? (ny - 1) * sy : -sy;
        yp = j == ny - 1 ? -(ny - 1) * sy : sy;
        zm = k == 0 ? (nz - 1) * sz : -sz;
        zp = k == nz - 1 ? -(nz - 1) * sz : sz;
        zf_m = dzf_at(G, k - 1);
        zf_0 = G.dzf[k];
        zf_p = dzf_at(G, k + 1);
        zc_m = dzc_at(G, k - 1);
        zc_0 = dzc_at(G, k);
        hx = G.h[0];
        hy = G.h[1];
        // reciprocals from the host tables (one scalar load each: k is
        // uniform over a workgroup) instead of eight divisions per thread
        ihx = G.ih[0];
        ihy = G.ih[1];
        const double *r = G.rz + 6 * (size_t)k;
        izf_0 = r[0];
        izf_p = r[1];
        izc_m = r[2];
        izc_0 = r[3];
        izc2_ = r[4];
        izf2_ = r[5];
    }
    __device__ __forceinline__ long off(int a, int b, int c) const
    {
        return (a < 0 ? xm : (a > 0 ? xp : 0)) + (b < 0 ? ym : (b > 0 ? yp : 0)) + (c < 0 ? zm : (c > 0 ? zp : 0));
    }
    __device__ __forceinline__ double cv(const double *q, int a, int b, int c) const { return q[c0 + off(a, b, c)]; }
    template <int C>
    __device__ __forceinline__ double fv(const double *q, int a, int b, int c) const
    {
        return q[c0 + off(a, b, c)];
    }
    template <int D> __device__ __forceinline__ bool wall(int) const { return false; }
    __device__ __forceinline__ double dzf(int s) const { return s < 0 ? zf_m : (s > 0 ? zf_p : zf_0); }
    __device__ __forceinline__ double dzc(int s) const { return s < 0 ? zc_m : zc_0; }
    __device__ __forceinline__ double h(int d) const { return d == 0 ? hx : hy; }
    __device__ __forceinline__ double ih(int d) const { return d == 0 ? ihx : ihy; }
    __device__ __forceinline__ double izf(int s) const { return s > 0 ? izf_p : izf_0; } // s in {0, 1}
    __device__ __forceinline__ double izc(int s) const { return s < 0 ? izc_m : izc_0; }
    __device__ __forceinline__ double izc2() const { return izc2_; }
    __device__ __forceinline__ double izf2() const { return izf2_; }
    __device__ __forceinline__ size_t idx(int a, int b, int c) const { return c0 + off(a, b, c); }
};

// offset (a, b, c) of s steps along direction D
#define DOFF(D, s) ((D) == 0 ? (s) : 0), ((D) == 1 ? (s) : 0), ((D) == 2 ? (s) : 0)

// cell width along D; centre spacing from the cell s steps along D to the next
template <class X> __device__ __forceinline__ double ihcell(const X &x, int D) { return D < 2 ? x.ih(D) : x.izf(0); }
template <class X> __device__ __forceinline__ double ihcen(const X &x, int D, int s) { return D < 2 ? x.ih(D) : x.izc(s); }

// cell quantity b0 + b1 q on the +D face of the cell s steps along D: mean
// in x, y, linear interpolation in z
template <int D, class X, class Q>
__device__ __forceinline__ double cface(const X &x, Q q, int s, double b0 = 0.0, double b1 = 1.0)
{
    const double q0 = b0 + b1 * x.cv(q, DOFF(D, s)), q1 = b0 + b1 * x.cv(q, DOFF(D, s + 1));
    if constexpr (D < 2) return 0.5 * (q0 + q1);
    else return (q0 * x.dzf(s + 1) + q1 * x.dzf(s)) * (0.5 * x.izc(s));
}

// difference quotient of a cell quantity across that face
template <int D, class X, class Q> __device__ __forceinline__ double cgrad(const X &x, Q q, int s)
{
    return (x.cv(q, DOFF(D, s + 1)) - x.cv(q, DOFF(D, s))) * ihcen(x, D, s);
}

// psi of phi clamped to [0, 1] (rounding can leave phi a few ulps outside,
// where the logarithm is undefined)
__device__ __forceinline__ double psi_of(const FParams &P, double phi)
{
    const double q = fmin(fmax(phi, 0.0), 1.0);
    return P.eps * log((q + P.eps_s) / (1.0 - q + P.eps_s));
}

// The three velocity components as the momentum stencils take them (get<C>()
// is component C): device pointers, or the workgroup-staged copies below.
struct PVel {
    const double *u, *v, *w;
    template <int C> __device__ __forceinline__ const double *get() const { return C == 0 ? u : (C == 1 ? v : w); }
};

// pointer triple with get<C>() (the regularization flux components)
using PVec = PVel;

// A field staged for the workgroup (F: its place in the stage: 0..3 in LDS,
// the others in registers, see StageAcc)
template <int F> struct SField {};
// staged u, v, w (the velocity) and a (the regularization flux) components
template <int F0> struct SVec {
    template <int C> __device__ __forceinline__ SField<F0 + C> get() const { return {}; }
};
using SVel = SVec<0>;

// Stage of an interior tile: u, v, w, phi (F = 0..3) in LDS over the tile
// and a one-cell halo in x, y and z; a_x, a_y, a_z and kappa (F = 4..7) in
// registers, each thread its own 3 x 3 x 3 neighbourhood (the loads of the
// values no stencil reads are dead and removed by the compiler).
constexpr int SLX = 64 + 2, SLY = 4 + 2, SPL = SLX * SLY, SFLD = 3 * SPL, SNF = 4, SNR = 4;

// Interior accessor whose staged fields come from the stages and all others
// from memory (as Fast): fields F < NL from the LDS stage (l0: the thread's
// cell in its middle plane), the others from the register stage rg[F - NL]
// (rg[f][n]: offset (a, b, c) at n = 9 (c + 1) + 3 (b + 1) + a + 1).
template <int NL> struct StageAcc : Fast {
    const double *st;
    int l0;
    const double (*rg)[27];
    __device__ __forceinline__ StageAcc(const FGrid &G, int i, int j, int k, const double *stage, int l,
                                        const double (*regs)[27])
        : Fast(G, i, j, k), st(stage), l0(l), rg(regs)
    {
    }
    using Fast::cv;
    using Fast::fv;
    template <int F> __device__ __forceinline__ double cv(SField<F>, int a, int b, int c) const
    {
        if constexpr (F < NL) return st[F * SFLD + l0 + c * SPL + b * SLX + a];
        else return rg[F - NL][9 * (c + 1) + 3 * (b + 1) + a + 1];
    }
    template <int C, int F> __device__ __forceinline__ double fv(SField<F> q, int a, int b, int c) const
    {
        return cv(q, a, b, c);
    }
};

// ---------------------------------------------------------------- passes

// g / |g| (0 where g = 0), with the fused multiply-adds written out, so that
// every kernel that evaluates a normal rounds it the same way; one
// reciprocal square root instead of a square root and a division
__device__ __forceinline__ void unit_normal(double gx, double gy, double gz, double &nx, double &ny, double &nz)
{
    const double m2 = fma(gx, gx, fma(gy, gy, gz * gz));
    if (m2 > 0.0) {
        const double im = rsqrt(m2);
        nx = gx * im;
        ny = gy * im;
        nz = gz * im;
    } else {
        nx = ny = nz = 0.0;
    }
}

// the unit normal grad psi / |grad psi| at the cell, from stored psi
template <class X, class PS>
__device__ __forceinline__ void normal_cell(const X &x, PS psi, double &nx, double &ny, double &nz)
{
    const double gx = (x.cv(psi, 1, 0, 0) - x.cv(psi, -1, 0, 0)) * (0.5 * x.ih(0));
    const double gy = (x.cv(psi, 0, 1, 0) - x.cv(psi, 0, -1, 0)) * (0.5 * x.ih(1));
    const double gz = (x.cv(psi, 0, 0, 1) - x.cv(psi, 0, 0, -1)) * x.izc2();
    unit_normal(gx, gy, gz, nx, ny, nz);
}

// regularization flux on the +D face of the cell (0 on a wall face)
template <int D, class X, class PH, class PS, class ND>
__device__ __forceinline__ double flux_face(const X &x, const FParams &P, PH phi, PS psi, ND nd)
{
    if (x.template wall<D>(0)) return 0.0;
    // (1 - tanh^2 z) / 4 = y / (1 + y)^2 with y = exp(-2 |z|): one
    // exponential instead of a hyperbolic tangent, and no cancellation
    // where tanh z is near +-1
    const double y = exp(-2.0 * fabs(cface<D>(x, psi, 0) * P.ihe));
    const double w = y / ((1.0 + y) * (1.0 + y));
    return P.gamma * (P.eps * cgrad<D>(x, phi, 0) - w * cface<D>(x, nd, 0));
}

// normal component D on the +D face of the cell s steps along D (0 on walls)
template <int D, class X, class ND> __device__ __forceinline__ double nface(const X &x, ND nd, int s)
{
    return x.template wall<D>(s) ? 0.0 : cface<D>(x, nd, s);
}

// curvature -div n_f at the cell
template <class X, class NV> __device__ __forceinline__ double curvature_cell(const X &x, const NV &n)
{
    const auto n0 = n.template get<0>();
    const auto n1 = n.template get<1>();
    const auto n2 = n.template get<2>();
    const double sx = nface<0>(x, n0, 0) - nface<0>(x, n0, -1);
    const double sy = nface<1>(x, n1, 0) - nface<1>(x, n1, -1);
    const double sz = nface<2>(x, n2, 0) - nface<2>(x, n2, -1);
    return -(sx * x.ih(0) + sy * x.ih(1) + sz * x.izf(0));
}

// net phase flux u phi_f - a through the +D face of the cell s steps along D
template <int D, class X, class PH, class VD, class AD>
__device__ __forceinline__ double jface(const X &x, PH phi, VD vel, AD ad, int s)
{
    if (x.template wall<D>(s)) return 0.0;
    return x.template fv<D>(vel, DOFF(D, s)) * cface<D>(x, phi, s) - x.cv(ad, DOFF(D, s));
}

// -div(u phi_f - a) at the cell
template <class X, class PH, class V, class AV>
__device__ __forceinline__ double acdi_cell(const X &x, PH phi, const V &vel, const AV &a)
{
    const auto u = vel.template get<0>();
    const auto v = vel.template get<1>();
    const auto w = vel.template get<2>();
    const auto a0 = a.template get<0>();
    const auto a1 = a.template get<1>();
    const auto a2 = a.template get<2>();
    double r = -(jface<0>(x, phi, u, a0, 0) - jface<0>(x, phi, u, a0, -1)) * x.ih(0);
    r -= (jface<1>(x, phi, v, a1, 0) - jface<1>(x, phi, v, a1, -1)) * x.ih(1);
    r -= (jface<2>(x, phi, w, a2, 0) - jface<2>(x, phi, w, a2, -1)) * x.izf(0);
    return r;
}

// mean of b0 + b1 q over the four cells around the edge touching the +A and
// +B faces of the cell s steps along B
template <int A, int B, class X, class Q>
__device__ __forceinline__ double edge_mean(const X &x, Q q, double b0, double b1, int s)
{
    constexpr int ai = A == 0, aj = A == 1, ak = A == 2, bi = B == 0, bj = B == 1, bk = B == 2;
    return 0.25 * ((b0 + b1 * x.cv(q, s * bi, s * bj, s * bk)) + (b0 + b1 * x.cv(q, ai + s * bi, aj + s * bj, ak + s * bk)) +
                   (b0 + b1 * x.cv(q, (s + 1) * bi, (s + 1) * bj, (s + 1) * bk)) +
                   (b0 + b1 * x.cv(q, ai + (s + 1) * bi, aj + (s + 1) * bj, ak + (s + 1) * bk)));
}

// component D of the regularization flux at the position of the +C face:
// its own value when D == C, else the mean of the four D faces around
// (wall faces carry none)
template <int C, int D, class X, class Q> __device__ __forceinline__ double a_at(const X &x, Q ad)
{
    if constexpr (C == D) {
        return x.cv(ad, 0, 0, 0);
    } else {
        constexpr int ci = C == 0, cj = C == 1, ck = C == 2, di = D == 0, dj = D == 1, dk = D == 2;
        double s = 0.0;
        if (!x.template wall<D>(0)) s += x.cv(ad, 0, 0, 0) + x.cv(ad, ci, cj, ck);
        if (!x.template wall<D>(-1)) s += x.cv(ad, -di, -dj, -dk) + x.cv(ad, ci - di, cj - dj, ck - dk);
        return 0.25 * s;
    }
}

// Transverse (D != C) contribution to the advection and viscous terms of
// component C on its +C face.
template <int C, int D, class X, class V, class PH>
__device__ __forceinline__ void mom_transverse(const X &x, const FParams &P, const V &vel, PH phi, double q0,
                                               double ihc, double &adv, double &visc)
{
    constexpr int ci = C == 0, cj = C == 1, ck = C == 2, di = D == 0, dj = D == 1, dk = D == 2;
    const auto q = vel.template get<C>();
    const auto p = vel.template get<D>();
    const double pu0 = x.template fv<D>(p, 0, 0, 0), pu1 = x.template fv<D>(p, ci, cj, ck);
    const double pd0 = x.template fv<D>(p, -di, -dj, -dk), pd1 = x.template fv<D>(p, ci - di, cj - dj, ck - dk);
    const double qu = x.template fv<C>(q, di, dj, dk), qd = x.template fv<C>(q, -di, -dj, -dk);
    const double ihd = ihcell(x, D);
    adv += (0.5 * (pu0 + pu1) * 0.5 * (q0 + qu) - 0.5 * (pd0 + pd1) * 0.5 * (qd + q0)) * ihd;
    const double m0 = P.mu2, m1 = P.mu1 - P.mu2;
    const double muu = edge_mean<C, D>(x, phi, m0, m1, 0);
    const double mud = edge_mean<C, D>(x, phi, m0, m1, -1);
    const double tu = muu * ((qu - q0) * ihcen(x, D, 0) + (pu1 - pu0) * ihc);
    const double td = mud * ((q0 - qd) * ihcen(x, D, -1) + (pd1 - pd0) * ihc);
    visc += (tu - td) * ihd;
}

template <int C, int D, class X, class V, class AV>
__device__ __forceinline__ double mom_reg(const X &x, const V &vel, const AV &a)
{
    constexpr int di = D == 0, dj = D == 1, dk = D == 2;
    const auto q = vel.template get<C>();
    const double qp = x.template fv<C>(q, di, dj, dk), qm = x.template fv<C>(q, -di, -dj, -dk);
    double ih;
    if constexpr (C == D) ih = D < 2 ? 0.5 * x.ih(D) : x.izf2();
    else ih = D < 2 ? 0.5 * x.ih(D) : x.izc2();
    return a_at<C, D>(x, a.template get<D>()) * (qp - qm) * ih;
}

// Momentum right-hand side per unit mass of component C on the +C face of
// the cell, which is not a wall face.
template <int C, class X, class V, class PH, class KP, class AV>
__device__ __forceinline__ double mom_face(const X &x, const FParams &P, PH phi, KP kap, const V &vel, const AV &a)
{
    constexpr int ci = C == 0, cj = C == 1, ck = C == 2;
    const auto q = vel.template get<C>();
    const double q0 = x.template fv<C>(q, 0, 0, 0);
    const double ihc = ihcen(x, C, 0);
    double adv, visc;
    {
        const double qm = x.template fv<C>(q, -ci, -cj, -ck), qp = x.template fv<C>(q, ci, cj, ck);
        const double cm = 0.5 * (qm + q0), cp = 0.5 * (q0 + qp);
        adv = (cp * cp - cm * cm) * ihc;
        const double ih1 = C < 2 ? x.ih(C) : x.izf(1), ih0 = C < 2 ? x.ih(C) : x.izf(0);
        const double mu1 = P.mu2 + (P.mu1 - P.mu2) * x.cv(phi, ci, cj, ck);
        const double mu0 = P.mu2 + (P.mu1 - P.mu2) * x.cv(phi, 0, 0, 0);
        const double tp = 2.0 * mu1 * (qp - q0) * ih1;
        const double tm = 2.0 * mu0 * (q0 - qm) * ih0;
        visc = (tp - tm) * ihc;
    }
    if constexpr (C != 0) mom_transverse<C, 0>(x, P, vel, phi, q0, ihc, adv, visc);
    if constexpr (C != 1) mom_transverse<C, 1>(x, P, vel, phi, q0, ihc, adv, visc);
    if constexpr (C != 2) mom_transverse<C, 2>(x, P, vel, phi, q0, ihc, adv, visc);
    const double reg = mom_reg<C, 0>(x, vel, a) + mom_reg<C, 1>(x, vel, a) + mom_reg<C, 2>(x, vel, a);
    const double st = P.sigma * cface<C>(x, kap, 0) * cgrad<C>(x, phi, 0);
    const double rf = cface<C>(x, phi, 0, P.rho2, P.rho1 - P.rho2);
    return -adv + (visc + st + (P.rho1 - P.rho2) * reg) / rf + P.g[C];
}

} // namespace flow
} // namespace pcx
