// pcx_passes.hpp -- the passes of one pressure-correction step, as device
// functions over one tile of one domain.  The same bodies serve the
// one-kernel-per-pass launches of a single domain and the persistent
// multi-domain kernel.
//
//   rhs    : splitting right-hand side f (FP64 stencil, k-marching)  (-> f)
//   resid  : r = f - L p (FP64 stencil, k-marching)                  (-> r)
//   xfwd   : real FFT in x of f or r, x->y corner turn              (-> S1)
//   yfwd   : complex FFT in y, y->z corner turn                  (S1 -> S2)
//   zsolve : tridiagonal solve per (l, m) line in z, in place        (S2)
//   yinv   : inverse complex FFT in y, z->y corner turn          (S2 -> S1)
//   xinv   : inverse real FFT in x, store or accumulate p        (S1 -> p)
//   corr   : velocity correction with the divergence check (k-marching)
#pragma once

#include <type_traits>

#include "pcx_dev.hpp"

namespace pcx {

// ------------------------------------------------------------- marching
// Stencil tiles: TI x TJ cells of a plane (one thread per (i, j) column,
// TI = min(nx, 64) so a wave holds one row segment when nx >= 64) marching
// over a chunk of planes.  The planes a cell needs above it are loaded once
// as the "k+1" neighbour and kept in registers for the next step; x
// neighbours come from the adjacent lanes, y neighbours through LDS; only
// tile-edge threads load neighbours from memory.
struct MTile {
    int i, j, ti, tj, kb, ke, lane;
    bool act;
};

__device__ __forceinline__ MTile march_tile(const Dom &d, const MGeo &g, int tile)
{
    MTile t;
    const int per = g.cnti * g.cntj;
    const int kc = tile / per;
    const int rem = tile - kc * per;
    const int jt = rem / g.cnti, it = rem - jt * g.cnti;
    t.tj = (int)fdiv(threadIdx.x, g.dcti);
    t.ti = threadIdx.x - t.tj * g.cti;
    const int i = it * g.cti + t.ti, j = jt * g.ctj + t.tj;
    t.act = t.tj < g.ctj && i < d.nx && j < d.ny;
    t.i = min(i, d.nx - 1); // clamped so that idle threads load valid cells
    t.j = min(j, d.ny - 1);
    t.kb = kc * g.ckc;
    t.ke = min(d.nz, t.kb + g.ckc);
    t.lane = threadIdx.x & 63;
    return t;
}

struct MNbr {
    int oe, ow, on, os;   // in-plane offsets of the four neighbours (wrapped)
    bool we, ww, wn, ws;  // wall faces
    bool she, shw;        // x neighbour held by the adjacent lane
    bool lyn, lys;        // y neighbour held in LDS by the tile
};

__device__ __forceinline__ MNbr march_nbr(const Dom &d, const MGeo &g, const MTile &t)
{
    MNbr n;
    const int nx = d.nx, ny = d.ny, i = t.i, j = t.j;
    n.oe = (i == nx - 1) ? -(nx - 1) : 1;
    n.ow = (i == 0) ? (nx - 1) : -1;
    n.on = (j == ny - 1) ? -(ny - 1) * nx : nx;
    n.os = (j == 0) ? (ny - 1) * nx : -nx;
    n.we = d.bcx == BC_WALL && i == nx - 1;
    n.ww = d.bcx == BC_WALL && i == 0;
    n.wn = d.bcy == BC_WALL && j == ny - 1;
    n.ws = d.bcy == BC_WALL && j == 0;
    n.she = t.ti < g.cti - 1 && t.lane < 63 && i + 1 < nx;
    n.shw = t.ti > 0 && t.lane > 0;
    n.lyn = t.tj < g.ctj - 1 && j + 1 < ny;
    n.lys = t.tj > 0;
    return n;
}

// Plane prefetched during plane k: k + 1, or k itself on the last plane of
// the chunk (a redundant read whose values are never used).  The prefetch
// loads, halo items included, are all unconditional, at addresses that are
// valid for every thread: a load under a branch inside the marching loop
// makes the compiler wait for every outstanding load (the next plane's
// included) before the plane's first LDS write.
__device__ __forceinline__ int march_next(int k, const MTile &t) { return min(k + 1, t.ke - 1); }

// z-metric coefficient of plane k (uniform) by a scalar load: the plan's
// tables are never written by a kernel, and a scalar load does not queue
// behind the vector prefetch (waiting for a vector load waits for every
// vector load issued before it).
__device__ __forceinline__ double ztab(const double *p, int k)
{
    return ((const __attribute__((address_space(4))) double *)p)[__builtin_amdgcn_readfirstlane(k)];
}

__device__ __forceinline__ double amax_nan(double m, double v)
{
    double a = fabs(v);
    return (a > m || a != a) ? a : m;
}

// Halo of an RHS tile (see the correction's halo below for the layout
// rules), 5 (TI + TJ) items:
//   north row: p*, rho      items [0, 2 TI)
//   south row: v*, p*, rho  items [2 TI, 5 TI)
//   east col:  p*, rho      items [5 TI, 5 TI + 2 TJ)
//   west col:  u*, p*, rho  items [5 TI + 2 TJ, 5 (TI + TJ))
struct Halo {
    const double *fp[2];
    int off[2];
};

__device__ __forceinline__ Halo rhs_halo(const Dom &d, const MGeo &g, int tile, int nth)
{
    const int per = g.cnti * g.cntj;
    const int rem = tile - (tile / per) * per;
    const int jt = rem / g.cnti, it = rem - jt * g.cnti;
    const int TI = g.cti, TJ = g.ctj, nx = d.nx, ny = d.ny;
    const int i0 = it * TI, j0 = jt * TJ;
    const int w = min(TI, nx - i0), h = min(TJ, ny - j0);
    const int ie = (i0 + w == nx) ? 0 : i0 + w, je = (j0 + h == ny) ? 0 : j0 + h;
    const int iw = (i0 == 0) ? nx - 1 : i0 - 1, js = (j0 == 0) ? ny - 1 : j0 - 1;
    auto pr = [&](int f) { return f == 0 ? d.ps : d.rho; };
    Halo H;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int q = threadIdx.x + s * nth;
        int i = 0, j = 0;
        const double *fp = d.ps;
        if (q < 2 * TI) {
            const int f = q / TI, x = min(q - f * TI, w - 1);
            fp = pr(f); i = i0 + x; j = je;
        } else if (q < 5 * TI) {
            const int f = (q - 2 * TI) / TI, x = min(q - 2 * TI - f * TI, w - 1);
            fp = f == 0 ? d.v : pr(f - 1); i = i0 + x; j = js;
        } else if (q < 5 * TI + 2 * TJ) {
            const int f = (q - 5 * TI) / TJ, y = min(q - 5 * TI - f * TJ, h - 1);
            fp = pr(f); i = ie; j = j0 + y;
        } else {
            const int qq = min(q - 5 * TI - 2 * TJ, 3 * TJ - 1);
            const int f = qq / TJ, y = min(qq - f * TJ, h - 1);
            fp = f == 0 ? d.u : pr(f - 1); i = iw; j = j0 + y;
        }
        H.fp[s] = fp;
        H.off[s] = j * nx + i;
    }
    return H;
}

// f = (rho0/dt) D u* + D[(1 - rho0/rho_face) G p*], stored in FP64 to d.f.
// Marching in k; the neighbours in x and y come through LDS (the tile's own
// plane) or from the halo; the z flux and w* below are carried from the
// previous plane.  Every global read of plane k+1 is issued while plane k
// is computed.  LDS: 16 reduction slots, p* / rho / u* / v* of the plane and
// the halo items.
template <int NTH = NT, bool TWO = true>
__device__ __forceinline__ void pass_rhs(const Dom &d, int tile, char *smem)
{
    constexpr int MG = 0;
    double *red = (double *)smem;
    double *sP = red + 16, *sR = sP + NTH, *sU = sR + NTH, *sV = sU + NTH, *hal = sV + NTH;
    const MGeo &g = d.mg[MG];
    const MTile t = march_tile(d, g, tile);
    const MNbr n = march_nbr(d, g, t);
    const int nx = d.nx, ny = d.ny, nz = d.nz, sz = nx * ny, TI = g.cti, TJ = g.ctj;
    const int col = t.j * nx + t.i;
    const double rr0 = d.rho0, tr0 = 2.0 * d.rho0;
    const double idx2 = d.idx * d.idx, idy2 = d.idy * d.idy, cdiv = d.rho0 / d.dt;
    const int nh = 5 * (TI + TJ);
    const Halo H = rhs_halo(d, g, tile, NTH);
    // TWO: a thread may own a second halo item (more halo items than
    // threads); without it the second item's load is not issued at all
    const bool hv0 = threadIdx.x < nh, hv1 = TWO && threadIdx.x + NTH < nh;
    // tile origin from the tile index (t.i, t.j are clamped for idle threads)
    const int per = g.cnti * g.cntj, rem = tile - (tile / per) * per;
    const int i0 = (rem % g.cnti) * TI, j0 = (rem / g.cnti) * TJ;
    const bool inE = t.ti + 1 < min(TI, nx - i0), inN = t.tj + 1 < min(TJ, ny - j0);
    const int me = threadIdx.x;
    auto kp = [&](int k) { return k == nz - 1 ? 0 : k + 1; };
    int k = t.kb;
    double Pc = d.ps[k * sz + col], Rc = d.rho[k * sz + col];
    double Pp = d.ps[kp(k) * sz + col], Rp = d.rho[kp(k) * sz + col];
    double U = d.u[k * sz + col], V = d.v[k * sz + col], W = d.w[k * sz + col];
    double h0 = H.fp[0][k * sz + H.off[0]], h1 = TWO ? H.fp[1][k * sz + H.off[1]] : 0.0;
    double Fb = 0.0, Wb = 0.0; // flux of (1 - rho0/rho) G p* and w* on face k - 1/2
    if (!(d.bcz == BC_WALL && k == 0)) {
        const int km = (k == 0) ? nz - 1 : k - 1;
        const double Pm = d.ps[km * sz + col], Rm = d.rho[km * sz + col];
        Fb = (1.0 - rr0 * rcp_nr(Rm * d.rzlo[km] + Rc * d.rzhi[km])) * (Pc - Pm) * d.idzc[km];
        Wb = d.w[km * sz + col];
    }
    double amax = 0.0;
    for (; k < t.ke; ++k) {
        // prefetch plane k+1 (no load is under a branch; see march_next)
        const int k1 = march_next(k, t), k2 = kp(k1);
        const double P2 = d.ps[k2 * sz + col], R2 = d.rho[k2 * sz + col];
        const double U1 = d.u[k1 * sz + col], V1 = d.v[k1 * sz + col], W1 = ld_stream(d.w + k1 * sz + col);
        const double g0 = H.fp[0][k1 * sz + H.off[0]], g1 = TWO ? H.fp[1][k1 * sz + H.off[1]] : 0.0;
        const int c = k * sz + col;
        const bool wt = d.bcz == BC_WALL && k == nz - 1;
        sP[me] = Pc; sR[me] = Rc; sU[me] = U; sV[me] = V;
        if (hv0) hal[me] = h0;
        if (hv1) hal[me + NTH] = h1;
        __syncthreads();
        double Pe, Re, Pn, Rn, Pw, Rw, uw, Ps, Rs, vs;
        if (inE) { Pe = sP[me + 1]; Re = sR[me + 1]; }
        else { const double *e2 = hal + 5 * TI + t.tj; Pe = e2[0]; Re = e2[TJ]; }
        if (inN) { Pn = sP[me + TI]; Rn = sR[me + TI]; }
        else { const double *n2 = hal + t.ti; Pn = n2[0]; Rn = n2[TI]; }
        if (t.ti > 0) { Pw = sP[me - 1]; Rw = sR[me - 1]; uw = sU[me - 1]; }
        else { const double *w3 = hal + 5 * TI + 2 * TJ + t.tj; uw = w3[0]; Pw = w3[TJ]; Rw = w3[2 * TJ]; }
        if (t.tj > 0) { Ps = sP[me - TI]; Rs = sR[me - TI]; vs = sV[me - TI]; }
        else { const double *s3 = hal + 2 * TI + t.ti; vs = s3[0]; Ps = s3[TI]; Rs = s3[2 * TI]; }
        __syncthreads();
        const double Fe = n.we ? 0.0 : (1.0 - tr0 * rcp_nr(Rc + Re)) * (Pe - Pc);
        const double Fw = n.ww ? 0.0 : (1.0 - tr0 * rcp_nr(Rw + Rc)) * (Pc - Pw);
        const double Fn = n.wn ? 0.0 : (1.0 - tr0 * rcp_nr(Rc + Rn)) * (Pn - Pc);
        const double Fs = n.ws ? 0.0 : (1.0 - tr0 * rcp_nr(Rs + Rc)) * (Pc - Ps);
        const double Ft = wt ? 0.0 : (1.0 - rr0 * rcp_nr(Rc * ztab(d.rzlo, k) + Rp * ztab(d.rzhi, k))) * (Pp - Pc) * ztab(d.idzc, k);
        const double ue = n.we ? 0.0 : U, uwf = n.ww ? 0.0 : uw;
        const double vn = n.wn ? 0.0 : V, vsf = n.ws ? 0.0 : vs;
        const double wt_ = wt ? 0.0 : W;
        const double idzf = ztab(d.idzf, k);
        const double f = cdiv * ((ue - uwf) * d.idx + (vn - vsf) * d.idy + (wt_ - Wb) * idzf) + (Fe - Fw) * idx2 +
                         (Fn - Fs) * idy2 + (Ft - Fb) * idzf;
        if (t.act) {
            st_stream(d.f + c, f);
            amax = amax_nan(amax, f);
        }
        Fb = Ft;
        Wb = wt_;
        Pc = Pp; Rc = Rp;
        Pp = P2; Rp = R2;
        U = U1; V = V1; W = W1;
        h0 = g0; h1 = g1;
    }
    block_max2_to<NTH>(d.stats + ST_FINF, amax, d.stats + ST_SOLVE0, amax, red);
}

// r = f - L p (FP64, 7-point operator with variable z spacing) -> d.r.
// Marching like the RHS: x and y neighbours of p through LDS or from the
// halo (p on the four sides of the tile, 2 (TI + TJ) items: north row,
// south row, east column, west column); the z gradient below is carried.
template <int NTH = NT>
__device__ __forceinline__ void pass_resid(const Dom &d, int tile, char *smem, int solve)
{
    constexpr int MG = 0;
    double *red = (double *)smem;
    double *sP = red + 16, *hal = sP + NTH;
    const MGeo &g = d.mg[MG];
    const MTile t = march_tile(d, g, tile);
    const MNbr n = march_nbr(d, g, t);
    const int nx = d.nx, ny = d.ny, nz = d.nz, sz = nx * ny, TI = g.cti, TJ = g.ctj;
    const int col = t.j * nx + t.i;
    const double idx2 = d.idx * d.idx, idy2 = d.idy * d.idy;
    // tile origin from the tile index (t.i, t.j are clamped for idle threads)
    const int per = g.cnti * g.cntj, rem = tile - (tile / per) * per;
    const int i0 = (rem % g.cnti) * TI, j0 = (rem / g.cnti) * TJ;
    const int w = min(TI, nx - i0), h = min(TJ, ny - j0);
    const bool inE = t.ti + 1 < w, inN = t.tj + 1 < h;
    // halo item of this thread (nh = 2 (TI + TJ) <= NTH)
    const int nh = 2 * (TI + TJ);
    const bool hv = threadIdx.x < nh;
    int hoff;
    {
        const int q = min((int)threadIdx.x, nh - 1);
        const int ie = (i0 + w == nx) ? 0 : i0 + w, je = (j0 + h == ny) ? 0 : j0 + h;
        const int iw = (i0 == 0) ? nx - 1 : i0 - 1, js = (j0 == 0) ? ny - 1 : j0 - 1;
        int i, j;
        if (q < TI) { i = i0 + min(q, w - 1); j = je; }
        else if (q < 2 * TI) { i = i0 + min(q - TI, w - 1); j = js; }
        else if (q < 2 * TI + TJ) { i = ie; j = j0 + min(q - 2 * TI, h - 1); }
        else { i = iw; j = j0 + min(q - 2 * TI - TJ, h - 1); }
        hoff = j * nx + i;
    }
    const int me = threadIdx.x;
    auto kp = [&](int k) { return k == nz - 1 ? 0 : k + 1; };
    int k = t.kb;
    double Pc = d.po[k * sz + col], Pp = d.po[kp(k) * sz + col], F = d.f[k * sz + col];
    double hc = d.po[k * sz + hoff];
    double Gb = 0.0;
    if (!(d.bcz == BC_WALL && k == 0)) {
        const int km = (k == 0) ? nz - 1 : k - 1;
        Gb = (Pc - d.po[km * sz + col]) * d.idzc[km];
    }
    double amax = 0.0;
    for (; k < t.ke; ++k) {
        const int k1 = march_next(k, t);
        const double P2 = d.po[kp(k1) * sz + col], F1 = ld_stream(d.f + k1 * sz + col), hn = d.po[k1 * sz + hoff];
        const int c = k * sz + col;
        const bool wt = d.bcz == BC_WALL && k == nz - 1;
        sP[me] = Pc;
        if (hv) hal[me] = hc;
        __syncthreads();
        const double Pe = inE ? sP[me + 1] : hal[2 * TI + t.tj];
        const double Pn = inN ? sP[me + TI] : hal[t.ti];
        const double Pw = t.ti > 0 ? sP[me - 1] : hal[2 * TI + TJ + t.tj];
        const double Ps = t.tj > 0 ? sP[me - TI] : hal[TI + t.ti];
        __syncthreads();
        const double ge = n.we ? 0.0 : Pe - Pc, gw = n.ww ? 0.0 : Pc - Pw;
        const double gn = n.wn ? 0.0 : Pn - Pc, gs = n.ws ? 0.0 : Pc - Ps;
        const double Gt = wt ? 0.0 : (Pp - Pc) * ztab(d.idzc, k);
        const double r = F - ((ge - gw) * idx2 + (gn - gs) * idy2 + (Gt - Gb) * ztab(d.idzf, k));
        if (t.act) {
            st_stream(d.r + c, r);
            amax = amax_nan(amax, r);
        }
        Gb = Gt;
        Pc = Pp; Pp = P2; F = F1; hc = hn;
    }
    block_max_to<NTH>(d.stats + ST_SOLVE0 + 4 * solve, amax, red);
}

// Halo of a marching tile: the cells just outside its TI x TJ extent that
// its stencil reads, one value per item, 7 (TI + TJ) items:
//   north row  (je, i0 + x): p, p*, rho          items [0, 3 TI)
//   south row  (j0 - 1, i0 + x): v*, p, p*, rho  items [3 TI, 7 TI)
//   east col   (j0 + y, ie): p, p*, rho          items [7 TI, 7 TI + 3 TJ)
//   west col   (j0 + y, i0 - 1): u*, p, p*, rho  items [7 TI + 3 TJ, 7 (TI + TJ))
// with je, ie one past the tile's last row/column, wrapped in periodic
// directions.  Items whose cell is outside a wall, or beyond a partial tile,
// read a clamped cell and are never used.  Each thread owns at most two
// items; the host keeps 7 (TI + TJ) <= 2 x threads.

__device__ __forceinline__ Halo corr_halo(const Dom &d, const MGeo &g, int tile, int nth)
{
    const int per = g.cnti * g.cntj;
    const int rem = tile - (tile / per) * per;
    const int jt = rem / g.cnti, it = rem - jt * g.cnti;
    const int TI = g.cti, TJ = g.ctj, nx = d.nx, ny = d.ny;
    const int i0 = it * TI, j0 = jt * TJ;
    const int w = min(TI, nx - i0), h = min(TJ, ny - j0);
    const int ie = (i0 + w == nx) ? 0 : i0 + w, je = (j0 + h == ny) ? 0 : j0 + h;
    const int iw = (i0 == 0) ? nx - 1 : i0 - 1, js = (j0 == 0) ? ny - 1 : j0 - 1;
    // p, p*, rho by index (no local array: it would live in scratch)
    auto psr = [&](int f) { return f == 0 ? d.po : (f == 1 ? d.ps : d.rho); };
    Halo H;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int q = threadIdx.x + s * nth;
        int i = 0, j = 0;
        const double *fp = d.po;
        if (q < 3 * TI) {
            const int f = q / TI, x = min(q - f * TI, w - 1);
            fp = psr(f); i = i0 + x; j = je;
        } else if (q < 7 * TI) {
            const int f = (q - 3 * TI) / TI, x = min(q - 3 * TI - f * TI, w - 1);
            fp = f == 0 ? d.v : psr(f - 1); i = i0 + x; j = js;
        } else if (q < 7 * TI + 3 * TJ) {
            const int f = (q - 7 * TI) / TJ, y = min(q - 7 * TI - f * TJ, h - 1);
            fp = psr(f); i = ie; j = j0 + y;
        } else {
            const int qq = min(q - 7 * TI - 3 * TJ, 4 * TJ - 1);
            const int f = qq / TJ, y = min(qq - f * TJ, h - 1);
            fp = f == 0 ? d.u : psr(f - 1); i = iw; j = j0 + y;
        }
        H.fp[s] = fp;
        H.off[s] = j * nx + i;
    }
    return H;
}

// Velocity correction of the +faces of each column, marching in k:
//   u_out = u* - dt [ (1/rho0) G p + (1/rho_face - 1/rho0) G p* ], 0 on walls.
// With `divcheck`, also max |D u_out|: the -x and -y faces of a cell are the
// +faces of its neighbours (through LDS), recomputed from the halo at the
// tile's west and south edges; the -z face is carried from the plane below.
// Every global read of plane k+1 (centre values, halo) is issued while
// plane k is computed, so each workgroup keeps a plane of loads in flight.
// LDS: 16 reduction slots, p / p* / rho / u_out / v_out of the plane (one per
// thread), and the halo items.
template <int NTH = NT, bool TWO = true>
__device__ __forceinline__ void pass_corr(const Dom &d, int tile, char *smem, bool divcheck)
{
    constexpr int MG = 1;
    double *red = (double *)smem;
    double *sP = red + 16, *sS = sP + NTH, *sR = sS + NTH, *sE = sR + NTH, *sF = sE + NTH, *hal = sF + NTH;
    const MGeo &g = d.mg[MG];
    const MTile t = march_tile(d, g, tile);
    const MNbr n = march_nbr(d, g, t);
    const int nx = d.nx, ny = d.ny, nz = d.nz, sz = nx * ny, TI = g.cti, TJ = g.ctj;
    const int col = t.j * nx + t.i;
    const double dt = d.dt, ir0 = d.irho0;
    const int nh = 7 * (TI + TJ);
    const Halo H = corr_halo(d, g, tile, NTH);
    // TWO: a thread may own a second halo item (more halo items than
    // threads); without it the second item's load is not issued at all
    const bool hv0 = threadIdx.x < nh, hv1 = TWO && threadIdx.x + NTH < nh;
    // tile extent and where the neighbours of this cell live
    // tile origin from the tile index (t.i, t.j are clamped for idle threads)
    const int per = g.cnti * g.cntj, rem = tile - (tile / per) * per;
    const int i0 = (rem % g.cnti) * TI, j0 = (rem / g.cnti) * TJ;
    const bool inE = t.ti + 1 < min(TI, nx - i0), inN = t.tj + 1 < min(TJ, ny - j0);
    const int me = threadIdx.x;
    auto kp = [&](int k) { return k == nz - 1 ? 0 : k + 1; };
    int k = t.kb;
    // plane k (centre), plane k+1 (centre p, p*, rho), u*, v*, w* and halo of plane k
    double P0 = d.po[k * sz + col], S0 = d.ps[k * sz + col], R0 = d.rho[k * sz + col];
    double P1 = d.po[kp(k) * sz + col], S1 = d.ps[kp(k) * sz + col], R1 = d.rho[kp(k) * sz + col];
    double U = d.u[k * sz + col], V = d.v[k * sz + col], W = d.w[k * sz + col];
    double h0 = H.fp[0][k * sz + H.off[0]], h1 = TWO ? H.fp[1][k * sz + H.off[1]] : 0.0;
    double fb = 0.0;
    if (divcheck && !(d.bcz == BC_WALL && k == 0)) fb = corr_face(d, 2, t.i, t.j, (k == 0) ? nz - 1 : k - 1);
    double dmax = 0.0, omax = 0.0;
    for (; k < t.ke; ++k) {
        // prefetch plane k+1 (no load is under a branch; see march_next)
        const int k1 = march_next(k, t), k2 = kp(k1);
        const double P2 = d.po[k2 * sz + col], S2 = d.ps[k2 * sz + col], R2 = d.rho[k2 * sz + col];
        const double U1 = d.u[k1 * sz + col], V1 = d.v[k1 * sz + col], W1 = ld_stream(d.w + k1 * sz + col);
        const double g0 = H.fp[0][k1 * sz + H.off[0]], g1 = TWO ? H.fp[1][k1 * sz + H.off[1]] : 0.0;
        const int c = k * sz + col;
        const bool wt = d.bcz == BC_WALL && k == nz - 1;
        sP[me] = P0; sS[me] = S0; sR[me] = R0;
        if (hv0) hal[me] = h0;
        if (hv1) hal[me + NTH] = h1;
        __syncthreads();
        double Pe, Se, Re, Pn, Sn, Rn;
        if (inE) { Pe = sP[me + 1]; Se = sS[me + 1]; Re = sR[me + 1]; }
        else { const double *e3 = hal + 7 * TI + t.tj; Pe = e3[0]; Se = e3[TJ]; Re = e3[2 * TJ]; }
        if (inN) { Pn = sP[me + TI]; Sn = sS[me + TI]; Rn = sR[me + TI]; }
        else { const double *n3 = hal + t.ti; Pn = n3[0]; Sn = n3[TI]; Rn = n3[2 * TI]; }
        const double fe = n.we ? 0.0 : U - dt * (ir0 * (Pe - P0) * d.idx + (2.0 * rcp_nr(R0 + Re) - ir0) * (Se - S0) * d.idx);
        const double fn = n.wn ? 0.0 : V - dt * (ir0 * (Pn - P0) * d.idy + (2.0 * rcp_nr(R0 + Rn) - ir0) * (Sn - S0) * d.idy);
        const double hz = ztab(d.idzc, k);
        const double ft = wt ? 0.0 : W - dt * (ir0 * (P1 - P0) * hz + (rcp_nr(R0 * ztab(d.rzlo, k) + R1 * ztab(d.rzhi, k)) - ir0) * (S1 - S0) * hz);
        if (t.act) {
            st_stream(d.uo + c, fe);
            st_stream(d.vo + c, fn);
            st_stream(d.wo + c, ft);
            omax = amax_nan(amax_nan(amax_nan(omax, fe), fn), ft);
        }
        // faces below and west of the tile, from the halo (before the halo is rewritten)
        double fw = 0.0, fs = 0.0;
        if (divcheck) {
            if (t.ti == 0 && !n.ww) {
                const double *w4 = hal + 7 * TI + 3 * TJ + t.tj;
                const double Uw = w4[0], Pw = w4[TJ], Sw = w4[2 * TJ], Rw = w4[3 * TJ];
                fw = Uw - dt * (ir0 * (P0 - Pw) * d.idx + (2.0 * rcp_nr(Rw + R0) - ir0) * (S0 - Sw) * d.idx);
            }
            if (t.tj == 0 && !n.ws) {
                const double *s4 = hal + 3 * TI + t.ti;
                const double Vs = s4[0], Ps = s4[TI], Ss = s4[2 * TI], Rs = s4[3 * TI];
                fs = Vs - dt * (ir0 * (P0 - Ps) * d.idy + (2.0 * rcp_nr(Rs + R0) - ir0) * (S0 - Ss) * d.idy);
            }
            sE[me] = fe;
            sF[me] = fn;
        }
        __syncthreads();
        if (divcheck) {
            if (t.ti > 0) fw = sE[me - 1];
            if (t.tj > 0) fs = sF[me - TI];
            const double dv = (fe - fw) * d.idx + (fn - fs) * d.idy + (ft - fb) * ztab(d.idzf, k);
            if (t.act) dmax = amax_nan(dmax, dv);
            fb = ft;
        }
        P0 = P1; S0 = S1; R0 = R1;
        P1 = P2; S1 = S2; R1 = R2;
        U = U1; V = V1; W = W1;
        h0 = g0; h1 = g1;
    }
    block_max2_to<NTH>(divcheck ? d.stats + ST_DIV : nullptr, dmax, d.stats + ST_NONFIN, omax, red);
}

// Divergence of the stored output velocity (used when outputs alias inputs);
// tiles of NT consecutive cells (d.ndiv_tiles of them).
__device__ __forceinline__ void pass_div(const Dom &d, int tile, char *smem)
{
    double *red = (double *)smem;
    const size_t ncell = (size_t)d.nx * d.ny * d.nz;
    const size_t c = (size_t)tile * NT + threadIdx.x;
    double dmax = 0.0;
    if (c < ncell) {
        size_t plane = (size_t)d.nx * d.ny;
        int k = (int)(c / plane);
        size_t rem = c - (size_t)k * plane;
        int j = (int)(rem / d.nx);
        int i = (int)(rem - (size_t)j * d.nx);
        double fw = (i > 0) ? d.uo[c - 1] : (d.bcx == BC_WALL ? 0.0 : d.uo[c + d.nx - 1]);
        double fs = (j > 0) ? d.vo[c - d.nx] : (d.bcy == BC_WALL ? 0.0 : d.vo[c + (size_t)(d.ny - 1) * d.nx]);
        double fb = (k > 0) ? d.wo[c - plane] : (d.bcz == BC_WALL ? 0.0 : d.wo[c + (size_t)(d.nz - 1) * plane]);
        double dv = (d.uo[c] - fw) * d.idx + (d.vo[c] - fs) * d.idy + (d.wo[c] - fb) * d.idzf[k];
        dmax = fabs(dv);
    }
    block_max_to(d.stats + ST_DIV, dmax, red);
}

// ------------------------------------------------------- fused stencils
// The RHS f (SRC_RHS_ST) or the residual r = f - L p (SRC_RESID_ST) at the
// cells of row j of plane k, evaluated by the calling wave straight from the
// fields, as the pairs (2h, 2h+1) the real x FFT takes (lane: h = lane + 64 t),
// handed to put(h, value).  Same stencil and wall rules as pass_rhs and
// pass_resid; the neighbours in y and z are read from memory (the tiles of
// the neighbouring rows and planes run at the same time, so these reads are
// mostly cache hits), the x neighbours of a pair are its two outer cells.
// Returns the lane's max |value|.
struct SxRow {
    int c, cn, cs, cu, cd;       // offsets of row j / j+1 / j-1 of plane k, row j of planes k+1 / k-1
    bool wn, ws, wt, wb;         // wall faces north, south, top, bottom
};

__device__ __forceinline__ SxRow sx_row(const Dom &d, int j, int k)
{
    SxRow r;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const size_t sz = (size_t)nx * ny;
    const bool wy = d.bcy == BC_WALL, wz = d.bcz == BC_WALL;
    r.wn = wy && j == ny - 1;
    r.ws = wy && j == 0;
    r.wt = wz && k == nz - 1;
    r.wb = wz && k == 0;
    // neighbours across a wall are never used: a valid (clamped) row instead
    const int jn = j == ny - 1 ? (wy ? j : 0) : j + 1;
    const int js = j == 0 ? (wy ? j : ny - 1) : j - 1;
    const int ku = k == nz - 1 ? (wz ? k : 0) : k + 1;
    const int kd = k == 0 ? (wz ? k : nz - 1) : k - 1;
    r.c = (int)(k * sz) + j * nx;
    r.cn = (int)(k * sz) + jn * nx;
    r.cs = (int)(k * sz) + js * nx;
    r.cu = (int)(ku * sz) + j * nx;
    r.cd = (int)(kd * sz) + j * nx;
    return r;
}

template <int SRC, typename Put>
__device__ __forceinline__ double stencil_row(const Dom &d, int j, int k, int lane, Put put)
{
    const SxRow R = sx_row(d, j, k);
    const int nx = d.nx, hx = nx >> 1;
    const bool wx = d.bcx == BC_WALL;
    const int kd = k == 0 ? d.nz - 1 : k - 1; // z face below (unused on a bottom wall)
    const double idzf = ztab(d.idzf, k), idzc = ztab(d.idzc, k), idzcb = ztab(d.idzc, kd);
    const double idx2 = d.idx * d.idx, idy2 = d.idy * d.idy;
    double amax = 0.0;
    if constexpr (SRC == SRC_RHS_ST) {
        const double rr0 = d.rho0, tr0 = 2.0 * d.rho0, cdiv = d.rho0 / d.dt;
        const double rlo = ztab(d.rzlo, k), rhi = ztab(d.rzhi, k), rlob = ztab(d.rzlo, kd), rhib = ztab(d.rzhi, kd);
        auto ld2 = [](const double *p, int o) { return *(const double2 *)(p + o); };
#pragma unroll 1
        for (int h = lane; h < hx; h += 64) {
            const int i0 = 2 * h;
            const int iw = h == 0 ? nx - 1 : i0 - 1, ie = h == hx - 1 ? 0 : i0 + 2;
            const double2 P = ld2(d.ps, R.c + i0), Rh = ld2(d.rho, R.c + i0);
            const double Pw = d.ps[R.c + iw], Rw = d.rho[R.c + iw], Pe = d.ps[R.c + ie], Re = d.rho[R.c + ie];
            const double2 Pn = ld2(d.ps, R.cn + i0), Rn = ld2(d.rho, R.cn + i0);
            const double2 Ps = ld2(d.ps, R.cs + i0), Rs = ld2(d.rho, R.cs + i0);
            const double2 Pu = ld2(d.ps, R.cu + i0), Ru = ld2(d.rho, R.cu + i0);
            const double2 Pd = ld2(d.ps, R.cd + i0), Rd = ld2(d.rho, R.cd + i0);
            const double2 U = ld2(d.u, R.c + i0), V = ld2(d.v, R.c + i0), Vs = ld2(d.v, R.cs + i0);
            const double2 W = ld2(d.w, R.c + i0), Wd = ld2(d.w, R.cd + i0); // w is re-read by the plane above
            const double Uw = d.u[R.c + iw];
            const bool ww = wx && h == 0, we = wx && h == hx - 1;
            // x fluxes: face between the pair's cells, west of cell 0, east of cell 1
            const double Fm = (1.0 - tr0 * rcp_nr(Rh.x + Rh.y)) * (P.y - P.x);
            const double Fw = ww ? 0.0 : (1.0 - tr0 * rcp_nr(Rw + Rh.x)) * (P.x - Pw);
            const double Fe = we ? 0.0 : (1.0 - tr0 * rcp_nr(Rh.y + Re)) * (Pe - P.y);
            double f[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double Pc = q ? P.y : P.x, Rc = q ? Rh.y : Rh.x;
                const double pn = q ? Pn.y : Pn.x, rn = q ? Rn.y : Rn.x, ps = q ? Ps.y : Ps.x, rs = q ? Rs.y : Rs.x;
                const double pu = q ? Pu.y : Pu.x, ru = q ? Ru.y : Ru.x, pd = q ? Pd.y : Pd.x, rd = q ? Rd.y : Rd.x;
                const double Fn = R.wn ? 0.0 : (1.0 - tr0 * rcp_nr(Rc + rn)) * (pn - Pc);
                const double Fs = R.ws ? 0.0 : (1.0 - tr0 * rcp_nr(rs + Rc)) * (Pc - ps);
                const double Ft = R.wt ? 0.0 : (1.0 - rr0 * rcp_nr(Rc * rlo + ru * rhi)) * (pu - Pc) * idzc;
                const double Fb = R.wb ? 0.0 : (1.0 - rr0 * rcp_nr(rd * rlob + Rc * rhib)) * (Pc - pd) * idzcb;
                const double ue = q ? (we ? 0.0 : U.y) : U.x, uw = q ? U.x : (ww ? 0.0 : Uw);
                const double vn = R.wn ? 0.0 : (q ? V.y : V.x), vs = R.ws ? 0.0 : (q ? Vs.y : Vs.x);
                const double wt = R.wt ? 0.0 : (q ? W.y : W.x), wb = R.wb ? 0.0 : (q ? Wd.y : Wd.x);
                const double fe = q ? Fe : Fm, fw = q ? Fm : Fw;
                f[q] = cdiv * ((ue - uw) * d.idx + (vn - vs) * d.idy + (wt - wb) * idzf) + (fe - fw) * idx2 +
                       (Fn - Fs) * idy2 + (Ft - Fb) * idzf;
            }
            const double2 v = double2{f[0], f[1]};
            if (d.r) st_stream((double2 *)(d.f + R.c + i0), v); // refined form: the residual needs f
            put(h, v);
            amax = amax_nan(amax_nan(amax, f[0]), f[1]);
        }
    } else {
        auto ld2 = [](const double *p, int o) { return *(const double2 *)(p + o); };
#pragma unroll 1
        for (int h = lane; h < hx; h += 64) {
            const int i0 = 2 * h;
            const int iw = h == 0 ? nx - 1 : i0 - 1, ie = h == hx - 1 ? 0 : i0 + 2;
            const double2 P = ld2(d.po, R.c + i0);
            const double Pw = d.po[R.c + iw], Pe = d.po[R.c + ie];
            const double2 Pn = ld2(d.po, R.cn + i0), Ps = ld2(d.po, R.cs + i0);
            const double2 Pu = ld2(d.po, R.cu + i0), Pd = ld2(d.po, R.cd + i0);
            const double2 F = ld_stream((const double2 *)(d.f + R.c + i0));
            const bool ww = wx && h == 0, we = wx && h == hx - 1;
            const double gm = P.y - P.x;
            const double gw = ww ? 0.0 : P.x - Pw, ge = we ? 0.0 : Pe - P.y;
            double r[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double Pc = q ? P.y : P.x;
                const double gn = R.wn ? 0.0 : (q ? Pn.y : Pn.x) - Pc, gs = R.ws ? 0.0 : Pc - (q ? Ps.y : Ps.x);
                const double Gt = R.wt ? 0.0 : ((q ? Pu.y : Pu.x) - Pc) * idzc;
                const double Gb = R.wb ? 0.0 : (Pc - (q ? Pd.y : Pd.x)) * idzcb;
                const double gee = q ? ge : gm, gww = q ? gm : gw;
                r[q] = (q ? F.y : F.x) - ((gee - gww) * idx2 + (gn - gs) * idy2 + (Gt - Gb) * idzf);
            }
            put(h, double2{r[0], r[1]});
            amax = amax_nan(amax_nan(amax, r[0]), r[1]);
        }
    }
    return amax;
}

// Maximum of the fused stencil passes' per-wave partials into stats slot
// sa (and sb when >= 0): workgroup wg of nwg takes every nwg-th block.
__device__ __forceinline__ void pass_smax(const Dom &d, int sa, int sb, int wg, int nwg, char *smem)
{
    double *red = (double *)smem;
    const int nt = sslots(d);
    double a = 0.0;
    for (int q0 = wg * NT; q0 < nt; q0 += 8 * nwg * NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = d.spart[min(q0 + u * nwg * NT + (int)threadIdx.x, nt - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q0 + u * nwg * NT + (int)threadIdx.x < nt) a = (v[u] != v[u] || v[u] > a) ? v[u] : a;
    }
    block_max2_to<NT>(d.stats + sa, a, sb >= 0 ? d.stats + sb : nullptr, a, red);
}

// ------------------------------------------------------------------ xfwd
// Tile = (j tile, k): rows j0 .. j0+rows-1 of plane k of f (or r).  Real
// FFT by a half-length complex FFT of z[n] = s[2n] + i s[2n+1] and the split
// X[l] = E + W^l O, X[M-l] = conj(E - W^l O); then the corner turn into S1.
template <typename T, int SRC, int NTH = NT, bool WV = true>
__device__ __forceinline__ void pass_xfwd(const Dom &d, int tile, char *smem)
{
    using C = c2<T>;
    C *buf = (C *)smem;
    const int ldr = lds_line(d.nl);
    C *ltw = buf + d.tj * ldr;
    const int jt = tile % d.ntj, k = tile / d.ntj;
    const int j0 = jt * d.tj;
    const int rows = min(d.tj, d.ny - j0);
    const int nx = d.nx, M = d.M, half = M / 2;
    constexpr bool ST = SRC == SRC_RHS_ST || SRC == SRC_RESID_ST;
    const double *src = (SRC == SRC_RHS || SRC == SRC_RHS_ST ? d.f : d.r) + ((size_t)k * d.ny + j0) * nx;
    // LDS: the tile's rows, the FFT roots, the split twiddles (M/2 + 1)
    C *ltr = ltw + tw_half(d.fx.n);
    TwStage<T, NTH> tws;
    TabStage<T, NTH> trs;
    tws.fetch(d.fx);
    trs.fetch((const C *)d.twr, M / 2 + 1);
    const bool wx = d.bcx != BC_PER;
    // Dirichlet x: the sine transform is the cosine one of (-1)^i s_i (its
    // modes come out in reverse order, which only the eigenvalues see)
    const T odd = d.bcx == BC_DIR ? T(-1) : T(1);
    const int hx = nx >> 1;
    const double2 *src2 = (const double2 *)src;
    const C *twr = ltr;
    const C *wd = (const C *)d.dctx;
    // pairs (s[2h], s[2h+1]) form complex point h of the half-length FFT;
    // wall x: cosine transform by reordering v[h] = s[2h], v[N-1-h] = s[2h+1]
    auto put_pair = [&](C *row, int h, double2 s) {
        if (!wx) {
            row[pidx(h)] = C{(T)s.x, (T)s.y};
        } else {
            int n1 = nx - 1 - h;
            ((T *)(row + pidx(h >> 1)))[h & 1] = (T)s.x;
            ((T *)(row + pidx(n1 >> 1)))[n1 & 1] = odd * (T)s.y;
        }
    };
    // split of the half-length spectrum, l in [0, M/2]
    auto split = [&](C *row, int l) {
        if (l == 0) {
            C z0 = row[0];
            row[0] = C{z0.x + z0.y, T(0)};
            row[pidx(M)] = C{z0.x - z0.y, T(0)};
        } else if (2 * l == M) {
            row[pidx(l)] = cconj(row[pidx(l)]);
        } else {
            C zl = row[pidx(l)], zm = row[pidx(M - l)];
            C e = {T(0.5) * (zl.x + zm.x), T(0.5) * (zl.y - zm.y)};
            // o = (zl - conj(zm)) / (2i)
            C o = {T(0.5) * (zl.y + zm.y), T(-0.5) * (zl.x - zm.x)};
            C wo = cmul(twr[l], o);
            row[pidx(l)] = cadd(e, wo);
            row[pidx(M - l)] = cconj(csub(e, wo));
        }
    };
    // DCT-II from the real FFT V of the reordered row: A_k = W_{4N}^k V_k,
    // X_k = Re A_k, X_{N-k} = -Im A_k (k in [0, M]); stored as real modes
    auto dct = [&](C *row, int kk) {
        C a = cmul(wd[kk], row[pidx(kk)]);
        row[pidx(kk)] = C{a.x, T(0)};
        if (kk >= 1 && kk < M) row[pidx(nx - kk)] = C{-a.y, T(0)};
    };
    // one wave per row when the tile has at most one row per wave and the
    // half length has the fixed wave plan (which must be the descriptor's)
    constexpr int NW = NTH / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const bool wv = WV && d.tj <= NW && wave_plan(d.fx);
    if (ST && !wv) return; // the host enables the fused forms only on the wave path
    if (wv) {
        if (wid < rows) {
            C *row = buf + wid * ldr;
            if constexpr (ST) {
                const double m = stencil_row<SRC>(d, j0 + wid, k, lane, [&](int h, double2 s) { put_pair(row, h, s); });
                const double wm = wave_max1(m);
                if (lane == 0) d.spart[tile * NW + wid] = wm;
            } else {
                const double2 *sr = src2 + (size_t)wid * hx;
                staged_copy_t<64, 8, double2>(
                    lane, hx, [&](int h) { return sr[h]; }, [&](int h, double2 s) { put_pair(row, h, s); });
            }
        } else if (ST && lane == 0 && wid < NW) {
            d.spart[tile * NW + wid] = 0.0;
        }
        tws.put(ltw, d.fx);
        trs.put(ltr, (const C *)d.twr, M / 2 + 1);
        __syncthreads(); // the twiddles
        if (wid < rows) {
            C *row = buf + wid * ldr;
            wave_fft<T, false>(row, ltw, d.fx, lane);
            for (int l = lane; l <= half; l += 64) split(row, l);
            if (wx) {
                wave_sync();
                for (int kk = lane; kk <= M; kk += 64) dct(row, kk);
            }
        }
        __syncthreads();
    } else {
        staged_copy<NTH, 8, double2>(
            rows * hx, [&](int e) { return src2[e]; },
            [&](int e, double2 s) {
                int r = (int)fdiv((uint32_t)e, d.dM);
                put_pair(buf + r * ldr, e - r * hx, s);
            });
        tws.put(ltw, d.fx);
        trs.put(ltr, (const C *)d.twr, M / 2 + 1);
        __syncthreads();
        lds_fft<T, false, NTH>(buf, ldr, rows, d.fx, ltw);
        for (int idx = threadIdx.x; idx < rows * (half + 1); idx += NTH) {
            int r = (int)fdiv((uint32_t)idx, d.dH1);
            split(buf + r * ldr, idx - r * (half + 1));
        }
        __syncthreads();
        if (wx) {
            for (int idx = threadIdx.x; idx < rows * (M + 1); idx += NTH) {
                int r = (int)fdiv((uint32_t)idx, d.dM1);
                dct(buf + r * ldr, idx - r * (M + 1));
            }
            __syncthreads();
        }
    }
    C *s1 = (C *)d.s1;
    const int tj = d.tj, nl = d.nl;
    staged_copy<NTH, 8, C>(
        tj * nl,
        [&](int e) {
            int l = (int)fdiv((uint32_t)e, d.dtj);
            int r = e - l * tj;
            return buf[min(r, rows - 1) * ldr + pidx(l)];
        },
        [&](int e, C v) {
            int l = (int)fdiv((uint32_t)e, d.dtj);
            int r = e - l * tj;
            if (r < rows) st_stream(s1 + ((size_t)k * nl + l) * d.ny + j0 + r, v);
        });
}

// Y pass, tile = (k tile, l).  Forward: columns (k, l) of S1 -> LDS -> FFT
// (DCT-II for a wall) -> corner turn into the z-lines of S2; inverse the
// reverse.
template <typename T, bool INV, int NTH = NT, bool WV = true>
__device__ __forceinline__ void pass_y(const Dom &d, int tile, char *smem)
{
    using C = c2<T>;
    C *buf = (C *)smem;
    const int ny = d.ny, nz = d.nz, nl = d.nl, tk = d.tk, ntk = d.ntk;
    const FastDiv dtk = d.dtk;
    const int ldc = lds_line(ny);
    C *ltw = buf + tk * ldc;
    const bool wy = d.bcy != BC_PER;
    // wall y: cosine transform by reordering v[n] = c[2n], v[N-1-n] = c[2n+1];
    // Dirichlet y: the same on (-1)^j c_j (forward) and for the result (inverse)
    auto pos = [&](int j) { return wy ? ((j & 1) ? ny - 1 - (j >> 1) : (j >> 1)) : j; };
    const bool dy = d.bcy == BC_DIR;
    auto sgn = [&](int j, C v) { return (dy && (j & 1)) ? C{-v.x, -v.y} : v; };
    C *s1 = (C *)d.s1;
    C *s2 = (C *)d.s2;
    const C *wd = (const C *)d.dcty;
    const int hy = ny / 2;
    const int kt = tile % ntk, l = tile / ntk;
    const int k0 = kt * tk;
    const int cols = min(tk, nz - k0);
    TwStage<T, NTH> tws;
    tws.fetch(d.fy);
    // one wave per column when the tile has at most one column per wave and
    // the length has the fixed wave plan (which must be the descriptor's)
    constexpr int NW = NTH / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const bool wv = WV && tk <= NW && wave_plan(d.fy);
    if (!INV && wv) {
        if (wid < cols) {
            const C *src = s1 + ((size_t)(k0 + wid) * nl + l) * ny;
            C *col = buf + wid * ldc;
            staged_copy_t<64, 8, C>(
                lane, ny, [&](int j) { return ld_stream(src + j); }, [&](int j, C v) { col[pidx(pos(j))] = sgn(j, v); });
        }
    } else if (!INV) {
        staged_copy<NTH, 8, C>(
            cols * ny,
            [&](int e) {
                const int c = (int)fdiv((uint32_t)e, d.dnyc), j = e - c * ny;
                return ld_stream(s1 + ((size_t)(k0 + c) * nl + l) * ny + j);
            },
            [&](int e, C v) {
                const int c = (int)fdiv((uint32_t)e, d.dnyc), j = e - c * ny;
                buf[c * ldc + pidx(pos(j))] = sgn(j, v);
            });
    } else {
        staged_copy<NTH, 8, C>(
            tk * ny,
            [&](int e) {
                const int m = (int)fdiv((uint32_t)e, dtk), c = e - m * tk;
                return ld_stream(s2 + ((size_t)l * ny + m) * nz + k0 + min(c, cols - 1));
            },
            [&](int e, C v) {
                const int m = (int)fdiv((uint32_t)e, dtk), c = e - m * tk;
                if (c < cols) buf[c * ldc + pidx(m)] = v;
            });
        if (wy && !wv) {
            // inverse DCT-II of complex columns: V_k = conj(w_k)(X_k - i X_{N-k}),
            // V_{N-k} = i w_k (X_{N-k} - i X_k), w_k = W_{4N}^k, X_N = 0
            __syncthreads();
            for (int idx = threadIdx.x; idx < cols * hy; idx += NTH) {
                const int c = (int)fdiv((uint32_t)idx, d.dhy);
                const int kk = idx - c * hy + 1;
                C *col = buf + c * ldc;
                const int kn = ny - kk;
                C w = wd[kk];
                C xk = col[pidx(kk)], xn = col[pidx(kn)];
                C a = {xk.x + xn.y, xk.y - xn.x};   // X_k - i X_{N-k}
                col[pidx(kk)] = cmul(cconj(w), a);
                if (kn != kk) {
                    C b = {xn.x + xk.y, xn.y - xk.x}; // X_{N-k} - i X_k
                    C wb = cmul(w, b);
                    col[pidx(kn)] = C{-wb.y, wb.x};   // i w b
                }
            }
        }
    }
    tws.put(ltw, d.fy);
    __syncthreads();
    if (wv) {
        if (wid < cols) {
            C *col = buf + wid * ldc;
            if (INV && wy) {
                // inverse DCT-II pre-step of this column (as in the workgroup path below)
                for (int kk = 1 + lane; kk <= hy; kk += 64) {
                    const int kn = ny - kk;
                    C w = wd[kk];
                    C xk = col[pidx(kk)], xn = col[pidx(kn)];
                    C a = {xk.x + xn.y, xk.y - xn.x};
                    col[pidx(kk)] = cmul(cconj(w), a);
                    if (kn != kk) {
                        C b = {xn.x + xk.y, xn.y - xk.x};
                        C wb = cmul(w, b);
                        col[pidx(kn)] = C{-wb.y, wb.x};
                    }
                }
            }
            wave_fft<T, INV>(col, ltw, d.fy, lane);
            if (!INV && wy) {
                for (int kk = 1 + lane; kk <= hy; kk += 64) {
                    const int kn = ny - kk;
                    C w = wd[kk];
                    C p = cmul(w, col[pidx(kk)]), q = cmul(cconj(w), col[pidx(kn)]);
                    col[pidx(kk)] = C{T(0.5) * (p.x + q.x), T(0.5) * (p.y + q.y)};
                    if (kn != kk) col[pidx(kn)] = C{T(-0.5) * (p.y - q.y), T(0.5) * (p.x - q.x)};
                }
            }
            if (INV) {
                // the column goes back to S1 by its own wave
                wave_sync();
                C *dst = s1 + ((size_t)(k0 + wid) * nl + l) * ny;
                // eight LDS reads in flight per lane, then the stores
                staged_copy_t<64, 8, C>(
                    lane, ny, [&](int j) { return sgn(j, col[pidx(pos(j))]); }, [&](int j, C v) { st_stream(dst + j, v); });
            }
        }
        if (INV) return;
        __syncthreads();
    } else {
        lds_fft<T, INV, NTH>(buf, ldc, cols, d.fy, ltw);
    }
    if (!INV) {
        if (wy && !wv) {
            // DCT-II of complex columns from the FFT V of the reordered data:
            // X_k = (w_k V_k + conj(w_k) V_{N-k}) / 2,
            // X_{N-k} = i (w_k V_k - conj(w_k) V_{N-k}) / 2, X_0 = V_0
            for (int idx = threadIdx.x; idx < cols * hy; idx += NTH) {
                const int c = (int)fdiv((uint32_t)idx, d.dhy);
                const int kk = idx - c * hy + 1;
                C *col = buf + c * ldc;
                const int kn = ny - kk;
                C w = wd[kk];
                C p = cmul(w, col[pidx(kk)]), q = cmul(cconj(w), col[pidx(kn)]);
                col[pidx(kk)] = C{T(0.5) * (p.x + q.x), T(0.5) * (p.y + q.y)};
                if (kn != kk) col[pidx(kn)] = C{T(-0.5) * (p.y - q.y), T(0.5) * (p.x - q.x)};
            }
            __syncthreads();
        }
        staged_copy<NTH, 8, C>(
            tk * ny,
            [&](int e) {
                const int m = (int)fdiv((uint32_t)e, dtk), c = e - m * tk;
                return buf[min(c, cols - 1) * ldc + pidx(m)];
            },
            [&](int e, C v) {
                const int m = (int)fdiv((uint32_t)e, dtk), c = e - m * tk;
                if (c < cols) st_stream(s2 + ((size_t)l * ny + m) * nz + k0 + c, v);
            });
    } else {
        staged_copy<NTH, 8, C>(
            cols * ny,
            [&](int e) {
                const int c = (int)fdiv((uint32_t)e, d.dnyc), j = e - c * ny;
                return sgn(j, buf[c * ldc + pidx(pos(j))]);
            },
            [&](int e, C v) {
                const int c = (int)fdiv((uint32_t)e, d.dnyc), j = e - c * ny;
                st_stream(s1 + ((size_t)(k0 + c) * nl + l) * ny + j, v);
            });
    }
}

// --------------------------------------------------------------- z solve
// Lines (l, m) are contiguous in S2.  G lanes cooperate on one line, lane t
// owning a contiguous chunk of S_t levels (sizes differ by at most one).  The
// first S_t - 1 levels of a chunk are eliminated locally (Thomas with two
// extra right-hand sides giving the response to the neighbouring chunks'
// last unknowns E_{t-1}, E_t), leaving one equation per lane in the E's:
//   alpha_t E_{t-1} + beta_t E_t + gamma_t E_{t+1} = rho_t,
// solved by parallel cyclic reduction across the G lanes (cyclic when z is
// periodic).  The singular mode (l, m) = (0, 0) is made compatible, pinned
// (last level = 0), solved without wrap, then shifted to zero dzf-weighted
// mean.  The right-hand side is scaled by 1/(nx ny) (inverse transforms are
// unnormalised).
template <typename T, int SMAX>
__device__ __forceinline__ void pass_z(const Dom &d, int tile, char *smem)
{
    using C = c2<T>;
    C *buf = (C *)smem;
    const int nz = d.nz, G = d.zg;
    const int lpw = 64 / G;                      // lines per wave
    const int lpg = d.zlpw;                      // lines per workgroup
    const long nlines_tot = (long)d.nl * d.ny;
    const long q0 = (long)tile * lpg;
    const int nlin = (int)min((long)lpg, nlines_tot - q0);
    C *s2 = (C *)d.s2;
    const size_t gbase = (size_t)q0 * nz;
    // Each wave stages, solves and writes back its own lines through its own
    // LDS region, with no workgroup barrier: the waves of a workgroup drift
    // apart, so one wave's loads overlap another's arithmetic.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wl0 = wv * lpw;                    // first line of this wave
    const int wlines = min(lpw, nlin - wl0);
    if (wlines <= 0) return;
    const int wb = wl0 * nz, wn = wlines * nz;   // element range of the wave
    // padded LDS index: one spare slot per 16 elements
#define ZP(e) ((e) + ((e) >> 4))
    staged_copy_t<64, 8, C>(lane, wn, [&](int e) { return s2[gbase + wb + e]; },
                            [&](int e, C v) { buf[ZP(wb + e)] = v; });
    wave_sync();

    const int t = lane & (G - 1);
    const int gl = wl0 + (lane / G);             // line within the workgroup
    const bool active = gl < nlin;
    const int gls = active ? gl : wl0;
    const long q = q0 + gls;
    const int l = (int)(q / d.ny), m = (int)(q - (long)l * d.ny);
    const bool sing_line = !d.nosing && l == 0 && m == 0;
    const T *za = (const T *)d.za, *zb = (const T *)d.zb, *zc = (const T *)d.zc, *dzf = (const T *)d.dzf_s;
    const T sh = ((const T *)d.lamx)[l] + ((const T *)d.lamy)[m];
    const T scale = (T)d.scale;
    const int base = nz / G, rem = nz - base * G;
    const int lbase = lane & ~(G - 1);
    // The solve body, FULL: every lane holds SMAX levels and no line of the
    // wave is the singular mode (all but one wave of the grid), so the
    // per-level guards and the singular-mode steps fold away at compile
    // time; CY: 1 periodic, 2 not, 0 decided at run time.
    auto solve = [&](auto full_tag, auto cy_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        constexpr int CY = decltype(cy_tag)::value;
        const bool sing = FULL ? false : sing_line;
        const bool cyc = CY == 1 ? true : (CY == 2 ? false : (d.bcz == BC_PER) && !sing);
        const int S = FULL ? SMAX : base + (t < rem ? 1 : 0);
        const int k0 = FULL ? t * SMAX : t * base + min(t, rem);
        const int mi = S - 1;                        // interior rows
        C y[SMAX];
        T g[SMAX], cp[SMAX];
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
            if (s < S) {
                C v = buf[ZP(gls * nz + k0 + s)];
                y[s] = C{v.x * scale, v.y * scale};
            }
        }
        // compatibility of the singular mode: remove the dzf-weighted mean
        if (sing) {
            C acc = {T(0), T(0)};
#pragma unroll
            for (int s = 0; s < SMAX; ++s)
                if (s < S) { T w = dzf[k0 + s]; acc.x += w * y[s].x; acc.y += w * y[s].y; }
            for (int o = 1; o < G; o <<= 1) { acc.x += __shfl_xor(acc.x, o, 64); acc.y += __shfl_xor(acc.y, o, 64); }
            T il = T(1) / (T)d.lz;
#pragma unroll
            for (int s = 0; s < SMAX; ++s)
                if (s < S) { y[s].x -= acc.x * il; y[s].y -= acc.y * il; }
            // the pinned level nz-1 is the identity row x = 0
#pragma unroll
            for (int s = 0; s < SMAX; ++s)
                if (s < S && k0 + s == nz - 1) y[s] = C{T(0), T(0)};
        }
        // row coefficients (pinned system for the singular mode)
        auto coef = [&](int k, T &A, T &B, T &Cc) {
            A = za[k]; Cc = zc[k]; B = zb[k] + sh;
            if (sing) {
                if (k == nz - 1) { A = T(0); Cc = T(0); B = T(1); }
                if (k == nz - 2) Cc = T(0);
                if (k == 0) A = T(0);
            }
        };
        // local elimination of the interior rows k0 .. k0+mi-1
        T hlast = T(0);
        {
            T cpp = T(0), gp = T(0);
            C yp = {T(0), T(0)};
#pragma unroll
            for (int s = 0; s < SMAX - 1; ++s) {
                if (s < mi) {
                    T A, B, Cc;
                    coef(k0 + s, A, B, Cc);
                    T a = (s == 0) ? T(0) : A;
                    T inv = rcp_t(B - a * cpp);
                    cp[s] = Cc * inv;
                    y[s] = C{(y[s].x - a * yp.x) * inv, (y[s].y - a * yp.y) * inv};
                    g[s] = ((s == 0) ? -A : -a * gp) * inv;
                    if (s == mi - 1) hlast = -Cc * inv;
                    cpp = cp[s]; yp = y[s]; gp = g[s];
                }
            }
        }
        T h0 = hlast;
#pragma unroll
        for (int s = SMAX - 3; s >= 0; --s) {
            if (s < mi - 1) {
                y[s].x -= cp[s] * y[s + 1].x;
                y[s].y -= cp[s] * y[s + 1].y;
                g[s] -= cp[s] * g[s + 1];
                h0 = -cp[s] * h0;
            }
        }
        // E-row of this lane: row ke = k0 + mi
        T Ae, Be, Ce;
        coef(k0 + mi, Ae, Be, Ce);
        C ye = y[0];
        T gl_last = T(0), hl_last = hlast;
        C yl_last = {T(0), T(0)};
#pragma unroll
        for (int s = 0; s < SMAX; ++s) {
            if (s == mi) ye = y[s];
            if (s == mi - 1) { yl_last = y[s]; gl_last = g[s]; }
        }
        // first interior unknown of the next lane (wraps for a cyclic line)
        const int nxt = lbase | ((t + 1) & (G - 1));
        C y0n = {__shfl(y[0].x, nxt, 64), __shfl(y[0].y, nxt, 64)};
        T g0n = __shfl(g[0], nxt, 64);
        T h0n = __shfl(h0, nxt, 64);
        T al = Ae * gl_last;
        T be = Be + Ae * hl_last + Ce * g0n;
        T ga = Ce * h0n;
        C rh = {ye.x - Ae * yl_last.x - Ce * y0n.x, ye.y - Ae * yl_last.y - Ce * y0n.y};
        // parallel cyclic reduction over the G lanes of the line
        for (int dd = 1; dd < G; dd <<= 1) {
            int lo = t - dd, hi = t + dd;
            bool vlo = cyc || lo >= 0, vhi = cyc || hi < G;
            int slo = lbase | (lo & (G - 1)), shi = lbase | (hi & (G - 1));
            T al_lo = __shfl(al, slo, 64), be_lo = __shfl(be, slo, 64), ga_lo = __shfl(ga, slo, 64);
            T rx_lo = __shfl(rh.x, slo, 64), ry_lo = __shfl(rh.y, slo, 64);
            T al_hi = __shfl(al, shi, 64), be_hi = __shfl(be, shi, 64), ga_hi = __shfl(ga, shi, 64);
            T rx_hi = __shfl(rh.x, shi, 64), ry_hi = __shfl(rh.y, shi, 64);
            if (!vlo) { al_lo = T(0); be_lo = T(1); ga_lo = T(0); rx_lo = T(0); ry_lo = T(0); }
            if (!vhi) { al_hi = T(0); be_hi = T(1); ga_hi = T(0); rx_hi = T(0); ry_hi = T(0); }
            T k1 = al * rcp_t(be_lo), k2 = ga * rcp_t(be_hi);
            T nal = -k1 * al_lo, nga = -k2 * ga_hi;
            T nbe = be - k1 * ga_lo - k2 * al_hi;
            rh = C{rh.x - k1 * rx_lo - k2 * rx_hi, rh.y - k1 * ry_lo - k2 * ry_hi};
            al = nal; be = nbe; ga = nga;
        }
        T den = cyc ? (al + be + ga) : be;
        const T iden = rcp_t(den);
        C E = {rh.x * iden, rh.y * iden};
        const int prv = lbase | ((t - 1) & (G - 1));
        C Ep = {__shfl(E.x, prv, 64), __shfl(E.y, prv, 64)};
        // reconstruction x_s = y_s + g_s E_{t-1} + h_s E_t
        {
            T h = hlast;
#pragma unroll
            for (int s = SMAX - 2; s >= 0; --s) {
                if (s < mi) {
                    y[s] = C{y[s].x + g[s] * Ep.x + h * E.x, y[s].y + g[s] * Ep.y + h * E.y};
                    if (s > 0) h = -cp[s - 1] * h;
                }
            }
#pragma unroll
            for (int s = 0; s < SMAX; ++s)
                if (s == mi) y[s] = E;
        }
        // gauge of the singular mode: zero dzf-weighted mean
        if (sing) {
            C acc = {T(0), T(0)};
#pragma unroll
            for (int s = 0; s < SMAX; ++s)
                if (s < S) { T w = dzf[k0 + s]; acc.x += w * y[s].x; acc.y += w * y[s].y; }
            for (int o = 1; o < G; o <<= 1) { acc.x += __shfl_xor(acc.x, o, 64); acc.y += __shfl_xor(acc.y, o, 64); }
            T il = T(1) / (T)d.lz;
#pragma unroll
            for (int s = 0; s < SMAX; ++s)
                if (s < S) { y[s].x -= acc.x * il; y[s].y -= acc.y * il; }
        }
        wave_sync();
        if (active) {
#pragma unroll
            for (int s = 0; s < SMAX; ++s)
                if (s < S) buf[ZP(gl * nz + k0 + s)] = y[s];
        }
    };
    using std::integral_constant;
    const bool full = rem == 0 && base == SMAX && !__any(sing_line ? 1 : 0);
    if (full && d.bcz == BC_PER) solve(integral_constant<bool, true>{}, integral_constant<int, 1>{});
    else if (full) solve(integral_constant<bool, true>{}, integral_constant<int, 2>{});
    else solve(integral_constant<bool, false>{}, integral_constant<int, 0>{});
    wave_sync();
    staged_copy_t<64, 8, C>(lane, wn, [&](int e) { return buf[ZP(wb + e)]; },
                            [&](int e, C v) { st_stream(s2 + gbase + wb + e, v); });
#undef ZP
}

// ------------------------------------------------------------------ xinv
// Tile = (j tile, k).  Inverse real FFT of rows j0.. of plane k from S1;
// MODE store: p = value; accum: p += value (refinement update).
template <typename T, int MODE, int NTH = NT, bool WV = true>
__device__ __forceinline__ void pass_xinv(const Dom &d, int tile, char *smem, int solve)
{
    using C = c2<T>;
    C *buf = (C *)smem;
    const int ldr = lds_line(d.nl);
    // LDS: the tile's rows, the FFT roots, the split twiddles (M/2 + 1), the
    // reduction slots
    C *ltw = buf + d.tj * ldr;
    C *ltr = ltw + tw_half(d.fx.n);
    double *red = (double *)(ltr + d.M / 2 + 1);
    TwStage<T, NTH> tws;
    TabStage<T, NTH> trs;
    tws.fetch(d.fx);
    trs.fetch((const C *)d.twr, d.M / 2 + 1);
    const int jt = tile % d.ntj, k = tile / d.ntj;
    const int j0 = jt * d.tj;
    const int rows = min(d.tj, d.ny - j0);
    const int nx = d.nx, nl = d.nl, tj = d.tj, M = d.M, half = M / 2;
    const C *s1 = (const C *)d.s1;
    staged_copy<NTH, 8, C>(
        tj * nl,
        [&](int e) {
            int l = (int)fdiv((uint32_t)e, d.dtj);
            int r = e - l * tj;
            return s1[((size_t)k * nl + l) * d.ny + j0 + min(r, rows - 1)];
        },
        [&](int e, C v) {
            int l = (int)fdiv((uint32_t)e, d.dtj);
            int r = e - l * tj;
            if (r < rows) buf[r * ldr + pidx(l)] = v;
        });
    // accumulate: the old p of this thread's first output pairs is fetched
    // now, so the loads are in flight during the transform (fewer in the
    // 256-thread batch kernel, whose register budget is tighter)
    constexpr int PF = NTH >= 512 ? 8 : 2;
    const int npair = rows * (d.nx >> 1);
    double2 oldv[PF];
    double2 *po2 = (double2 *)(d.po + ((size_t)k * d.ny + j0) * d.nx);
    // one wave per row (see below) when the tile has at most one row per
    // wave and the half length has the fixed wave plan
    constexpr int NW = NTH / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const bool wv = WV && d.tj <= NW && wave_plan(d.fx) && (M >> 6) <= PF;
    if (MODE == XOUT_ACCUM) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            // pair of this thread: (row wid, lane + 64 q) on the wave path
            const int e = wv ? (wid < rows && lane + 64 * q < (M) ? wid * M + lane + 64 * q : npair)
                             : threadIdx.x + q * NTH;
            oldv[q] = e < npair ? po2[e] : double2{0.0, 0.0};
        }
    }
    tws.put(ltw, d.fx);
    trs.put(ltr, (const C *)d.twr, M / 2 + 1);
    __syncthreads();
    const bool wx = d.bcx != BC_PER;
    const double odd = d.bcx == BC_DIR ? -1.0 : 1.0; // Dirichlet x: (-1)^i on the result
    const C *wd = (const C *)d.dctx;
    const C *twr = ltr;
    // inverse DCT-II: half spectrum of the reordered row,
    // V_k = conj(W_{4N}^k) (X_k - i X_{N-k}), X_N = 0, k in [0, M]
    auto dct_pre = [&](C *row, int kk) {
        T xk = row[pidx(kk)].x;
        T xn = kk == 0 ? T(0) : row[pidx(nx - kk)].x;
        row[pidx(kk)] = cmul(cconj(wd[kk]), C{xk, -xn});
    };
    // Z[l] = E + i O,  E = X[l] + conj(X[M-l]),  O = (X[l] - conj(X[M-l])) conj(W^l)
    auto c2r_pre = [&](C *row, int l) {
        if (l == 0) {
            T a = row[0].x, b = row[pidx(M)].x;
            row[0] = C{a + b, a - b};
        } else {
            C xl = row[pidx(l)], xm = row[pidx(M - l)];
            C e = {xl.x + xm.x, xl.y - xm.y};
            C df = {xl.x - xm.x, xl.y + xm.y};
            C o = cmul(df, cconj(twr[l]));
            C io = {-o.y, o.x};
            row[pidx(l)] = cadd(e, io);
            if (2 * l != M) {
                // Z[M-l] = conj(E) + i conj(O)
                C ioc = {o.y, o.x};
                row[pidx(M - l)] = cadd(cconj(e), ioc);
            }
        }
    };
    // accumulation also removes the FP64 volume mean of the previous p: the
    // residual cannot see a constant, so the FP32 gauge error of earlier
    // solves is cancelled here
    const double shift = (MODE == XOUT_ACCUM) ? d.pmean[0] : 0.0;
    double emax = 0.0, pmax = 0.0, psum = 0.0;
    const int hx = nx >> 1;
    // output pairs p[2h], p[2h+1] of row r: complex point h of the
    // half-length FFT, or (wall x) points h and N-1-h of the reordered sequence
    auto value = [&](const C *row, int h) {
        if (!wx) {
            C z = row[pidx(h)];
            return double2{(double)z.x, (double)z.y};
        }
        int n1 = nx - 1 - h;
        return double2{(double)((const T *)(row + pidx(h >> 1)))[h & 1],
                       odd * (double)((const T *)(row + pidx(n1 >> 1)))[n1 & 1]};
    };
    auto emit = [&](int e, double2 val, double2 old) {
        double2 pv = (MODE == XOUT_STORE) ? val : double2{(old.x - shift) + val.x, (old.y - shift) + val.y};
        st_stream(po2 + e, pv);
        psum += pv.x + pv.y;
        emax = amax_nan(amax_nan(emax, val.x), val.y);
        // a stored p is the update itself: its maximum is emax
        if (MODE != XOUT_STORE) pmax = amax_nan(amax_nan(pmax, pv.x), pv.y);
    };
    if (wv) {
        // one wave per row: pre-steps, transform and output of its row
        if (wid < rows) {
            C *row = buf + wid * ldr;
            if (wx) {
                for (int kk = lane; kk <= M; kk += 64) dct_pre(row, kk);
                wave_sync();
            }
            for (int l = lane; l <= half; l += 64) c2r_pre(row, l);
            wave_fft<T, true>(row, ltw, d.fx, lane);
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int h = lane + 64 * q;
                if (h < hx) emit(wid * hx + h, value(row, h), MODE == XOUT_STORE ? double2{0.0, 0.0} : oldv[q]);
            }
        }
    } else {
        if (wx) {
            for (int idx = threadIdx.x; idx < rows * (M + 1); idx += NTH) {
                int r = (int)fdiv((uint32_t)idx, d.dM1);
                dct_pre(buf + r * ldr, idx - r * (M + 1));
            }
            __syncthreads();
        }
        for (int idx = threadIdx.x; idx < rows * (half + 1); idx += NTH) {
            int r = (int)fdiv((uint32_t)idx, d.dH1);
            c2r_pre(buf + r * ldr, idx - r * (half + 1));
        }
        __syncthreads();
        lds_fft<T, true, NTH>(buf, ldr, rows, d.fx, ltw);
        if (MODE == XOUT_STORE) {
            for (int e = threadIdx.x; e < rows * hx; e += NTH) {
                int r = (int)fdiv((uint32_t)e, d.dM);
                emit(e, value(buf + r * ldr, e - r * hx), double2{0.0, 0.0});
            }
        } else {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int e = threadIdx.x + q * NTH;
                if (e < npair) {
                    int r = (int)fdiv((uint32_t)e, d.dM);
                    emit(e, value(buf + r * ldr, e - r * hx), oldv[q]);
                }
            }
            // pairs beyond the prefetched ones (tiles of more than PF x NTH pairs)
            for (int e = threadIdx.x + PF * NTH; e < npair; e += NTH) {
                int r = (int)fdiv((uint32_t)e, d.dM);
                emit(e, value(buf + r * ldr, e - r * hx), po2[e]);
            }
        }
    }
    if (MODE == XOUT_STORE) pmax = emax;
    // per-wave partials, reduced by pass_xmax / pass_pmean (one atomic per
    // statistic per launch, and no workgroup barrier at the end of a tile);
    // the slot of wave wid of this tile (the launch has d.xth threads)
    const int slot = tile * (d.xth >> 6) + wid;
    if (d.ppart) {
        const double ws = wave_sum(psum);
        if (lane == 0) d.ppart[slot] = ws * d.dzf[k];
    }
    if (d.xpart) {
        emax = wave_max1(emax);
        pmax = MODE == XOUT_STORE ? emax : wave_max1(pmax);
        if (lane == 0) {
            d.xpart[2 * slot] = emax;
            d.xpart[2 * slot + 1] = pmax;
        }
    } else {
        block_max2_to<NTH>(d.stats + ST_SOLVE0 + 4 * solve + 1, emax, d.stats + ST_SOLVE0 + 4 * solve + 2, pmax, red);
    }
}

// Maxima of the x-inverse partials into the solve's statistics slots and,
// when the plan tracks the mean of p, their sum: workgroup `wg` of `nwg`
// (nwg <= XMAX_WG) takes every nwg-th block of NT partials, sums them in a
// fixed order and stores the sum in pmean[8 + wg].
__device__ __forceinline__ void pass_xmax(const Dom &d, int solve, int wg, int nwg, char *smem)
{
    double *red = (double *)smem;
    const int nt = xslots(d);
    double a = 0.0, b = 0.0, s = 0.0;
    const double2 *xp = (const double2 *)d.xpart;
    const double *pp = d.ppart ? d.ppart : d.xpart; // a valid address for the unused loads
    for (int q0 = wg * NT; q0 < nt; q0 += 8 * nwg * NT) {
        double2 v[8];
        double w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = min(q0 + u * nwg * NT + (int)threadIdx.x, nt - 1);
            v[u] = xp[q];
            w[u] = pp[q];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (q0 + u * nwg * NT + (int)threadIdx.x >= nt) continue;
            a = (v[u].x != v[u].x || v[u].x > a) ? v[u].x : a;
            b = (v[u].y != v[u].y || v[u].y > b) ? v[u].y : b;
            s += w[u];
        }
    }
    if (d.ppart) {
        const double tot = block_sum(s, red);
        if (threadIdx.x == 0) d.pmean[8 + wg] = tot;
        __syncthreads(); // red is reused below
    }
    block_max2_to<NT>(d.stats + ST_SOLVE0 + 4 * solve + 1, a, d.stats + ST_SOLVE0 + 4 * solve + 2, b, red);
}

// Volume mean of p from the nwg workgroup sums of pass_xmax, added in a
// fixed order by one thread: pmean[0] = sum / (nx ny lz).
__device__ __forceinline__ void pass_pmean(const Dom &d, int nwg)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int w = 0; w < nwg; ++w) s += d.pmean[8 + w];
    d.pmean[0] = s / ((double)d.nx * (double)d.ny * d.lz);
}

} // namespace pcx
