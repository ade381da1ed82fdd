// flow_tile.hpp -- tiling of the one-thread-per-cell stencil launches of
// the substep and of the variable-coefficient projection: 256-thread
// workgroups of 64 x 4 cells of one plane.
//
// The tiles of a grid are split into boxes (ranges of x tiles, y tiles and
// planes): one interior box whose stencils reach no wall, run by a kernel
// instantiated with the branch-free interior accessor only, and up to six
// boxes around it, run by the same kernel instantiated with the general
// accessor.  Kept apart, the interior kernel gets the register budget of its
// own short code (the general accessor's wall cases raised the register
// count and cut occupancy for every tile).  Within a launch consecutive
// workgroups go to different XCDs, so XCD x gets a contiguous range of the
// box's tiles in the order below.
#pragma once

#include <vector>

#include "flow_dev.hpp"

namespace pcx {
namespace flow {

constexpr int FT = 256, FTI = 64, FTJ = FT / FTI;

// tiles [it0, it0 + nit) x [jt0, jt0 + njt) x planes [k0, k0 + nk)
struct TileBox {
    int it0, jt0, k0, nit, njt, nk;
};

__host__ __device__ inline long box_tiles(const TileBox &b) { return (long)b.nit * b.njt * b.nk; }

// workgroups of a launch over a box (a multiple of 8, the XCD count)
inline int box_grid(const TileBox &b)
{
    const long n = box_tiles(b);
    return (int)(((n + 7) >> 3) << 3);
}

// The launches of one grid: box b runs with the interior accessor when
// fast[b]; its workgroups own partial-result slots [slot0[b], slot0[b] +
// box_grid(box[b])); nslots in all.
struct TilePlan {
    int n;
    TileBox box[7];
    bool fast[7];
    int slot0[7];
    int nslots;
    int zlow; // first interior plane with walls in z (tile_plan's argument)
};

// Host tables of a grid's z metrics: dzf (nz), dzc (nz, the periodic wrap
// at nz-1), then the 6 nz reciprocals of FGrid::rz, each computed in the
// order and from the values the device accessors would use.
inline std::vector<double> metric_tables(const double *zf, int nz, bool zper)
{
    std::vector<double> t(8 * (size_t)nz);
    double *dzf = t.data(), *dzc = dzf + nz, *rz = dzc + nz;
    for (int k = 0; k < nz; ++k) dzf[k] = zf[k + 1] - zf[k];
    for (int k = 0; k < nz - 1; ++k) dzc[k] = 0.5 * (dzf[k] + dzf[k + 1]);
    dzc[nz - 1] = 0.5 * (dzf[nz - 1] + dzf[0]);
    auto fat = [&](int k) { return k < 0 ? dzf[zper ? nz - 1 : 0] : (k >= nz ? dzf[zper ? 0 : nz - 1] : dzf[k]); };
    auto cat = [&](int k) {
        if (k < 0) return zper ? dzc[nz - 1] : dzf[0];
        if (k >= nz - 1) return zper ? dzc[nz - 1] : dzf[nz - 1];
        return dzc[k];
    };
    for (int k = 0; k < nz; ++k) {
        double *r = rz + 6 * (size_t)k;
        const double f0 = fat(k), fp = fat(k + 1), cm = cat(k - 1), c0 = cat(k);
        r[0] = 1.0 / f0;
        r[1] = 1.0 / fp;
        r[2] = 1.0 / cm;
        r[3] = 1.0 / c0;
        r[4] = 1.0 / (c0 + cm);
        r[5] = 1.0 / (f0 + fp);
    }
    return t;
}

// Tile boxes of a grid.  The stencils reach one cell (and one face) beyond
// their cell, so a wall direction's interior tiles lie within [1, n-3]: x
// tiles it >= 1 with (it + 1) FTI <= nx - 2, likewise y, planes 1 .. nz-3.
// With zlow = 2 the interior planes start at 2 (wall z; x and y tiles are
// at least 4 cells from a wall anyway): the flux kernel's interior form
// evaluates the normals of its neighbours, whose stencils reach two cells.
inline TilePlan tile_plan(const FGrid &G, int zlow = 1)
{
    const int ti = (G.n[0] + FTI - 1) / FTI, tj = (G.n[1] + FTJ - 1) / FTJ, nz = G.n[2];
    const int it0 = G.per[0] ? 0 : 1, it1 = G.per[0] ? ti : (G.n[0] - 2) / FTI;
    const int jt0 = G.per[1] ? 0 : 1, jt1 = G.per[1] ? tj : (G.n[1] - 2) / FTJ;
    const int k0 = G.per[2] ? 0 : zlow, k1 = G.per[2] ? nz : nz - 2;
    TilePlan p{};
    p.zlow = zlow;
    auto add = [&](TileBox b, bool fast) {
        if (b.nit <= 0 || b.njt <= 0 || b.nk <= 0) return;
        p.box[p.n] = b;
        p.fast[p.n] = fast;
        p.slot0[p.n] = p.nslots;
        p.nslots += box_grid(b);
        ++p.n;
    };
    // the interior kernels' stages wrap a halo index by at most one period
    const bool small = (G.per[0] && G.n[0] < FTI + 2) || (G.per[1] && G.n[1] < FTJ + 2) || (G.per[2] && nz < 3);
    if (small || it1 <= it0 || jt1 <= jt0 || k1 <= k0) {
        add(TileBox{0, 0, 0, ti, tj, nz}, false);
        return p;
    }
    add(TileBox{it0, jt0, k0, it1 - it0, jt1 - jt0, k1 - k0}, true);
    add(TileBox{0, 0, 0, ti, tj, k0}, false);                            // planes below
    add(TileBox{0, 0, k1, ti, tj, nz - k1}, false);                      // planes above
    add(TileBox{0, 0, k0, ti, jt0, k1 - k0}, false);                     // rows south
    add(TileBox{0, jt1, k0, ti, tj - jt1, k1 - k0}, false);              // rows north
    add(TileBox{0, jt0, k0, it0, jt1 - jt0, k1 - k0}, false);            // columns west
    add(TileBox{it1, jt0, k0, ti - it1, jt1 - jt0, k1 - k0}, false);     // columns east
    return p;
}

struct FTile {
    int i, j, k;
    bool act;   // the thread's cell is in the grid
    bool valid; // the workgroup has a tile (uniform over the workgroup)
};

// Order of the tiles within a box: chunks of TKC planes; within a chunk, x
// tiles fastest, then planes, then y tiles.  A tile's z neighbours are then
// nit tiles away in the launch order and its y neighbours nit * TKC tiles
// away, inside the window of workgroups an XCD runs at once, so the planes
// and rows a tile re-reads are still in that XCD's L2 (ordered plane by
// plane, the next plane of the same tile came a whole plane of tiles later
// and every z neighbour was fetched again).
constexpr int TKC = 16;

// tile t (0 <= t < box_tiles(b)) of a box in the order above
__host__ __device__ inline void box_tile(const TileBox &b, long t, int &it, int &jt, int &k)
{
    const long chunk = (long)b.nit * b.njt * TKC;
    const int kc = (int)(t / chunk);
    const int rem = (int)(t - (long)kc * chunk);
    const int kb = kc * TKC;
    const int nkc = b.nk - kb < TKC ? b.nk - kb : TKC; // planes in this chunk
    const int ii = rem % b.nit;
    const int q = rem / b.nit;
    it = b.it0 + ii;
    jt = b.jt0 + q / nkc;
    k = b.k0 + kb + q % nkc;
}

// the thread's cell in the launch over box b (act false past the box or the grid)
__device__ __forceinline__ FTile btile(const FGrid &G, const TileBox &b)
{
    const long n = box_tiles(b);
    const long per = (n + 7) >> 3;
    const long t = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    FTile c;
    c.act = false;
    c.valid = t < n;
    c.i = c.j = c.k = 0;
    if (!c.valid) return c;
    int it, jt;
    box_tile(b, t, it, jt, c.k);
    c.i = it * FTI + (threadIdx.x % FTI);
    c.j = jt * FTJ + (threadIdx.x / FTI);
    c.act = c.i < G.n[0] && c.j < G.n[1];
    return c;
}

// runs body(accessor): the interior accessor in the FAST instantiation, the
// general one otherwise
template <bool FAST, class Body> __device__ __forceinline__ void with_acc(const FGrid &G, const FTile &t, Body body)
{
    if constexpr (FAST) body(Fast(G, t.i, t.j, t.k));
    else body(Gen{G, t.i, t.j, t.k});
}

// register stage of the listed fields: each thread's 3 x 3 x 3 neighbourhood
// (loads whose values no stencil reads are removed by the compiler), all
// issued before the first use; threads past the grid read a clamped cell
template <int N>
__device__ __forceinline__ void stage_regs(const FGrid &G, const FTile &t, const double *const (&src)[N],
                                           double (&rg)[N][27])
{
    const Fast f(G, t.act ? t.i : G.n[0] - 1, t.act ? t.j : G.n[1] - 1, t.k);
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
        for (int n = 0; n < 27; ++n) rg[q][n] = src[q][f.idx(n % 3 - 1, (n / 3) % 3 - 1, n / 9 - 1)];
}

// Launches kernel<true> on the interior box and kernel<false> on the others;
// every kernel takes (box, first slot, args...).
#define FLOW_LAUNCH_PLAN(TP, KERNEL, STREAM, ...)                                                          \
    ([&]() -> hipError_t {                                                                                \
        for (int b_ = 0; b_ < (TP).n; ++b_) {                                                             \
            if ((TP).fast[b_])                                                                            \
                hipLaunchKernelGGL(KERNEL<true>, dim3(box_grid((TP).box[b_])), dim3(FT), 0, (STREAM),     \
                                   (TP).box[b_], (TP).slot0[b_], __VA_ARGS__);                            \
            else                                                                                          \
                hipLaunchKernelGGL(KERNEL<false>, dim3(box_grid((TP).box[b_])), dim3(FT), 0, (STREAM),    \
                                   (TP).box[b_], (TP).slot0[b_], __VA_ARGS__);                            \
            const hipError_t e_ = hipGetLastError();                                                      \
            if (e_ != hipSuccess) return e_;                                                              \
        }                                                                                                 \
        return hipSuccess;                                                                                \
    }())

} // namespace flow
} // namespace pcx
