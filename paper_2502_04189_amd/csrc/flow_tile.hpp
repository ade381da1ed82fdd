// flow_tile.hpp -- tiling of the one-thread-per-cell stencil launches of
// the substep and of the variable-coefficient projection: 256-thread
// workgroups of 64 x 4 cells of one plane; consecutive workgroups go to
// different XCDs, so the launch hands XCD x a contiguous range of tiles (its
// planes), and a tile's y and z neighbours are mostly in that XCD's L2.
#pragma once

#include "flow_dev.hpp"

namespace pcx {
namespace flow {

constexpr int FT = 256, FTI = 64, FTJ = FT / FTI;

struct FTile {
    int i, j, k;
    bool act;
    bool fast; // no stencil of the tile reaches a wall (uniform over the workgroup)
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
    // the stencils reach one cell (and one face) beyond the cell: a wall
    // direction needs the tile within [1, n-3]
    const int i0 = it * FTI, j0 = jt * FTJ;
    c.fast = (G.per[0] || (i0 >= 1 && i0 + FTI - 1 <= G.n[0] - 3)) &&
             (G.per[1] || (j0 >= 1 && j0 + FTJ - 1 <= G.n[1] - 3)) && (G.per[2] || (k >= 1 && k <= G.n[2] - 3));
    return c;
}

// runs body(accessor) with the branch-free interior accessor on tiles that
// reach no wall, the general one elsewhere
template <class Body> __device__ __forceinline__ void with_acc(const FGrid &G, const FTile &t, Body body)
{
    if (t.fast) body(Fast(G, t.i, t.j, t.k));
    else body(Gen{G, t.i, t.j, t.k});
}

// workgroups of a one-thread-per-cell tile launch over the grid (a multiple
// of 8, the XCD count)
inline int ngrid(const FGrid &G)
{
    const long nt = (long)((G.n[0] + FTI - 1) / FTI) * ((G.n[1] + FTJ - 1) / FTJ) * G.n[2];
    return (int)(((nt + 7) >> 3) << 3);
}

} // namespace flow
} // namespace pcx
