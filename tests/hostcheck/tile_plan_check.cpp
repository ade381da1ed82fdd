// Host-only check of the substep's tile plan and z-metric tables (no device
// call): for many grids and boundary mixes, every tile of the grid is
// launched exactly once, the interior boxes satisfy the interior accessor's
// conditions, partial-result slots do not overlap, and the metric tables
// hold the reciprocals the general accessor computes.  Prints "ok" or the
// first failure and exits non-zero.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "flow_tile.hpp"

using namespace pcx::flow;

static int fail(const char *what, int nx, int ny, int nz, int px, int py, int pz)
{
    std::printf("FAIL %s: grid %d x %d x %d periodic %d%d%d\n", what, nx, ny, nz, px, py, pz);
    return 1;
}

static int check(int nx, int ny, int nz, int px, int py, int pz, int zlow)
{
    FGrid G{};
    G.n[0] = nx; G.n[1] = ny; G.n[2] = nz;
    G.per[0] = px; G.per[1] = py; G.per[2] = pz;
    const TilePlan p = tile_plan(G, zlow);
    if (p.zlow != zlow) return fail("plan's zlow", nx, ny, nz, px, py, pz);
    const int ti = (nx + FTI - 1) / FTI, tj = (ny + FTJ - 1) / FTJ;
    std::vector<int> seen((size_t)ti * tj * nz, 0);
    int slot = 0;
    for (int b = 0; b < p.n; ++b) {
        const TileBox &x = p.box[b];
        if (p.slot0[b] != slot) return fail("slot ranges", nx, ny, nz, px, py, pz);
        slot += box_grid(x);
        const long n = box_tiles(x);
        if (n <= 0 || box_grid(x) < n || box_grid(x) % 8) return fail("box launch size", nx, ny, nz, px, py, pz);
        for (long t = 0; t < n; ++t) {
            int it, jt, k;
            box_tile(x, t, it, jt, k);
            if (it < x.it0 || it >= x.it0 + x.nit || jt < x.jt0 || jt >= x.jt0 + x.njt || k < x.k0 || k >= x.k0 + x.nk)
                return fail("tile outside its box", nx, ny, nz, px, py, pz);
            if (it < 0 || it >= ti || jt < 0 || jt >= tj || k < 0 || k >= nz)
                return fail("tile outside the grid", nx, ny, nz, px, py, pz);
            ++seen[((size_t)k * tj + jt) * ti + it];
            if (p.fast[b]) {
                const int i0 = it * FTI, j0 = jt * FTJ;
                const bool okx = px ? nx >= FTI + 2 : (i0 >= 1 && i0 + FTI - 1 <= nx - 3);
                const bool oky = py ? ny >= FTJ + 2 : (j0 >= 1 && j0 + FTJ - 1 <= ny - 3);
                const bool okz = pz ? nz >= 3 : (k >= zlow && k <= nz - 3);
                if (!okx || !oky || !okz) return fail("interior tile reaches a wall", nx, ny, nz, px, py, pz);
                // zlow = 2: the normals of the neighbours read cells two steps
                // away, which must exist (wall) or wrap once (periodic)
                if (zlow == 2) {
                    const bool rx = px ? nx >= 2 : (i0 >= 2 && i0 + FTI - 1 <= nx - 3);
                    const bool ry = py ? ny >= 2 : (j0 >= 2 && j0 + FTJ - 1 <= ny - 3);
                    const bool rz = pz ? nz >= 3 : (k >= 2 && k <= nz - 3);
                    if (!rx || !ry || !rz) return fail("interior tile's two-cell reach leaves the grid", nx, ny, nz, px, py, pz);
                }
            }
        }
    }
    if (slot != p.nslots) return fail("slot count", nx, ny, nz, px, py, pz);
    if ((long)p.nslots * FT < (long)nx * ny * nz) return fail("slots cover the cells", nx, ny, nz, px, py, pz);
    for (int v : seen)
        if (v != 1) return fail("tile not launched exactly once", nx, ny, nz, px, py, pz);
    return 0;
}

static int check_metrics(int nz, int pz, unsigned seed)
{
    std::vector<double> zf(nz + 1);
    zf[0] = 0.0;
    for (int k = 0; k < nz; ++k) {
        seed = seed * 1103515245u + 12345u;
        zf[k + 1] = zf[k] + 0.5 + (seed >> 16) / 65536.0;
    }
    const std::vector<double> t = metric_tables(zf.data(), nz, pz);
    const double *dzf = t.data(), *dzc = dzf + nz, *rz = dzc + nz;
    // the general accessor's rules (dzf_at, dzc_at) written out again
    auto fat = [&](int k) { return k < 0 ? (pz ? dzf[nz - 1] : dzf[0]) : (k >= nz ? (pz ? dzf[0] : dzf[nz - 1]) : dzf[k]); };
    auto cat = [&](int k) {
        if (k < 0) return pz ? dzc[nz - 1] : dzf[0];
        if (k >= nz - 1) return pz ? dzc[nz - 1] : dzf[nz - 1];
        return dzc[k];
    };
    for (int k = 0; k < nz; ++k) {
        if (dzf[k] != zf[k + 1] - zf[k]) return 1;
        const double want[6] = {1.0 / fat(k), 1.0 / fat(k + 1), 1.0 / cat(k - 1), 1.0 / cat(k),
                                1.0 / (cat(k) + cat(k - 1)), 1.0 / (fat(k) + fat(k + 1))};
        for (int q = 0; q < 6; ++q)
            if (rz[6 * k + q] != want[q]) {
                std::printf("FAIL metric table k %d entry %d nz %d periodic %d\n", k, q, nz, pz);
                return 1;
            }
    }
    return 0;
}

int main()
{
    const int ns[] = {2, 3, 4, 5, 6, 9, 17, 64, 65, 66, 67, 96, 128, 129, 130, 131, 192, 200};
    long grids = 0;
    for (int nx : ns)
        for (int ny : {2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 18, 33})
            for (int nz : {2, 3, 4, 5, 8, 17, 33})
                for (int m = 0; m < 8; ++m) {
                    for (int zl = 1; zl <= 2; ++zl)
                        if (check(nx, ny, nz, m & 1, (m >> 1) & 1, (m >> 2) & 1, zl)) return 1;
                    ++grids;
                }
    // a large grid (tile counts past a chunk of planes)
    for (int m = 0; m < 8; ++m)
        for (int zl = 1; zl <= 2; ++zl)
            if (check(512, 512, 40, m & 1, (m >> 1) & 1, (m >> 2) & 1, zl)) return 1;
    for (int nz : {2, 3, 5, 64, 129})
        for (int pz = 0; pz < 2; ++pz)
            if (check_metrics(nz, pz, 7u * nz + pz)) return 1;
    std::printf("ok %ld grids\n", grids);
    return 0;
}
