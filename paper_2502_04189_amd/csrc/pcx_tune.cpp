// pcx_tune.cpp -- per-size-class autotuner.  Each pass family is tuned on
// its own parameters (x passes: rows per tile and the radix split of the
// half-length x FFT; y passes: columns per tile and the y radix split; z
// solve: lanes per line), by timing candidates with HIP events on scratch
// data of the grid's size and keeping the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <sstream>
#include <vector>

#include "pcx_launch.hpp"
#include "pcx_tune.hpp"

namespace pcx {

std::string TuneCache::key(const pcx_grid &g, int prec)
{
    char b[128];
    std::snprintf(b, sizeof(b), "%d %d %d %d %d %d %d", g.nx, g.ny, g.nz, g.bc_x, g.bc_y, g.bc_z, prec);
    return b;
}

bool TuneCache::load(const char *path)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        // "nx ny nz bcx bcy bcz prec : tj tk zg : rx.. : ry.."
        size_t c1 = line.find(':'), c2 = line.find(':', c1 + 1), c3 = line.find(':', c2 + 1);
        if (c1 == std::string::npos || c2 == std::string::npos || c3 == std::string::npos) continue;
        std::string k = line.substr(0, c1);
        while (!k.empty() && k.back() == ' ') k.pop_back();
        TuneParams tp;
        RadixChoice rc;
        std::istringstream a(line.substr(c1 + 1, c2 - c1 - 1)), bx(line.substr(c2 + 1, c3 - c2 - 1)), by(line.substr(c3 + 1));
        a >> tp.tj >> tp.tk >> tp.zg;
        int r;
        while (bx >> r) rc.x.push_back(r);
        while (by >> r) rc.y.push_back(r);
        m[k] = {tp, rc};
    }
    return true;
}

bool TuneCache::save(const char *path) const
{
    std::ofstream f(path);
    if (!f) return false;
    f << "# nx ny nz bcx bcy bcz prec : tj tk zg : x radices : y radices\n";
    for (auto &kv : m) {
        f << kv.first << " : " << kv.second.first.tj << " " << kv.second.first.tk << " " << kv.second.first.zg << " :";
        for (int r : kv.second.second.x) f << " " << r;
        f << " :";
        for (int r : kv.second.second.y) f << " " << r;
        f << "\n";
    }
    return true;
}

bool TuneCache::lookup(const pcx_grid &g, int prec, TuneParams &tp, RadixChoice &rc) const
{
    auto it = m.find(key(g, prec));
    if (it == m.end()) return false;
    tp = it->second.first;
    rc = it->second.second;
    return true;
}

void TuneCache::store(const pcx_grid &g, int prec, const TuneParams &tp, const RadixChoice &rc)
{
    m[key(g, prec)] = {tp, rc};
}

static std::vector<std::vector<int>> radix_variants(int n)
{
    std::vector<std::vector<int>> out;
    out.push_back(default_radices(n));
    int a = 0, b = 0, t = n;
    while (t % 2 == 0) { t /= 2; ++a; }
    while (t % 3 == 0) { t /= 3; ++b; }
    std::vector<int> v4;
    int aa = a;
    while (aa >= 2) { v4.push_back(4); aa -= 2; }
    if (aa == 1) v4.push_back(2);
    for (int i = 0; i < b; ++i) v4.push_back(3);
    std::vector<int> rev = out[0];
    std::reverse(rev.begin(), rev.end());
    for (auto &v : {v4, rev})
        if (std::find(out.begin(), out.end(), v) == out.end()) out.push_back(v);
    return out;
}

namespace {
struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    void *alloc(size_t n)
    {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 256)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
};
} // namespace

pcx_status autotune_class(const pcx_grid &g, int prec, hipStream_t s, TuneParams &best, RadixChoice &brc, bool grouped)
{
    const size_t ncell = (size_t)g.nx * g.ny * g.nz;
    const int M = g.nx / 2;
    const size_t csz = prec == PREC_F64 ? 16 : 8;
    const int nlx = g.bc_x != PCX_BC_PERIODIC ? g.nx : M + 1;
    const size_t nspec = (size_t)nlx * g.ny * g.nz;
    Scratch sc;
    std::vector<double> ones(ncell, 1.0);
    double *fld[9];
    for (int i = 0; i < 9; ++i) {
        fld[i] = (double *)sc.alloc(ncell * 8);
        if (!fld[i]) return fail(PCX_ERR_NOMEM, "autotune scratch allocation failed");
        if (hipMemcpy(fld[i], ones.data(), ncell * 8, hipMemcpyHostToDevice) != hipSuccess)
            return fail(PCX_ERR_HIP, "autotune scratch copy failed");
    }
    void *s1 = sc.alloc(nspec * csz), *s2 = sc.alloc(nspec * csz);
    double *f = (double *)sc.alloc(ncell * 8);
    double *rr = (double *)sc.alloc(ncell * 8);
    unsigned long long *stats = (unsigned long long *)sc.alloc(NSTAT * 8);
    // partial sums of the x inverse: at most one per wave of a 1024-thread
    // workgroup per row, plus the mean
    double *ppart = (double *)sc.alloc(((size_t)g.ny * g.nz * 16 + PMEAN_LEN) * 8);
    if (!s1 || !s2 || !f || !rr || !stats || !ppart) return fail(PCX_ERR_NOMEM, "autotune scratch allocation failed");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(PCX_ERR_HIP, "hipEventCreate");
    // grouped launches (the batch's kernels): a one-entry domain table and an
    // item list of every tile of the pass, as the batch builds them
    Dom *ddom = (Dom *)sc.alloc(sizeof(Dom));
    const size_t max_items = (size_t)std::max<long>({(long)g.ny * g.nz, (long)nlx * g.nz, (long)nlx * g.ny,
                                                     (long)(ncell / 64 + 64)}) + 64;
    GItem *ditems = (GItem *)sc.alloc(max_items * sizeof(GItem));
    if (!ddom || !ditems) return fail(PCX_ERR_NOMEM, "autotune scratch allocation failed");
    std::vector<GItem> hitems;
    // uploads d and the tile list of pass `kind`; returns false when it does not fit
    auto prep_group = [&](const Dom &d, int kind, int smax, GVariant &v, GArgs &a, size_t &lds) {
        const long t = group_tiles(d, kind);
        if (t <= 0 || (size_t)t > max_items) return false;
        hitems.resize(t);
        for (long q = 0; q < t; ++q) hitems[q] = GItem{0u, (uint32_t)(kind == PK_Z ? t - 1 - q : q)};
        if (hipMemcpy(ddom, &d, sizeof(Dom), hipMemcpyHostToDevice) != hipSuccess) return false;
        if (hipMemcpy(ditems, hitems.data(), t * sizeof(GItem), hipMemcpyHostToDevice) != hipSuccess) return false;
        v = variant_of(d, kind, smax);
        a = GArgs{ddom, ditems, (int)t, 0};
        lds = group_lds(d, kind, prec);
        return true;
    };
    // launches of pass kinds k1 (and k2) of d, grouped or single-domain
    auto passes = [&](const Dom &d, int smax, size_t lx, size_t ly, size_t lz, int k1, int k2) {
        std::vector<std::pair<GVariant, std::pair<GArgs, size_t>>> gl;
        if (grouped) {
            // two passes share the item buffer only when they have the same tiles
            for (int k : {k1, k2}) {
                if (k < 0) continue;
                GVariant v; GArgs a; size_t lds;
                if (!prep_group(d, k, smax, v, a, lds)) return std::function<hipError_t()>();
                gl.push_back({v, {a, lds}});
            }
        }
        return std::function<hipError_t()>([=, &d]() {
            hipError_t e = hipSuccess;
            if (grouped) {
                for (auto &x : gl)
                    if (e == hipSuccess) e = launch_group(x.first, prec, x.second.first, group_tiles(d, x.first.kind),
                                                          x.second.second, s);
                return e;
            }
            for (int k : {k1, k2}) {
                if (k < 0 || e != hipSuccess) continue;
                switch (k) {
                case PK_XFWD_RHS: e = launch_xfwd(d, prec, SRC_RHS, lx, s); break;
                case PK_XINV_STORE: e = launch_xinv(d, prec, XOUT_STORE, 0, lx, s); break;
                case PK_YF: e = launch_y(d, prec, false, ly, s); break;
                case PK_YI: e = launch_y(d, prec, true, ly, s); break;
                case PK_Z: e = launch_z(d, prec, smax, lz, s); break;
                default: break;
                }
            }
            return e;
        });
    };

    auto make = [&](const TuneParams &tp, const RadixChoice &rc, Dom &d, DomTables &tb, size_t &lx, size_t &ly, size_t &lz, int &smax) {
        Shapes sh;
        choose_shapes(g, prec, &tp, sh, false);
        pcx_status st = build_domain(g, prec, sh, &rc, tb, d);
        if (st != PCX_OK) return st;
        d.dt = 1e-3; d.rho0 = 1.0; d.irho0 = 1.0;
        d.rho = fld[0]; d.ps = fld[1]; d.u = fld[2]; d.v = fld[3]; d.w = fld[4];
        d.uo = fld[5]; d.vo = fld[6]; d.wo = fld[7]; d.po = fld[8];
        d.f = f; d.r = rr; d.s1 = s1; d.s2 = s2; d.stats = stats;
        d.ppart = prec == PREC_F32 ? ppart : nullptr;
        d.pmean = prec == PREC_F32 ? ppart + (size_t)xslots(d) : nullptr;
        lx = lds_x(d, prec); ly = lds_y(d, prec); lz = lds_z(d, prec); smax = sh.smax;
        return PCX_OK;
    };
    // time fn() (best of 3 after one warm-up)
    auto timeit = [&](auto fn) -> float {
        float bestt = 1e30f;
        if (fn() != hipSuccess) return bestt;
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, s);
            if (fn() != hipSuccess) return 1e30f;
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            bestt = std::min(bestt, t);
        }
        return bestt;
    };
    const long cap = 96 * 1024;
    Shapes base;
    choose_shapes(g, prec, nullptr, base, false);
    best.tj = base.tj; best.tk = base.tk; best.zg = base.zg;
    brc.x = default_radices(M);
    brc.y = default_radices(g.ny);
    // x passes
    {
        float bt = 1e30f;
        for (int tj = 1; tj <= 64; tj *= 2) {
            if ((long)tj * M > MAXPTS || (long)tj * lds_line(nlx) * (long)csz > cap) continue;
            if (tj > 2 * g.ny) continue;
            for (auto &rx : radix_variants(M)) {
                TuneParams tp = best;
                tp.tj = tj;
                RadixChoice rc = brc;
                rc.x = rx;
                Dom d; DomTables tb; size_t lx, ly, lz; int smax;
                if (make(tp, rc, d, tb, lx, ly, lz, smax) != PCX_OK) { if (tb.dev) (void)hipFree(tb.dev); continue; }
                // x forward and inverse have the same tiles, so the item list is shared
                auto fn = passes(d, smax, lx, ly, lz, PK_XFWD_RHS, PK_XINV_STORE);
                float t = fn ? timeit(fn) : 1e30f;
                (void)hipFree(tb.dev);
                if (t < bt) { bt = t; best.tj = tj; brc.x = rx; }
            }
        }
    }
    // y passes
    {
        float bt = 1e30f;
        for (int tk = 1; tk <= 64; tk *= 2) {
            if ((long)tk * g.ny > MAXPTS || (long)tk * lds_line(g.ny) * (long)csz > cap) continue;
            if (tk > 2 * g.nz) continue;
            for (auto &ry : radix_variants(g.ny)) {
                TuneParams tp = best;
                tp.tk = tk;
                RadixChoice rc = brc;
                rc.y = ry;
                Dom d; DomTables tb; size_t lx, ly, lz; int smax;
                if (make(tp, rc, d, tb, lx, ly, lz, smax) != PCX_OK) { if (tb.dev) (void)hipFree(tb.dev); continue; }
                auto fn = passes(d, smax, lx, ly, lz, PK_YF, PK_YI);
                float t = fn ? timeit(fn) : 1e30f;
                (void)hipFree(tb.dev);
                if (t < bt) { bt = t; best.tk = tk; brc.y = ry; }
            }
        }
    }
    // z solve
    {
        float bt = 1e30f;
        for (int G = 1; G <= 64; G *= 2) {
            if (G > std::max(1, g.nz / 2) || (g.nz + G - 1) / G > 16) continue;
            TuneParams tp = best;
            tp.zg = G;
            Dom d; DomTables tb; size_t lx, ly, lz; int smax;
            if (make(tp, brc, d, tb, lx, ly, lz, smax) != PCX_OK) { if (tb.dev) (void)hipFree(tb.dev); continue; }
            auto fn = passes(d, smax, lx, ly, lz, PK_Z, -1);
            float t = fn ? timeit(fn) : 1e30f;
            (void)hipFree(tb.dev);
            if (t < bt) { bt = t; best.zg = G; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
    return PCX_OK;
}

} // namespace pcx
