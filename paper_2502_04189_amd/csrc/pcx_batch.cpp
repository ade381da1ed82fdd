// pcx_batch.cpp -- batched form: many independent domains of uneven size,
// solved by one HIP graph launch.
//
// At create time every domain gets its own tables and workspace.  Two
// schedules of the same pass bodies can be captured into the graph:
//   phased (default): one node per pass of the step, each a grouped launch
//     over the tiles of every domain for that pass (domains largest first),
//     each kernel with its own workgroup size and register budget; with
//     PCX_BATCH_MODE=persistent the same nodes run persistent grids (one
//     workgroup slot per resident workgroup, items taken in a fixed stride);
//   mega (PCX_BATCH_MODE=mega): a single persistent kernel pulling
//     (domain, pass, tile) items from a device queue, with per-domain phase
//     counters for the dependencies.
// The graph starts with a reset kernel (queue head, phase counters,
// reduction slots; no memset nodes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "pcx.h"
#include "pcx_launch.hpp"
#include "pcx_plan.hpp"
#include "pcx_tune.hpp"

using namespace pcx;

struct pcx_batch_s {
    int n = 0;
    int prec = 0;
    int solves = 1;
    pcx_options opt;
    std::vector<pcx_grid> grids;
    std::vector<std::vector<double>> zfs;
    std::vector<double> dts, rho0s;
    std::vector<Dom> doms;
    std::vector<DomTables> tables;
    std::vector<double *> pouts;
    Dom *d_doms = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    Item *items = nullptr;
    int nitems = 0;
    unsigned *ctl = nullptr;        // [0] head, [1] err, [2..] done counters
    unsigned *need = nullptr;
    int nctl = 0;
    unsigned long long *stats = nullptr; // n * NSTAT
    double *psum = nullptr;
    int blocks = 0, smax = 4;
    size_t lds = 0;
    PhaseTab tab;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;     // stream of the last launch (reports run on it)
    int mode = 0;                   // 0 phased, 1 phased persistent, 2 mega
    GItem *gitems = nullptr;        // phased: items of every group, in launch order
    struct Group {
        GVariant v;
        int first, count, grid, solve;
        size_t lds;
    };
    std::vector<Group> groups;
    std::vector<int> smaxs;         // z levels per lane of each domain
};

static void batch_free(pcx_batch B)
{
    if (!B) return;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (auto &t : B->tables)
        if (t.dev) (void)hipFree(t.dev);
    if (B->d_doms) (void)hipFree(B->d_doms);
    if (B->ws) (void)hipFree(B->ws);
    if (B->items) (void)hipFree(B->items);
    if (B->gitems) (void)hipFree(B->gitems);
    if (B->ctl) (void)hipFree(B->ctl);
    if (B->need) (void)hipFree(B->need);
    if (B->stats) (void)hipFree(B->stats);
    if (B->psum) (void)hipFree(B->psum);
    delete B;
}

#define BCHK(x)                                                                                   \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) {                                                                   \
            batch_free(B);                                                                        \
            return fail(PCX_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));             \
        }                                                                                         \
    } while (0)

static long tiles_of(const Dom &d, int kind)
{
    switch (kind) {
    case PK_RHS:
    case PK_RESID: return d.mg[0].ntiles; // pass_rhs, pass_resid walk mg[0]
    case PK_CORR: return d.mg[1].ntiles;  // pass_corr walks mg[1]
    case PK_XFWD_RHS:
    case PK_XFWD_RESID:
    case PK_XINV_STORE:
    case PK_XINV_ACCUM: return (long)d.ntj * d.nz;
    case PK_YF:
    case PK_YI: return (long)d.ntk * d.nl;
    case PK_Z: return d.nzt;
    case PK_PMEAN: return 1;
    default: return d.mg[0].ntiles;
    }
}

// Schedule of the batch, from PCX_BATCH_MODE: "phased" (default),
// "persistent" (phased with persistent grids) or "mega".
static int batch_mode()
{
    const char *m = std::getenv("PCX_BATCH_MODE");
    if (!m) return 0;
    if (!std::strcmp(m, "persistent")) return 1;
    if (!std::strcmp(m, "mega")) return 2;
    return 0;
}

namespace pcx {

// Kernel variant of pass `kind` for domain d (see launch_group).
GVariant variant_of(const Dom &d, int kind, int smax)
{
    GVariant v{kind, NT, 0, 0};
    switch (kind) {
    case PK_RHS: v.nth = march_threads(0); v.two = 5 * (d.mg[0].cti + d.mg[0].ctj) > v.nth; break;
    case PK_RESID: v.nth = march_threads(0); break;
    case PK_CORR: v.nth = march_threads(1); v.two = 7 * (d.mg[1].cti + d.mg[1].ctj) > v.nth; break;
    case PK_XFWD_RHS:
    case PK_XFWD_RESID:
    case PK_XINV_STORE:
    case PK_XINV_ACCUM: v.nth = d.xth; break;
    case PK_YF:
    case PK_YI: v.nth = d.yth; break;
    case PK_Z: v.smax = smax; break;
    case PK_PMEAN: v.nth = 64; break;
    default: break;
    }
    return v;
}

long group_tiles(const Dom &d, int kind)
{
    switch (kind) {
    case PK_XMAX: return xmax_wgs(d);
    case PK_PMEAN: return 1;
    default: return ::tiles_of(d, kind);
    }
}

size_t group_lds(const Dom &d, int kind, int prec)
{
    switch (kind) {
    case PK_XFWD_RHS:
    case PK_XFWD_RESID:
    case PK_XINV_STORE:
    case PK_XINV_ACCUM: return lds_x(d, prec);
    case PK_YF:
    case PK_YI: return lds_y(d, prec);
    case PK_Z: return lds_z(d, prec);
    default: return 0;
    }
}

} // namespace pcx

// Phased schedule: one grouped launch per (pass, kernel variant), in the
// order of the single-domain step, captured into the graph after the reset
// of the reduction slots.  Within a launch the domains come largest first;
// the stencil passes hand each XCD a contiguous range of tiles (consecutive
// workgroups go to different XCDs), so tiles adjacent in a domain share an
// L2 for their halos, as in the single-domain launches.
static pcx_status build_phased(pcx_batch B)
{
    const int n = B->n;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    auto cells = [&](int i) { return (long)B->grids[i].nx * B->grids[i].ny * B->grids[i].nz; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cells(a) > cells(b); });
    struct Ph {
        int kind, solve;
    };
    std::vector<Ph> phs;
    const bool ref = B->prec == PREC_F32;
    phs.push_back({PK_RHS, 0});
    phs.push_back({PK_XFWD_RHS, 0});
    for (int k : {PK_YF, PK_Z, PK_YI, PK_XINV_STORE, PK_XMAX}) phs.push_back({k, 0});
    if (ref) phs.push_back({PK_PMEAN, 0});
    for (int sv = 1; sv < B->solves; ++sv)
        for (int k : {PK_RESID, PK_XFWD_RESID, PK_YF, PK_Z, PK_YI, PK_XINV_ACCUM, PK_XMAX, PK_PMEAN})
            phs.push_back({k, sv});
    phs.push_back({PK_CORR, 0});

    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(PCX_ERR_HIP, "hipGetDeviceProperties failed");
    std::vector<GItem> all;
    for (const Ph &ph : phs) {
        // domains of each kernel variant, in first-appearance order
        std::vector<std::pair<GVariant, std::vector<int>>> grp;
        for (int i : order) {
            const GVariant v = variant_of(B->doms[i], ph.kind, B->smaxs[i]);
            auto it = std::find_if(grp.begin(), grp.end(), [&](const std::pair<GVariant, std::vector<int>> &g) {
                return g.first.nth == v.nth && g.first.two == v.two && g.first.smax == v.smax;
            });
            if (it == grp.end()) grp.push_back({v, {i}});
            else it->second.push_back(i);
        }
        for (auto &g : grp) {
            std::vector<GItem> lst;
            size_t lds = 0;
            for (int i : g.second) {
                const Dom &d = B->doms[i];
                const long t = group_tiles(d, ph.kind);
                for (long q = 0; q < t; ++q)
                    lst.push_back(GItem{(uint32_t)i, (uint32_t)(ph.kind == PK_Z ? t - 1 - q : q)});
                lds = std::max(lds, group_lds(d, ph.kind, B->prec));
            }
            const bool stencil = ph.kind == PK_RHS || ph.kind == PK_RESID || ph.kind == PK_CORR;
            if (stencil) {
                const size_t cnt = lst.size(), per = (cnt + 7) / 8;
                std::vector<GItem> perm(8 * per, GItem{GSKIP, 0});
                for (size_t b = 0; b < 8 * per; ++b) {
                    const size_t L = (b & 7) * per + (b >> 3);
                    if (L < cnt) perm[b] = lst[L];
                }
                lst.swap(perm);
            }
            int grid = (int)lst.size();
            if (B->mode == 1) {
                int per_cu = 0;
                if (group_occupancy(g.first, B->prec, lds, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
                long cap = std::max(8L, ((long)prop.multiProcessorCount * per_cu) & ~7L);
                grid = (int)std::min<long>(grid, cap);
            }
            B->groups.push_back({g.first, (int)all.size(), (int)lst.size(), grid, ph.solve, lds});
            all.insert(all.end(), lst.begin(), lst.end());
        }
    }
    if (hipMalloc(&B->gitems, std::max<size_t>(all.size(), 1) * sizeof(GItem)) != hipSuccess)
        return fail(PCX_ERR_NOMEM, "batch item list allocation failed");
    if (hipMemcpy(B->gitems, all.data(), all.size() * sizeof(GItem), hipMemcpyHostToDevice) != hipSuccess)
        return fail(PCX_ERR_HIP, "batch item list copy failed");
    B->nctl = 2;
    if (hipMalloc(&B->ctl, (size_t)B->nctl * sizeof(unsigned)) != hipSuccess)
        return fail(PCX_ERR_NOMEM, "batch control allocation failed");

    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(PCX_ERR_HIP, "stream create");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_reset(B->ctl, B->nctl, cs);
    if (e == hipSuccess) e = launch_reset((unsigned *)B->stats, n * NSTAT * 2, cs);
    for (const auto &g : B->groups) {
        if (e != hipSuccess) break;
        GArgs a{B->d_doms, B->gitems + g.first, g.count, g.solve};
        e = launch_group(g.v, B->prec, a, g.grid, g.lds, cs);
    }
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &gr);
    if (e == hipSuccess) e = e2;
    B->graph = gr;
    if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    return PCX_OK;
}

extern "C" pcx_status pcx_batch_create(const pcx_domain *domains, int32_t n, const pcx_options *opts, void *stream,
                                       pcx_batch *out)
{
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!domains || n <= 0 || n > 65535) return fail(PCX_ERR_INVALID, "need 1..65535 domains");
    pcx_options o = {PCX_FP32_REFINED, 1e-10, 8, 0, 0, 0, nullptr};
    if (opts) o = *opts;
    if (o.precision != PCX_FP64 && o.precision != PCX_FP32_REFINED) return fail(PCX_ERR_INVALID, "unknown precision");
    if (!(o.rtol > 0.0)) o.rtol = 1e-10;
    if (o.max_iters <= 0) o.max_iters = 8;
    if (o.max_iters > MAXIT) o.max_iters = MAXIT;
    if (o.fixed_iters <= 0) o.fixed_iters = 3;
    if (o.fixed_iters > o.max_iters) o.fixed_iters = o.max_iters;
    for (int i = 0; i < n; ++i) {
        const pcx_domain &dm = domains[i];
        pcx_status st = validate_grid(&dm.grid);
        if (st != PCX_OK) return fail(st, "domain " + std::to_string(i) + ": " + g_err);
        if (dm.grid.bc_x == PCX_BC_DIRICHLET || dm.grid.bc_y == PCX_BC_DIRICHLET || dm.grid.bc_z == PCX_BC_DIRICHLET)
            return fail(PCX_ERR_UNSUPPORTED, "domain " + std::to_string(i) + ": Dirichlet boundaries are for pcx_poisson_solve");
        if (!(dm.dt > 0.0) || !(dm.rho0 > 0.0)) return fail(PCX_ERR_INVALID, "domain " + std::to_string(i) + ": dt, rho0 must be > 0");
        const void *f[] = {dm.rho, dm.p_star, dm.u, dm.v, dm.w, dm.u_out, dm.v_out, dm.w_out, dm.p_out};
        for (const void *q : f)
            if (!q) return fail(PCX_ERR_INVALID, "domain " + std::to_string(i) + ": NULL field pointer");
        const void *ins[] = {dm.rho, dm.p_star, dm.u, dm.v, dm.w};
        for (const void *q : ins)
            if (q == dm.u_out || q == dm.v_out || q == dm.w_out || q == dm.p_out)
                return fail(PCX_ERR_INVALID, "domain " + std::to_string(i) + ": outputs must not alias inputs in a batch");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PCX_ERR_HIP, "no HIP device available");

    pcx_batch B = new pcx_batch_s();
    B->n = n;
    B->opt = o;
    B->prec = o.precision == PCX_FP64 ? PREC_F64 : PREC_F32;
    B->solves = B->prec == PREC_F64 ? 1 : o.fixed_iters;
    B->grids.resize(n);
    B->zfs.resize(n);
    B->doms.resize(n);
    B->tables.resize(n);
    B->dts.resize(n);
    B->rho0s.resize(n);
    B->pouts.resize(n);
    TuneCache cache;
    if (o.tune_cache) cache.load(o.tune_cache);
    B->mode = batch_mode();
    B->smaxs.assign(n, 4);

    // phases
    PhaseTab &tab = B->tab;
    std::memset(&tab, 0, sizeof(tab));
    bool ph_over = false;
    auto addph = [&](int kind, int solve) {
        if (tab.nphase >= MAXPH) { ph_over = true; return; }
        tab.kind[tab.nphase] = (uint8_t)kind; tab.solve[tab.nphase] = (uint8_t)solve; tab.nphase++;
    };
    addph(PK_RHS, 0);
    addph(PK_XFWD_RHS, 0);
    addph(PK_YF, 0); addph(PK_Z, 0); addph(PK_YI, 0); addph(PK_XINV_STORE, 0);
    // after every x-inverse phase: the maxima of its wave partials (and, refined, the
    // volume mean of p), one workgroup per domain
    addph(PK_PMEAN, 0);
    for (int s = 1; s < B->solves; ++s) {
        addph(PK_RESID, s);
        addph(PK_XFWD_RESID, s);
        addph(PK_YF, s); addph(PK_Z, s); addph(PK_YI, s); addph(PK_XINV_ACCUM, s);
        addph(PK_PMEAN, s);
    }
    addph(PK_CORR, 0);
    if (ph_over) { batch_free(B); return fail(PCX_ERR_UNSUPPORTED, "too many solves for the batch phase table"); }

    // per-domain tables, shapes and workspace layout
    const size_t csz = B->prec == PREC_F64 ? 16 : 8;
    std::vector<size_t> off_s1(n), off_s2(n), off_f(n), off_r(n), off_pp(n), off_xp(n);
    size_t total = 0;
    auto take = [&](size_t bytes) { size_t o2 = (total + 255) & ~(size_t)255; total = o2 + bytes; return o2; };
    for (int i = 0; i < n; ++i) {
        B->zfs[i].assign(domains[i].grid.zf, domains[i].grid.zf + domains[i].grid.nz + 1);
        B->grids[i] = domains[i].grid;
        B->grids[i].zf = B->zfs[i].data();
        Shapes sh;
        TuneParams tp;
        RadixChoice rc;
        bool have = cache.lookup(B->grids[i], B->prec, tp, rc);
        if (!have && o.autotune) {
            pcx_status st = autotune_class(B->grids[i], B->prec, (hipStream_t)stream, tp, rc, B->mode != 2);
            if (st != PCX_OK) { batch_free(B); return st; }
            cache.store(B->grids[i], B->prec, tp, rc);
        }
        // the phased schedule runs the single-domain pass shapes; the mega
        // kernel runs every pass in NT-thread workgroups
        choose_shapes(B->grids[i], B->prec, have || o.autotune ? &tp : nullptr, sh, B->mode == 2);
        B->smaxs[i] = sh.smax;
        pcx_status st = build_domain(B->grids[i], B->prec, sh, have || o.autotune ? &rc : nullptr, B->tables[i], B->doms[i]);
        if (st != PCX_OK) { batch_free(B); return st; }
        B->smax = std::max(B->smax, sh.smax);
        B->lds = std::max({B->lds, lds_x(B->doms[i], B->prec), lds_y(B->doms[i], B->prec), lds_z(B->doms[i], B->prec),
                           (size_t)(16 + 7 * NT) * sizeof(double)});
        const size_t nspec = (size_t)B->doms[i].nl * B->grids[i].ny * B->grids[i].nz;
        const size_t ncell = (size_t)B->grids[i].nx * B->grids[i].ny * B->grids[i].nz;
        off_s1[i] = take(nspec * csz);
        off_s2[i] = take(nspec * csz);
        off_f[i] = take(ncell * 8);
        off_r[i] = B->prec == PREC_F32 ? take(ncell * 8) : 0;
        off_pp[i] = B->prec == PREC_F32 ? take(((size_t)xslots(B->doms[i]) + PMEAN_LEN) * 8) : 0;
        off_xp[i] = take((size_t)2 * xslots(B->doms[i]) * 8);
    }
    if (o.tune_cache && o.autotune) cache.save(o.tune_cache);
    if (hipMalloc(&B->ws, std::max<size_t>(total, 256)) != hipSuccess) { batch_free(B); return fail(PCX_ERR_NOMEM, "batch workspace allocation failed"); }
    B->ws_bytes = total;
    BCHK(hipMalloc(&B->stats, (size_t)n * NSTAT * sizeof(unsigned long long)));
    size_t maxnz = 0;
    for (int i = 0; i < n; ++i) maxnz = std::max(maxnz, (size_t)B->grids[i].nz);
    BCHK(hipMalloc(&B->psum, maxnz * sizeof(double)));
    for (int i = 0; i < n; ++i) {
        Dom &d = B->doms[i];
        const pcx_domain &dm = domains[i];
        d.s1 = (char *)B->ws + off_s1[i];
        d.s2 = (char *)B->ws + off_s2[i];
        d.f = (double *)((char *)B->ws + off_f[i]);
        d.r = B->prec == PREC_F32 ? (double *)((char *)B->ws + off_r[i]) : nullptr;
        d.ppart = B->prec == PREC_F32 ? (double *)((char *)B->ws + off_pp[i]) : nullptr;
        d.pmean = d.ppart ? d.ppart + (size_t)xslots(d) : nullptr;
        d.xpart = (double *)((char *)B->ws + off_xp[i]);
        d.stats = B->stats + (size_t)i * NSTAT;
        d.dt = dm.dt; d.rho0 = dm.rho0; d.irho0 = 1.0 / dm.rho0;
        d.rho = dm.rho; d.ps = dm.p_star; d.u = dm.u; d.v = dm.v; d.w = dm.w;
        d.uo = dm.u_out; d.vo = dm.v_out; d.wo = dm.w_out; d.po = dm.p_out;
        B->dts[i] = dm.dt; B->rho0s[i] = dm.rho0; B->pouts[i] = dm.p_out;
    }
    BCHK(hipMalloc(&B->d_doms, (size_t)n * sizeof(Dom)));
    BCHK(hipMemcpy(B->d_doms, B->doms.data(), (size_t)n * sizeof(Dom), hipMemcpyHostToDevice));
    if (B->mode != 2) {
        pcx_status st = build_phased(B);
        if (st != PCX_OK) { batch_free(B); return st; }
        *out = B;
        return PCX_OK;
    }

    // work list: phase-major, largest domains first within a phase
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long)B->grids[a].nx * B->grids[a].ny * B->grids[a].nz > (long)B->grids[b].nx * B->grids[b].ny * B->grids[b].nz;
    });
    // items: runs of consecutive tiles of one (domain, phase), sized to about
    // 256 KB of HBM traffic so that the per-item queue and fence cost stays
    // small next to the work
    std::vector<Item> items;
    std::vector<unsigned> need((size_t)n * tab.nphase);
    const size_t target = 256 * 1024;
    for (int p = 0; p < tab.nphase; ++p)
        for (int i : order) {
            const Dom &d = B->doms[i];
            const long t = tiles_of(d, tab.kind[p]);
            const size_t sp = (size_t)d.nl * d.ny * d.nz * csz;
            const size_t cells = (size_t)d.nx * d.ny * d.nz;
            size_t bytes = 0;
            switch (tab.kind[p]) {
            case PK_RHS: bytes = 48 * cells; break;
            case PK_RESID: bytes = 24 * cells; break;
            case PK_CORR: bytes = 72 * cells; break;
            case PK_XINV_ACCUM: bytes = sp + 16 * cells; break;
            case PK_PMEAN: bytes = 0; break;
            case PK_XFWD_RHS:
            case PK_XFWD_RESID:
            case PK_XINV_STORE: bytes = sp + 8 * cells; break;
            default: bytes = 2 * sp; break;
            }
            const size_t per_tile = std::max<size_t>(1, bytes / (size_t)t);
            const long g = std::max(1L, std::min(t, (long)(target / per_tile)));
            long cnt = 0;
            for (long k = 0; k < t; k += g, ++cnt)
                items.push_back(Item{(uint16_t)i, (uint16_t)p, (uint32_t)k, (uint32_t)std::min(g, t - k), 0u});
            need[(size_t)i * tab.nphase + p] = (unsigned)cnt;
        }
    B->nitems = (int)items.size();
    BCHK(hipMalloc(&B->items, items.size() * sizeof(Item)));
    BCHK(hipMemcpy(B->items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
    BCHK(hipMalloc(&B->need, need.size() * sizeof(unsigned)));
    BCHK(hipMemcpy(B->need, need.data(), need.size() * sizeof(unsigned), hipMemcpyHostToDevice));
    B->nctl = 2 + n * tab.nphase;
    BCHK(hipMalloc(&B->ctl, (size_t)B->nctl * sizeof(unsigned)));

    // persistent grid: every resident workgroup slot of the device
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    BCHK(hipGetDevice(&dev));
    BCHK(hipGetDeviceProperties(&prop, dev));
    BCHK(persist_occupancy(B->prec, B->smax, B->lds, &per_cu));
    if (per_cu < 1) per_cu = 1;
    B->blocks = std::min((long)prop.multiProcessorCount * per_cu, (long)B->nitems);

    // capture: reset kernels then the persistent kernel
    hipStream_t cs = nullptr;
    BCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    PersistArgs a;
    a.doms = B->d_doms;
    a.items = B->items;
    a.nitems = B->nitems;
    a.head = B->ctl;
    a.err = B->ctl + 1;
    a.done = B->ctl + 2;
    a.need = B->need;
    a.spin_limit = 1u << 20;
    a.tab = tab;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_reset(B->ctl, B->nctl, cs);
    if (e == hipSuccess) e = launch_reset((unsigned *)B->stats, n * NSTAT * 2, cs);
    if (e == hipSuccess) e = launch_persist(a, B->prec, B->smax, B->blocks, B->lds, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    B->graph = g;
    if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        batch_free(B);
        return fail(PCX_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = B;
    return PCX_OK;
}

extern "C" pcx_status pcx_batch_launch(pcx_batch B, void *stream)
{
    if (!B) return fail(PCX_ERR_INVALID, "batch is NULL");
    hipError_t e = hipGraphLaunch(B->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    B->last = (hipStream_t)stream;
    return PCX_OK;
}

extern "C" pcx_status pcx_batch_reports(pcx_batch B, pcx_report *out_n)
{
    if (!B || !out_n) return fail(PCX_ERR_INVALID, "NULL argument");
    // everything runs on the stream of the last launch, in its order
    const hipStream_t s = B->last;
    std::vector<unsigned long long> h((size_t)B->n * NSTAT);
    unsigned err = 0;
    hipError_t e = hipMemcpyAsync(h.data(), B->stats, h.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&err, B->ctl + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("batch stats: ") + hipGetErrorString(e));
    bool all_conv = true;
    for (int i = 0; i < B->n; ++i) {
        const pcx_grid &g = B->grids[i];
        auto sd = [&](int k) { double v; std::memcpy(&v, &h[(size_t)i * NSTAT + k], 8); return v; };
        e = launch_plane_sums(B->pouts[i], g.nx * g.ny, g.nz, B->psum, s);
        std::vector<double> ps(g.nz);
        if (e == hipSuccess) e = hipMemcpyAsync(ps.data(), B->psum, g.nz * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("plane sums: ") + hipGetErrorString(e));
        double num = 0.0, lz = g.zf[g.nz] - g.zf[0];
        for (int k = 0; k < g.nz; ++k) num += (g.zf[k + 1] - g.zf[k]) * ps[k];
        pcx_report &r = out_n[i];
        std::memset(&r, 0, sizeof(r));
        r.solves = B->solves;
        r.f_inf = sd(ST_FINF);
        r.max_div_abs = sd(ST_DIV);
        r.rel_residual = r.max_div_abs / ((B->dts[i] / B->rho0s[i]) * r.f_inf);
        r.max_div_rel = r.rel_residual;
        r.mean_p = num / ((double)g.nx * g.ny * lz);
        r.last_update_inf = sd(ST_SOLVE0 + 4 * (B->solves - 1) + 1);
        double eprev = B->solves >= 2 ? sd(ST_SOLVE0 + 4 * (B->solves - 2) + 1) : 0.0;
        double pinf = sd(ST_SOLVE0 + 4 * (B->solves - 1) + 2);
        r.converged = B->prec == PREC_F64 ? (r.rel_residual <= B->opt.rtol)
                                          : pcx_refine_should_stop(r.rel_residual, r.last_update_inf, eprev, pinf, B->opt.rtol);
        all_conv = all_conv && r.converged;
    }
    if (err) return fail(PCX_ERR_HIP, "a dependency wait of the persistent kernel timed out");
    if (!all_conv) return fail(PCX_ERR_NOT_CONVERGED, "some domains missed rtol with the fixed number of solves");
    return PCX_OK;
}

extern "C" pcx_status pcx_batch_destroy(pcx_batch B)
{
    batch_free(B);
    return PCX_OK;
}
