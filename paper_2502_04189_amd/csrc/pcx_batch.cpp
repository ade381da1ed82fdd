// pcx_batch.cpp -- batched form: many independent domains of uneven size in
// one persistent kernel launch, captured once into a HIP graph.
//
// At create time every domain gets its own tables and workspace, and a
// device work list is built: phase by phase, domains in decreasing size
// (longest first), every tile of a (domain, phase) in a row.  The graph holds
// a reset kernel (queue head, phase counters, reduction slots; no memset
// nodes) followed by the persistent kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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
            pcx_status st = autotune_class(B->grids[i], B->prec, (hipStream_t)stream, tp, rc);
            if (st != PCX_OK) { batch_free(B); return st; }
            cache.store(B->grids[i], B->prec, tp, rc);
        }
        choose_shapes(B->grids[i], B->prec, have || o.autotune ? &tp : nullptr, sh, true);
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
