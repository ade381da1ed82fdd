// pcx_host.cpp -- host runtime behind the C ABI: validation, tables
// (eigenvalues, z coefficients, twiddles), workspace, pass sequencing, the
// refinement loop and reports.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pcx.h"
#include "pcx_launch.hpp"
#include "pcx_plan.hpp"
#include "pcx_tune.hpp"

namespace pcx {

thread_local std::string g_err;

pcx_status fail(pcx_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

static bool is_2a3b(int n)
{
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

FastDiv mkdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    f.m = d <= 1 ? 0u : (uint32_t)((0x100000000ull / d) + 1ull);
    return f;
}

std::vector<int> default_radices(int n)
{
    // 256 as four radix-4 stages: the wave-level FFT then has one butterfly
    // on every lane in every stage (8.8.4 leaves half the lanes idle in the
    // radix-8 stages)
    if (n == 256) return {4, 4, 4, 4};
    std::vector<int> r;
    int a = 0, b = 0;
    while (n % 2 == 0) { n /= 2; ++a; }
    while (n % 3 == 0) { n /= 3; ++b; }
    while (a >= 3) { r.push_back(8); a -= 3; }
    if (a == 2) r.push_back(4);
    else if (a == 1) r.push_back(2);
    for (int i = 0; i < b; ++i) r.push_back(3);
    return r;
}

void fill_fft(FftDesc &fd, int n, const std::vector<int> &rad)
{
    std::memset(&fd, 0, sizeof(fd));
    fd.n = n;
    fd.nst = (int)rad.size();
    int ns = 1;
    for (int s = 0; s < fd.nst; ++s) {
        int R = rad[s];
        fd.rad[s] = R;
        fd.ns[s] = ns;
        fd.tws[s] = n / (ns * R);
        fd.dnb[s] = mkdiv((uint32_t)(n / R));
        fd.dns[s] = mkdiv((uint32_t)ns);
        ns *= R;
    }
}

// ---------------------------------------------------------------- tables
struct Blob {
    std::vector<char> bytes;
    size_t add(const void *p, size_t n)
    {
        size_t off = (bytes.size() + 255) & ~(size_t)255;
        bytes.resize(off + n);
        if (n) std::memcpy(bytes.data() + off, p, n);
        return off;
    }
};

template <typename T> static std::vector<T> cast_vec(const std::vector<long double> &v)
{
    std::vector<T> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
    return o;
}

template <typename T> static std::vector<T> roots(int n, bool extra)
{
    // exp(-2 pi i e / n), e in [0, n) (+1 entry when extra), two T per entry
    int cnt = n + (extra ? 1 : 0);
    std::vector<T> o(2 * (size_t)cnt);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int e = 0; e < cnt; ++e) {
        long double a = 2.0L * pi * (long double)e / (long double)n;
        o[2 * e] = (T)cosl(a);
        o[2 * e + 1] = (T)(-sinl(a));
    }
    return o;
}

pcx_status validate_grid(const pcx_grid *g)
{
    if (!g) return fail(PCX_ERR_INVALID, "grid is NULL");
    if (!g->zf) return fail(PCX_ERR_INVALID, "grid.zf is NULL");
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return fail(PCX_ERR_INVALID, "nx, ny, nz must be >= 2");
    if (!(g->lx > 0.0) || !(g->ly > 0.0)) return fail(PCX_ERR_INVALID, "lx and ly must be > 0");
    for (int b : {g->bc_x, g->bc_y, g->bc_z})
        if (b != PCX_BC_PERIODIC && b != PCX_BC_WALL && b != PCX_BC_DIRICHLET)
            return fail(PCX_ERR_INVALID, "unknown boundary condition");
    if (g->nx % 2) return fail(PCX_ERR_INVALID, "nx must be even");
    if (g->bc_y == PCX_BC_PERIODIC && (g->ny % 2)) return fail(PCX_ERR_INVALID, "ny must be even in a periodic direction");
    for (int k = 0; k < g->nz; ++k)
        if (!(g->zf[k + 1] > g->zf[k])) return fail(PCX_ERR_INVALID, "zf must be strictly increasing");
    if (!is_2a3b(g->nx) || !is_2a3b(g->ny) || g->nx > 4096 || g->ny > 4096)
        return fail(PCX_ERR_UNSUPPORTED, "transform lengths must be 2^a 3^b and at most 4096");
    if (g->nz > 1024) return fail(PCX_ERR_UNSUPPORTED, "nz above 1024 is not supported");
    // cell offsets inside the kernels are 32-bit: nx ny nz (which bounds the
    // spectral count nl ny nz as well, nl <= nx) must fit in int32
    if ((int64_t)g->nx * g->ny * g->nz > (int64_t)INT32_MAX)
        return fail(PCX_ERR_UNSUPPORTED, "grids of more than 2^31 - 1 cells are not supported");
    return PCX_OK;
}

static int pow2_floor(long v)
{
    int p = 1;
    while ((long)p * 2 <= v) p *= 2;
    return p;
}

// Tile shapes: rows per x tile, columns per y tile (with the y workgroup
// size), z lanes per line, marching workgroup size.  Corner-turn segments are
// kept at 128 bytes (8 FP64 or 16 FP32 complex values).  The batched form runs
// every pass in 256-thread workgroups.
void choose_shapes(const pcx_grid &g, int prec, const TuneParams *tp, Shapes &sh, bool batch)
{
    const int M = g.nx / 2;
    const size_t csz = prec == PREC_F64 ? 16 : 8;
    const long lds_cap = 80 * 1024;
    const int seg = prec == PREC_F64 ? 8 : 16;
    const int nlx = g.bc_x != PCX_BC_PERIODIC ? g.nx : M + 1;
    int tj = pow2_floor(std::max(1, MAXPTS / std::max(M, 1)));
    tj = std::min(tj, pow2_floor(lds_cap / (long)(lds_line(nlx) * csz)));
    tj = std::min(tj, seg);
    int tk = pow2_floor(std::max(1, MAXPTS / g.ny));
    tk = std::min(tk, pow2_floor(lds_cap / (long)(lds_line(g.ny) * csz)));
    tk = std::min(tk, seg);
    int G = std::min(64, pow2_floor(std::max(1, g.nz / 2)));
    if (tp) {
        if (tp->tj > 0) tj = tp->tj;
        if (tp->tk > 0) tk = tp->tk;
        if (tp->zg > 0) G = tp->zg;
    }
    // a tile never holds more than MAXPTS points (register staging of the
    // pipelined passes assumes it), whatever a tune cache says
    while (tj > 1 && (long)tj * std::max(M, 1) > MAXPTS) tj >>= 1;
    while (tk > 1 && (long)tk * g.ny > MAXPTS) tk >>= 1;
    sh.tj = std::max(1, tj);
    sh.tk = std::max(1, tk);
    sh.zg = G;
    int smax_need = (g.nz + G - 1) / G;
    sh.smax = smax_need <= 4 ? 4 : (smax_need <= 8 ? 8 : 16);
    sh.mth = batch ? NT : 512;
    sh.mthc = batch ? NT : 1024;
    // wider y workgroups when a tile holds many columns: more waves per CU
    // 512-thread y workgroups when a tile holds many columns (more waves per
    // CU), and when its columns fit one per wave on the wave-level FFT path
    sh.yth = (!batch && ((long)sh.tk * (lds_line(g.ny) * (long)csz) > 48 * 1024 ||
                         (wave_len(g.ny) && sh.tk > NT / 64 && sh.tk <= 8)))
                 ? 512
                 : NT;
    sh.xth = batch ? NT : 512;
    sh.batch = batch;
}

// Domain descriptor and the host image of its device tables (eigenvalues, z
// coefficients, twiddles); the table pointers of d are bound by bind_tables
// once the image sits in device memory.
void make_domain(const pcx_grid &g, int prec, const Shapes &sh, const RadixChoice *rc, HostTables &ht, Dom &d)
{
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int M = nx / 2;
    // x modes: half spectrum of a real FFT (periodic) or nx cosine modes (wall)
    const int nl = g.bc_x != PCX_BC_PERIODIC ? nx : M + 1;
    std::memset(&d, 0, sizeof(d));
    d.nx = nx; d.ny = ny; d.nz = nz; d.nl = nl; d.M = M;
    d.bcx = g.bc_x; d.bcy = g.bc_y; d.bcz = g.bc_z;
    d.nosing = g.bc_x == PCX_BC_DIRICHLET || g.bc_y == PCX_BC_DIRICHLET || g.bc_z == PCX_BC_DIRICHLET;
    d.tj = sh.tj; d.ntj = (ny + sh.tj - 1) / sh.tj;
    d.tk = sh.tk; d.ntk = (nz + sh.tk - 1) / sh.tk;
    d.zg = sh.zg; d.zlpw = (NT / 64) * (64 / sh.zg);
    long nlines = (long)nl * ny;
    d.nzt = (int)((nlines + d.zlpw - 1) / d.zlpw);
    d.ndiv_tiles = (int)(((long)nx * ny * nz + NT - 1) / NT);
    // marching stencils: TI x TJ cell tiles over chunks of ckc planes
    d.mth = sh.mth;
    // marching tiles: [0] RHS and residual with sh.mth threads, [1] the
    // correction with sh.mthc threads; each halo (7 (TI + TJ) items at most)
    // fits two items per thread
    for (int q = 0; q < 2; ++q) {
        MGeo &m = d.mg[q];
        const int th = q == 0 ? sh.mth : sh.mthc;
        m.cti = std::min(nx, 64);
        m.ctj = std::max(1, std::min({ny, th / m.cti, 2 * th / 7 - m.cti}));
        m.cnti = (nx + m.cti - 1) / m.cti;
        m.cntj = (ny + m.ctj - 1) / m.ctj;
        if (sh.batch) {
            m.ckc = nz; // whole columns: batch items stay large
        } else {
            long txy = (long)m.cnti * m.cntj;
            long target = 2048L * 512 / th;
            long chunks = std::max(1L, std::min((long)std::max(1, nz / 16), (target + txy - 1) / txy));
            m.ckc = (int)((nz + chunks - 1) / chunks);
        }
        m.cnk = (nz + m.ckc - 1) / m.ckc;
        m.ntiles = m.cnti * m.cntj * m.cnk;
        m.dcti = mkdiv(m.cti);
    }
    d.yth = sh.yth;
    d.xth = sh.xth;
    d.dnx = mkdiv(nx); d.dny = mkdiv(ny); d.dtj = mkdiv(sh.tj); d.dtk = mkdiv(sh.tk); d.dnyc = mkdiv(ny);
    d.dM = mkdiv(M);
    d.dH1 = mkdiv(M / 2 + 1);
    d.dM1 = mkdiv(M + 1);
    d.dhy = mkdiv(std::max(1, ny / 2));
    d.dx = g.lx / nx; d.dy = g.ly / ny;
    d.idx = 1.0 / d.dx; d.idy = 1.0 / d.dy;
    d.lz = g.zf[nz] - g.zf[0];
    d.scale = 1.0 / ((double)nx * (double)ny);

    // z metrics
    std::vector<long double> dzf(nz), zc(nz), dzc(nz);
    for (int k = 0; k < nz; ++k) {
        dzf[k] = (long double)g.zf[k + 1] - (long double)g.zf[k];
        zc[k] = 0.5L * ((long double)g.zf[k] + (long double)g.zf[k + 1]);
    }
    for (int k = 0; k < nz - 1; ++k) dzc[k] = zc[k + 1] - zc[k];
    dzc[nz - 1] = 0.5L * (dzf[nz - 1] + dzf[0]);
    std::vector<long double> idzf(nz), idzc(nz), rzlo(nz), rzhi(nz), za(nz), zb(nz), zcc(nz);
    const bool per = g.bc_z == PCX_BC_PERIODIC;
    for (int k = 0; k < nz; ++k) {
        int kp = (k + 1) % nz, km = (k + nz - 1) % nz;
        idzf[k] = 1.0L / dzf[k];
        idzc[k] = 1.0L / dzc[k];
        rzlo[k] = dzf[kp] / (2.0L * dzc[k]);
        rzhi[k] = dzf[k] / (2.0L * dzc[k]);
        bool lo = per || k > 0, hi = per || k < nz - 1;
        za[k] = lo ? 1.0L / (dzf[k] * dzc[km]) : 0.0L;
        zcc[k] = hi ? 1.0L / (dzf[k] * dzc[k]) : 0.0L;
        zb[k] = -(za[k] + zcc[k]);
        // Dirichlet z: ghost -p one cell width beyond the boundary face
        if (g.bc_z == PCX_BC_DIRICHLET && !lo) zb[k] -= 2.0L / (dzf[k] * dzf[k]);
        if (g.bc_z == PCX_BC_DIRICHLET && !hi) zb[k] -= 2.0L / (dzf[k] * dzf[k]);
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> lamx(nl), lamy(ny);
    // eigenvalues of the second difference: periodic -(4/h^2) sin^2(pi l/n)
    // (folded to min(l, n-l)), cell-centred Neumann -(4/h^2) sin^2(pi l/(2n)),
    // Dirichlet (sign-alternated cosine mode l = sine mode n-1-l)
    // -(4/h^2) cos^2(pi l/(2n))
    auto eig = [&](int bc, int n, int l) {
        if (bc == PCX_BC_WALL) { long double s = sinl(pi * (long double)l / (2.0L * n)); return s * s; }
        if (bc == PCX_BC_DIRICHLET) { long double c = cosl(pi * (long double)l / (2.0L * n)); return c * c; }
        long double s = sinl(pi * (long double)std::min(l, n - l) / (long double)n);
        return s * s;
    };
    for (int l = 0; l < nl; ++l) lamx[l] = -4.0L / ((long double)d.dx * d.dx) * eig(g.bc_x, nx, l);
    for (int m = 0; m < ny; ++m) lamy[m] = -4.0L / ((long double)d.dy * d.dy) * eig(g.bc_y, ny, m);

    Blob b;
    auto addd = [&](const std::vector<long double> &v) { auto c = cast_vec<double>(v); return b.add(c.data(), c.size() * 8); };
    auto adds = [&](const std::vector<long double> &v) {
        if (prec == PREC_F64) { auto c = cast_vec<double>(v); return b.add(c.data(), c.size() * 8); }
        auto c = cast_vec<float>(v);
        return b.add(c.data(), c.size() * 4);
    };
    auto addr = [&](int n, bool extra) {
        if (prec == PREC_F64) { auto c = roots<double>(n, extra); return b.add(c.data(), c.size() * 8); }
        auto c = roots<float>(n, extra);
        return b.add(c.data(), c.size() * 4);
    };
    size_t o_dzf = addd(dzf), o_idzf = addd(idzf), o_idzc = addd(idzc), o_rzlo = addd(rzlo), o_rzhi = addd(rzhi);
    size_t o_za = adds(za), o_zb = adds(zb), o_zc = adds(zcc), o_dzfs = adds(dzf);
    size_t o_lx = adds(lamx), o_ly = adds(lamy);
    size_t o_twr = addr(nx, false); // first M+1 entries of the nx roots are W_nx^l
    size_t o_twx = addr(M, false);
    size_t o_twy = addr(ny, false);
    // cosine-transform twiddles exp(-i pi k / (2N)) = W_{4N}^k
    size_t o_dcx = g.bc_x != PCX_BC_PERIODIC ? addr(4 * nx, false) : 0;
    size_t o_dcy = g.bc_y != PCX_BC_PERIODIC ? addr(4 * ny, false) : 0;

    ht.o_dzf = o_dzf; ht.o_idzf = o_idzf; ht.o_idzc = o_idzc; ht.o_rzlo = o_rzlo; ht.o_rzhi = o_rzhi;
    ht.o_za = o_za; ht.o_zb = o_zb; ht.o_zc = o_zc; ht.o_dzfs = o_dzfs; ht.o_lx = o_lx; ht.o_ly = o_ly;
    ht.o_twr = o_twr; ht.o_twx = o_twx; ht.o_twy = o_twy; ht.o_dcx = o_dcx; ht.o_dcy = o_dcy;
    ht.bytes.swap(b.bytes);
    fill_fft(d.fx, M, rc && !rc->x.empty() ? rc->x : default_radices(M));
    fill_fft(d.fy, ny, rc && !rc->y.empty() ? rc->y : default_radices(ny));
}

void bind_tables(Dom &d, const HostTables &ht, char *base)
{
    d.dzf = (const double *)(base + ht.o_dzf);
    d.idzf = (const double *)(base + ht.o_idzf);
    d.idzc = (const double *)(base + ht.o_idzc);
    d.rzlo = (const double *)(base + ht.o_rzlo);
    d.rzhi = (const double *)(base + ht.o_rzhi);
    d.za = base + ht.o_za; d.zb = base + ht.o_zb; d.zc = base + ht.o_zc; d.dzf_s = base + ht.o_dzfs;
    d.lamx = base + ht.o_lx; d.lamy = base + ht.o_ly;
    d.twr = base + ht.o_twr;
    d.dctx = d.bcx != BC_PER ? base + ht.o_dcx : nullptr;
    d.dcty = d.bcy != BC_PER ? base + ht.o_dcy : nullptr;
    d.fx.tw = base + ht.o_twx;
    d.fy.tw = base + ht.o_twy;
}

pcx_status build_domain(const pcx_grid &g, int prec, const Shapes &sh, const RadixChoice *rc, DomTables &tb, Dom &d)
{
    HostTables ht;
    make_domain(g, prec, sh, rc, ht, d);
    tb.bytes = ht.bytes.size();
    hipError_t e = hipMalloc(&tb.dev, tb.bytes);
    if (e != hipSuccess) { tb.dev = nullptr; return fail(PCX_ERR_NOMEM, "hipMalloc(tables) failed"); }
    e = hipMemcpy(tb.dev, ht.bytes.data(), tb.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("hipMemcpy(tables): ") + hipGetErrorString(e));
    bind_tables(d, ht, (char *)tb.dev);
    return PCX_OK;
}

size_t lds_x(const Dom &d, int prec)
{
    // rows, FFT roots, split twiddles, then (x inverse) 16 reduction doubles
    return ((size_t)d.tj * lds_line(d.nl) + tw_half(d.M) + d.M / 2 + 1) * (prec == PREC_F64 ? 16 : 8) + 128;
}
size_t lds_y(const Dom &d, int prec)
{
    return ((size_t)d.tk * lds_line(d.ny) + tw_half(d.ny)) * (prec == PREC_F64 ? 16 : 8) + 64;
}
size_t lds_z(const Dom &d, int prec)
{
    size_t e = (size_t)d.zlpw * d.nz;
    return (e + e / 16 + 1) * (prec == PREC_F64 ? 16 : 8) + 64;
}

} // namespace pcx

using namespace pcx;

// =================================================================== plan

static pcx_status plan_free(pcx_plan P)
{
    if (!P) return PCX_OK;
    if (P->tables.dev) (void)hipFree(P->tables.dev);
    if (P->ws) (void)hipFree(P->ws);
    for (auto e : P->ev) (void)hipEventDestroy(e);
    delete P;
    return PCX_OK;
}

namespace pcx {

pcx_status plan_options(const pcx_options *opts, pcx_options &o)
{
    o = {PCX_FP64, 1e-10, 8, 0, 0, 0, nullptr};
    if (opts) o = *opts;
    if (o.precision != PCX_FP64 && o.precision != PCX_FP32_REFINED) return fail(PCX_ERR_INVALID, "unknown precision");
    if (!(o.rtol > 0.0)) o.rtol = 1e-10;
    if (o.max_iters <= 0) o.max_iters = 8;
    if (o.max_iters > MAXIT) o.max_iters = MAXIT;
    if (o.fixed_iters <= 0) o.fixed_iters = 3;
    if (o.fixed_iters > o.max_iters) o.fixed_iters = o.max_iters;
    return PCX_OK;
}

pcx_status plan_prepare(pcx_plan_s *P, const pcx_grid *grid, const pcx_options &o, HostTables &ht)
{
    P->grid = *grid;
    P->zf.assign(grid->zf, grid->zf + grid->nz + 1);
    P->grid.zf = P->zf.data();
    P->opt = o;
    P->prec = o.precision == PCX_FP64 ? PREC_F64 : PREC_F32;
    TuneParams tp;
    RadixChoice rc;
    TuneCache cache;
    bool have = o.tune_cache && cache.load(o.tune_cache) && cache.lookup(P->grid, P->prec, tp, rc);
    if (!have && o.autotune) {
        pcx_status st = autotune_class(P->grid, P->prec, nullptr, tp, rc, false);
        if (st != PCX_OK) return st;
        have = true;
        if (o.tune_cache) {
            cache.store(P->grid, P->prec, tp, rc);
            cache.save(o.tune_cache);
        }
    }
    choose_shapes(P->grid, P->prec, have ? &tp : nullptr, P->sh, false);
    make_domain(P->grid, P->prec, P->sh, have ? &rc : nullptr, ht, P->dom);
    return PCX_OK;
}

WsLayout plan_layout(const pcx_plan_s *P)
{
    const size_t csz = P->prec == PREC_F64 ? 16 : 8;
    const size_t nspec = (size_t)P->dom.nl * P->grid.ny * P->grid.nz;
    const size_t ncell = (size_t)P->grid.nx * P->grid.ny * P->grid.nz;
    const bool ref = P->prec == PREC_F32;
    WsLayout L;
    size_t off = 0;
    auto put = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    L.s1 = put(nspec * csz);
    L.s2 = put(nspec * csz);
    L.f = put(ncell * sizeof(double));
    L.r = ref ? put(ncell * sizeof(double)) : 0;
    L.stats = put(NSTAT * sizeof(unsigned long long));
    L.psum = put((size_t)P->grid.nz * sizeof(double));
    L.xpart = put((size_t)2 * xslots(P->dom) * sizeof(double));
    L.ppart = ref ? put(((size_t)xslots(P->dom) + PMEAN_LEN) * sizeof(double)) : 0;
    L.spart = put((size_t)sslots(P->dom) * sizeof(double));
    L.total = off;
    return L;
}

void plan_bind(pcx_plan_s *P, const HostTables &ht, char *tables, char *ws, const WsLayout &L)
{
    const bool ref = P->prec == PREC_F32;
    bind_tables(P->dom, ht, tables);
    P->s1 = ws + L.s1;
    P->s2 = ws + L.s2;
    P->f = (double *)(ws + L.f);
    P->r = ref ? (double *)(ws + L.r) : nullptr;
    P->stats = (unsigned long long *)(ws + L.stats);
    P->psum = (double *)(ws + L.psum);
    P->xpart = (double *)(ws + L.xpart);
    P->ppart = ref ? (double *)(ws + L.ppart) : nullptr;
    P->ws_bytes = L.total + ht.bytes.size();
    P->dom.s1 = P->s1;
    P->dom.s2 = P->s2;
    P->dom.f = P->f;
    P->dom.r = P->r;
    P->dom.stats = P->stats;
    P->dom.ppart = P->ppart;
    P->dom.xpart = P->xpart;
    P->dom.pmean = P->ppart ? P->ppart + (size_t)xslots(P->dom) : nullptr;
    P->spart = (double *)(ws + L.spart);
    P->dom.spart = P->spart;
    // The fused stencil + x passes need an x pass with one row per wave.
    // The residual's is the default (r is never stored: 0.63 ms against
    // 0.59 + 0.33 ms per extra solve at 512^3); the RHS's is opt-in
    // (PCX_FUSE_RHS=1): its stencil, which reads five fields and their
    // neighbours straight from memory, is slower than the marching RHS
    // kernel plus the x pass (1.74 against 1.21 + 0.40 ms at 512^3 FP64).
    // PCX_FUSE=0 turns both off.
    const char *fz = std::getenv("PCX_FUSE"), *fr = std::getenv("PCX_FUSE_RHS");
    const bool fuse = !(fz && fz[0] == '0') && sx_supported(P->dom);
    P->fuse_resid = fuse;
    P->fuse_rhs = fuse && fr && fr[0] == '1';
    P->lx = lds_x(P->dom, P->prec);
    P->ly = lds_y(P->dom, P->prec);
    P->lzs = lds_z(P->dom, P->prec);
}

} // namespace pcx

extern "C" pcx_status pcx_plan_create(const pcx_grid *grid, const pcx_options *opts, pcx_plan *out)
{
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    pcx_status st = validate_grid(grid);
    if (st != PCX_OK) return st;
    pcx_options o;
    st = plan_options(opts, o);
    if (st != PCX_OK) return st;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(PCX_ERR_HIP, "no HIP device available");

    pcx_plan P = new pcx_plan_s();
    (void)hipGetDevice(&P->device);
    HostTables ht;
    st = plan_prepare(P, grid, o, ht);
    if (st != PCX_OK) { delete P; return st; }
    P->tables.bytes = ht.bytes.size();
    if (hipMalloc(&P->tables.dev, P->tables.bytes) != hipSuccess) {
        P->tables.dev = nullptr;
        plan_free(P);
        return fail(PCX_ERR_NOMEM, "hipMalloc(tables) failed");
    }
    e = hipMemcpy(P->tables.dev, ht.bytes.data(), P->tables.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        plan_free(P);
        return fail(PCX_ERR_HIP, std::string("hipMemcpy(tables): ") + hipGetErrorString(e));
    }
    const WsLayout L = plan_layout(P);
    if (hipMalloc(&P->ws, L.total) != hipSuccess) {
        P->ws = nullptr;
        plan_free(P);
        return fail(PCX_ERR_NOMEM, "workspace allocation failed");
    }
    plan_bind(P, ht, (char *)P->tables.dev, (char *)P->ws, L);
    *out = P;
    return PCX_OK;
}

extern "C" pcx_status pcx_plan_workspace_bytes(pcx_plan P, size_t *bytes)
{
    if (!P || !bytes) return fail(PCX_ERR_INVALID, "NULL argument");
    *bytes = P->ws_bytes;
    return PCX_OK;
}

extern "C" pcx_status pcx_plan_destroy(pcx_plan P) { return plan_free(P); }

// --------------------------------------------------------------- timing
// When timing is on, every step appends HIP events recorded on its stream
// between passes (mode 1), or only around the velocity correction (mode 2:
// two events per step); pcx_plan_pass_times returns the durations of the
// timed passes of all steps since timing was (re)enabled.  An unnamed event
// starts an interval that is not reported.
static void tmark_record(pcx_plan P, hipStream_t s, const char *name);

static void tmark(pcx_plan P, hipStream_t s, const char *name)
{
    if (!P->timing) return;
    if (P->timing == 2 && !(name && !std::strcmp(name, "correct_div"))) return;
    tmark_record(P, s, name);
}

static void tmark_record(pcx_plan P, hipStream_t s, const char *name)
{
    if (P->nev >= (int)P->ev.size()) {
        if (P->ev.size() >= 4096) return;
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        P->ev.push_back(e);
        P->names.push_back("");
    }
    (void)hipEventRecord(P->ev[P->nev], s);
    P->names[P->nev] = name ? name : "";
    P->nev++;
}

extern "C" pcx_status pcx_plan_set_timing(pcx_plan P, int32_t enable)
{
    if (!P) return fail(PCX_ERR_INVALID, "plan is NULL");
    P->timing = enable == 2 ? 2 : (enable != 0 ? 1 : 0);
    P->nev = 0;
    P->npass = 0;
    return PCX_OK;
}

extern "C" pcx_status pcx_plan_pass_times(pcx_plan P, double *ms, int32_t cap, int32_t *n_out)
{
    if (!P || !n_out) return fail(PCX_ERR_INVALID, "NULL argument");
    *n_out = 0;
    if (P->nev == 0) return PCX_OK;
    hipError_t e = hipEventSynchronize(P->ev[P->nev - 1]);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    P->pass_names.clear();
    int n = 0;
    for (int i = 1; i < P->nev; ++i) {
        if (P->names[i].empty()) continue; // step start marker
        float t = 0.f;
        e = hipEventElapsedTime(&t, P->ev[i - 1], P->ev[i]);
        if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
        if (n < cap && ms) ms[n] = t;
        P->pass_names.push_back(P->names[i]);
        ++n;
    }
    *n_out = n;
    return PCX_OK;
}

extern "C" const char *pcx_plan_pass_name(pcx_plan P, int32_t i)
{
    if (!P || i < 0 || i >= (int)P->pass_names.size()) return "";
    return P->pass_names[i].c_str();
}

// ----------------------------------------------------------------- step
#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(PCX_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// One FP32/FP64 solve: transforms and tridiagonal solve on the right-hand
// side already placed (x-transformed) in S1, ending with p stored/accumulated.
static pcx_status solve_tail(pcx_plan P, const Dom &d, int solve, int mode, hipStream_t s)
{
    HIPCHK(launch_y(d, P->prec, false, P->ly, s));
    tmark(P, s, "y_fft_fwd");
    HIPCHK(launch_z(d, P->prec, P->sh.smax, P->lzs, s));
    tmark(P, s, "z_solve");
    HIPCHK(launch_y(d, P->prec, true, P->ly, s));
    tmark(P, s, "y_fft_inv");
    HIPCHK(launch_xinv(d, P->prec, mode, solve, P->lx, s));
    tmark(P, s, mode == XOUT_STORE ? "x_fft_inv_store_p" : "x_fft_inv_accum_p");
    HIPCHK(launch_xmax(d, solve, s));
    tmark(P, s, "x_max");
    if (d.ppart) {
        HIPCHK(launch_pmean(d, s));
        tmark(P, s, "p_mean");
    }
    return PCX_OK;
}

static double stat_d(const std::vector<unsigned long long> &h, int i)
{
    double v;
    std::memcpy(&v, &h[i], 8);
    return v;
}

// Stop test of the refinement: the relative residual must be within rtol and
// the error left after the last update, estimated from the observed
// contraction q = |e_s| / |e_{s-1}| as q |e_s| / (1 - q), must be below
// 0.1 rtol |p|.  The first solve alone never stops (no rate is known).
extern "C" int32_t pcx_refine_should_stop(double rel_residual, double update_inf, double prev_update_inf, double p_inf,
                                          double rtol)
{
    if (!(rel_residual <= rtol)) return 0;
    if (!(prev_update_inf > 0.0) || !(update_inf >= 0.0)) return 0;
    const double q = update_inf / prev_update_inf;
    if (!(q < 1.0)) return 0;
    const double est = q * update_inf / (1.0 - q);
    return est <= 0.1 * rtol * p_inf ? 1 : 0;
}

extern "C" pcx_status pcx_step(pcx_plan P, double dt, double rho0, const double *rho, const double *p_star,
                               const double *u_in, const double *v_in, const double *w_in, double *u_out,
                               double *v_out, double *w_out, double *p_out, void *stream, pcx_report *report)
{
    if (!P) return fail(PCX_ERR_INVALID, "plan is NULL");
    if (P->dom.nosing)
        return fail(PCX_ERR_UNSUPPORTED, "the pressure-correction step has no rule for a Dirichlet boundary "
                                         "(use pcx_poisson_solve)");
    if (!rho || !p_star || !u_in || !v_in || !w_in || !u_out || !v_out || !w_out || !p_out)
        return fail(PCX_ERR_INVALID, "NULL field pointer");
    if (!(dt > 0.0) || !(rho0 > 0.0) || !std::isfinite(dt) || !std::isfinite(rho0))
        return fail(PCX_ERR_INVALID, "dt and rho0 must be finite and > 0");
    const void *ins[] = {rho, p_star, u_in, v_in, w_in, u_out, v_out, w_out};
    for (const void *q : ins)
        if (q == p_out) return fail(PCX_ERR_INVALID, "p_out aliases another field");
    const double *velin[] = {u_in, v_in, w_in};
    const double *velout[] = {u_out, v_out, w_out};
    bool inplace = false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            if (velout[a] == velin[b]) {
                if (a != b) return fail(PCX_ERR_INVALID, "velocity output aliases a different input component");
                inplace = true;
            }
            if (velout[a] == rho || velout[a] == p_star) return fail(PCX_ERR_INVALID, "velocity output aliases rho or p_star");
            if (a != b && velout[a] == velout[b]) return fail(PCX_ERR_INVALID, "velocity outputs alias each other");
        }
    hipStream_t s = (hipStream_t)stream;
    Dom d = P->dom;
    d.dt = dt; d.rho0 = rho0; d.irho0 = 1.0 / rho0;
    d.rho = rho; d.ps = p_star; d.u = u_in; d.v = v_in; d.w = w_in;
    d.uo = u_out; d.vo = v_out; d.wo = w_out; d.po = p_out;
    tmark(P, s, nullptr);
    HIPCHK(launch_zero(P->stats, NSTAT, s));
    int solves = 0;
    if (P->fuse_rhs) {
        HIPCHK(launch_sx(d, P->prec, SRC_RHS_ST, P->lx, s));
        tmark(P, s, "rhs_fftx");
        HIPCHK(launch_smax(d, ST_FINF, ST_SOLVE0, s));
        tmark(P, s, "f_max");
    } else {
        HIPCHK(launch_rhs(d, s));
        tmark(P, s, "rhs_stencil");
        HIPCHK(launch_xfwd(d, P->prec, SRC_RHS, P->lx, s));
        tmark(P, s, "x_fft_fwd");
    }
    pcx_status st0 = solve_tail(P, d, 0, XOUT_STORE, s);
    if (st0 != PCX_OK) return st0;
    solves = 1;
    auto refine_once = [&](int solve) -> pcx_status {
        if (P->fuse_resid) {
            HIPCHK(launch_sx(d, P->prec, SRC_RESID_ST, P->lx, s));
            tmark(P, s, "resid_fftx");
            HIPCHK(launch_smax(d, ST_SOLVE0 + 4 * solve, -1, s));
            tmark(P, s, "r_max");
        } else {
            HIPCHK(launch_resid(d, solve, s));
            tmark(P, s, "resid_stencil");
            HIPCHK(launch_xfwd(d, P->prec, SRC_RESID, P->lx, s));
            tmark(P, s, "x_fft_fwd_resid");
        }
        return solve_tail(P, d, solve, XOUT_ACCUM, s);
    };
    if (P->prec == PREC_F32) {
        for (; solves < P->opt.fixed_iters; ++solves) {
            pcx_status st = refine_once(solves);
            if (st != PCX_OK) return st;
        }
    }
    auto correct = [&]() -> pcx_status {
        if (P->timing == 2) tmark_record(P, s, nullptr); // start of the correction
        HIPCHK(launch_corr(d, !inplace, s));
        tmark(P, s, "correct_div");
        if (inplace) {
            HIPCHK(launch_div(d, s));
            tmark(P, s, "div_check");
        }
        return PCX_OK;
    };
    // With a report the refined form keeps refining until rtol is met.  The
    // correction is computed from p only after the decision: the step is
    // re-corrected after each extra solve (u* is untouched unless in place,
    // where no extra solve can be taken after the first correction).
    pcx_status st = PCX_OK;
    std::vector<unsigned long long> h(NSTAT);
    if (!report) return correct();
    while (true) {
        st = correct();
        if (st != PCX_OK) return st;
        HIPCHK(hipMemcpyAsync(h.data(), P->stats, NSTAT * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double finf = stat_d(h, ST_FINF), dv = stat_d(h, ST_DIV);
        double rel = dv / ((dt / rho0) * finf);
        double einf = stat_d(h, ST_SOLVE0 + 4 * (solves - 1) + 1);
        double eprev = solves >= 2 ? stat_d(h, ST_SOLVE0 + 4 * (solves - 2) + 1) : 0.0;
        double pinf = stat_d(h, ST_SOLVE0 + 4 * (solves - 1) + 2);
        bool stop = P->prec == PREC_F64 || pcx_refine_should_stop(rel, einf, eprev, pinf, P->opt.rtol);
        if (stop || solves >= P->opt.max_iters || inplace) break;
        HIPCHK(launch_zero(P->stats + ST_DIV, 1, s));
        st = refine_once(solves);
        if (st != PCX_OK) return st;
        ++solves;
    }
    // report
    HIPCHK(launch_plane_sums(p_out, P->grid.nx * P->grid.ny, P->grid.nz, P->psum, s));
    std::vector<double> ps(P->grid.nz);
    HIPCHK(hipMemcpyAsync(ps.data(), P->psum, ps.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double num = 0.0, lz = P->zf[P->grid.nz] - P->zf[0];
    for (int k = 0; k < P->grid.nz; ++k) num += (P->zf[k + 1] - P->zf[k]) * ps[k];
    pcx_report r;
    std::memset(&r, 0, sizeof(r));
    r.solves = solves;
    r.f_inf = stat_d(h, ST_FINF);
    r.max_div_abs = stat_d(h, ST_DIV);
    r.rel_residual = r.max_div_abs / ((dt / rho0) * r.f_inf);
    r.max_div_rel = r.rel_residual;
    r.mean_p = num / ((double)P->grid.nx * P->grid.ny * lz);
    r.last_update_inf = stat_d(h, ST_SOLVE0 + 4 * (solves - 1) + 1);
    double eprev = solves >= 2 ? stat_d(h, ST_SOLVE0 + 4 * (solves - 2) + 1) : 0.0;
    double pinf = stat_d(h, ST_SOLVE0 + 4 * (solves - 1) + 2);
    r.converged = P->prec == PREC_F64 ? (r.rel_residual <= P->opt.rtol)
                                      : pcx_refine_should_stop(r.rel_residual, r.last_update_inf, eprev, pinf, P->opt.rtol);
    *report = r;
    if (P->opt.check_finite) {
        double om = stat_d(h, ST_NONFIN);
        if (!std::isfinite(om) || !std::isfinite(r.f_inf) || !std::isfinite(r.max_div_abs))
            return fail(PCX_ERR_NONFINITE, "non-finite value in the outputs");
    }
    if (P->prec == PREC_F32 && !r.converged) return fail(PCX_ERR_NOT_CONVERGED, "refinement did not reach rtol within max_iters");
    return PCX_OK;
}

// L p = f with the plan's boundary conditions (periodic, Neumann wall or
// homogeneous Dirichlet per direction): the transforms and tridiagonal
// solves of the step on a given right-hand side.  Without a Dirichlet
// direction, the compatible part f - <f> is solved and <p> = 0.
extern "C" pcx_status pcx_poisson_solve(pcx_plan P, const double *f, double *p, void *stream)
{
    if (!P || !f || !p) return fail(PCX_ERR_INVALID, "NULL argument");
    if (f == p) return fail(PCX_ERR_INVALID, "p must not alias f");
    if (P->prec != PREC_F64) return fail(PCX_ERR_UNSUPPORTED, "pcx_poisson_solve runs FP64 plans only");
    hipStream_t s = (hipStream_t)stream;
    Dom d = P->dom;
    d.f = const_cast<double *>(f); // read only: the forward x pass reads its source
    d.po = p;
    HIPCHK(launch_zero(P->stats, NSTAT, s));
    HIPCHK(launch_xfwd(d, P->prec, SRC_RHS, P->lx, s));
    return solve_tail(P, d, 0, XOUT_STORE, s);
}

// ------------------------------------------------------------------ misc

static std::mutex g_min_mutex;

extern "C" pcx_status pcx_rho_min(const double *rho, int64_t n, void *stream, double *out)
{
    if (!rho || !out || n <= 0) return fail(PCX_ERR_INVALID, "bad argument");
    // one reduction slot per device in static device memory: calls are
    // serialised here, and each synchronises its stream before returning
    std::lock_guard<std::mutex> lk(g_min_mutex);
    hipError_t e = min_to_host(rho, (long long)n, (hipStream_t)stream, out);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("rho_min: ") + hipGetErrorString(e));
    return PCX_OK;
}

extern "C" const char *pcx_status_str(pcx_status s)
{
    switch (s) {
    case PCX_OK: return "PCX_OK";
    case PCX_ERR_INVALID: return "PCX_ERR_INVALID";
    case PCX_ERR_UNSUPPORTED: return "PCX_ERR_UNSUPPORTED";
    case PCX_ERR_NOMEM: return "PCX_ERR_NOMEM";
    case PCX_ERR_HIP: return "PCX_ERR_HIP";
    case PCX_ERR_NOT_CONVERGED: return "PCX_ERR_NOT_CONVERGED";
    case PCX_ERR_NONFINITE: return "PCX_ERR_NONFINITE";
    }
    return "PCX_ERR_UNKNOWN";
}

extern "C" const char *pcx_last_error(void) { return g_err.c_str(); }

extern "C" int32_t pcx_abi_version(void) { return PCX_ABI_VERSION; }
