// pcx_plan.hpp -- host-side plan objects shared by the single-domain and
// batched forms.
#pragma once

#include <string>
#include <vector>

#include "pcx.h"
#include "pcx_dev.hpp"

namespace pcx {

struct Shapes {
    int tj = 8, tk = 8, zg = 64, smax = 8;
    int yth = 256, mth = 512, mthc = 1024, xth = 512;
    bool batch = false;
};

// Optional overrides picked by the autotuner (0 / empty = default).
struct TuneParams {
    int tj = 0, tk = 0, zg = 0;
};
struct RadixChoice {
    std::vector<int> x, y;
};

struct DomTables {
    void *dev = nullptr;
    size_t bytes = 0;
};

// Host image of a domain's device tables and the byte offset of each table
// in it (each 256-byte aligned).
struct HostTables {
    std::vector<char> bytes;
    size_t o_dzf = 0, o_idzf = 0, o_idzc = 0, o_rzlo = 0, o_rzhi = 0, o_za = 0, o_zb = 0, o_zc = 0, o_dzfs = 0,
           o_lx = 0, o_ly = 0, o_twr = 0, o_twx = 0, o_twy = 0, o_dcx = 0, o_dcy = 0;
};

// Byte offsets of a single-domain step's workspace pieces inside one region
// (each 256-byte aligned; r and ppart are used by the refined form only).
struct WsLayout {
    size_t s1 = 0, s2 = 0, f = 0, r = 0, stats = 0, psum = 0, xpart = 0, ppart = 0, spart = 0, total = 0;
};

extern thread_local std::string g_err;
pcx_status fail(pcx_status s, const std::string &msg);
FastDiv mkdiv(uint32_t d);
std::vector<int> default_radices(int n);
void fill_fft(FftDesc &fd, int n, const std::vector<int> &rad);
pcx_status validate_grid(const pcx_grid *g);
void choose_shapes(const pcx_grid &g, int prec, const TuneParams *tp, Shapes &sh, bool batch);
void make_domain(const pcx_grid &g, int prec, const Shapes &sh, const RadixChoice *rc, HostTables &ht, Dom &d);
void bind_tables(Dom &d, const HostTables &ht, char *base);
pcx_status build_domain(const pcx_grid &g, int prec, const Shapes &sh, const RadixChoice *rc, DomTables &tb, Dom &d);
size_t lds_x(const Dom &d, int prec);
size_t lds_y(const Dom &d, int prec);
size_t lds_z(const Dom &d, int prec);
// grouped (batched) launches: the kernel variant, tile count and LDS bytes
// of pass `kind` for domain d
struct GVariant;
GVariant variant_of(const Dom &d, int kind, int smax);
long group_tiles(const Dom &d, int kind);
size_t group_lds(const Dom &d, int kind, int prec);

} // namespace pcx

struct pcx_plan_s;

namespace pcx {
// Pieces of plan creation shared by pcx_plan_create and the allocation-free
// step: option defaults, the host part of a plan (grid copy, shapes, domain
// descriptor and table image; no device call unless autotuning), the
// workspace layout of a prepared plan, and the binding of a plan to its
// tables and workspace in device memory.
pcx_status plan_options(const pcx_options *opts, pcx_options &o);
pcx_status plan_prepare(pcx_plan_s *P, const pcx_grid *grid, const pcx_options &o, HostTables &ht);
WsLayout plan_layout(const pcx_plan_s *P);
void plan_bind(pcx_plan_s *P, const HostTables &ht, char *tables, char *ws, const WsLayout &L);
} // namespace pcx

struct pcx_plan_s {
    int device = 0;
    pcx_grid grid;
    std::vector<double> zf;
    pcx_options opt;
    int prec = 0;
    pcx::Shapes sh;
    pcx::DomTables tables;
    pcx::Dom dom;
    void *ws = nullptr;             // owned workspace region (pcx_plan_create); NULL when borrowed
    void *s1 = nullptr, *s2 = nullptr;
    double *f = nullptr;
    double *r = nullptr;
    double *psum = nullptr;
    double *ppart = nullptr;
    double *xpart = nullptr;
    double *spart = nullptr;
    bool fuse_rhs = false;          // RHS evaluated inside the forward x pass
    bool fuse_resid = false;        // residual evaluated inside the forward x pass
    unsigned long long *stats = nullptr;
    size_t ws_bytes = 0;
    size_t lx = 0, ly = 0, lzs = 0;
    int timing = 0; // 0 off, 1 every pass, 2 the velocity correction only
    std::vector<hipEvent_t> ev;
    std::vector<std::string> names, pass_names;
    int nev = 0, npass = 0;
};
