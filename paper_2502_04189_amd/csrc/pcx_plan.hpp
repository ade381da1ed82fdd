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

extern thread_local std::string g_err;
pcx_status fail(pcx_status s, const std::string &msg);
FastDiv mkdiv(uint32_t d);
std::vector<int> default_radices(int n);
void fill_fft(FftDesc &fd, int n, const std::vector<int> &rad);
pcx_status validate_grid(const pcx_grid *g);
void choose_shapes(const pcx_grid &g, int prec, const TuneParams *tp, Shapes &sh, bool batch);
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

struct pcx_plan_s {
    int device = 0;
    pcx_grid grid;
    std::vector<double> zf;
    pcx_options opt;
    int prec = 0;
    pcx::Shapes sh;
    pcx::DomTables tables;
    pcx::Dom dom;
    void *s1 = nullptr, *s2 = nullptr;
    double *f = nullptr;
    double *r = nullptr;
    double *psum = nullptr;
    double *ppart = nullptr;
    double *xpart = nullptr;
    unsigned long long *stats = nullptr;
    size_t ws_bytes = 0;
    size_t lx = 0, ly = 0, lzs = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<std::string> names, pass_names;
    int nev = 0, npass = 0;
};
