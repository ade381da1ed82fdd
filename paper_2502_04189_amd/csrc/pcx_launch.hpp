// pcx_launch.hpp -- host-side launchers of the device passes.
#pragma once

#include "pcx_dev.hpp"

namespace pcx {

hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_rhs(const Dom &d, hipStream_t s);
hipError_t launch_resid(const Dom &d, int solve, hipStream_t s);
hipError_t launch_xfwd(const Dom &d, int prec, int src, size_t lds, hipStream_t s);
// fused stencil + forward x pass (src SRC_RHS_ST or SRC_RESID_ST), with its
// per-wave maxima reduced by launch_smax into stats slots sa (and sb >= 0)
bool sx_supported(const Dom &d);
hipError_t launch_sx(const Dom &d, int prec, int src, size_t lds, hipStream_t s);
hipError_t launch_smax(const Dom &d, int sa, int sb, hipStream_t s);
hipError_t launch_y(const Dom &d, int prec, bool inv, size_t lds, hipStream_t s);
hipError_t launch_z(const Dom &d, int prec, int smax, size_t lds, hipStream_t s);
hipError_t launch_xinv(const Dom &d, int prec, int mode, int solve, size_t lds, hipStream_t s);
hipError_t launch_corr(const Dom &d, bool divcheck, hipStream_t s);
hipError_t launch_div(const Dom &d, hipStream_t s);
hipError_t launch_pmean(const Dom &d, hipStream_t s);
hipError_t launch_xmax(const Dom &d, int solve, hipStream_t s);
hipError_t launch_plane_sums(const double *p, int nxy, int nz, double *out, hipStream_t s);
// min over n doubles into *out (host); synchronises s
hipError_t min_to_host(const double *a, long long n, hipStream_t s, double *out);

} // namespace pcx

namespace pcx {

// ------------------------------------------------------ grouped (batched)
// One launch of one pass over tiles of many domains: item i of the launch is
// tile items[i].tile of domain items[i].dom (dom == GSKIP: no work).  Items
// are processed by workgroup b in the order b, b + grid, b + 2 grid, ...
constexpr uint32_t GSKIP = 0xffffffffu;
struct GItem {
    uint32_t dom, tile;
};
struct GArgs {
    const Dom *doms;
    const GItem *items;
    int nitems;
    int solve;
};
// Which kernel a group runs: the pass kind (PK_*), its workgroup size, and
// the per-pass template choice (RHS / correction: a second halo item per
// thread; z: levels per lane).
struct GVariant {
    int kind, nth, two, smax;
};
hipError_t launch_group(const GVariant &v, int prec, const GArgs &a, int grid, size_t lds, hipStream_t s);
// resident workgroups per CU of a group's kernel
hipError_t group_occupancy(const GVariant &v, int prec, size_t lds, int *blocks_per_cu);
// workgroup size of the marching stencil kernels (RHS and residual; correction)
int march_threads(int corr);

// ---------------------------------------------------------------- batched
// phases of a batch: 8 for the first solve (RHS, x, y, z, y, x, maxima,
// correction) and 7 per further solve, for up to MAXIT solves
constexpr int MAXPH = 96;
static_assert(MAXPH >= 8 + 7 * (MAXIT - 1), "phase table too small for MAXIT solves");
enum { PK_RHS = 0, PK_RESID, PK_XFWD_RHS, PK_XFWD_RESID, PK_YF, PK_Z, PK_YI, PK_XINV_STORE, PK_XINV_ACCUM, PK_PMEAN, PK_CORR,
       PK_XMAX };

struct Item {
    uint16_t dom, phase;
    uint32_t tile;   // first tile
    uint32_t count;  // consecutive tiles in this item
    uint32_t pad;
};

// Pass kind and solve index of each phase (the same for every domain).
struct PhaseTab {
    int nphase;
    uint8_t kind[MAXPH];
    uint8_t solve[MAXPH];
};

struct PersistArgs {
    const Dom *doms;
    const Item *items;
    int nitems;
    unsigned *head;           // queue head
    unsigned *done;           // [ndom * nphase] finished tiles
    const unsigned *need;     // [ndom * nphase] tiles of each phase
    unsigned *err;            // set when a dependency wait gives up
    unsigned spin_limit;      // max polls of one dependency wait
    PhaseTab tab;
};

hipError_t launch_persist(const PersistArgs &a, int prec, int smax, int blocks, size_t lds, hipStream_t s);
hipError_t launch_reset(unsigned *p, int n, hipStream_t s);
hipError_t persist_occupancy(int prec, int smax, size_t lds, int *blocks_per_cu);

} // namespace pcx
