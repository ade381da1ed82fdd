// Host-side checks of libpcx built with AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; no device is needed): plan
// preparation over a sweep of grids, boundary conditions and precisions
// (tables, shapes, workspace layout), descriptor validation, the
// allocation-free step's size rejection, the refinement stop test, and the
// create calls on a host without a GPU.
#include <cmath>
#include <cstdio>
#include <vector>

#include "pcx.h"

static int g_fail = 0;
#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                            \
        }                                                                        \
    } while (0)

static std::vector<double> zf_of(int nz, double lz, bool stretched)
{
    std::vector<double> z(nz + 1);
    for (int k = 0; k <= nz; ++k) {
        double s = (double)k / nz;
        z[k] = stretched ? lz * 0.5 * (1.0 + std::tanh(1.8 * (s - 0.5)) / std::tanh(0.9)) : lz * s;
    }
    z[0] = 0.0;
    z[nz] = lz;
    return z;
}

int main()
{
    const int xs[] = {2, 4, 6, 8, 12, 18, 32, 48, 96, 128, 256, 384, 512, 1024, 3072, 4096, 8192};
    const int ys[] = {2, 3, 5, 9, 27, 64, 96, 512, 4096};
    const int zs[] = {2, 3, 17, 64, 1024, 2048};
    long ok = 0, unsup = 0, inval = 0;
    for (int nx : xs)
        for (int ny : ys)
            for (int nz : zs)
                for (int bc = 0; bc < 8; ++bc)
                    for (int prec = 0; prec < 2; ++prec) {
                        std::vector<double> zf = zf_of(nz, 1.0, bc & 1);
                        pcx_grid g{nx, ny, nz, 1.0, 2.0, zf.data(), (bc >> 2) & 1, (bc >> 1) & 1, bc & 1};
                        pcx_options o{prec, 1e-10, 8, 0, 0, 0, nullptr};
                        size_t need = 0;
                        pcx_status st = pcx_noalloc_scratch_need(&g, &o, &need);
                        if (st == PCX_OK) {
                            ++ok;
                            CHECK(need > 0);
                        } else if (st == PCX_ERR_UNSUPPORTED) {
                            ++unsup;
                        } else {
                            CHECK(st == PCX_ERR_INVALID);
                            ++inval;
                        }
                    }
    CHECK(ok > 1000 && unsup > 0 && inval > 0);

    // descriptor validation
    std::vector<double> zf = zf_of(16, 1.0, false);
    pcx_grid g{32, 32, 16, 1.0, 1.0, zf.data(), 0, 0, 1};
    size_t need = 0;
    CHECK(pcx_noalloc_scratch_need(nullptr, nullptr, &need) == PCX_ERR_INVALID);
    CHECK(pcx_noalloc_scratch_need(&g, nullptr, nullptr) == PCX_ERR_INVALID);
    pcx_grid b = g;
    b.zf = nullptr;
    CHECK(pcx_noalloc_scratch_need(&b, nullptr, &need) == PCX_ERR_INVALID);
    b = g;
    b.bc_z = 7;
    CHECK(pcx_noalloc_scratch_need(&b, nullptr, &need) == PCX_ERR_INVALID);
    std::vector<double> zbad = zf;
    zbad[3] = zbad[2];
    b = g;
    b.zf = zbad.data();
    CHECK(pcx_noalloc_scratch_need(&b, nullptr, &need) == PCX_ERR_INVALID);
    pcx_options bad_prec{7, 1e-10, 8, 0, 0, 0, nullptr};
    CHECK(pcx_noalloc_scratch_need(&g, &bad_prec, &need) == PCX_ERR_INVALID);

    // the allocation-free step rejects a grid beyond its array before any
    // device call; dummy pointers are never dereferenced
    std::vector<double> zbig = zf_of(256, 1.0, false);
    pcx_grid big{256, 256, 256, 1.0, 1.0, zbig.data(), 0, 0, 1};
    double *d = (double *)(uintptr_t)4096;
    CHECK(pcx_step_noalloc(&big, nullptr, 1e-3, 1.0, d, d + 1, d + 2, d + 3, d + 4, d + 5, d + 6, d + 7, d + 8,
                           nullptr, nullptr) == PCX_ERR_UNSUPPORTED);

    // create calls: no device on this host
    pcx_plan p = nullptr;
    pcx_status st = pcx_plan_create(&g, nullptr, &p);
    CHECK(st == PCX_ERR_HIP || st == PCX_OK);
    if (p) pcx_plan_destroy(p);
    CHECK(pcx_plan_create(nullptr, nullptr, &p) == PCX_ERR_INVALID);
    pcx_domain dom{};
    dom.grid = g;
    dom.dt = 1e-3;
    dom.rho0 = 1.0;
    pcx_batch bt = nullptr;
    CHECK(pcx_batch_create(&dom, 1, nullptr, nullptr, &bt) == PCX_ERR_INVALID); // NULL fields
    CHECK(pcx_batch_create(nullptr, 1, nullptr, nullptr, &bt) == PCX_ERR_INVALID);
    pcx_options many{PCX_FP32_REFINED, 1e-10, 12, 12, 0, 0, nullptr};
    dom.rho = dom.p_star = dom.u = dom.v = dom.w = d;
    dom.u_out = d + 1; dom.v_out = d + 2; dom.w_out = d + 3; dom.p_out = d + 4;
    st = pcx_batch_create(&dom, 1, &many, nullptr, &bt);
    CHECK(st == PCX_ERR_HIP || st == PCX_ERR_UNSUPPORTED || st == PCX_ERR_INVALID);

    // refinement stop test
    CHECK(pcx_refine_should_stop(1e-11, 1e-12, 1e-6, 1.0, 1e-10) == 1);
    CHECK(pcx_refine_should_stop(1e-9, 1e-12, 1e-6, 1.0, 1e-10) == 0);
    CHECK(pcx_refine_should_stop(1e-11, 1e-12, 0.0, 1.0, 1e-10) == 0);
    CHECK(pcx_refine_should_stop(1e-11, 1e-6, 1e-6, 1.0, 1e-10) == 0);
    CHECK(pcx_refine_should_stop(NAN, 1e-12, 1e-6, 1.0, 1e-10) == 0);
    for (int s = 0; s < 8; ++s) CHECK(pcx_status_str((pcx_status)s)[0] == 'P');
    CHECK(pcx_last_error() != nullptr);
    CHECK(pcx_abi_version() == PCX_ABI_VERSION);

    std::printf("host checks: %ld grids prepared, %ld unsupported, %ld invalid; %d failures\n", ok, unsup, inval,
                g_fail);
    return g_fail ? 1 : 0;
}
