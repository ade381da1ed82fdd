// pcx_noalloc.cpp -- the allocation-free single-domain step.
//
// pcx_step_noalloc runs the same passes as pcx_plan_create + pcx_step, with
// the plan's tables and workspace placed in one file-scope device array
// (`scratch`) instead of memory from hipMalloc.  Each device the library runs
// on holds its own copy of the array for the life of the process; its device
// address is looked up once per device (hipGetSymbolAddress, with that
// device current) and kept, and only that address is ever handed to kernels
// or copies: in host code the array's name is not a device address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "pcx.h"
#include "pcx_launch.hpp"
#include "pcx_plan.hpp"

using namespace pcx;

namespace {

static_assert(PCX_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) unsigned char scratch[PCX_NOALLOC_SCRATCH_BYTES];

constexpr int MAXDEV = 64;
std::mutex g_ptr_mu;
char *g_ptr[MAXDEV] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device).
pcx_status scratch_ptr(int dev, char **out)
{
    if (dev < 0 || dev >= MAXDEV) return fail(PCX_ERR_HIP, "device ordinal beyond the supported range");
    std::lock_guard<std::mutex> lk(g_ptr_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PCX_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = (char *)p;
    }
    *out = g_ptr[dev];
    return PCX_OK;
}

} // namespace

extern "C" pcx_status pcx_noalloc_scratch_need(const pcx_grid *grid, const pcx_options *opts, size_t *bytes)
{
    if (!bytes) return fail(PCX_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    pcx_status st = validate_grid(grid);
    if (st != PCX_OK) return st;
    pcx_options o;
    st = plan_options(opts, o);
    if (st != PCX_OK) return st;
    if (o.autotune) return fail(PCX_ERR_INVALID, "autotune is not available without allocation");
    pcx_plan_s P;
    HostTables ht;
    st = plan_prepare(&P, grid, o, ht);
    if (st != PCX_OK) return st;
    const size_t tab = (ht.bytes.size() + 255) & ~(size_t)255;
    *bytes = tab + plan_layout(&P).total;
    return PCX_OK;
}

extern "C" pcx_status pcx_step_noalloc(const pcx_grid *grid, const pcx_options *opts, double dt, double rho0,
                                       const double *rho, const double *p_star, const double *u_in,
                                       const double *v_in, const double *w_in, double *u_out, double *v_out,
                                       double *w_out, double *p_out, void *stream, pcx_report *report)
{
    pcx_status st = validate_grid(grid);
    if (st != PCX_OK) return st;
    pcx_options o;
    st = plan_options(opts, o);
    if (st != PCX_OK) return st;
    if (o.autotune) return fail(PCX_ERR_INVALID, "autotune is not available without allocation");
    // host part first: a grid too large for the scratch array is rejected
    // before any device call
    pcx_plan_s P;
    HostTables ht;
    st = plan_prepare(&P, grid, o, ht);
    if (st != PCX_OK) return st;
    const size_t tab = (ht.bytes.size() + 255) & ~(size_t)255;
    const WsLayout L = plan_layout(&P);
    if (tab + L.total > (size_t)PCX_NOALLOC_SCRATCH_BYTES)
        return fail(PCX_ERR_UNSUPPORTED, "grid needs " + std::to_string(tab + L.total) +
                                             " bytes of scratch; the allocation-free step holds " +
                                             std::to_string((size_t)PCX_NOALLOC_SCRATCH_BYTES));
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(PCX_ERR_HIP, "no HIP device available");
    if (hipGetDevice(&P.device) != hipSuccess) return fail(PCX_ERR_HIP, "hipGetDevice failed");
    char *base = nullptr;
    st = scratch_ptr(P.device, &base);
    if (st != PCX_OK) return st;
    // The tables go in front of the workspace.  The copy is queued on the
    // caller's stream (after any earlier call's kernels that still read the
    // array) and waited for, since its source is this call's host memory.
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(base, ht.bytes.data(), ht.bytes.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(PCX_ERR_HIP, std::string("table upload: ") + hipGetErrorString(e));
    plan_bind(&P, ht, base, base + tab, L);
    return pcx_step(&P, dt, rho0, rho, p_star, u_in, v_in, w_in, u_out, v_out, w_out, p_out, stream, report);
}
