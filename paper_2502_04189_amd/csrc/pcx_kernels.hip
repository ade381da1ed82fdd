// pcx_kernels.hip -- __global__ entry points and their host launchers.
// One kernel per pass for a single domain (the descriptor travels by value
// in the kernel arguments), small reduction helpers, and the persistent
// multi-domain kernel of the batched form.
#include <algorithm>

#include "pcx_launch.hpp"
#include "pcx_passes.hpp"

namespace pcx {

// Logical tile of a marching stencil launch: consecutive blockIdx values go
// to different XCDs (round-robin), so the launch hands XCD x a contiguous
// range of tiles; tiles adjacent in j then share that XCD's L2 for their halo
// rows.  The grid is padded to a multiple of 8; surplus blocks exit.
__device__ __forceinline__ int xcd_tile(int ntiles)
{
    const int per = (ntiles + 7) >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// Marching stencil launches of a single domain use 512-thread workgroups
// (64 x 8 cells per plane) for the RHS and the residual, and 1024 threads
// (64 x 16) for the correction, whose halo (seven fields) is the largest.
constexpr int MT = 512;
constexpr int MTC = 1024;

template <bool TWO>
__global__ __launch_bounds__(MT) void k_rhs(Dom d)
{
    __shared__ double sm[16 + 6 * MT];
    const int t = xcd_tile(d.mg[0].ntiles);
    if (t >= d.mg[0].ntiles) return;
    pass_rhs<MT, TWO>(d, t, (char *)sm);
}

__global__ __launch_bounds__(MT) void k_resid(Dom d, int solve)
{
    __shared__ double sm[16 + 2 * MT];
    const int t = xcd_tile(d.mg[0].ntiles);
    if (t >= d.mg[0].ntiles) return;
    pass_resid<MT>(d, t, (char *)sm, solve);
}

template <typename T, int SRC, int NTH>
__global__ __launch_bounds__(NTH) void k_xfwd(Dom d)
{
    extern __shared__ __align__(16) char smem[];
    pass_xfwd<T, SRC, NTH>(d, blockIdx.x, smem);
}

// Tile of a fused stencil x pass (tile = k ntj + jt, as pass_xfwd reads it).
// The launch is ordered so that the tiles that read each other's rows run
// together on one XCD: groups of SXG consecutive j tiles, every plane k of
// a group in turn (k fastest after the SXG tiles of a plane), and each XCD
// a contiguous range of that order (consecutive workgroups go to different
// XCDs).  Returns -1 for the surplus workgroups of the padded grid.
constexpr int SXG = 4;
__host__ __device__ inline long sx_order_len(const Dom &d) { return (long)((d.ntj + SXG - 1) / SXG) * d.nz * SXG; }

__device__ __forceinline__ int sx_tile(const Dom &d)
{
    const long n = sx_order_len(d);
    const long per = (n + 7) >> 3;
    const long L = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (L >= n) return -1;
    const int jj = (int)(L % SXG);
    const long q = L / SXG;
    const int k = (int)(q % d.nz), g = (int)(q / d.nz);
    const int jt = g * SXG + jj;
    if (jt >= d.ntj) return -1;
    return k * d.ntj + jt;
}

template <typename T, int SRC, int NTH>
__global__ __launch_bounds__(NTH) void k_sx(Dom d)
{
    extern __shared__ __align__(16) char smem[];
    const int t = sx_tile(d);
    if (t < 0) return;
    pass_xfwd<T, SRC, NTH>(d, t, smem);
}

__global__ __launch_bounds__(NT) void k_smax(Dom d, int sa, int sb)
{
    __shared__ double red[2 * NT / 64];
    pass_smax(d, sa, sb, blockIdx.x, gridDim.x, (char *)red);
}

template <typename T, bool INV, int NTH>
__global__ __launch_bounds__(NTH) void k_y(Dom d)
{
    extern __shared__ __align__(16) char smem[];
    pass_y<T, INV, NTH>(d, blockIdx.x, smem);
}

template <typename T, int SMAX>
__global__ __launch_bounds__(NT) void k_z(Dom d)
{
    extern __shared__ __align__(16) char smem[];
    // lines in the reverse of the order the forward y pass wrote them, so the
    // first tiles read what the device-side cache still holds
    pass_z<T, SMAX>(d, d.nzt - 1 - (int)blockIdx.x, smem);
}

template <typename T, int MODE, int NTH>
__global__ __launch_bounds__(NTH) void k_xinv(Dom d, int solve)
{
    extern __shared__ __align__(16) char smem[];
    pass_xinv<T, MODE, NTH>(d, blockIdx.x, smem, solve);
}

template <bool TWO>
__global__ __launch_bounds__(MTC) void k_corr(Dom d, int divcheck)
{
    __shared__ double sm[16 + 7 * MTC];
    const int t = xcd_tile(d.mg[1].ntiles);
    if (t >= d.mg[1].ntiles) return;
    pass_corr<MTC, TWO>(d, t, (char *)sm, divcheck != 0);
}

__global__ __launch_bounds__(NT) void k_div(Dom d)
{
    __shared__ double red[NT / 64];
    pass_div(d, blockIdx.x, (char *)red);
}

__global__ __launch_bounds__(NT) void k_xmax(Dom d, int solve)
{
    __shared__ double red[2 * NT / 64];
    pass_xmax(d, solve, blockIdx.x, gridDim.x, (char *)red);
}

__global__ void k_pmean(Dom d, int nwg)
{
    pass_pmean(d, nwg);
}

__global__ void k_zero(unsigned long long *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Per-plane sums of p in a fixed order (deterministic), one workgroup per k.
__global__ __launch_bounds__(NT) void k_plane_sums(const double *p, int nxy, double *out)
{
    __shared__ double part[NT];
    const double *pl = p + (size_t)blockIdx.x * nxy;
    double s = 0.0;
    for (int i = threadIdx.x; i < nxy; i += NT) s += pl[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// min over doubles via an order-preserving uint64 key and atomicMin.
__device__ __forceinline__ unsigned long long dkey(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// ----------------------------------------------------------------- launch

static hipError_t lds_attr(const void *fn, size_t lds)
{
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

#define PCX_LAUNCH_B(fn, grid, block, lds, st, ...)                                     \
    do {                                                                                \
        hipError_t e_ = lds_attr((const void *)(fn), (lds));                            \
        if (e_ != hipSuccess) return e_;                                                \
        hipLaunchKernelGGL(fn, dim3(grid), dim3(block), (lds), (st), __VA_ARGS__);      \
        return hipGetLastError();                                                       \
    } while (0)
#define PCX_LAUNCH(fn, grid, lds, st, ...) PCX_LAUNCH_B(fn, grid, NT, lds, st, __VA_ARGS__)

hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

static int xcd_grid(int ntiles) { return ((ntiles + 7) >> 3) << 3; }

hipError_t launch_rhs(const Dom &d, hipStream_t s)
{
    // a second halo item per thread only when the halo outnumbers the threads
    if (5 * (d.mg[0].cti + d.mg[0].ctj) > MT) PCX_LAUNCH_B(k_rhs<true>, xcd_grid(d.mg[0].ntiles), MT, 0, s, d);
    PCX_LAUNCH_B(k_rhs<false>, xcd_grid(d.mg[0].ntiles), MT, 0, s, d);
}

hipError_t launch_resid(const Dom &d, int solve, hipStream_t s)
{
    PCX_LAUNCH_B(k_resid, xcd_grid(d.mg[0].ntiles), MT, 0, s, d, solve);
}

template <int NTH> static hipError_t launch_xfwd_t(const Dom &d, int prec, int src, size_t lds, hipStream_t s)
{
    const int grid = d.ntj * d.nz;
    if (prec == PREC_F64) {
        if (src == SRC_RHS) PCX_LAUNCH_B((k_xfwd<double, SRC_RHS, NTH>), grid, NTH, lds, s, d);
        PCX_LAUNCH_B((k_xfwd<double, SRC_RESID, NTH>), grid, NTH, lds, s, d);
    }
    if (src == SRC_RHS) PCX_LAUNCH_B((k_xfwd<float, SRC_RHS, NTH>), grid, NTH, lds, s, d);
    PCX_LAUNCH_B((k_xfwd<float, SRC_RESID, NTH>), grid, NTH, lds, s, d);
}

hipError_t launch_xfwd(const Dom &d, int prec, int src, size_t lds, hipStream_t s)
{
    return d.xth == 512 ? launch_xfwd_t<512>(d, prec, src, lds, s) : launch_xfwd_t<NT>(d, prec, src, lds, s);
}

bool sx_supported(const Dom &d)
{
    return (d.tj == 8 || d.tj == 16) && wave_plan(d.fx) && d.spart != nullptr;
}

hipError_t launch_sx(const Dom &d, int prec, int src, size_t lds, hipStream_t s)
{
    if (!sx_supported(d)) return hipErrorInvalidValue;
    const int grid = (int)(((sx_order_len(d) + 7) >> 3) << 3);
    if (d.tj == 8) {
        if (prec == PREC_F64) {
            if (src == SRC_RHS_ST) PCX_LAUNCH_B((k_sx<double, SRC_RHS_ST, 512>), grid, 512, lds, s, d);
            return hipErrorInvalidValue; // the FP64 form has no residual pass
        }
        if (src == SRC_RHS_ST) PCX_LAUNCH_B((k_sx<float, SRC_RHS_ST, 512>), grid, 512, lds, s, d);
        PCX_LAUNCH_B((k_sx<float, SRC_RESID_ST, 512>), grid, 512, lds, s, d);
    }
    if (prec == PREC_F64) {
        if (src == SRC_RHS_ST) PCX_LAUNCH_B((k_sx<double, SRC_RHS_ST, 1024>), grid, 1024, lds, s, d);
        return hipErrorInvalidValue;
    }
    if (src == SRC_RHS_ST) PCX_LAUNCH_B((k_sx<float, SRC_RHS_ST, 1024>), grid, 1024, lds, s, d);
    PCX_LAUNCH_B((k_sx<float, SRC_RESID_ST, 1024>), grid, 1024, lds, s, d);
}

hipError_t launch_smax(const Dom &d, int sa, int sb, hipStream_t s)
{
    const int v = (sslots(d) + 4 * NT - 1) / (4 * NT);
    const int nwg = v < 1 ? 1 : (v > XMAX_WG ? XMAX_WG : v);
    PCX_LAUNCH(k_smax, nwg, 0, s, d, sa, sb);
}

hipError_t launch_y(const Dom &d, int prec, bool inv, size_t lds, hipStream_t s)
{
    const int grid = d.ntk * d.nl;
    if (d.yth == 512) {
        if (prec == PREC_F64) {
            if (inv) PCX_LAUNCH_B((k_y<double, true, 512>), grid, 512, lds, s, d);
            PCX_LAUNCH_B((k_y<double, false, 512>), grid, 512, lds, s, d);
        }
        if (inv) PCX_LAUNCH_B((k_y<float, true, 512>), grid, 512, lds, s, d);
        PCX_LAUNCH_B((k_y<float, false, 512>), grid, 512, lds, s, d);
    }
    if (prec == PREC_F64) {
        if (inv) PCX_LAUNCH((k_y<double, true, NT>), grid, lds, s, d);
        PCX_LAUNCH((k_y<double, false, NT>), grid, lds, s, d);
    }
    if (inv) PCX_LAUNCH((k_y<float, true, NT>), grid, lds, s, d);
    PCX_LAUNCH((k_y<float, false, NT>), grid, lds, s, d);
}

hipError_t launch_z(const Dom &d, int prec, int smax, size_t lds, hipStream_t s)
{
    const int grid = d.nzt;
    if (prec == PREC_F64) {
        if (smax <= 4) PCX_LAUNCH((k_z<double, 4>), grid, lds, s, d);
        if (smax <= 8) PCX_LAUNCH((k_z<double, 8>), grid, lds, s, d);
        PCX_LAUNCH((k_z<double, 16>), grid, lds, s, d);
    }
    if (smax <= 4) PCX_LAUNCH((k_z<float, 4>), grid, lds, s, d);
    if (smax <= 8) PCX_LAUNCH((k_z<float, 8>), grid, lds, s, d);
    PCX_LAUNCH((k_z<float, 16>), grid, lds, s, d);
}

template <int NTH> static hipError_t launch_xinv_t(const Dom &d, int prec, int mode, int solve, size_t lds, hipStream_t s)
{
    const int grid = d.ntj * d.nz;
    if (prec == PREC_F64) {
        if (mode == XOUT_STORE) PCX_LAUNCH_B((k_xinv<double, XOUT_STORE, NTH>), grid, NTH, lds, s, d, solve);
        PCX_LAUNCH_B((k_xinv<double, XOUT_ACCUM, NTH>), grid, NTH, lds, s, d, solve);
    }
    if (mode == XOUT_STORE) PCX_LAUNCH_B((k_xinv<float, XOUT_STORE, NTH>), grid, NTH, lds, s, d, solve);
    PCX_LAUNCH_B((k_xinv<float, XOUT_ACCUM, NTH>), grid, NTH, lds, s, d, solve);
}

hipError_t launch_xinv(const Dom &d, int prec, int mode, int solve, size_t lds, hipStream_t s)
{
    return d.xth == 512 ? launch_xinv_t<512>(d, prec, mode, solve, lds, s)
                        : launch_xinv_t<NT>(d, prec, mode, solve, lds, s);
}

hipError_t launch_corr(const Dom &d, bool divcheck, hipStream_t s)
{
    if (7 * (d.mg[1].cti + d.mg[1].ctj) > MTC)
        PCX_LAUNCH_B(k_corr<true>, xcd_grid(d.mg[1].ntiles), MTC, 0, s, d, divcheck ? 1 : 0);
    PCX_LAUNCH_B(k_corr<false>, xcd_grid(d.mg[1].ntiles), MTC, 0, s, d, divcheck ? 1 : 0);
}

static int xmax_grid(const Dom &d) { return xmax_wgs(d); }

hipError_t launch_xmax(const Dom &d, int solve, hipStream_t s)
{
    PCX_LAUNCH(k_xmax, xmax_grid(d), 0, s, d, solve);
}

hipError_t launch_pmean(const Dom &d, hipStream_t s)
{
    PCX_LAUNCH_B(k_pmean, 1, 64, 0, s, d, xmax_grid(d));
}

hipError_t launch_div(const Dom &d, hipStream_t s)
{
    PCX_LAUNCH(k_div, d.ndiv_tiles, 0, s, d);
}

hipError_t launch_plane_sums(const double *p, int nxy, int nz, double *out, hipStream_t s)
{
    PCX_LAUNCH(k_plane_sums, nz, 0, s, p, nxy, out);
}

// The 8-byte key of pcx_rho_min: a file-scope device variable (one per
// device, held for the process lifetime), so the helper allocates nothing.
// Its kernels name it directly; the host reads it back by symbol.  Calls are
// serialised by the caller (a host mutex) and each one synchronises its
// stream before the next may start.
__device__ unsigned long long g_min_key;

__global__ void k_min_init() { g_min_key = ~0ull; }

__global__ __launch_bounds__(NT) void k_min_slot(const double *a, long long n)
{
    __shared__ unsigned long long part[NT / 64];
    unsigned long long m = ~0ull;
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
        unsigned long long kk = dkey(a[i]);
        m = kk < m ? kk : m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long x = __shfl_xor(m, o, 64);
        m = x < m ? x : m;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NT / 64; ++i) m = part[i] < m ? part[i] : m;
        m = part[0] < m ? part[0] : m;
        atomicMin(&g_min_key, m);
    }
}

hipError_t min_to_host(const double *a, long long n, hipStream_t s, double *out)
{
    long long blocks = (n + NT - 1) / NT;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_min_init, dim3(1), dim3(1), 0, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_min_slot, dim3((unsigned)blocks), dim3(NT), 0, s, a, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long hk = 0;
    e = hipMemcpyFromSymbolAsync(&hk, HIP_SYMBOL(g_min_key), sizeof(hk), 0, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    // invert the order-preserving key
    const unsigned long long u = (hk >> 63) ? (hk & 0x7fffffffffffffffull) : ~hk;
    __builtin_memcpy(out, &u, 8);
    return hipSuccess;
}

} // namespace pcx

namespace pcx {

// ------------------------------------------------------------------ grouped
// Kernels of the batched form: one launch runs one pass over tiles of many
// domains (a graph node per pass), each kernel with its own workgroup size
// and register budget.  The domain table is read through the constant
// address space (scalar loads, no registers held for it across the pass).
__device__ __forceinline__ const Dom &gdom(const GArgs &a, int i)
{
    return *(const Dom *)((const __attribute__((address_space(4))) Dom *)a.doms + i);
}

// Runs body(domain, tile) for the items of this workgroup; every value that
// steers the loop is wave-uniform, and a barrier separates consecutive items
// (the next item rewrites the LDS the last one read).
template <typename Body>
__device__ __forceinline__ void gloop(const GArgs &a, Body body)
{
    for (int it = blockIdx.x; it < a.nitems; it += gridDim.x) {
        const int dom = __builtin_amdgcn_readfirstlane((int)a.items[it].dom);
        const int tile = __builtin_amdgcn_readfirstlane((int)a.items[it].tile);
        if ((uint32_t)dom == GSKIP) continue;
        body(gdom(a, dom), tile);
        if (it + (int)gridDim.x < a.nitems) __syncthreads();
    }
}

template <bool TWO>
__global__ __launch_bounds__(MT) void kg_rhs(GArgs a)
{
    __shared__ double sm[16 + 6 * MT];
    gloop(a, [&](const Dom &d, int t) { pass_rhs<MT, TWO>(d, t, (char *)sm); });
}

__global__ __launch_bounds__(MT) void kg_resid(GArgs a)
{
    __shared__ double sm[16 + 2 * MT];
    gloop(a, [&](const Dom &d, int t) { pass_resid<MT>(d, t, (char *)sm, a.solve); });
}

template <bool TWO>
__global__ __launch_bounds__(MTC) void kg_corr(GArgs a)
{
    __shared__ double sm[16 + 7 * MTC];
    gloop(a, [&](const Dom &d, int t) { pass_corr<MTC, TWO>(d, t, (char *)sm, true); });
}

template <typename T, int SRC, int NTH>
__global__ __launch_bounds__(NTH) void kg_xfwd(GArgs a)
{
    extern __shared__ __align__(16) char smem[];
    gloop(a, [&](const Dom &d, int t) { pass_xfwd<T, SRC, NTH>(d, t, smem); });
}

template <typename T, bool INV, int NTH>
__global__ __launch_bounds__(NTH) void kg_y(GArgs a)
{
    extern __shared__ __align__(16) char smem[];
    gloop(a, [&](const Dom &d, int t) { pass_y<T, INV, NTH>(d, t, smem); });
}

template <typename T, int SMAX>
__global__ __launch_bounds__(NT) void kg_z(GArgs a)
{
    extern __shared__ __align__(16) char smem[];
    gloop(a, [&](const Dom &d, int t) { pass_z<T, SMAX>(d, t, smem); });
}

template <typename T, int MODE, int NTH>
__global__ __launch_bounds__(NTH) void kg_xinv(GArgs a)
{
    extern __shared__ __align__(16) char smem[];
    gloop(a, [&](const Dom &d, int t) { pass_xinv<T, MODE, NTH>(d, t, smem, a.solve); });
}

// x-inverse maxima: item tile = reduction workgroup wg of the domain
__global__ __launch_bounds__(NT) void kg_xmax(GArgs a)
{
    __shared__ double red[2 * NT / 64];
    gloop(a, [&](const Dom &d, int wg) { pass_xmax(d, a.solve, wg, xmax_wgs(d), (char *)red); });
}

__global__ __launch_bounds__(64) void kg_pmean(GArgs a)
{
    gloop(a, [&](const Dom &d, int) { pass_pmean(d, xmax_wgs(d)); });
}

int march_threads(int corr) { return corr ? MTC : MT; }

template <typename T>
static const void *group_fn(const GVariant &v)
{
    switch (v.kind) {
    case PK_RHS: return v.two ? (const void *)kg_rhs<true> : (const void *)kg_rhs<false>;
    case PK_RESID: return (const void *)kg_resid;
    case PK_CORR: return v.two ? (const void *)kg_corr<true> : (const void *)kg_corr<false>;
    case PK_XFWD_RHS: return v.nth == 512 ? (const void *)kg_xfwd<T, SRC_RHS, 512> : (const void *)kg_xfwd<T, SRC_RHS, NT>;
    case PK_XFWD_RESID:
        return v.nth == 512 ? (const void *)kg_xfwd<T, SRC_RESID, 512> : (const void *)kg_xfwd<T, SRC_RESID, NT>;
    case PK_YF: return v.nth == 512 ? (const void *)kg_y<T, false, 512> : (const void *)kg_y<T, false, NT>;
    case PK_YI: return v.nth == 512 ? (const void *)kg_y<T, true, 512> : (const void *)kg_y<T, true, NT>;
    case PK_Z:
        return v.smax <= 4 ? (const void *)kg_z<T, 4> : (v.smax <= 8 ? (const void *)kg_z<T, 8> : (const void *)kg_z<T, 16>);
    case PK_XINV_STORE:
        return v.nth == 512 ? (const void *)kg_xinv<T, XOUT_STORE, 512> : (const void *)kg_xinv<T, XOUT_STORE, NT>;
    case PK_XINV_ACCUM:
        return v.nth == 512 ? (const void *)kg_xinv<T, XOUT_ACCUM, 512> : (const void *)kg_xinv<T, XOUT_ACCUM, NT>;
    case PK_XMAX: return (const void *)kg_xmax;
    case PK_PMEAN: return (const void *)kg_pmean;
    }
    return nullptr;
}

static int group_threads(const GVariant &v)
{
    switch (v.kind) {
    case PK_RHS:
    case PK_RESID: return MT;
    case PK_CORR: return MTC;
    case PK_Z:
    case PK_XMAX: return NT;
    case PK_PMEAN: return 64;
    default: return v.nth;
    }
}

hipError_t launch_group(const GVariant &v, int prec, const GArgs &a, int grid, size_t lds, hipStream_t s)
{
    const void *fn = prec == PREC_F64 ? group_fn<double>(v) : group_fn<float>(v);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    GArgs arg = a;
    void *args[] = {&arg};
    return hipLaunchKernel(fn, dim3(grid), dim3(group_threads(v)), args, lds, s);
}

hipError_t group_occupancy(const GVariant &v, int prec, size_t lds, int *blocks_per_cu)
{
    const void *fn = prec == PREC_F64 ? group_fn<double>(v) : group_fn<float>(v);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, group_threads(v), lds);
}

} // namespace pcx

namespace pcx {

// Persistent multi-domain kernel.  Workgroups pull items (domain, phase,
// tile) from one queue in list order; the list holds every tile of phase p
// of a domain before any tile of phase p+1 of that domain, so a workgroup
// only ever waits for items already taken by running workgroups and the
// queue drains.  Each dependency wait is bounded by spin_limit polls; on
// expiry the error flag is set and the item runs anyway, so every workgroup
// exits.  Stores are released with a device-scope fence before the phase
// counter is incremented, and acquired with a device-scope fence after the
// wait.
template <typename T, int SMAX>
__global__ __launch_bounds__(NT) void k_persist(PersistArgs a)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int s_item;
    // All control flow of the work loop is uniform: the queue fetch, the
    // dependency wait and the completion count are done by the whole of wave
    // 0 under a wave-uniform branch, with only lane 0 contributing 1 to each
    // atomic, and every value that steers a branch or a loop around a barrier
    // goes through readfirstlane.  (With a per-lane loop exit or a
    // `threadIdx.x == 0` block next to the back edge, the compiler may
    // restructure the loop so that lane 0 and the rest of its wave run
    // different iterations around the barriers.)
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const unsigned one = (threadIdx.x & 63) == 0 ? 1u : 0u;
    for (;;) {
        if (wid == 0) {
            unsigned old = atomicAdd(a.head, one);
            s_item = __builtin_amdgcn_readfirstlane((int)old);
        }
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads(); // s_item is rewritten only after every wave has read it
        if (it >= a.nitems) break;
        const Item X = a.items[it];
        const int dom = __builtin_amdgcn_readfirstlane((int)X.dom);
        const int ph = __builtin_amdgcn_readfirstlane((int)X.phase);
        const int tile0 = __builtin_amdgcn_readfirstlane((int)X.tile);
        const int count = __builtin_amdgcn_readfirstlane((int)X.count);
        const unsigned slot = (unsigned)dom * a.tab.nphase + ph;
        if (ph > 0 && wid == 0) {
            const unsigned want = (unsigned)__builtin_amdgcn_readfirstlane((int)a.need[slot - 1]);
            for (unsigned polls = 0;; ++polls) {
                unsigned cur = __builtin_amdgcn_readfirstlane(
                    (int)__hip_atomic_load(&a.done[slot - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                if (cur >= want) break;
                if (polls >= a.spin_limit) {
                    atomicOr(a.err, one);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __syncthreads();
        __threadfence();
        // the descriptor table is read-only for the kernel's lifetime: read it
        // through the constant address space, so its fields are scalar loads
        // that need no registers held across the pass
        const Dom &d = *(const Dom *)((const __attribute__((address_space(4))) Dom *)a.doms + dom);
        const int sv = a.tab.solve[ph];
        const int kind = a.tab.kind[ph];
        for (int tile = tile0; tile < tile0 + count; ++tile) {
            switch (kind) {
            case PK_RHS: pass_rhs(d, tile, smem); break;
            case PK_RESID: pass_resid(d, tile, smem, sv); break;
            case PK_XFWD_RHS: pass_xfwd<T, SRC_RHS, NT, false>(d, tile, smem); break;
            case PK_XFWD_RESID: pass_xfwd<T, SRC_RESID, NT, false>(d, tile, smem); break;
            case PK_YF: pass_y<T, false, NT, false>(d, tile, smem); break;
            case PK_Z: pass_z<T, SMAX>(d, tile, smem); break;
            case PK_YI: pass_y<T, true, NT, false>(d, tile, smem); break;
            case PK_XINV_STORE: pass_xinv<T, XOUT_STORE, NT, false>(d, tile, smem, sv); break;
            case PK_XINV_ACCUM: pass_xinv<T, XOUT_ACCUM, NT, false>(d, tile, smem, sv); break;
            case PK_PMEAN:
                pass_xmax(d, sv, 0, 1, smem);
                __syncthreads();
                if (d.ppart) pass_pmean(d, 1);
                break;
            default: pass_corr(d, tile, smem, true); break;
            }
            __syncthreads(); // the next tile rewrites LDS the last one read
        }
        __threadfence();
        __syncthreads();
        if (wid == 0) atomicAdd(&a.done[slot], one);
    }
}

__global__ void k_reset(unsigned *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_reset(unsigned *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename T, int SMAX> static const void *persist_fn() { return (const void *)k_persist<T, SMAX>; }

static const void *persist_sel(int prec, int smax)
{
    if (prec == PREC_F64) return smax <= 4 ? persist_fn<double, 4>() : (smax <= 8 ? persist_fn<double, 8>() : persist_fn<double, 16>());
    return smax <= 4 ? persist_fn<float, 4>() : (smax <= 8 ? persist_fn<float, 8>() : persist_fn<float, 16>());
}

hipError_t persist_occupancy(int prec, int smax, size_t lds, int *blocks_per_cu)
{
    const void *fn = persist_sel(prec, smax);
    hipError_t e = lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, NT, lds);
}

hipError_t launch_persist(const PersistArgs &a, int prec, int smax, int blocks, size_t lds, hipStream_t s)
{
    if (prec == PREC_F64) {
        if (smax <= 4) PCX_LAUNCH((k_persist<double, 4>), blocks, lds, s, a);
        if (smax <= 8) PCX_LAUNCH((k_persist<double, 8>), blocks, lds, s, a);
        PCX_LAUNCH((k_persist<double, 16>), blocks, lds, s, a);
    }
    if (smax <= 4) PCX_LAUNCH((k_persist<float, 4>), blocks, lds, s, a);
    if (smax <= 8) PCX_LAUNCH((k_persist<float, 8>), blocks, lds, s, a);
    PCX_LAUNCH((k_persist<float, 16>), blocks, lds, s, a);
}

} // namespace pcx
