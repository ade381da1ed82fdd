// pcx_dev.hpp -- device-side building blocks of the pressure-correction step
// for gfx950 (CDNA4, wave64).
//
// The step (CaNS-Fizzy, "Methods and Implementation strategy"): the
// right-hand side of the constant-coefficient pressure equation obtained by
// the splitting, a fast direct solve (real FFT in x, complex FFT in y, one
// tridiagonal solve in z per wavenumber pair on a possibly stretched z grid),
// and the staggered velocity correction.
//
// Spectral data live in two workspace layouts, chosen so that every pass
// reads or writes long contiguous runs and does its corner turn in LDS:
//   S1 "y-columns": ((k*NL + l)*NY + j)   one (k,l) column contiguous in j/m
//   S2 "z-lines"  : ((l*NY + m)*NZ + k)   one (l,m) line contiguous in k
// with NL = nx/2 + 1 half-spectrum x modes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcx {

constexpr int NT = 256;       // threads per workgroup (4 wave64)
constexpr int MAXST = 16;     // max FFT stages
constexpr int PPT = 16;       // complex points per thread per FFT stage (at NT threads)
constexpr int MAXPTS = PPT * NT; // most complex points one workgroup transforms at once
constexpr int NSTAT = 64;     // reduction slots per domain
constexpr int MAXIT = 12;     // max refinement solves tracked

enum { PREC_F64 = 0, PREC_F32 = 1 };
// boundary conditions: periodic; wall (zero normal velocity, Neumann
// pressure); homogeneous Dirichlet pressure (the solve alone)
enum { BC_PER = 0, BC_WALL = 1, BC_DIR = 2 };
// x-transform source: the stored f or r, or (the fused forms) f or r
// evaluated by the stencil inside the x pass, never stored (f is still
// stored in the refined form, whose residual needs it)
enum { SRC_RHS = 0, SRC_RESID = 1, SRC_RHS_ST = 2, SRC_RESID_ST = 3 };
enum { XOUT_STORE = 0, XOUT_ACCUM = 1 };

// reduction slots (uint64 bit patterns of non-negative doubles, atomicMax)
enum {
    ST_FINF = 0,      // ||f||inf
    ST_DIV = 1,       // max |D u_out|
    ST_NONFIN = 2,    // max over outputs of |.| (NaN/Inf show up here)
    ST_SOLVE0 = 8     // per solve s: [8+4s] ||rhs||, [9+4s] ||e||, [10+4s] ||p||
};

// Division by a runtime constant d < 2^16 for numerators a < 2^16 via a
// multiply-high: q = umulhi(a, m), m = floor(2^32/d) + 1 (exact when a*d < 2^32).
struct FastDiv {
    uint32_t d, m;
};
__device__ __forceinline__ uint32_t fdiv(uint32_t a, FastDiv f) { return f.d == 1 ? a : __umulhi(a, f.m); }

struct FftDesc {
    int n;                 // length
    int nst;               // number of stages
    int rad[MAXST];        // radix of each stage (2, 3, 4 or 8)
    int ns[MAXST];         // product of the radices before the stage
    int tws[MAXST];        // table stride n / (ns * rad)
    FastDiv dnb[MAXST];    // division by n / rad
    FastDiv dns[MAXST];    // division by ns
    const void *tw;        // n roots exp(-2 pi i e / n), T2
};

// Tiling of a marching stencil launch: TI x TJ cells of a plane (one thread
// per column) over chunks of ckc planes; ntiles = cnti cntj cnk.
struct MGeo {
    int cti, ctj, cnti, cntj, ckc, cnk, ntiles;
    FastDiv dcti;
};

// Everything one domain needs on the device.
struct Dom {
    int nx, ny, nz, nl, M;            // M = nx/2 (half-length complex FFT)
    int bcx, bcy, bcz;
    int nosing;                       // a Dirichlet direction: no singular (0, 0) mode
    int tj, ntj;                      // x-pass rows per tile, j tiles
    int tk, ntk;                      // y-pass columns per tile, k tiles
    int zg, zlpw, nzt;                // z lanes per line, lines per WG, z tiles
    MGeo mg[2];                       // marching tiles: [0] RHS and residual, [1] correction
    int ndiv_tiles;                   // divergence-only tiles (NT cells each)
    int mth, yth, xth;                // threads of the marching, y and x workgroups
    FastDiv dnx, dny, dtj, dtk, dnyc, dM, dH1, dM1, dhy; // dH1: M/2+1, dM1: M+1, dhy: ny/2
    double dx, dy, idx, idy, dt, rho0, irho0, lz, scale;
    // z tables (FP64): dzf, 1/dzf, 1/dzc, rho interpolation weights
    const double *dzf, *idzf, *idzc, *rzlo, *rzhi;
    // z tridiagonal coefficients and eigenvalues in the solve precision
    const void *za, *zb, *zc, *dzf_s, *lamx, *lamy;
    const void *twr;                  // post-twiddles exp(-2 pi i l / nx), l in [0, M]
    const void *dctx, *dcty;          // wall x / wall y: exp(-i pi k / (2N)), else NULL
    FftDesc fx, fy;
    // fields
    const double *rho, *ps, *u, *v, *w;
    double *uo, *vo, *wo, *po;
    double *f;                        // FP64 right-hand side
    double *r;                        // FP64 residual f - L p (refined form)
    void *s1, *s2;                    // spectral workspaces
    unsigned long long *stats;        // NSTAT slots
    double *ppart;                    // per x-tile wave dzf-weighted sums of p
    double *pmean;                    // [0]: volume mean of p after the last xinv pass
    double *xpart;                    // per x-tile wave max |update|, max |p| (NULL: atomics)
    double *spart;                    // per x-tile wave max |f| or |r| of the fused stencil passes
};

// Partial-result slots of the x inverse: one per wave of each x tile.  They
// are reduced by at most XMAX_WG workgroups, whose sums of p go to
// pmean[8 ..]; pmean[0] is the mean (PMEAN_LEN doubles in all).
constexpr int XMAX_WG = 64;
constexpr int PMEAN_LEN = 8 + XMAX_WG;
__host__ __device__ inline int xslots(const Dom &d) { return d.ntj * d.nz * (d.xth >> 6); }
// partial-maximum slots of the fused stencil x passes: one per wave, one
// wave per row of a tile
__host__ __device__ inline int sslots(const Dom &d) { return d.ntj * d.nz * d.tj; }
// workgroups of the reduction of those slots (pass_xmax), at most XMAX_WG
__host__ __device__ inline int xmax_wgs(const Dom &d)
{
    const int v = (xslots(d) + 4 * NT - 1) / (4 * NT);
    return v < 1 ? 1 : (v > XMAX_WG ? XMAX_WG : v);
}


// ------------------------------------------------------------ complex math
template <typename T> struct T2;
template <> struct T2<double> { using type = double2; };
template <> struct T2<float> { using type = float2; };
template <typename T> using c2 = typename T2<T>::type;

// Store of a streamed output (written once, not read again by the pass that
// writes it): non-temporal, so it does not displace lines still being read.
__device__ __forceinline__ void st_stream(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(double2 *p, double2 v)
{
    typedef double v2d __attribute__((ext_vector_type(2)));
    v2d w = {v.x, v.y};
    __builtin_nontemporal_store(w, (v2d *)p);
}
__device__ __forceinline__ void st_stream(float2 *p, float2 v)
{
    typedef float v2f __attribute__((ext_vector_type(2)));
    v2f w = {v.x, v.y};
    __builtin_nontemporal_store(w, (v2f *)p);
}

// Non-temporal load, for a streamed input no other tile of the pass reads
// (inputs that neighbouring tiles re-read as halo stay cached normally).
__device__ __forceinline__ double ld_stream(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
    typedef double v2d __attribute__((ext_vector_type(2)));
    v2d w = __builtin_nontemporal_load((const v2d *)p);
    return double2{w.x, w.y};
}
__device__ __forceinline__ float2 ld_stream(const float2 *p)
{
    typedef float v2f __attribute__((ext_vector_type(2)));
    v2f w = __builtin_nontemporal_load((const v2f *)p);
    return float2{w.x, w.y};
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return {a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return {a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename C> __device__ __forceinline__ C cconj(C a) { return {a.x, -a.y}; }
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot90(C a) { return INV ? C{-a.y, a.x} : C{a.y, -a.x}; }

// ---------------------------------------------------------- radix kernels
// In-register DFT of R points; forward uses exp(-2 pi i/R), INV the conjugate.
template <bool INV, typename C> __device__ __forceinline__ void bfly2(C &a0, C &a1)
{
    C t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <bool INV, typename C, typename T> __device__ __forceinline__ void bfly3(C &a0, C &a1, C &a2)
{
    const T c = T(-0.5);
    const T s = T(0.86602540378443864676); // sqrt(3)/2
    C sm = cadd(a1, a2), df = csub(a1, a2);
    C b = {a0.x + c * sm.x, a0.y + c * sm.y};
    // forward: y1 = b - i s df, y2 = b + i s df
    C isd = {-s * df.y, s * df.x}; // i * s * df
    a0 = cadd(a0, sm);
    if (INV) { a1 = cadd(b, isd); a2 = csub(b, isd); }
    else { a1 = csub(b, isd); a2 = cadd(b, isd); }
}

template <bool INV, typename C> __device__ __forceinline__ void bfly4(C &a0, C &a1, C &a2, C &a3)
{
    C t0 = cadd(a0, a2), t1 = csub(a0, a2);
    C t2 = cadd(a1, a3), t3 = rot90<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <bool INV, typename C, typename T> __device__ __forceinline__ void bfly8(C *a)
{
    const T r = T(0.70710678118654752440); // 1/sqrt(2)
    C e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    C o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    bfly4<INV>(e0, e1, e2, e3);
    bfly4<INV>(o0, o1, o2, o3);
    // twiddles W8^k on the odd half
    C w1 = INV ? C{r * (o1.x - o1.y), r * (o1.x + o1.y)} : C{r * (o1.x + o1.y), r * (o1.y - o1.x)};
    C w2 = rot90<INV>(o2);
    C w3 = INV ? C{-r * (o3.x + o3.y), r * (o3.x - o3.y)} : C{r * (o3.y - o3.x), -r * (o3.x + o3.y)};
    a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
    a[1] = cadd(e1, w1); a[5] = csub(e1, w1);
    a[2] = cadd(e2, w2); a[6] = csub(e2, w2);
    a[3] = cadd(e3, w3); a[7] = csub(e3, w3);
}

template <bool INV, int R, typename C, typename T> __device__ __forceinline__ void bfly(C *a)
{
    if constexpr (R == 2) bfly2<INV>(a[0], a[1]);
    else if constexpr (R == 3) bfly3<INV, C, T>(a[0], a[1], a[2]);
    else if constexpr (R == 4) bfly4<INV>(a[0], a[1], a[2], a[3]);
    else bfly8<INV, C, T>(a);
}

// LDS position of element e of a line: one spare slot after every 8
// elements, so that the stride-R stores of the early Stockham stages (and the
// strided corner-turn accesses) spread over the LDS banks.
__device__ __forceinline__ int pidx(int e) { return e + (e >> 3); }
// Line stride for n elements: padded length rounded to 16 slots, plus one,
// so consecutive lines start in different banks.
__host__ __device__ constexpr int lds_line(int n) { return (((n - 1) + ((n - 1) >> 3) + 1 + 15) & ~15) + 1; }

// Twiddle table of a length-n FFT as held in LDS: for even n only the first
// n/2 roots, since W_n^(e + n/2) = -W_n^e.
__host__ __device__ constexpr int tw_half(int n) { return (n & 1) ? n : n / 2; }

// One Stockham autosort stage over `nlines` LDS lines of length n (line
// stride ldb, padded positions): butterfly b = (line, j), j in [0, n/R):
//   inputs  x[line][j + r n/R], r < R
//   twiddle W_{ns R}^{(j mod ns) r}
//   outputs y[line][(j / ns) ns R + (j mod ns) + r ns]
// Results are held in registers across a barrier, so the stage is in place.
// Twiddles come from an LDS copy of the first th roots (see TwStage).
template <typename T, bool INV, int R, int NTH>
__device__ __forceinline__ void fft_stage(c2<T> *buf, int ldb, int nlines, const FftDesc &fd, int s,
                                          const c2<T> *tw, int th)
{
    using C = c2<T>;
    constexpr int K = (MAXPTS / NTH + R - 1) / R;
    const int nb = fd.n / R;
    const int total = nlines * nb;
    const int ns = fd.ns[s];
    const int tws = fd.tws[s];
    C v[K][R];
    int lo[K], oo[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        int b = threadIdx.x + t * NTH;
        lo[t] = -1;
        oo[t] = 0;
        if (b < total) {
            int line = (int)fdiv((uint32_t)b, fd.dnb[s]);
            int j = b - line * nb;
            const C *src = buf + line * ldb;
#pragma unroll
            for (int r = 0; r < R; ++r) v[t][r] = src[pidx(j + r * nb)];
            int jq = (int)fdiv((uint32_t)j, fd.dns[s]);
            int jm = j - jq * ns;
            if (ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const int e = jm * r * tws;
                    C w = e < th ? tw[e] : C{-tw[e - th].x, -tw[e - th].y};
                    if (INV) w.y = -w.y;
                    v[t][r] = cmul(v[t][r], w);
                }
            }
            lo[t] = line * ldb;
            oo[t] = jq * ns * R + jm;
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < K; ++t) {
        if (lo[t] >= 0) {
            bfly<INV, R, C, T>(v[t]);
            C *dst = buf + lo[t];
#pragma unroll
            for (int r = 0; r < R; ++r) dst[pidx(oo[t] + r * ns)] = v[t][r];
        }
    }
    __syncthreads();
}

// Complex FFT (unnormalised) of nlines LDS lines; all threads participate.
// Entry and exit are barrier-separated from the caller's LDS traffic.
template <typename T, bool INV, int NTH = NT>
__device__ void lds_fft(c2<T> *buf, int ldb, int nlines, const FftDesc &fd, const c2<T> *tw)
{
    const int th = tw_half(fd.n);
    for (int s = 0; s < fd.nst; ++s) {
        switch (fd.rad[s]) {
        case 2: fft_stage<T, INV, 2, NTH>(buf, ldb, nlines, fd, s, tw, th); break;
        case 3: fft_stage<T, INV, 3, NTH>(buf, ldb, nlines, fd, s, tw, th); break;
        case 4: fft_stage<T, INV, 4, NTH>(buf, ldb, nlines, fd, s, tw, th); break;
        default: fft_stage<T, INV, 8, NTH>(buf, ldb, nlines, fd, s, tw, th); break;
        }
    }
}

// Copies a table of n complex values into LDS (no barrier: the caller's next
// barrier publishes them), in two halves: fetch() reads this thread's entry
// into a register, put() stores it, so a pass can issue the read ahead of its
// tile's reads and store it after them (one memory latency instead of two).
// Entries beyond the first NTH are copied by put() directly.  TwStage: the
// first tw_half(n) roots of an FFT descriptor.
template <typename T, int NTH>
struct TabStage {
    c2<T> v;
    __device__ __forceinline__ void fetch(const c2<T> *tab, int n) { v = tab[min((int)threadIdx.x, n - 1)]; }
    __device__ __forceinline__ void put(c2<T> *lds, const c2<T> *tab, int n) const
    {
        if ((int)threadIdx.x < n) lds[threadIdx.x] = v;
        for (int e = threadIdx.x + NTH; e < n; e += NTH) lds[e] = tab[e];
    }
};
template <typename T, int NTH>
struct TwStage {
    TabStage<T, NTH> t;
    __device__ __forceinline__ void fetch(const FftDesc &fd) { t.fetch((const c2<T> *)fd.tw, tw_half(fd.n)); }
    __device__ __forceinline__ void put(c2<T> *ltw, const FftDesc &fd) const
    {
        t.put(ltw, (const c2<T> *)fd.tw, tw_half(fd.n));
    }
};

// ------------------------------------------------------ wave-level FFT
// Lengths 256 and 512 (plans 4.4.4.4 or 8.8.4, and 8.8.8; see wave_plan) can also be
// transformed by one wave per line: butterfly j of a stage is lane j mod 64,
// every index is a compile-time shift or mask, and no workgroup barrier is
// needed between stages (the LDS operations of one wave execute in order;
// the fences keep the compiler from moving them across a stage boundary).
// Same arithmetic, in the same order, as fft_stage with the same radices.
__host__ __device__ constexpr bool wave_len(int n) { return n == 256 || n == 512; }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS position of element e + r S: for S a multiple of 8 the padding adds
// exactly S/8 per step, so the offsets are constants.
template <int S> __device__ __forceinline__ int pstep(int pe, int e, int r)
{
    if constexpr (S % 8 == 0) return pe + r * (S + S / 8);
    else return pidx(e + r * S);
}

template <typename T, bool INV, int N, int R, int NS>
__device__ __forceinline__ void wstage(c2<T> *ln, const c2<T> *tw, int lane)
{
    using C = c2<T>;
    constexpr int NB = N / R, TS = N / (NS * R);
    static_assert(NB <= 64, "one butterfly per lane");
    const int j = lane;
    const bool on = NB == 64 || j < NB;
    C v[R];
    if (on) {
        const int pj = pidx(j);
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = ln[pstep<NB>(pj, j, r)];
        if constexpr (NS > 1) {
            const int jm = j & (NS - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int e = jm * r * TS;
                C w = e < N / 2 ? tw[e] : C{-tw[e - N / 2].x, -tw[e - N / 2].y};
                if (INV) w.y = -w.y;
                v[r] = cmul(v[r], w);
            }
        }
    }
    wave_sync();
    if (on) {
        bfly<INV, R, C, T>(v);
        const int o = (j / NS) * NS * R + (j & (NS - 1));
        const int po = pidx(o);
#pragma unroll
        for (int r = 0; r < R; ++r) ln[pstep<NS>(po, o, r)] = v[r];
    }
    wave_sync();
}

// Whole line of length n (wave_len(n)) by the calling wave.
// The plans the wave path has: 256 as 4.4.4.4 (every lane holds one
// butterfly in every stage) or 8.8.4, 512 as 8.8.8.
__host__ __device__ inline bool wave_plan(const FftDesc &fd)
{
    if (fd.n == 512) return fd.nst == 3 && fd.rad[0] == 8 && fd.rad[1] == 8 && fd.rad[2] == 8;
    if (fd.n != 256) return false;
    if (fd.nst == 4) return fd.rad[0] == 4 && fd.rad[1] == 4 && fd.rad[2] == 4 && fd.rad[3] == 4;
    return fd.nst == 3 && fd.rad[0] == 8 && fd.rad[1] == 8 && fd.rad[2] == 4;
}

template <typename T, bool INV>
__device__ __forceinline__ void wave_fft(c2<T> *ln, const c2<T> *tw, const FftDesc &fd, int lane)
{
    wave_sync();
    if (fd.n == 256 && fd.nst == 4) {
        wstage<T, INV, 256, 4, 1>(ln, tw, lane);
        wstage<T, INV, 256, 4, 4>(ln, tw, lane);
        wstage<T, INV, 256, 4, 16>(ln, tw, lane);
        wstage<T, INV, 256, 4, 64>(ln, tw, lane);
    } else if (fd.n == 256) {
        wstage<T, INV, 256, 8, 1>(ln, tw, lane);
        wstage<T, INV, 256, 8, 8>(ln, tw, lane);
        wstage<T, INV, 256, 4, 64>(ln, tw, lane);
    } else {
        wstage<T, INV, 512, 8, 1>(ln, tw, lane);
        wstage<T, INV, 512, 8, 8>(ln, tw, lane);
        wstage<T, INV, 512, 8, 64>(ln, tw, lane);
    }
}

// ------------------------------------------------------- staged copies
// Moves `total` elements with all of a thread's reads of one round issued
// before its first write, CNT per thread per round: a global -> LDS copy
// then waits for one memory latency per round instead of one per element.
// get(e) returns element e, put(e, v) stores it.  The reads are not under a
// branch (a worker past the end re-reads the last element) and stay ahead of
// the writes: a read in a conditional block makes the compiler wait for
// every earlier read before it, which would serialise the round.
// staged_copy_t: the same for worker `tid` of STRIDE workers (a wave's lanes).
template <int STRIDE, int CNT, typename V, typename Get, typename Put>
__device__ __forceinline__ void staged_copy_t(int tid, int total, Get get, Put put)
{
    auto round = [&](int b) {
        V v[CNT];
#pragma unroll
        for (int t = 0; t < CNT; ++t) v[t] = get(min(b + tid + t * STRIDE, total - 1));
        // keeps the compiler from sinking a read into the conditional write
        // that consumes it
        asm volatile("" ::: "memory");
#pragma unroll
        for (int t = 0; t < CNT; ++t) {
            int e = b + tid + t * STRIDE;
            if (e < total) put(e, v[t]);
        }
    };
    // the first round is peeled: at the head of a loop the compiler cannot
    // tell which reads of the previous round are still pending, and waits
    // for all of them (including reads the caller issued just before)
    if (total <= 0) return;
    round(0);
    for (int b = CNT * STRIDE; b < total; b += CNT * STRIDE) round(b);
}

template <int NTH, int CNT, typename V, typename Get, typename Put>
__device__ __forceinline__ void staged_copy(int total, Get get, Put put)
{
    staged_copy_t<NTH, CNT, V>((int)threadIdx.x, total, get, put);
}

// ------------------------------------------------------------- reductions
// Block-wide max of non-negative values (NaN propagates), then one atomicMax
// on the uint64 bit pattern (order-preserving for non-negative doubles).
template <int NTH = NT>
__device__ __forceinline__ void block_max_to(unsigned long long *slot, double v, double *red)
{
    // keep NaN visible: fmax drops NaN, so map NaN to +Inf-plus pattern
    if (v != v) v = __longlong_as_double(0x7ff8000000000000LL);
    double w = v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double x = __shfl_xor(w, o, 64);
        w = (x != x || x > w) ? x : w;
    }
    int wid = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wid] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int i = 1; i < NTH / 64; ++i) m = (red[i] != red[i] || red[i] > m) ? red[i] : m;
        atomicMax(slot, (unsigned long long)__double_as_longlong(m));
    }
}

// Two block-wide maxima in one pass (one pair of barriers), valid in thread
// 0.  Same NaN handling as block_max_to.
template <int NTH = NT>
__device__ __forceinline__ void block_max2(double &a, double &b, double *red)
{
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    if (a != a) a = qnan;
    if (b != b) b = qnan;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double x = __shfl_xor(a, o, 64), y = __shfl_xor(b, o, 64);
        a = (x != x || x > a) ? x : a;
        b = (y != y || y > b) ? y : b;
    }
    const int wid = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[wid] = a; red[NTH / 64 + wid] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ma = red[0], mb = red[NTH / 64];
        for (int i = 1; i < NTH / 64; ++i) {
            const double x = red[i], y = red[NTH / 64 + i];
            ma = (x != x || x > ma) ? x : ma;
            mb = (y != y || y > mb) ? y : mb;
        }
        a = ma;
        b = mb;
    }
}

// block_max2, then one atomicMax per slot (either slot may be NULL).
template <int NTH = NT>
__device__ __forceinline__ void block_max2_to(unsigned long long *sa, double a, unsigned long long *sb, double b,
                                              double *red)
{
    block_max2<NTH>(a, b, red);
    if (threadIdx.x == 0) {
        if (sa) atomicMax(sa, (unsigned long long)__double_as_longlong(a));
        if (sb) atomicMax(sb, (unsigned long long)__double_as_longlong(b));
    }
}

// Wave-wide reductions by DPP lane moves (VALU operations, no LDS round
// trips): xor 1 and xor 2 within quads, mirrors within 8 and 16 lanes, then
// row 0 -> row 1, row 2 -> row 3 and row 1 -> rows 2, 3 broadcasts.  The
// result is complete in lane 63 only (wave_last reads it); the combination
// order is fixed, so sums are deterministic.  A lane a move does not write
// keeps its own value.
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, RM, 0xf, false);
    const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, RM, 0xf, false);
    return __hiloint2double(h2, l2);
}

template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op)
{
    v = op(v, dpp_d<0xB1>(v));       // quad_perm [1,0,3,2]
    v = op(v, dpp_d<0x4E>(v));       // quad_perm [2,3,0,1]
    v = op(v, dpp_d<0x141>(v));      // row_half_mirror
    v = op(v, dpp_d<0x140>(v));      // row_mirror
    v = op(v, dpp_d<0x142, 0xA>(v)); // row_bcast:15
    v = op(v, dpp_d<0x143, 0xC>(v)); // row_bcast:31
    return v;
}

// value of lane 63, in every lane
__device__ __forceinline__ double wave_last(double v)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// max of non-negative values, NaN propagating (as block_max2)
__device__ __forceinline__ double wave_max1(double a)
{
    if (a != a) a = __longlong_as_double(0x7ff8000000000000LL);
    return wave_last(wave_reduce(a, [](double x, double y) { return (y != y || y > x) ? y : x; }));
}

__device__ __forceinline__ double wave_sum(double v)
{
    return wave_last(wave_reduce(v, [](double x, double y) { return x + y; }));
}

// Deterministic block-wide sum (fixed shuffle tree, then waves in order);
// the result is valid in thread 0.
template <int NTH = NT>
__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NTH / 64; ++i) t += red[i];
    return t;
}

// -------------------------------------------------------------- stencils
// 1/x for positive normal x: hardware estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r) (about one ulp; no scaling is needed for the
// densities and spacings this is used on).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Reciprocal in the solve precision: FP64 as rcp_nr; FP32 correctly rounded
// (the FP32 solve's accuracy sets how fast the refinement contracts).
__device__ __forceinline__ float rcp_t(float x) { return 1.0f / x; }
__device__ __forceinline__ double rcp_t(double x) { return rcp_nr(x); }

// Corrected +x (dir 0), +y (1) or +z (2) face velocity of cell (i,j,k):
// u* - dt [ (1/rho0) G p + (1/rho_face - 1/rho0) G p* ], 0 on wall faces.
__device__ __forceinline__ double corr_face(const Dom &d, int dir, int i, int j, int k)
{
    const int nx = d.nx, ny = d.ny, nz = d.nz, sz = nx * ny;
    const int c = k * sz + j * nx + i;
    int o;
    double h, irf;
    const double *rho = d.rho + c;
    if (dir == 0) {
        if (d.bcx == BC_WALL && i == nx - 1) return 0.0;
        o = (i == nx - 1) ? -(nx - 1) : 1;
        h = d.idx;
        irf = 2.0 * rcp_nr(rho[0] + rho[o]);
    } else if (dir == 1) {
        if (d.bcy == BC_WALL && j == ny - 1) return 0.0;
        o = (j == ny - 1) ? -(ny - 1) * nx : nx;
        h = d.idy;
        irf = 2.0 * rcp_nr(rho[0] + rho[o]);
    } else {
        if (d.bcz == BC_WALL && k == nz - 1) return 0.0;
        o = (k == nz - 1) ? -(nz - 1) * sz : sz;
        h = d.idzc[k];
        irf = rcp_nr(rho[0] * d.rzlo[k] + rho[o] * d.rzhi[k]);
    }
    const double *vin = (dir == 0 ? d.u : (dir == 1 ? d.v : d.w)) + c;
    const double *p = d.po + c, *ps = d.ps + c;
    const double gp = (p[o] - p[0]) * h;
    const double gs = (ps[o] - ps[0]) * h;
    return vin[0] - d.dt * (d.irho0 * gp + (irf - d.irho0) * gs);
}

} // namespace pcx
