/*
 * pcx.h -- C ABI of the MI355X (gfx950) pressure-correction library.
 *
 * The library computes the pressure-correction step of one Runge-Kutta
 * substep of a one-fluid two-phase incompressible solver (CaNS-Fizzy,
 * "Methods and Implementation strategy"): second-order finite differences
 * on a staggered Cartesian grid, a projection enforcing mass conservation,
 * and a splitting that replaces the variable-coefficient pressure equation
 * by a constant-coefficient one, solved directly with transforms in x and y
 * and a tridiagonal solve in z.  For a grid with cell-centred density rho,
 * extrapolated pressure p*, predicted face velocity u* and a scalar rho0:
 *
 *   f     = (rho0/dt) D u* + D[(1 - rho0/rho_face) G p*]
 *   L p   = f - <f>,  <p> = 0           (L = D G, <.> volume-weighted mean)
 *   u_out = u* - dt [ (1/rho0) G p + (1/rho_face - 1/rho0) G p* ]
 *
 * on every non-wall face, and u_out = 0 on wall faces.  rho_face is the
 * arithmetic mean of the two adjacent cells in x and y and the linear
 * interpolation to the face in z.
 *
 * Layout of every field argument: FP64, C-contiguous [nz][ny][nx] (x
 * fastest), nx*ny*nz elements, device memory of the plan's device.
 * u[k][j][i] is the +x face of cell (i,j,k), v the +y face, w the +z face.
 * In a wall direction the last face index (e.g. w[nz-1][..][..]) is the wall
 * face: it is ignored on input and written 0 on output; the face below cell 0
 * is an implicit 0.
 *
 * Errors: every call returns a pcx_status and never throws or aborts;
 * pcx_last_error() gives a thread-local message for the last failure.
 * Streams are passed as `void *` holding a hipStream_t (NULL = the null
 * stream).  The library allocates device memory only in *_create calls.
 */
#ifndef PCX_H
#define PCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCX_ABI_VERSION 1

typedef enum {
    PCX_OK = 0,
    PCX_ERR_INVALID = 1,       /* bad argument, descriptor, or aliasing      */
    PCX_ERR_UNSUPPORTED = 2,   /* valid, but a size the library does not run */
    PCX_ERR_NOMEM = 3,         /* device or host allocation failed            */
    PCX_ERR_HIP = 4,           /* HIP runtime failure, including "no device"  */
    PCX_ERR_NOT_CONVERGED = 5, /* refinement missed rtol; outputs written     */
    PCX_ERR_NONFINITE = 6      /* NaN/Inf found in the outputs (check_finite) */
} pcx_status;

/* Boundary condition of a direction.  WALL: zero normal velocity and zero
 * normal pressure gradient (cosine transform in x/y, Neumann rows in z).
 * DIRICHLET: p = 0 on the boundary faces (ghost value -p; sine transform in
 * x/y, Dirichlet rows in z); accepted by pcx_plan_create for
 * pcx_poisson_solve only -- pcx_step, the batch and the substep reject it
 * (UNSUPPORTED), since what the velocity correction does on an open
 * boundary is not part of the method. */
typedef enum { PCX_BC_PERIODIC = 0, PCX_BC_WALL = 1, PCX_BC_DIRICHLET = 2 } pcx_bc;

/* FP64: every pass in double precision.
 * FP32_REFINED: transforms and tridiagonal solves in single precision inside
 * an iterative refinement whose right-hand side, residual (7-point operator
 * with variable z spacing), pressure accumulation, velocity correction and
 * divergence check are double precision. */
typedef enum { PCX_FP64 = 0, PCX_FP32_REFINED = 1 } pcx_precision;

/* Grid and boundary descriptor.  x and y are uniform (dx = lx/nx,
 * dy = ly/ny); z is given by its nz+1 strictly increasing face coordinates
 * zf (host memory, copied at plan creation).  Rules: nx, ny, nz >= 2;
 * nx even (its transform is a half-length complex FFT, also for the cosine
 * transform of a wall x); ny even when periodic (any ny with a wall in y);
 * transform lengths nx, ny of the form 2^a 3^b
 * and at most 4096 (else UNSUPPORTED); nz <= 1024 (else UNSUPPORTED);
 * nx*ny*nz <= 2^31 - 1 cells (else UNSUPPORTED: cell offsets in the kernels
 * are 32-bit). */
typedef struct {
    int32_t nx, ny, nz;
    double lx, ly;
    const double *zf;
    int32_t bc_x, bc_y, bc_z; /* pcx_bc */
} pcx_grid;

/* Options.  rtol: stop test of the refinement on ||f - L p||inf/||f||inf
 * (default 1e-10).  fixed_iters: FP32 solves always run per step (0 = the
 * default, 3); with a report the single-domain step keeps refining, up to
 * max_iters solves (default 8), until rtol is met.  check_finite: scan
 * outputs for NaN/Inf when a report is requested.  autotune: time candidate
 * tile shapes, FFT radix splits and z lanes per line for each distinct grid
 * (size class) at create time; tune_cache: optional path of a text cache of
 * those choices, read at create time and (re)written after tuning. */
typedef struct {
    int32_t precision; /* pcx_precision */
    double rtol;
    int32_t max_iters;
    int32_t fixed_iters;
    int32_t check_finite;
    int32_t autotune;
    const char *tune_cache;
} pcx_options;

/* Diagnostics of one step.  rel_residual = max|D u_out| / ((dt/rho0)
 * ||f||inf) equals ||f - L p||inf/||f||inf (D u_out = (dt/rho0)(f - L p)). */
typedef struct {
    int32_t solves;      /* number of transform + tridiagonal solves     */
    int32_t converged;   /* 1 if rel_residual <= rtol (FP32_REFINED)     */
    double f_inf;        /* ||f||inf                                      */
    double rel_residual; /* as above                                      */
    double max_div_abs;  /* max |D u_out|                                 */
    double max_div_rel;  /* same value as rel_residual                    */
    double mean_p;       /* volume-weighted mean of p (gauge check)       */
    double last_update_inf; /* ||e||inf of the last refinement update     */
} pcx_report;

typedef struct pcx_plan_s *pcx_plan;
typedef struct pcx_batch_s *pcx_batch;

/* Validates the grid, builds the tables (eigenvalues, z coefficients,
 * twiddles) and allocates the plan's workspace on the current HIP device.
 * opts may be NULL (FP64 defaults).  Errors: INVALID, UNSUPPORTED, NOMEM,
 * HIP.  On error *out is NULL. */
pcx_status pcx_plan_create(const pcx_grid *grid, const pcx_options *opts, pcx_plan *out);

/* Device bytes held by the plan (workspace and tables). */
pcx_status pcx_plan_workspace_bytes(pcx_plan plan, size_t *bytes);

/* One pressure-correction step.  dt > 0 is the substep's time step, rho0 > 0
 * the splitting density (normally min(rho), see pcx_rho_min).  Inputs rho,
 * p_star, u_in, v_in, w_in; outputs u_out, v_out, w_out, p_out (all device
 * FP64 [nz][ny][nx]).  u_out may equal u_in (likewise v, w): the update is
 * then in place.  p_out must not alias any input or velocity output
 * (INVALID).  With report == NULL the call only enqueues work on `stream`;
 * with a report it synchronizes the stream and fills it.  Returns
 * NOT_CONVERGED (outputs written) when a refined step misses rtol within
 * max_iters, NONFINITE when check_finite finds NaN/Inf. */
pcx_status pcx_step(pcx_plan plan, double dt, double rho0,
                    const double *rho, const double *p_star,
                    const double *u_in, const double *v_in, const double *w_in,
                    double *u_out, double *v_out, double *w_out, double *p_out,
                    void *stream, pcx_report *report);

pcx_status pcx_plan_destroy(pcx_plan plan);

/* The plan's constant-coefficient Poisson solve alone (the direct solver of
 * the method: transforms in x and y, tridiagonal solves in z): L p = f for
 * the 7-point operator with variable z spacing and the plan's boundary
 * conditions.  With a Dirichlet direction L is non-singular and p is the
 * solution; without one, the compatible part f - <f> is solved and <p> = 0.
 * f and p: device FP64 [nz][ny][nx], p must not alias f.  FP64 plans only
 * (else UNSUPPORTED).  Enqueues on stream. */
pcx_status pcx_poisson_solve(pcx_plan plan, const double *f, double *p, void *stream);

/* Per-pass device timing of a plan: with enable = 1 pcx_step records HIP
 * events on its stream between passes; with enable = 2 only around the
 * velocity correction (two events per step, for timing that kernel inside a
 * timed loop at the least cost); 0 turns timing off (other values act as 1).
 * pcx_plan_pass_times synchronizes on the last recorded step and returns up
 * to cap durations (ms) of the timed passes and, in *n_out, their number;
 * pcx_plan_pass_name names pass i. */
pcx_status pcx_plan_set_timing(pcx_plan plan, int32_t enable);
pcx_status pcx_plan_pass_times(pcx_plan plan, double *ms, int32_t cap, int32_t *n_out);
const char *pcx_plan_pass_name(pcx_plan plan, int32_t i);

/* Batched form: n independent domains of (possibly) different sizes and
 * boundary conditions, solved together.  Each domain has its own grid, dt,
 * rho0 and device buffers (same rules as pcx_step), which must stay valid
 * until pcx_batch_destroy.  The work of all domains is captured at create
 * time into one HIP graph: one grouped launch per pass of the step (per
 * kernel variant), each running that pass over the tiles of every domain,
 * in dependency order.  opts->precision selects the solve precision of every
 * domain; every domain runs opts->fixed_iters solves in the refined form.
 * Outputs must not alias inputs (INVALID).  opts->autotune times tile
 * shapes per size class on the batch's own kernels at create time. */
typedef struct {
    pcx_grid grid;
    double dt, rho0;
    const double *rho, *p_star, *u, *v, *w;
    double *u_out, *v_out, *w_out, *p_out;
} pcx_domain;

pcx_status pcx_batch_create(const pcx_domain *domains, int32_t n, const pcx_options *opts,
                            void *stream, pcx_batch *out);
/* Enqueues one solve of every domain (one graph launch) on `stream`. */
pcx_status pcx_batch_launch(pcx_batch batch, void *stream);
/* Fills n reports (one per domain) for the last launch: waits for the
 * stream that launch was enqueued on (not the whole device), and runs its
 * small report kernels and copies on that stream. */
pcx_status pcx_batch_reports(pcx_batch batch, pcx_report *out_n);
pcx_status pcx_batch_destroy(pcx_batch batch);

/* Helper: *out = min over n doubles of rho (device pointer), the splitting
 * density rho0 of the paper's constant-coefficient splitting.  Enqueues on
 * `stream` and synchronizes it.  Allocates nothing: the reduction key is a
 * static 8-byte device variable per device, so concurrent calls from several
 * host threads are serialized by the library. */
pcx_status pcx_rho_min(const double *rho, int64_t n, void *stream, double *out);

/* Allocation-free step, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same computation, arguments and report as pcx_plan_create +
 * pcx_step + pcx_plan_destroy on (grid, opts), with the plan's tables and
 * workspace placed in a fixed device array of PCX_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device it runs on until the process ends.  Calls
 * no hipMalloc/hipFree.  The grid's need (tables + workspace, see
 * pcx_noalloc_scratch_need) must fit the array, else UNSUPPORTED before any
 * device call: 128^3 fits in both precisions, 256^3 does not.
 * opts->autotune must be 0 (INVALID otherwise); a tune_cache is read, never
 * written.  The tables are uploaded from host memory on `stream`, and the
 * call waits for that upload (so for earlier work on the stream) before it
 * queues the step; with report == NULL the step itself is then only queued.
 * Every call on one device shares that device's array and leaves its last
 * contents there (each step clears what it accumulates): calls whose work
 * overlaps on one device -- on different streams, or from several host
 * threads -- race on it and must be serialized by the caller. */
#define PCX_NOALLOC_SCRATCH_BYTES (64u << 20)
pcx_status pcx_step_noalloc(const pcx_grid *grid, const pcx_options *opts, double dt, double rho0,
                            const double *rho, const double *p_star,
                            const double *u_in, const double *v_in, const double *w_in,
                            double *u_out, double *v_out, double *w_out, double *p_out,
                            void *stream, pcx_report *report);
/* Device bytes pcx_step_noalloc needs for (grid, opts); host-only. */
pcx_status pcx_noalloc_scratch_need(const pcx_grid *grid, const pcx_options *opts, size_t *bytes);

/* Refinement stop test used by the refined forms: nonzero when
 * rel_residual <= rtol and the error left after the last update, estimated
 * from the observed contraction q = update_inf / prev_update_inf (< 1) as
 * q * update_inf / (1 - q), is at most 0.1 * rtol * p_inf.  With
 * prev_update_inf <= 0 (first solve) it returns 0. */
int32_t pcx_refine_should_stop(double rel_residual, double update_inf, double prev_update_inf, double p_inf,
                               double rtol);

const char *pcx_status_str(pcx_status s);
const char *pcx_last_error(void);
int32_t pcx_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PCX_H */
