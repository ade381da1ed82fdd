/*
 * flow.c -- plain FP64 single-threaded reference for the phase-field
 * transport, the momentum predictor and the Runge-Kutta substep around the
 * pressure-correction step (CaNS-Fizzy, "Mathematical model", "Methods and
 * Implementation strategy"; the ACDI method it names, the CSF surface force,
 * second-order finite differences on the staggered grid, and the
 * low-storage three-step Runge-Kutta scheme).
 *
 * TEST INFRASTRUCTURE ONLY: the product library never links or calls this
 * file.  Written for clarity, face by face, with no blocking or fusion.
 *
 * Discretization (the paper prints no equations; these are the readings):
 *   psi    = eps ln((phi + eps_s)/(1 - phi + eps_s)), phi clamped to [0, 1]
 *   n      = grad psi / |grad psi| at cell centres, central differences
 *            (zero-gradient ghost cells across walls)
 *   a      = Gamma [eps grad phi - 1/4 (1 - tanh^2(psi_f/(2 eps))) n_f] on
 *            faces; phi_f, psi_f, n_f interpolated to the face (mean in x,
 *            y; linear in z), grad phi by the face difference
 *   d phi/dt = -div(u phi_f) + div a                 (0 flux on walls)
 *   kappa  = -div n_f
 *   momentum per unit mass on a face:
 *     -div(u u) + [div(mu (grad u + grad u^T)) + sigma kappa_f grad phi
 *                  + (rho1 - rho2)(a . grad) u] / rho_f + g
 *   rho, mu = phase-2 value + (phase-1 - phase-2 value) phi
 *   RK3: gamma = 8/15, 5/12, 3/4; zeta = 0, -17/60, -5/12.
 */
#include "flow.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, nz, bcx, bcy, bcz;
    double dx, dy;
    double *dzf, *dzc; /* dzc[k]: centre k to centre k+1 (periodic wrap at nz-1) */
} fgeo;

#define ID(i, j, k) ((((size_t)(k)) * (size_t)m->ny + (size_t)(j)) * (size_t)m->nx + (size_t)(i))

static void fgeo_free(fgeo *m)
{
    free(m->dzf);
    free(m->dzc);
}

static int fgeo_init(const or_grid *g, fgeo *m)
{
    if (oracle_check_grid(g)) return 1;
    const int nz = g->nz;
    m->nx = g->nx; m->ny = g->ny; m->nz = nz;
    m->bcx = g->bcx; m->bcy = g->bcy; m->bcz = g->bcz;
    m->dx = g->lx / g->nx;
    m->dy = g->ly / g->ny;
    m->dzf = malloc(sizeof(double) * nz);
    m->dzc = malloc(sizeof(double) * nz);
    if (!m->dzf || !m->dzc) { fgeo_free(m); return 1; }
    for (int k = 0; k < nz; ++k) m->dzf[k] = g->zf[k + 1] - g->zf[k];
    for (int k = 0; k < nz - 1; ++k) m->dzc[k] = 0.5 * (m->dzf[k] + m->dzf[k + 1]);
    m->dzc[nz - 1] = 0.5 * (m->dzf[nz - 1] + m->dzf[0]);
    return 0;
}

static int per(const fgeo *m, int d) { return (d == 0 ? m->bcx : (d == 1 ? m->bcy : m->bcz)) == 0; }
static int nof(const fgeo *m, int d) { return d == 0 ? m->nx : (d == 1 ? m->ny : m->nz); }

/* Cell-centred scalar at (i, j, k), any index one cell outside the grid:
 * periodic wrap, or the adjacent cell across a wall (zero gradient). */
static double cval(const fgeo *m, const double *q, int i, int j, int k)
{
    int ix[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) {
        int n = nof(m, d);
        if (ix[d] < 0) ix[d] = per(m, d) ? ix[d] + n : 0;
        else if (ix[d] >= n) ix[d] = per(m, d) ? ix[d] - n : n - 1;
    }
    return q[ID(ix[0], ix[1], ix[2])];
}

/* Velocity component c (0 u, 1 v, 2 w) on the +c face of cell (i, j, k),
 * for indices one outside the grid: in its own direction the faces -1 and
 * n-1 of a wall direction are the walls (0); across a wall in another
 * direction the no-slip ghost is minus the adjacent value. */
static double fval(const fgeo *m, const double *q, int c, int i, int j, int k)
{
    int ix[3] = {i, j, k};
    double sgn = 1.0;
    for (int d = 0; d < 3; ++d) {
        int n = nof(m, d);
        if (d == c) {
            if (per(m, d)) {
                if (ix[d] < 0) ix[d] += n;
                else if (ix[d] >= n) ix[d] -= n;
            } else if (ix[d] < 0 || ix[d] >= n - 1) {
                return 0.0;
            }
        } else if (ix[d] < 0 || ix[d] >= n) {
            if (per(m, d)) ix[d] = ix[d] < 0 ? ix[d] + n : ix[d] - n;
            else { ix[d] = ix[d] < 0 ? 0 : n - 1; sgn = -sgn; }
        }
    }
    return sgn * q[ID(ix[0], ix[1], ix[2])];
}

/* Is the +d face of cell index s (s in [-1, n-1]) a wall? */
static int wallface(const fgeo *m, int d, int s) { return !per(m, d) && (s < 0 || s >= nof(m, d) - 1); }

/* z spacing between cell centres k and k+1 for k in [-1, nz-1]: across a
 * wall the ghost centre is the mirror image, one cell width away. */
static double dzc_at(const fgeo *m, int k)
{
    const int nz = m->nz;
    if (k < 0) return per(m, 2) ? m->dzc[nz - 1] : m->dzf[0];
    if (k >= nz - 1) return per(m, 2) ? m->dzc[nz - 1] : m->dzf[nz - 1];
    return m->dzc[k];
}
static double dzf_at(const fgeo *m, int k)
{
    const int nz = m->nz;
    if (k < 0) return m->dzf[per(m, 2) ? nz - 1 : 0];
    if (k >= nz) return m->dzf[per(m, 2) ? 0 : nz - 1];
    return m->dzf[k];
}

/* Linear interpolation of cell values q_k, q_{k+1} to the face between them. */
static double zinterp(const fgeo *m, int k, double qk, double qk1)
{
    const double a = dzf_at(m, k + 1), b = dzf_at(m, k), h = dzc_at(m, k);
    return (qk * a + qk1 * b) / (2.0 * h);
}

/* Cell value interpolated to the +d face of cell (i, j, k). */
static double cface(const fgeo *m, const double *q, int d, int i, int j, int k)
{
    const double q0 = cval(m, q, i, j, k);
    if (d == 0) return 0.5 * (q0 + cval(m, q, i + 1, j, k));
    if (d == 1) return 0.5 * (q0 + cval(m, q, i, j + 1, k));
    return zinterp(m, k, q0, cval(m, q, i, j, k + 1));
}

/* Difference quotient of a cell quantity across the +d face of (i, j, k). */
static double cgrad(const fgeo *m, const double *q, int d, int i, int j, int k)
{
    const double q0 = cval(m, q, i, j, k);
    if (d == 0) return (cval(m, q, i + 1, j, k) - q0) / m->dx;
    if (d == 1) return (cval(m, q, i, j + 1, k) - q0) / m->dy;
    return (cval(m, q, i, j, k + 1) - q0) / dzc_at(m, k);
}

static double hcell(const fgeo *m, int d, int k) { return d == 0 ? m->dx : (d == 1 ? m->dy : m->dzf[k]); }

/* ---------------------------------------------------------------- ACDI */

static void psi_field(const fgeo *m, const or_acdi *a, const double *phi, double *psi)
{
    const size_t n = (size_t)m->nx * m->ny * m->nz;
    for (size_t c = 0; c < n; ++c) {
        /* the logarithm is defined for phi in [0, 1]; rounding can leave phi
           a few ulps outside, so psi takes phi clamped to that range */
        const double q = phi[c] < 0.0 ? 0.0 : (phi[c] > 1.0 ? 1.0 : phi[c]);
        psi[c] = a->eps * log((q + a->eps_s) / (1.0 - q + a->eps_s));
    }
}

static void normal_field(const fgeo *m, const double *psi, double *nx_, double *ny_, double *nz_)
{
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                const double gx = (cval(m, psi, i + 1, j, k) - cval(m, psi, i - 1, j, k)) / (2.0 * m->dx);
                const double gy = (cval(m, psi, i, j + 1, k) - cval(m, psi, i, j - 1, k)) / (2.0 * m->dy);
                const double gz = (cval(m, psi, i, j, k + 1) - cval(m, psi, i, j, k - 1)) / (dzc_at(m, k) + dzc_at(m, k - 1));
                const double mag = sqrt(gx * gx + gy * gy + gz * gz);
                const size_t c = ID(i, j, k);
                if (mag > 0.0) {
                    nx_[c] = gx / mag;
                    ny_[c] = gy / mag;
                    nz_[c] = gz / mag;
                } else {
                    nx_[c] = ny_[c] = nz_[c] = 0.0;
                }
            }
}

int oracle_acdi_normals(const or_grid *g, const or_acdi *a, const double *phi, double *psi, double *nx,
                        double *ny, double *nz)
{
    fgeo m;
    if (!a || !phi || !psi || !nx || !ny || !nz || fgeo_init(g, &m)) return 1;
    psi_field(&m, a, phi, psi);
    normal_field(&m, psi, nx, ny, nz);
    fgeo_free(&m);
    return 0;
}

/* The three face fluxes from phi, psi and the cell normals. */
static void flux_fields(const fgeo *m, const or_acdi *a, const double *phi, const double *psi, const double *const n[3],
                        double *const af[3])
{
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                const int s[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    const size_t c = ID(i, j, k);
                    if (wallface(m, d, s[d])) { af[d][c] = 0.0; continue; }
                    const double psf = cface(m, psi, d, i, j, k);
                    const double nf = cface(m, n[d], d, i, j, k);
                    const double t = tanh(psf / (2.0 * a->eps));
                    af[d][c] = a->gamma * (a->eps * cgrad(m, phi, d, i, j, k) - 0.25 * (1.0 - t * t) * nf);
                }
            }
}

static int acdi_all(const or_grid *g, const or_acdi *a, const double *phi, fgeo *m, double **psi, double *n[3],
                    double *af[3])
{
    if (!a || !phi || fgeo_init(g, m)) return 1;
    const size_t nc = (size_t)m->nx * m->ny * m->nz;
    *psi = malloc(nc * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        n[d] = malloc(nc * sizeof(double));
        af[d] = malloc(nc * sizeof(double));
    }
    psi_field(m, a, phi, *psi);
    normal_field(m, *psi, n[0], n[1], n[2]);
    flux_fields(m, a, phi, *psi, (const double *const *)n, af);
    return 0;
}

static void acdi_free(fgeo *m, double *psi, double *n[3], double *af[3])
{
    free(psi);
    for (int d = 0; d < 3; ++d) {
        free(n[d]);
        free(af[d]);
    }
    fgeo_free(m);
}

int oracle_acdi_flux(const or_grid *g, const or_acdi *a, const double *phi, double *ax, double *ay, double *az)
{
    fgeo m;
    double *psi, *n[3], *af[3];
    if (!ax || !ay || !az || acdi_all(g, a, phi, &m, &psi, n, af)) return 1;
    const size_t nc = (size_t)m.nx * m.ny * m.nz;
    memcpy(ax, af[0], nc * sizeof(double));
    memcpy(ay, af[1], nc * sizeof(double));
    memcpy(az, af[2], nc * sizeof(double));
    acdi_free(&m, psi, n, af);
    return 0;
}

int oracle_acdi_rhs(const or_grid *g, const or_acdi *a, const double *phi, const double *u, const double *v,
                    const double *w, double *rhs)
{
    fgeo mm;
    double *psi, *n[3], *af[3];
    if (!u || !v || !w || !rhs || acdi_all(g, a, phi, &mm, &psi, n, af)) return 1;
    const fgeo *m = &mm;
    const double *vel[3] = {u, v, w};
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                double r = 0.0;
                for (int d = 0; d < 3; ++d) {
                    /* net flux J = u phi_f - a through the +d and -d faces */
                    const int s[3] = {i, j, k};
                    int lo[3] = {i, j, k};
                    lo[d] -= 1;
                    double jp = 0.0, jm = 0.0;
                    if (!wallface(m, d, s[d]))
                        jp = fval(m, vel[d], d, i, j, k) * cface(m, phi, d, i, j, k) - af[d][ID(i, j, k)];
                    if (!wallface(m, d, s[d] - 1)) {
                        /* the -d face of this cell is the +d face of the neighbour */
                        int q[3] = {lo[0], lo[1], lo[2]};
                        const int nn = nof(m, d);
                        if (q[d] < 0) q[d] += nn; /* periodic */
                        jm = fval(m, vel[d], d, q[0], q[1], q[2]) * cface(m, phi, d, q[0], q[1], q[2]) -
                             af[d][ID(q[0], q[1], q[2])];
                    }
                    r -= (jp - jm) / hcell(m, d, k);
                }
                rhs[ID(i, j, k)] = r;
            }
    acdi_free(&mm, psi, n, af);
    return 0;
}

static void curvature_field(const fgeo *m, const double *const n[3], double *kappa)
{
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                double s = 0.0;
                const int ix[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    const double np = wallface(m, d, ix[d]) ? 0.0 : cface(m, n[d], d, i, j, k);
                    int q[3] = {i, j, k};
                    q[d] -= 1;
                    double nm = 0.0;
                    if (!wallface(m, d, ix[d] - 1)) {
                        if (q[d] < 0) q[d] += nof(m, d);
                        nm = cface(m, n[d], d, q[0], q[1], q[2]);
                    }
                    s += (np - nm) / hcell(m, d, k);
                }
                kappa[ID(i, j, k)] = -s;
            }
}

int oracle_curvature(const or_grid *g, const or_acdi *a, const double *phi, double *kappa)
{
    fgeo m;
    double *psi, *n[3], *af[3];
    if (!kappa || acdi_all(g, a, phi, &m, &psi, n, af)) return 1;
    curvature_field(&m, (const double *const *)n, kappa);
    acdi_free(&m, psi, n, af);
    return 0;
}

/* ------------------------------------------------------------ momentum */

/* Mean of a cell quantity over the four cells around the edge parallel to
 * direction e that touches the +a and +b faces of cell (i, j, k). */
static double edge4(const fgeo *m, const double *q, int a, int b, int i, int j, int k)
{
    int o1[3] = {0, 0, 0}, o2[3] = {0, 0, 0};
    o1[a] = 1;
    o2[b] = 1;
    return 0.25 * (cval(m, q, i, j, k) + cval(m, q, i + o1[0], j + o1[1], k + o1[2]) +
                   cval(m, q, i + o2[0], j + o2[1], k + o2[2]) +
                   cval(m, q, i + o1[0] + o2[0], j + o1[1] + o2[1], k + o1[2] + o2[2]));
}

/* Spacing between cell centres s and s+1 in direction d. */
static double hcen(const fgeo *m, int d, int s) { return d == 0 ? m->dx : (d == 1 ? m->dy : dzc_at(m, s)); }

/* Momentum right-hand side of component c on the +c face of cell (i, j, k). */
static double mom_face(const fgeo *m, const or_flow *f, const double *phi, const double *const vel[3],
                       const double *rho, const double *mu, const double *kappa, const double *const af[3], int c,
                       int i, int j, int k)
{
    const int ix[3] = {i, j, k};
    const double *q = vel[c];
    int e[3] = {0, 0, 0};
    e[c] = 1;
    /* own component at offsets along each direction */
#define Q(di, dj, dk) fval(m, q, c, i + (di), j + (dj), k + (dk))
    const double q0 = Q(0, 0, 0);
    /* width of the c-control volume in direction c: cell centre s to s+1 */
    const double hc = hcen(m, c, ix[c]);
    double adv = 0.0, visc = 0.0, reg = 0.0;
    /* normal direction d == c: fluxes at the cell centres s and s+1 */
    {
        const double qm = Q(-e[0], -e[1], -e[2]), qp = Q(e[0], e[1], e[2]);
        const double cm = 0.5 * (qm + q0), cp = 0.5 * (q0 + qp);
        adv += (cp * cp - cm * cm) / hc;
        const double mu0 = cval(m, mu, i, j, k), mu1 = cval(m, mu, i + e[0], j + e[1], k + e[2]);
        const double tp = 2.0 * mu1 * (qp - q0) / hcell(m, c, ix[c] + 1 < nof(m, c) ? ix[c] + 1 : 0);
        const double tm = 2.0 * mu0 * (q0 - qm) / hcell(m, c, ix[c]);
        visc += (tp - tm) / hc;
    }
    /* transverse directions: fluxes on the edges at s + 1/2 and s - 1/2 */
    for (int d = 0; d < 3; ++d) {
        if (d == c) continue;
        int ed[3] = {0, 0, 0};
        ed[d] = 1;
        const double *p = vel[d];
        /* transport velocity (component d) at the edges: mean of the d-faces
         * of the two cells along c, on the +d side and on the -d side */
        const double pu = 0.5 * (fval(m, p, d, i, j, k) + fval(m, p, d, i + e[0], j + e[1], k + e[2]));
        const double pd = 0.5 * (fval(m, p, d, i - ed[0], j - ed[1], k - ed[2]) +
                                 fval(m, p, d, i + e[0] - ed[0], j + e[1] - ed[1], k + e[2] - ed[2]));
        const double qu = Q(ed[0], ed[1], ed[2]), qd = Q(-ed[0], -ed[1], -ed[2]);
        adv += (pu * 0.5 * (q0 + qu) - pd * 0.5 * (qd + q0)) / hcell(m, d, ix[2]);
        /* stress on the edges: mu (dq/dd + dp/dc) */
        const double hu = hcen(m, d, ix[d]), hd = hcen(m, d, ix[d] - 1);
        const double dpu = (fval(m, p, d, i + e[0], j + e[1], k + e[2]) - fval(m, p, d, i, j, k)) / hc;
        const double dpd = (fval(m, p, d, i + e[0] - ed[0], j + e[1] - ed[1], k + e[2] - ed[2]) -
                            fval(m, p, d, i - ed[0], j - ed[1], k - ed[2])) / hc;
        const double muu = edge4(m, mu, c, d, i, j, k);
        const double mud = edge4(m, mu, c, d, i - ed[0], j - ed[1], k - ed[2]);
        const double tu = muu * ((qu - q0) / hu + dpu);
        const double td = mud * ((q0 - qd) / hd + dpd);
        visc += (tu - td) / hcell(m, d, ix[2]);
    }
    /* regularization (rho1 - rho2)(a . grad) q with a at this face: own
     * component directly, the others as the mean of the four faces around */
    for (int d = 0; d < 3; ++d) {
        double ad;
        if (d == c) {
            ad = af[c][ID(i, j, k)];
        } else {
            int ed[3] = {0, 0, 0};
            ed[d] = 1;
            /* faces (+d) of the cells (i,j,k), (+c neighbour), and their -d neighbours */
            double s = 0.0;
            const int cells[4][3] = {{i, j, k},
                                     {i + e[0], j + e[1], k + e[2]},
                                     {i - ed[0], j - ed[1], k - ed[2]},
                                     {i + e[0] - ed[0], j + e[1] - ed[1], k + e[2] - ed[2]}};
            for (int t = 0; t < 4; ++t) {
                int a0 = cells[t][0], a1 = cells[t][1], a2 = cells[t][2];
                int a3[3] = {a0, a1, a2};
                if (wallface(m, d, a3[d])) continue; /* wall faces carry no flux */
                for (int dd = 0; dd < 3; ++dd) {
                    const int nn = nof(m, dd);
                    if (a3[dd] < 0) a3[dd] += nn;
                    else if (a3[dd] >= nn) a3[dd] -= nn;
                }
                s += af[d][ID(a3[0], a3[1], a3[2])];
            }
            ad = 0.25 * s;
        }
        int ed[3] = {0, 0, 0};
        ed[d] = 1;
        double gq;
        if (d == c) gq = (Q(e[0], e[1], e[2]) - Q(-e[0], -e[1], -e[2])) / (hcell(m, c, ix[c]) + hcell(m, c, ix[c] + 1 < nof(m, c) ? ix[c] + 1 : 0));
        else gq = (Q(ed[0], ed[1], ed[2]) - Q(-ed[0], -ed[1], -ed[2])) / (hcen(m, d, ix[d]) + hcen(m, d, ix[d] - 1));
        reg += ad * gq;
    }
#undef Q
    /* surface tension on this face */
    const double kf = cface(m, kappa, c, i, j, k);
    const double st = f->sigma * kf * cgrad(m, phi, c, i, j, k);
    const double rf = cface(m, rho, c, i, j, k);
    const double g[3] = {f->gx, f->gy, f->gz};
    return -adv + (visc + st + (f->rho1 - f->rho2) * reg) / rf + g[c];
}

int oracle_momentum_rhs(const or_grid *g, const or_flow *f, const double *phi, const double *u, const double *v,
                        const double *w, double *ru, double *rv, double *rw)
{
    fgeo mm;
    double *psi, *n[3], *af[3];
    if (!f || !u || !v || !w || !ru || !rv || !rw || acdi_all(g, &f->acdi, phi, &mm, &psi, n, af)) return 1;
    const fgeo *m = &mm;
    const size_t nc = (size_t)m->nx * m->ny * m->nz;
    double *rho = malloc(nc * sizeof(double)), *mu = malloc(nc * sizeof(double)), *kap = malloc(nc * sizeof(double));
    for (size_t c = 0; c < nc; ++c) {
        rho[c] = f->rho2 + (f->rho1 - f->rho2) * phi[c];
        mu[c] = f->mu2 + (f->mu1 - f->mu2) * phi[c];
    }
    curvature_field(m, (const double *const *)n, kap);
    const double *vel[3] = {u, v, w};
    double *out[3] = {ru, rv, rw};
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                const int ix[3] = {i, j, k};
                for (int c = 0; c < 3; ++c)
                    out[c][ID(i, j, k)] = wallface(m, c, ix[c]) ? 0.0 :
                        mom_face(m, f, phi, vel, rho, mu, kap, (const double *const *)af, c, i, j, k);
            }
    free(rho);
    free(mu);
    free(kap);
    acdi_free(&mm, psi, n, af);
    return 0;
}

/* ------------------------------------------------------------ substep */

int oracle_rk3_coeffs(int s, double *gamma, double *zeta, double *alpha)
{
    static const double ga[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
    static const double ze[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
    if (s < 1 || s > 3) return 1;
    if (gamma) *gamma = ga[s - 1];
    if (zeta) *zeta = ze[s - 1];
    if (alpha) *alpha = ga[s - 1] + ze[s - 1];
    return 0;
}

int oracle_flow_substep(const or_grid *g, const or_flow *f, int s, double Dt, const double *phi, const double *u,
                        const double *v, const double *w, const double *p1, const double *p2, double r,
                        double *hphi, double *hu, double *hv, double *hw, double *phi_out, double *u_out,
                        double *v_out, double *w_out, double *p_out, or_diag *diag)
{
    double ga, ze, al;
    if (!f || oracle_rk3_coeffs(s, &ga, &ze, &al) || oracle_check_grid(g) || !(Dt > 0.0)) return 1;
    const size_t nc = (size_t)g->nx * g->ny * g->nz;
    double *A = malloc(nc * sizeof(double));
    double *M[3];
    for (int d = 0; d < 3; ++d) M[d] = malloc(nc * sizeof(double));
    /* right-hand sides at the start of the substep */
    if (oracle_acdi_rhs(g, &f->acdi, phi, u, v, w, A) ||
        oracle_momentum_rhs(g, f, phi, u, v, w, M[0], M[1], M[2])) {
        free(A);
        for (int d = 0; d < 3; ++d) free(M[d]);
        return 1;
    }
    const double *q0[4] = {phi, u, v, w};
    double *h[4] = {hphi, hu, hv, hw};
    double *R[4] = {A, M[0], M[1], M[2]};
    double *qs[4] = {phi_out, NULL, NULL, NULL};
    double *us[3];
    for (int d = 0; d < 3; ++d) us[d] = malloc(nc * sizeof(double));
    qs[1] = us[0]; qs[2] = us[1]; qs[3] = us[2];
    for (int q = 0; q < 4; ++q)
        for (size_t c = 0; c < nc; ++c) {
            const double old = s == 1 ? 0.0 : h[q][c];
            qs[q][c] = q0[q][c] + Dt * (ga * R[q][c] + ze * old);
            h[q][c] = R[q][c];
        }
    /* density of the new phase field, splitting density, extrapolated p */
    double *rho = malloc(nc * sizeof(double)), *ps = malloc(nc * sizeof(double));
    double rho0 = INFINITY;
    for (size_t c = 0; c < nc; ++c) {
        rho[c] = f->rho2 + (f->rho1 - f->rho2) * phi_out[c];
        if (rho[c] < rho0) rho0 = rho[c];
        ps[c] = (1.0 + r) * p1[c] - r * p2[c];
    }
    const int st = oracle_step(g, al * Dt, rho0, rho, ps, us[0], us[1], us[2], u_out, v_out, w_out, p_out, diag);
    free(A);
    free(rho);
    free(ps);
    for (int d = 0; d < 3; ++d) {
        free(M[d]);
        free(us[d]);
    }
    return st;
}
