/*
 * rf_oracle.c -- plain FP64 CPU oracle for the Richards-equation hot path of
 * Orgogozo et al., "An open source massively parallel solver for Richards
 * equation" (RichardsFOAM, arXiv:1809.10895).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * What it computes, in the paper's order:
 *   - van Genuchten retention theta(h), capacity C(h), Mualem K(h)
 *     (Sec. 1, Eqs. 2-4), with a storage term S*h added to theta for h >= 0
 *     so that C = S there is the derivative of the storage function;
 *   - one backward-Euler step (Sec. 2.2) linearised by classical Picard
 *     iteration with the chord-slope capacity (Sec. 2.2), implicit pressure
 *     diffusion and explicit gravity from the previous Picard iterate with
 *     arithmetic-mean face conductivity (Sec. 2.2, last paragraph),
 *     on a uniform cell-centred 7-point finite-volume grid (constant cell
 *     volume, programme summary "Restrictions");
 *   - each linear system solved by conjugate gradients preconditioned with
 *     diagonal incomplete Cholesky (DIC-PCG, Sec. 2.2), in natural storage
 *     order;
 *   - the Picard exit test evaluated over the whole domain (Sec. 2.3);
 *   - the empirically based adaptive time step (EBATS, Sec. 2.2);
 *   - a global water balance (storage vs. cumulative boundary inflow).
 *
 * Everything is written for clarity, not speed: the 7-point matrix is
 * assembled explicitly (diagonal + six neighbour coefficients per cell), the
 * preconditioner sweeps run serially, no loop is blocked or fused.
 *
 * Optional slab mode (orc_set_slabs, used only to time the method on many
 * host cores): the grid is cut into slabs of whole y-rows, one per
 * sub-domain, as the paper's 'simple' mesh decomposition does (Sec. 2.3);
 * the DIC factorisation and sweeps then ignore the couplings between slabs
 * (block Jacobi over sub-domains, like a decomposed OpenFOAM case whose
 * processor patches are left out of the preconditioner), and the slabs,
 * the assembly and the vector operations run on OpenMP threads.  The
 * converged solution is the same; only the PCG iteration count changes.
 * With one slab (the default) every loop is the serial one above.
 *
 * Layout of every per-cell array: cell (i,j,k) is at k + nz*(i + nx*j);
 * k = 0 is the bottom layer, z points up.  Column (i,j) is active for
 * k < ktop[i + nx*j].  Inactive cells are carried unchanged.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- public constants (mirrored by the Python wrapper) ---------------- */
enum { ORC_VGM = 0, ORC_GARDNER = 1 };
enum { ORC_XMIN = 0, ORC_XMAX, ORC_YMIN, ORC_YMAX, ORC_ZMIN, ORC_ZMAX };
enum { ORC_NOFLOW = 0, ORC_DIRICHLET = 1, ORC_FLUX = 2, ORC_FREE_DRAINAGE = 3 };
enum { ORC_PICARD_CHORD = 0, ORC_PICARD_MODIFIED = 1 };   /* linearisation, Sec. 2.2 */
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NOT_CONVERGED = -5,
       ORC_ERR_LINEAR = -6, ORC_ERR_NONFINITE = -7 };

#define ORC_MAX_LAYERS 16
#define ORC_MAX_PICARD_LOG 128

typedef struct {
    double tol_picard;   /* L-infinity of h^{m+1}-h^m [m] */
    double tol_cg;       /* L-infinity of diag(A)^-1 r [m] */
    int max_picard;
    int max_cg;
    double chord_eps;    /* |h^m-h^n| below this: analytic C(h^m) */
    double dt0, dt_max, dt_min;
    int ebats;           /* 1: adaptive steps in orc_run, 0: fixed dt0 */
    int inc_after;       /* consecutive "easy" steps before dt *= factor */
    int few_iters;       /* an easy step used at most this many Picard its */
    int max_iters;       /* a step needing more Picard its is rerun */
    double factor;       /* EBATS scaling factor */
    int picard_variant;  /* ORC_PICARD_CHORD (classical Picard, chord-slope
                            capacity) or ORC_PICARD_MODIFIED (Celia et al.) */
} orc_options;

typedef struct {
    int converged;
    int picard_iters;
    int cg_iters_total;
    int cg_iters[ORC_MAX_PICARD_LOG];
    double delta[ORC_MAX_PICARD_LOG];
    double dt;
    double t;
} orc_step_stats;

typedef struct {
    int accepted, rejected;
    long picard_total, cg_total;
    double dt_last, t;
} orc_run_stats;

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    double g[3];                     /* gradient of elevation, grid axes */
    int32_t *ktop;                   /* nx*ny */
    int model;
    int nlayer;
    double layer[ORC_MAX_LAYERS][6]; /* theta_r, theta_s, alpha, n, Ks, S */
    uint8_t *layer_of_cell;          /* N or NULL */
    double *lnks;                    /* N or NULL */
    int bc_type[6];
    double bc_value[6];
    int nseg[6];
    double *seg_t[6], *seg_q[6];
    orc_options opt;
    /* state */
    double *h;       /* h^n */
    double t;
    double dt_cur;
    int easy_count;
    /* water balance */
    double storage0, storage;
    double inflow[6];
    int have_storage0;
    int nslab;       /* sub-domains of whole y-rows (1 = the serial method) */
} orc_problem;

/* ======================================================================
 * Soil hydraulic functions, Sec. 1, Eqs. 2-4
 * p = {theta_r, theta_s, alpha, n, Ks, S}
 * ====================================================================== */

/* Eq. 2, plus S*h above saturation (storage function used by the chord
 * slope and by the water balance). */
double orc_theta(int model, double h, const double *p)
{
    double tr = p[0], ts = p[1], a = p[2], n = p[3], S = p[5];
    if (h >= 0.0) return ts + S * h;
    if (model == ORC_GARDNER) return tr + (ts - tr) * exp(a * h);
    double m = 1.0 - 1.0 / n;
    double u = pow(-a * h, n);
    return tr + (ts - tr) * pow(1.0 + u, -m);
}

/* Eq. 3: C = d theta / dh; C = S for h >= 0. */
double orc_capacity(int model, double h, const double *p)
{
    double tr = p[0], ts = p[1], a = p[2], n = p[3], S = p[5];
    if (h >= 0.0) return S;
    if (model == ORC_GARDNER) return a * (ts - tr) * exp(a * h);
    double m = 1.0 - 1.0 / n;
    double u = pow(-a * h, n);
    return (ts - tr) * a * n * m * pow(-a * h, n - 1.0) * pow(1.0 + u, -(1.0 + m));
}

/* Eq. 4 (Mualem): K = Ks Se^(1/2) (1 - (1 - Se^(1/m))^m)^2, Se = (1+u)^-m,
 * u = (-alpha h)^n, m = 1 - 1/n.  The exponent printed in Eq. 4 as
 * "(n/n-1)" is n/(n-1) = 1/m, so Se^(1/m) = 1/(1+u) and 1 - Se^(1/m) equals
 * u/(1+u) exactly.  (u/(1+u))^m is then formed as exp(-m*log1p(1/u)) and
 * 1 - (.)^m as -expm1(.) so that the dry end (u >> 1), where the printed
 * form cancels, keeps full precision.  Gardner's model (Appendix A, Eq. A6):
 * K = Ks exp(alpha h). */
double orc_conductivity(int model, double h, const double *p)
{
    double a = p[2], n = p[3], Ks = p[4];
    if (h >= 0.0) return Ks;
    if (model == ORC_GARDNER) return Ks * exp(a * h);
    double m = 1.0 - 1.0 / n;
    double u = pow(-a * h, n);
    double Se = pow(1.0 + u, -m);
    double one_minus = -expm1(-m * log1p(1.0 / u));
    return Ks * sqrt(Se) * one_minus * one_minus;
}

/* ======================================================================
 * Problem set-up
 * ====================================================================== */

static size_t ncell(const orc_problem *P) { return (size_t)P->nx * P->ny * P->nz; }

orc_problem *orc_create(int nx, int ny, int nz, double dx, double dy, double dz,
                        const int32_t *ktop, const double *g3)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !(dy > 0) || !(dz > 0)) return NULL;
    orc_problem *P = (orc_problem *)calloc(1, sizeof(orc_problem));
    P->nx = nx; P->ny = ny; P->nz = nz; P->dx = dx; P->dy = dy; P->dz = dz;
    P->g[0] = g3 ? g3[0] : 0.0; P->g[1] = g3 ? g3[1] : 0.0; P->g[2] = g3 ? g3[2] : 1.0;
    P->ktop = (int32_t *)malloc(sizeof(int32_t) * nx * ny);
    for (int c = 0; c < nx * ny; c++) {
        int kt = ktop ? ktop[c] : nz;
        if (kt < 0) kt = 0;
        if (kt > nz) kt = nz;
        P->ktop[c] = kt;
    }
    P->h = (double *)calloc(ncell(P), sizeof(double));
    P->opt.tol_picard = 1e-6; P->opt.tol_cg = 1e-8; P->opt.max_picard = 50;
    P->opt.max_cg = 10000; P->opt.chord_eps = 1e-9;
    P->opt.dt0 = 1.0; P->opt.dt_max = 3600.0; P->opt.dt_min = 1e-6;
    P->opt.ebats = 1; P->opt.inc_after = 10; P->opt.few_iters = 3;
    P->opt.max_iters = 8; P->opt.factor = 1.3;
    P->opt.picard_variant = ORC_PICARD_CHORD;
    P->dt_cur = P->opt.dt0;
    P->nslab = 1;
    return P;
}

/* Slab mode: nslab sub-domains of whole y-rows (1 <= nslab <= ny). */
int orc_set_slabs(orc_problem *P, int nslab)
{
    if (nslab < 1 || nslab > P->ny) return ORC_ERR_ARG;
    P->nslab = nslab;
    return ORC_OK;
}

/* Threads the slab mode's parallel loops use (OMP_NUM_THREADS). */
int orc_threads(void) { return omp_get_max_threads(); }

/* Rows [j0, j1) of slab s. */
static void slab_rows(const orc_problem *P, int s, int *j0, int *j1)
{
    *j0 = (int)((long)s * P->ny / P->nslab);
    *j1 = (int)((long)(s + 1) * P->ny / P->nslab);
}

void orc_free(orc_problem *P)
{
    if (!P) return;
    free(P->ktop); free(P->layer_of_cell); free(P->lnks); free(P->h);
    for (int f = 0; f < 6; f++) { free(P->seg_t[f]); free(P->seg_q[f]); }
    free(P);
}

int orc_set_soil(orc_problem *P, int model, int nlayer, const double *params,
                 const uint8_t *layer_of_cell, const double *lnks)
{
    if (nlayer < 1 || nlayer > ORC_MAX_LAYERS || !params) return ORC_ERR_ARG;
    P->model = model;
    P->nlayer = nlayer;
    for (int l = 0; l < nlayer; l++)
        for (int q = 0; q < 6; q++) P->layer[l][q] = params[6 * l + q];
    size_t N = ncell(P);
    free(P->layer_of_cell); P->layer_of_cell = NULL;
    free(P->lnks); P->lnks = NULL;
    if (layer_of_cell) {
        P->layer_of_cell = (uint8_t *)malloc(N);
        for (size_t c = 0; c < N; c++) {
            if (layer_of_cell[c] >= nlayer) return ORC_ERR_ARG;
            P->layer_of_cell[c] = layer_of_cell[c];
        }
    }
    if (lnks) {
        P->lnks = (double *)malloc(sizeof(double) * N);
        memcpy(P->lnks, lnks, sizeof(double) * N);
    }
    return ORC_OK;
}

int orc_set_bc(orc_problem *P, int face, int type, double value)
{
    if (face < 0 || face > 5 || type < 0 || type > 3) return ORC_ERR_ARG;
    P->bc_type[face] = type;
    P->bc_value[face] = value;
    return ORC_OK;
}

int orc_set_forcing(orc_problem *P, int face, int nseg, const double *t0, const double *q)
{
    if (face < 0 || face > 5 || nseg < 0) return ORC_ERR_ARG;
    free(P->seg_t[face]); free(P->seg_q[face]);
    P->seg_t[face] = P->seg_q[face] = NULL;
    P->nseg[face] = nseg;
    if (nseg) {
        P->seg_t[face] = (double *)malloc(sizeof(double) * nseg);
        P->seg_q[face] = (double *)malloc(sizeof(double) * nseg);
        memcpy(P->seg_t[face], t0, sizeof(double) * nseg);
        memcpy(P->seg_q[face], q, sizeof(double) * nseg);
    }
    return ORC_OK;
}

int orc_set_options(orc_problem *P, const orc_options *o)
{
    P->opt = *o;
    P->dt_cur = o->dt0;
    P->easy_count = 0;
    return ORC_OK;
}

/* Parameters of cell c (layer values, Ks scaled by exp(lnks[c])). */
static void cell_params(const orc_problem *P, size_t c, double *p)
{
    int l = P->layer_of_cell ? P->layer_of_cell[c] : 0;
    for (int q = 0; q < 6; q++) p[q] = P->layer[l][q];
    if (P->lnks) p[4] *= exp(P->lnks[c]);
}

static int active(const orc_problem *P, int i, int j, int k)
{
    if (i < 0 || i >= P->nx || j < 0 || j >= P->ny || k < 0) return 0;
    return k < P->ktop[i + P->nx * j];
}

/* Value carried by a flux face at time t: the forcing segment that contains
 * t (piecewise constant), else the constant from orc_set_bc. */
static double face_flux(const orc_problem *P, int f, double t)
{
    if (P->nseg[f] == 0 || t < P->seg_t[f][0]) return P->bc_value[f];
    int s = 0;
    while (s + 1 < P->nseg[f] && P->seg_t[f][s + 1] <= t) s++;
    return P->seg_q[f][s];
}

/* Storage S(h) = sum over active cells of V * theta~(h). */
static double storage_of(const orc_problem *P, const double *h)
{
    double V = P->dx * P->dy * P->dz, s = 0.0, p[6];
    for (int j = 0; j < P->ny; j++)
        for (int i = 0; i < P->nx; i++)
            for (int k = 0; k < P->ktop[i + P->nx * j]; k++) {
                size_t c = (size_t)k + (size_t)P->nz * (i + (size_t)P->nx * j);
                cell_params(P, c, p);
                s += V * orc_theta(P->model, h[c], p);
            }
    return s;
}

int orc_set_state(orc_problem *P, const double *h, double t)
{
    size_t N = ncell(P);
    for (size_t c = 0; c < N; c++)
        if (!isfinite(h[c])) return ORC_ERR_NONFINITE;
    memcpy(P->h, h, sizeof(double) * N);
    P->t = t;
    P->storage0 = P->storage = storage_of(P, P->h);
    for (int f = 0; f < 6; f++) P->inflow[f] = 0.0;
    P->easy_count = 0;
    P->dt_cur = P->opt.dt0;
    return ORC_OK;
}

int orc_get_state(const orc_problem *P, double *h, double *t)
{
    memcpy(h, P->h, sizeof(double) * ncell(P));
    if (t) *t = P->t;
    return ORC_OK;
}

/* ======================================================================
 * Assembly of the linearised system for one Picard iteration
 * ====================================================================== */

/* Six neighbour directions: -x,+x,-y,+y,-z,+z; face id of the domain
 * boundary crossed in that direction. */
static const int DI[6] = {-1, 1, 0, 0, 0, 0};
static const int DJ[6] = {0, 0, -1, 1, 0, 0};
static const int DK[6] = {0, 0, 0, 0, -1, 1};
static const int FACE_OF_DIR[6] = {ORC_XMIN, ORC_XMAX, ORC_YMIN, ORC_YMAX, ORC_ZMIN, ORC_ZMAX};

typedef struct {
    double *diag;     /* N */
    double *off;      /* 6*N: off[d*N + c] = A(c, neighbour in direction d) */
    double *b;        /* N */
    double *K;        /* N: K(h^m) */
    double *C;        /* N: capacity used (chord or analytic) */
} orc_system;

/* Builds A h^{m+1} = b for iterate hm of the step hn -> hn+dt, following the
 * paper's discretisation:
 *   V C^m (h^{m+1} - h^n)/dt = sum_f T_f (h_N^{m+1} - h_P^{m+1})
 *                             + sum_f A_f K_f (g . n_f) + boundary terms
 * with K_f = (K_P + K_N)/2 at h^m, T_f = A_f K_f / d_f, C^m the chord slope
 * (theta~(h^m)-theta~(h^n))/(h^m-h^n) (analytic Eq. 3 when |h^m-h^n| <
 * chord_eps).  The modified Picard variant (Sec. 2.2; Celia et al. 1990)
 * replaces the storage term by
 *   V [C(h^m) (h^{m+1} - h^m) + theta~(h^m) - theta~(h^n)] / dt
 * with the analytic capacity of Eq. 3; both reach the same fixed point,
 * V (theta~(h) - theta~(h^n)) / dt = fluxes.  Boundary faces: Dirichlet h_b with K(h_b) over a half cell;
 * prescribed flux q (positive into the domain) as A q; free drainage as the
 * gravity flux A K(h_P^m) (g . n) with zero pressure gradient; no-flow and
 * faces towards inactive cells carry nothing.  Inactive cells get the
 * identity row with b = hm so that they are carried unchanged. */
static void assemble(const orc_problem *P, const double *hm, const double *hn,
                     double dt, double t, orc_system *S)
{
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const size_t N = ncell(P);
    const double V = P->dx * P->dy * P->dz;
    const double area[3] = {P->dy * P->dz, P->dx * P->dz, P->dx * P->dy};
    const double dist[3] = {P->dx, P->dy, P->dz};
    double p[6];

    memset(S->off, 0, sizeof(double) * 6 * N);
    /* cell coefficients */
#pragma omp parallel for private(p) schedule(static) if (P->nslab > 1)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++)
            for (int k = 0; k < nz; k++) {
                size_t c = (size_t)k + (size_t)nz * (i + (size_t)nx * j);
                if (!active(P, i, j, k)) {
                    S->K[c] = 0.0; S->C[c] = 0.0;
                    S->diag[c] = 1.0; S->b[c] = hm[c];
                    continue;
                }
                cell_params(P, c, p);
                S->K[c] = orc_conductivity(P->model, hm[c], p);
                if (P->opt.picard_variant == ORC_PICARD_MODIFIED) {
                    double C = orc_capacity(P->model, hm[c], p);
                    double dtheta = orc_theta(P->model, hm[c], p) - orc_theta(P->model, hn[c], p);
                    S->C[c] = C;
                    S->diag[c] = V * C / dt;
                    S->b[c] = V * (C * hm[c] - dtheta) / dt;
                    continue;
                }
                double dh = hm[c] - hn[c];
                double C;
                if (fabs(dh) >= P->opt.chord_eps)
                    C = (orc_theta(P->model, hm[c], p) - orc_theta(P->model, hn[c], p)) / dh;
                else
                    C = orc_capacity(P->model, hm[c], p);
                S->C[c] = C;
                S->diag[c] = V * C / dt;
                S->b[c] = V * C * hn[c] / dt;
            }
    /* faces (each cell writes only its own row) */
#pragma omp parallel for private(p) schedule(static) if (P->nslab > 1)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++)
            for (int k = 0; k < nz; k++) {
                if (!active(P, i, j, k)) continue;
                size_t c = (size_t)k + (size_t)nz * (i + (size_t)nx * j);
                for (int d = 0; d < 6; d++) {
                    int ax = d / 2;                       /* axis 0,1,2 */
                    double sgn = (d % 2) ? 1.0 : -1.0;    /* outward normal sign */
                    double gn = sgn * P->g[ax];           /* g . n_f */
                    int in = i + DI[d], jn = j + DJ[d], kn = k + DK[d];
                    int outside = in < 0 || in >= nx || jn < 0 || jn >= ny || kn < 0 ||
                                  (d == 5 && kn >= P->ktop[i + nx * j]);
                    if (!outside) {
                        if (!active(P, in, jn, kn)) continue;    /* masked: no flow */
                        size_t cn = (size_t)kn + (size_t)nz * (in + (size_t)nx * jn);
                        double Kf = 0.5 * (S->K[c] + S->K[cn]);
                        double T = area[ax] * Kf / dist[ax];
                        S->diag[c] += T;
                        S->off[(size_t)d * N + c] = -T;
                        S->b[c] += area[ax] * Kf * gn;
                        continue;
                    }
                    int f = FACE_OF_DIR[d];
                    int type = P->bc_type[f];
                    if (type == ORC_DIRICHLET) {
                        cell_params(P, c, p);
                        double hb = P->bc_value[f];
                        double Kb = orc_conductivity(P->model, hb, p);
                        double T = area[ax] * Kb / (0.5 * dist[ax]);
                        S->diag[c] += T;
                        S->b[c] += T * hb + area[ax] * Kb * gn;
                    } else if (type == ORC_FLUX) {
                        S->b[c] += area[ax] * face_flux(P, f, t);
                    } else if (type == ORC_FREE_DRAINAGE) {
                        S->b[c] += area[ax] * S->K[c] * gn;
                    }
                }
            }
}

/* Boundary inflow per face for the converged iterate (h = h^{m+1}, K = K^m),
 * added with weight dt to acc[6]. */
static void boundary_inflow(const orc_problem *P, const double *h, const double *K,
                            double dt, double t, double *acc)
{
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const double area[3] = {P->dy * P->dz, P->dx * P->dz, P->dx * P->dy};
    const double dist[3] = {P->dx, P->dy, P->dz};
    double p[6];
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++)
            for (int k = 0; k < P->ktop[i + nx * j]; k++) {
                size_t c = (size_t)k + (size_t)nz * (i + (size_t)nx * j);
                for (int d = 0; d < 6; d++) {
                    int ax = d / 2;
                    double gn = ((d % 2) ? 1.0 : -1.0) * P->g[ax];
                    int in = i + DI[d], jn = j + DJ[d], kn = k + DK[d];
                    int outside = in < 0 || in >= nx || jn < 0 || jn >= ny || kn < 0 ||
                                  (d == 5 && kn >= P->ktop[i + nx * j]);
                    if (!outside) continue;
                    int f = FACE_OF_DIR[d];
                    double q = 0.0;
                    if (P->bc_type[f] == ORC_DIRICHLET) {
                        cell_params(P, c, p);
                        double hb = P->bc_value[f];
                        double Kb = orc_conductivity(P->model, hb, p);
                        q = area[ax] * Kb / (0.5 * dist[ax]) * (hb - h[c]) + area[ax] * Kb * gn;
                    } else if (P->bc_type[f] == ORC_FLUX) {
                        q = area[ax] * face_flux(P, f, t);
                    } else if (P->bc_type[f] == ORC_FREE_DRAINAGE) {
                        q = area[ax] * K[c] * gn;
                    }
                    acc[f] += dt * q;
                }
            }
}

/* ======================================================================
 * Linear algebra: y = A x, DIC preconditioner, PCG (Sec. 2.2)
 * ====================================================================== */

static void neighbour_index(const orc_problem *P, size_t c, int d, size_t *cn, int *ok)
{
    int nz = P->nz, nx = P->nx;
    int k = (int)(c % nz);
    int col = (int)(c / nz);
    int i = col % nx, j = col / nx;
    int in = i + DI[d], jn = j + DJ[d], kn = k + DK[d];
    *ok = (in >= 0 && in < P->nx && jn >= 0 && jn < P->ny && kn >= 0 && kn < P->nz);
    *cn = *ok ? (size_t)kn + (size_t)nz * (in + (size_t)nx * jn) : 0;
}

static void matvec(const orc_problem *P, const orc_system *S, const double *x, double *y)
{
    size_t N = ncell(P);
#pragma omp parallel for schedule(static) if (P->nslab > 1)
    for (size_t c = 0; c < N; c++) {
        double s = S->diag[c] * x[c];
        for (int d = 0; d < 6; d++) {
            double a = S->off[(size_t)d * N + c];
            if (a == 0.0) continue;
            size_t cn; int ok;
            neighbour_index(P, c, d, &cn, &ok);
            s += a * x[cn];
        }
        y[c] = s;
    }
}

/* Diagonal incomplete Cholesky, M = (Dt + L) Dt^-1 (Dt + L^T), where L is the
 * strictly lower part of A in natural order and Dt is chosen so that
 * Dt_c = A_cc - sum_{lower n} A_cn^2 / Dt_n.  rD = 1/Dt.
 * In slab mode each slab is factorised on its own: the y-couplings across a
 * slab boundary are left out (block Jacobi over the sub-domains). */

/* Whether the coupling of cell c (in slab rows [j0, j1)) in direction dd is
 * kept by the preconditioner: not when it crosses the slab boundary. */
static int in_slab(const orc_problem *P, size_t c, int dd, int j0, int j1)
{
    const int j = (int)(c / ((size_t)P->nz * P->nx));
    if (dd == 2) return j > j0;        /* -y */
    if (dd == 3) return j + 1 < j1;    /* +y */
    return 1;
}

static int dic_factor_slab(const orc_problem *P, const orc_system *S, double *rD, int j0, int j1)
{
    size_t N = ncell(P);
    const size_t row = (size_t)P->nz * P->nx;
    for (size_t c = (size_t)j0 * row; c < (size_t)j1 * row; c++) {
        double d = S->diag[c];
        for (int dd = 0; dd < 6; dd += 2) {      /* lower neighbours: -x, -y, -z */
            double a = S->off[(size_t)dd * N + c];
            if (a == 0.0 || !in_slab(P, c, dd, j0, j1)) continue;
            size_t cn; int ok;
            neighbour_index(P, c, dd, &cn, &ok);
            d -= a * a * rD[cn];
        }
        if (!(d > 0.0)) return ORC_ERR_LINEAR;
        rD[c] = 1.0 / d;
    }
    return ORC_OK;
}

static int dic_factor(const orc_problem *P, const orc_system *S, double *rD)
{
    int bad = 0;
#pragma omp parallel for schedule(static, 1) reduction(| : bad) if (P->nslab > 1)
    for (int sl = 0; sl < P->nslab; sl++) {
        int j0, j1;
        slab_rows(P, sl, &j0, &j1);
        if (dic_factor_slab(P, S, rD, j0, j1) != ORC_OK) bad = 1;
    }
    return bad ? ORC_ERR_LINEAR : ORC_OK;
}

static void dic_apply_slab(const orc_problem *P, const orc_system *S, const double *rD,
                           const double *r, double *w, double *z, int j0, int j1)
{
    size_t N = ncell(P);
    const size_t row = (size_t)P->nz * P->nx;
    const size_t c0 = (size_t)j0 * row, c1 = (size_t)j1 * row;
    for (size_t c = c0; c < c1; c++) {         /* forward: (Dt + L) w = r */
        double s = r[c];
        for (int dd = 0; dd < 6; dd += 2) {
            double a = S->off[(size_t)dd * N + c];
            if (a == 0.0 || !in_slab(P, c, dd, j0, j1)) continue;
            size_t cn; int ok;
            neighbour_index(P, c, dd, &cn, &ok);
            s -= a * w[cn];
        }
        w[c] = s * rD[c];
    }
    for (size_t cc = c1; cc-- > c0;) {         /* backward: (I + Dt^-1 L^T) z = w */
        double s = 0.0;
        for (int dd = 1; dd < 6; dd += 2) {    /* upper neighbours: +x, +y, +z */
            double a = S->off[(size_t)dd * N + cc];
            if (a == 0.0 || !in_slab(P, cc, dd, j0, j1)) continue;
            size_t cn; int ok;
            neighbour_index(P, cc, dd, &cn, &ok);
            s += a * z[cn];
        }
        z[cc] = w[cc] - rD[cc] * s;
    }
}

static void dic_apply(const orc_problem *P, const orc_system *S, const double *rD,
                      const double *r, double *w, double *z)
{
#pragma omp parallel for schedule(static, 1) if (P->nslab > 1)
    for (int sl = 0; sl < P->nslab; sl++) {
        int j0, j1;
        slab_rows(P, sl, &j0, &j1);
        dic_apply_slab(P, S, rD, r, w, z, j0, j1);
    }
}

static double dot(const orc_problem *P, const double *a, const double *b)
{
    size_t N = ncell(P);
    if (P->nslab == 1) {
        double s = 0.0;
        for (size_t c = 0; c < N; c++) s += a[c] * b[c];
        return s;
    }
    /* slab mode: one partial sum per slab, added in slab order */
    double part[P->nslab];
    const size_t row = (size_t)P->nz * P->nx;
#pragma omp parallel for schedule(static, 1)
    for (int sl = 0; sl < P->nslab; sl++) {
        int j0, j1;
        slab_rows(P, sl, &j0, &j1);
        double s = 0.0;
        for (size_t c = (size_t)j0 * row; c < (size_t)j1 * row; c++) s += a[c] * b[c];
        part[sl] = s;
    }
    double s = 0.0;
    for (int sl = 0; sl < P->nslab; sl++) s += part[sl];
    return s;
}

/* Jacobi-scaled residual max |r_c / A_cc|, in metres. */
static double scaled_res(const orc_problem *P, const double *r, const double *diag)
{
    size_t N = ncell(P);
    double m = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m) if (P->nslab > 1)
    for (size_t c = 0; c < N; c++) {
        double v = fabs(r[c] / diag[c]);
        if (v > m) m = v;
    }
    return m;
}

/* DIC-PCG for A x = b from the initial guess in x.  Stops when
 * max|r/diag| <= tol (checked before every iteration).  Returns the number
 * of iterations, or -1 on breakdown / no convergence. */
static int pcg_dic(const orc_problem *P, const orc_system *S, double *x, double tol, int max_it)
{
    size_t N = ncell(P);
    double *r = (double *)calloc(N, sizeof(double));
    double *z = (double *)calloc(N, sizeof(double));
    double *w = (double *)calloc(N, sizeof(double));
    double *p = (double *)calloc(N, sizeof(double));
    double *q = (double *)calloc(N, sizeof(double));
    double *rD = (double *)calloc(N, sizeof(double));
    int it = 0, failed = 0;
    if (dic_factor(P, S, rD) != ORC_OK) failed = 1;
    const int par = P->nslab > 1;
    if (!failed) {
        matvec(P, S, x, q);
        for (size_t c = 0; c < N; c++) r[c] = S->b[c] - q[c];
    }
    if (!failed && scaled_res(P, r, S->diag) > tol) {
        dic_apply(P, S, rD, r, w, z);
        memcpy(p, z, sizeof(double) * N);
        double rho = dot(P, r, z);
        for (;;) {
            if (it >= max_it) { failed = 1; break; }
            matvec(P, S, p, q);
            double pq = dot(P, p, q);
            if (!(pq > 0.0)) { failed = 1; break; }
            double alpha = rho / pq;
#pragma omp parallel for schedule(static) if (par)
            for (size_t c = 0; c < N; c++) { x[c] += alpha * p[c]; r[c] -= alpha * q[c]; }
            it++;
            if (scaled_res(P, r, S->diag) <= tol) break;
            dic_apply(P, S, rD, r, w, z);
            double rho_new = dot(P, r, z);
            double beta = rho_new / rho;
            rho = rho_new;
#pragma omp parallel for schedule(static) if (par)
            for (size_t c = 0; c < N; c++) p[c] = z[c] + beta * p[c];
        }
    }
    free(r); free(z); free(w); free(p); free(q); free(rD);
    return failed ? -1 : it;
}

/* ======================================================================
 * One backward-Euler step with the Picard loop (Sec. 2.2, Sec. 2.3)
 * ====================================================================== */

static void alloc_system(size_t N, orc_system *S)
{
    S->diag = (double *)malloc(sizeof(double) * N);
    S->off = (double *)malloc(sizeof(double) * 6 * N);
    S->b = (double *)malloc(sizeof(double) * N);
    S->K = (double *)malloc(sizeof(double) * N);
    S->C = (double *)malloc(sizeof(double) * N);
}

static void free_system(orc_system *S)
{
    free(S->diag); free(S->off); free(S->b); free(S->K); free(S->C);
}

/* h^{(0)} = guess (or h^n).  For m = 0.. : assemble at h^m, solve for
 * h^{m+1} by DIC-PCG started from h^m, delta = max|h^{m+1}-h^m| over active
 * cells; converged when delta < tol_picard.  On success the state advances
 * and the water balance is updated; on failure the state is untouched. */
static int picard_loop(orc_problem *P, double dt, const double *guess, int max_picard,
                       orc_step_stats *st, int stop_after, double *h_out);

static int picard_step(orc_problem *P, double dt, const double *guess, int max_picard,
                       orc_step_stats *st)
{
    return picard_loop(P, dt, guess, max_picard, st, 0, NULL);
}

/* The Picard loop of picard_step.  With stop_after > 0 the loop stops after
 * that many iterations (or earlier, on convergence or failure), copies the
 * last iterate into h_out and leaves the state untouched. */
static int picard_loop(orc_problem *P, double dt, const double *guess, int max_picard,
                       orc_step_stats *st, int stop_after, double *h_out)
{
    size_t N = ncell(P);
    memset(st, 0, sizeof(*st));
    st->dt = dt;
    st->t = P->t;
    if (!(dt > 0.0)) return ORC_ERR_ARG;
    double *hm = (double *)malloc(sizeof(double) * N);
    double *x = (double *)malloc(sizeof(double) * N);
    orc_system S;
    alloc_system(N, &S);
    memcpy(hm, guess ? guess : P->h, sizeof(double) * N);
    int status = ORC_ERR_NOT_CONVERGED;
    for (int m = 0; m < max_picard; m++) {
        assemble(P, hm, P->h, dt, P->t, &S);
        memcpy(x, hm, sizeof(double) * N);
        int its = pcg_dic(P, &S, x, P->opt.tol_cg, P->opt.max_cg);
        if (its < 0) { status = ORC_ERR_LINEAR; st->picard_iters = m + 1; break; }
        double delta = 0.0;
        int finite = 1;
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++)
                for (int k = 0; k < P->ktop[i + P->nx * j]; k++) {
                    size_t c = (size_t)k + (size_t)P->nz * (i + (size_t)P->nx * j);
                    double d = fabs(x[c] - hm[c]);
                    if (!isfinite(x[c])) finite = 0;
                    if (d > delta) delta = d;
                }
        if (m < ORC_MAX_PICARD_LOG) { st->cg_iters[m] = its; st->delta[m] = delta; }
        st->cg_iters_total += its;
        st->picard_iters = m + 1;
        memcpy(hm, x, sizeof(double) * N);
        if (!finite) { status = ORC_ERR_NONFINITE; break; }
        if (delta < P->opt.tol_picard) { status = ORC_OK; break; }
        if (stop_after > 0 && m + 1 >= stop_after) break;
    }
    if (stop_after > 0) {
        memcpy(h_out, hm, sizeof(double) * N);
        free(hm); free(x); free_system(&S);
        return status;
    }
    if (status == ORC_OK) {
        boundary_inflow(P, hm, S.K, dt, P->t, P->inflow);
        memcpy(P->h, hm, sizeof(double) * N);
        P->t += dt;
        P->storage = storage_of(P, P->h);
        st->converged = 1;
        st->t = P->t;
    }
    free(hm); free(x); free_system(&S);
    return status;
}

int orc_step(orc_problem *P, double dt, const double *guess, orc_step_stats *st)
{
    return picard_step(P, dt, guess, P->opt.max_picard, st);
}

/* The Picard iterate h^m of a step of size dt from the state hn at the
 * current time (the iterates of orc_step, for inspection): m >= 1 Picard
 * iterations from h^(0) = hn, fewer if the loop converges first.  The
 * problem's state is left as it was. */
int orc_picard_iterate(orc_problem *P, const double *hn, double dt, int m, double *out)
{
    if (m < 1 || !(dt > 0.0)) return ORC_ERR_ARG;
    const size_t N = ncell(P);
    double *saved = P->h;
    double *start = (double *)malloc(sizeof(double) * N);
    memcpy(start, hn, sizeof(double) * N);
    P->h = start;
    orc_step_stats st;
    const int s = picard_loop(P, dt, NULL, m, &st, m, out);
    P->h = saved;
    free(start);
    return s;
}

/* End of the forcing segment that contains t (infinity if none). */
static double next_forcing_change(const orc_problem *P, double t)
{
    double tn = INFINITY;
    for (int f = 0; f < 6; f++) {
        if (P->bc_type[f] != ORC_FLUX) continue;
        for (int s = 0; s < P->nseg[f]; s++)
            if (P->seg_t[f][s] > t * (1.0 + 1e-15) + 1e-12 && P->seg_t[f][s] < tn) tn = P->seg_t[f][s];
    }
    return tn;
}

/* Time loop to t_end.  With ebats = 0 every step uses dt0 (the last one is
 * clipped to t_end).  With ebats = 1 (Sec. 2.2): a step that fails, or
 * needs more than max_iters Picard iterations, is rerun with dt/factor; after
 * inc_after consecutive accepted steps with at most few_iters Picard
 * iterations dt is multiplied by factor (capped at dt_max) and the count
 * restarts.  Steps end on forcing-segment boundaries. */
int orc_run(orc_problem *P, double t_end, orc_run_stats *rs)
{
    memset(rs, 0, sizeof(*rs));
    orc_step_stats st;
    while (P->t < t_end * (1.0 - 1e-15) - 1e-12) {
        double dt = P->opt.ebats ? P->dt_cur : P->opt.dt0;
        double tf = next_forcing_change(P, P->t);
        int clipped = 0;
        if (P->t + dt > tf) { dt = tf - P->t; clipped = 1; }
        if (P->t + dt > t_end) { dt = t_end - P->t; clipped = 1; }
        int maxp = P->opt.ebats ? P->opt.max_iters : P->opt.max_picard;
        int s = picard_step(P, dt, NULL, maxp, &st);
        rs->picard_total += st.picard_iters;
        rs->cg_total += st.cg_iters_total;
        if (s == ORC_ERR_NONFINITE && !P->opt.ebats) return s;
        if (s != ORC_OK) {
            rs->rejected++;
            if (!P->opt.ebats) return s;
            P->dt_cur = dt / P->opt.factor;
            P->easy_count = 0;
            if (P->dt_cur < P->opt.dt_min) { rs->t = P->t; rs->dt_last = P->dt_cur; return ORC_ERR_NOT_CONVERGED; }
            continue;
        }
        rs->accepted++;
        if (P->opt.ebats) {
            if (!clipped) P->dt_cur = dt;
            if (st.picard_iters <= P->opt.few_iters) {
                if (++P->easy_count >= P->opt.inc_after) {
                    P->dt_cur = fmin(P->dt_cur * P->opt.factor, P->opt.dt_max);
                    P->easy_count = 0;
                }
            } else {
                P->easy_count = 0;
            }
        }
    }
    rs->t = P->t;
    rs->dt_last = P->opt.ebats ? P->dt_cur : P->opt.dt0;
    return ORC_OK;
}

/* out = {storage, storage0, inflow[6], error = storage - storage0 - sum inflow} */
int orc_mass_balance(const orc_problem *P, double *out)
{
    double in = 0.0;
    out[0] = P->storage;
    out[1] = P->storage0;
    for (int f = 0; f < 6; f++) { out[2 + f] = P->inflow[f]; in += P->inflow[f]; }
    out[8] = P->storage - P->storage0 - in;
    return ORC_OK;
}

/* ======================================================================
 * Introspection for per-stage parity checks
 * ====================================================================== */

/* System of the Picard iterate hm for the current state h^n and step dt:
 * diag[N], off[6N] (directions -x,+x,-y,+y,-z,+z), b[N], K[N], C[N]. */
int orc_assemble(orc_problem *P, const double *hm, double dt,
                 double *diag, double *off, double *b, double *K, double *C)
{
    orc_system S = {diag, off, b, K, C};
    if (!(dt > 0.0)) return ORC_ERR_ARG;
    assemble(P, hm, P->h, dt, P->t, &S);
    return ORC_OK;
}

/* Solve the system (diag, off, b) with DIC-PCG from x (in/out). */
int orc_pcg(orc_problem *P, const double *diag, const double *off, const double *b,
            double *x, double tol, int max_it)
{
    orc_system S = {(double *)diag, (double *)off, (double *)b, NULL, NULL};
    return pcg_dic(P, &S, x, tol, max_it);
}

/* y = A x for an assembled system. */
int orc_matvec(orc_problem *P, const double *diag, const double *off, const double *x, double *y)
{
    orc_system S = {(double *)diag, (double *)off, NULL, NULL, NULL};
    matvec(P, &S, x, y);
    return ORC_OK;
}

/* z = M^-1 r with the DIC preconditioner of the system. */
int orc_dic_apply(orc_problem *P, const double *diag, const double *off, const double *r, double *z)
{
    size_t N = ncell(P);
    orc_system S = {(double *)diag, (double *)off, NULL, NULL, NULL};
    double *rD = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    int s = dic_factor(P, &S, rD);
    if (s == ORC_OK) dic_apply(P, &S, rD, r, w, z);
    free(rD); free(w);
    return s;
}

double orc_storage(const orc_problem *P, const double *h) { return storage_of(P, h); }
double orc_time(const orc_problem *P) { return P->t; }
double orc_dt(const orc_problem *P) { return P->dt_cur; }

/* theta~, C (Eq. 3) and K (Eq. 4) of every cell of the problem at h. */
int orc_eval_cells(const orc_problem *P, const double *h, double *theta, double *C, double *K)
{
    size_t N = ncell(P);
    double p[6];
    for (size_t c = 0; c < N; c++) {
        cell_params(P, c, p);
        if (theta) theta[c] = orc_theta(P->model, h[c], p);
        if (C) C[c] = orc_capacity(P->model, h[c], p);
        if (K) K[c] = orc_conductivity(P->model, h[c], p);
    }
    return ORC_OK;
}
