/*
 * rf.h -- C ABI of the MI355X (gfx950) Richards-equation hot path.
 *
 * The library advances the 3-D transient Richards equation in pressure-head
 * form, C(h) dh/dt = div(K(h) grad(h + z))  (Orgogozo et al.,
 * arXiv:1809.10895, Sec. 1, Eq. 1), on a uniform structured grid of
 * constant-volume hexahedral cells (programme summary, "Restrictions").
 * Each backward-Euler step (Sec. 2.2) is linearised by classical Picard
 * iteration with the chord-slope capacity; pressure diffusion is implicit,
 * gravity explicit from the previous Picard iterate with arithmetic-mean
 * face conductivity (Sec. 2.2, last paragraph); each linear system is solved
 * by preconditioned conjugate gradients (Sec. 2.2); the Picard exit test is
 * global (Sec. 2.3); time steps adapt by EBATS (Sec. 2.2).  Soil properties
 * follow van Genuchten-Mualem, Eqs. 2-4.
 *
 * Conventions shared by every call:
 *   - Units are SI: metres, seconds, m/s.  z (and grad_elev) point upward.
 *   - Cell (i,j,k) of an nx*ny*nz grid is element k + nz*(i + nx*j) of every
 *     per-cell array (z fastest); k = 0 is the bottom layer.  Column (i,j)
 *     holds active cells k < k_top[i + nx*j]; the others are carried
 *     unchanged and never read.
 *   - Host pointers (grid, soil, forcing tables) are copied during the call;
 *     the caller keeps ownership.
 *   - Device pointers (workspace, states, outputs) belong to the caller.  The
 *     library never allocates device memory; all work is enqueued on the
 *     stream given to rf_create and the calls return when the stream has
 *     finished that work (rf_step/rf_run synchronise only to read scalars).
 *   - Every call returns an rf_status; rf_last_error() explains the last
 *     failure.  No call throws.  A context is not thread-safe.
 *   - Required order: rf_create -> rf_setup_grid -> rf_set_soil ->
 *     rf_bind_workspace -> rf_set_state -> rf_step / rf_run.  Boundary
 *     conditions, forcing and options may be set at any time after the grid.
 *     Calls out of order return RF_ERR_STATE.
 */
#ifndef RF_H
#define RF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RF_OK = 0,
    RF_ERR_ARG = -1,           /* invalid argument (NULL, size, range) */
    RF_ERR_STATE = -2,         /* call made out of the required order */
    RF_ERR_HIP = -3,           /* a HIP runtime call failed */
    RF_ERR_NOMEM = -4,         /* workspace smaller than rf_workspace_bytes */
    RF_ERR_NOT_CONVERGED = -5, /* Picard loop did not meet tol_picard */
    RF_ERR_LINEAR = -6,        /* PCG broke down or hit max_cg */
    RF_ERR_NONFINITE = -7      /* NaN/Inf in the state or an iterate */
} rf_status;

enum { RF_VGM = 0, RF_GARDNER = 1 };                           /* soil model */
enum { RF_XMIN = 0, RF_XMAX, RF_YMIN, RF_YMAX, RF_ZMIN, RF_ZMAX }; /* faces */
enum { RF_NOFLOW = 0, RF_DIRICHLET = 1, RF_FLUX = 2, RF_FREE_DRAINAGE = 3 };
enum { RF_PRECOND_JACOBI = 0, RF_PRECOND_ZLINE = 1 };
/* Arithmetic of the Picard / PCG loop.  RF_PREC_FP64: every array and
 * operation FP64.  RF_PREC_MIXED: soil coefficients, the Picard residual
 * b - A h^m and h stay FP64 (each Picard iteration is then one step of
 * iterative refinement of the FP32 solve); the PCG vectors, the operator's
 * K and D copies and the preconditioner are FP32; PCG reductions and
 * scalars stay FP64.  The paper's solver is FP64 throughout (Sec. 2.2):
 * RF_PREC_MIXED is an extension, with results that differ from FP64 by
 * about the PCG and Picard tolerances. */
enum { RF_PREC_FP64 = 0, RF_PREC_MIXED = 1 };
/* Picard linearisation of the storage term (Sec. 2.2).  RF_PICARD_CHORD, the
 * paper's choice: V C (h^{m+1} - h^n) / dt with the chord slope
 * C = (theta~(h^m) - theta~(h^n)) / (h^m - h^n) (Eq. 3 when the two heads are
 * closer than chord_eps).  RF_PICARD_MODIFIED, the mass-conservative form of
 * Celia et al. that Sec. 2.2 also mentions:
 * V [C(h^m) (h^{m+1} - h^m) + theta~(h^m) - theta~(h^n)] / dt with the
 * analytic capacity of Eq. 3.  Both converge to the same backward-Euler
 * solution; the iterations differ. */
enum { RF_PICARD_CHORD = 0, RF_PICARD_MODIFIED = 1 };
/* First Picard iterate of a step when rf_step gets no h_guess_dev.
 * RF_FIRST_PREVIOUS: h^{n+1,0} = h^n (the paper's Picard loop, Sec. 2.2).
 * RF_FIRST_EXTRAPOLATE: h^{n+1,0} = h^n + (dt / dt_prev) (h^n - h^{n-1}), the
 * linear extrapolation of the last accepted increment (h^n after rf_set_state
 * or a change of options); the loop still runs to tol_picard, so only the
 * number of iterations changes. */
enum { RF_FIRST_PREVIOUS = 0, RF_FIRST_EXTRAPOLATE = 1 };
/* When the z-line preconditioner (the exact LDL^T factorisation of each
 * column's vertical tridiagonal, standing in for the DIC of Sec. 2.2) is
 * factorised.
 * RF_REFACTOR_EVERY: every Picard iteration, from that iteration's matrix.
 * RF_REFACTOR_STEP: at the first Picard iteration of each step; the later
 * iterations of the step precondition with those factors.  A preconditioner
 * does not change the solution of the linear system (only how many PCG
 * iterations reach the tolerance), so the Picard iterates are those of
 * RF_REFACTOR_EVERY to within the PCG tolerance. */
enum { RF_REFACTOR_EVERY = 0, RF_REFACTOR_STEP = 1 };
/* How the host waits for the end of a step's enqueued work (once per step).
 * RF_WAIT_SPIN: polls the stream in a loop, keeping one host thread busy for
 * the duration of the step; the next step is enqueued as soon as the device
 * is done.
 * RF_WAIT_BLOCK: hipStreamSynchronize, which may put the thread to sleep and
 * wakes it later (3 % slower per step on a 1 M-cell grid). */
enum { RF_WAIT_SPIN = 0, RF_WAIT_BLOCK = 1 };
/* How the stencil kernels reach a cell's lateral neighbours (grids of at most
 * 64 cells per column; taller columns always use RF_STENCIL_COLUMNS).
 * RF_STENCIL_TILES: a workgroup stages a tile of 8 x tile_rows columns with
 * its one-column halo in LDS, each column read once per tile.
 * RF_STENCIL_COLUMNS: each wavefront loads its column's four neighbour
 * columns itself.
 * RF_STENCIL_AUTO: tiles on grids of more than 16384 columns, where they
 * measure faster; columns otherwise.
 * Results agree to rounding (the same arithmetic per cell, reductions
 * combined in a different order). */
enum { RF_STENCIL_COLUMNS = 0, RF_STENCIL_TILES = 1, RF_STENCIL_AUTO = 2 };

#define RF_MAX_LAYERS 16
#define RF_MAX_PICARD_LOG 128

typedef struct rf_ctx rf_ctx;

typedef struct {
    double tol_picard;  /* Picard exit: max |h^{m+1} - h^m| over the domain [m] (Sec. 2.3) */
    double tol_cg;      /* PCG exit: max |r_c / A_cc| [m] */
    int max_picard;     /* Picard iterations allowed per rf_step */
    int max_cg;         /* PCG iterations allowed per Picard iteration */
    double chord_eps;   /* |h^m - h^n| below this uses the analytic C(h^m) of Eq. 3 [m] */
    int precond;        /* RF_PRECOND_JACOBI or RF_PRECOND_ZLINE */
    int check_every;    /* PCG iterations enqueued between convergence polls (>= 1) */
    double dt0;         /* first time step of rf_run [s] (fixed step when ebats = 0) */
    double dt_max;      /* EBATS upper bound [s] */
    double dt_min;      /* EBATS gives up below this [s] */
    int ebats;          /* 1: adaptive steps in rf_run (Sec. 2.2); 0: fixed dt0 */
    int inc_after;      /* consecutive easy steps before dt *= factor (default 10) */
    int few_iters;      /* an easy step needs at most this many Picard its (default 3) */
    int max_iters;      /* under EBATS a step needing more Picard its is rerun (default 8) */
    double factor;      /* EBATS growth / shrink factor (default 1.3) */
    int cols_per_wave;  /* launch shape of the PCG kernels: z-columns per wavefront
                           (0 = chosen from the grid size) */
    int precision;      /* RF_PREC_FP64 (default) or RF_PREC_MIXED.  Sizes the
                           workspace: changing it on a bound context unbinds the
                           workspace (rf_bind_workspace and rf_set_state again) */
    double cg_rel_tol;  /* PCG also exits once max |r_c / A_cc| has fallen to
                           cg_rel_tol times its value at the start of the solve
                           (0 = the absolute test alone, the default) */
    int picard_variant; /* RF_PICARD_CHORD (default) or RF_PICARD_MODIFIED */
    int first_iterate;  /* RF_FIRST_PREVIOUS (default) or RF_FIRST_EXTRAPOLATE */
    int zline_refactor; /* RF_REFACTOR_EVERY (default) or RF_REFACTOR_STEP */
    int host_wait;      /* RF_WAIT_SPIN (default) or RF_WAIT_BLOCK */
    int stencil;        /* RF_STENCIL_AUTO (default), RF_STENCIL_TILES or RF_STENCIL_COLUMNS */
    int tile_rows;      /* launch shape of RF_STENCIL_TILES: columns of a tile along
                           y, 2 or 4 (0 = chosen: 2) */
} rf_options;

typedef struct {
    int converged;
    int picard_iters;
    int cg_iters_total;
    int cg_iters[RF_MAX_PICARD_LOG];     /* PCG iterations of each Picard iteration */
    double delta[RF_MAX_PICARD_LOG];     /* max |h^{m+1} - h^m| of each Picard iteration */
    double dt;
    double t;                            /* time after the step (before, if rejected) */
} rf_step_stats;

typedef struct {
    int accepted, rejected;
    long picard_total, cg_total;
    double dt_last;   /* step size EBATS will try next */
    double t;
} rf_run_stats;

typedef struct {
    double storage;      /* sum over active cells of V * theta~(h) now [m^3] */
    double storage0;     /* same at the last rf_set_state [m^3] */
    double inflow[6];    /* cumulative boundary inflow per face since rf_set_state [m^3] */
    double error;        /* storage - storage0 - sum(inflow) [m^3] */
} rf_mass;

/* Fills *o with the defaults: tol_picard 1e-6, tol_cg 1e-8 (1/100 of the
 * Picard tolerance, the ratio of Sec. 3.2, 4.2, App. A, App. B), max_picard
 * 50, max_cg 10000, chord_eps 1e-9, z-line preconditioner, check_every 8,
 * dt0 1, dt_max 3600, dt_min 1e-6, EBATS on with 10 / 3 / 8 / 1.3 (Sec. 2.2). */
void rf_default_options(rf_options *o);

/* Creates a context on HIP device `hip_device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *ctx receives the handle. */
rf_status rf_create(rf_ctx **ctx, int hip_device, void *hip_stream);
void rf_destroy(rf_ctx *ctx);
/* Message for the last non-OK status (static storage inside the context). */
const char *rf_last_error(const rf_ctx *ctx);

/* Grid (programme summary "Nature of problem", "Restrictions"): nx*ny*nz
 * cells of dx*dy*dz metres.  k_top (host, nx*ny int32, values clipped to
 * [0, nz]) masks cells above a surface; NULL = all active.  grad_elev (host,
 * 3 doubles) is grad z in grid axes, NULL = (0,0,1).  Invalidates any bound
 * workspace. */
rf_status rf_setup_grid(rf_ctx *ctx, int nx, int ny, int nz, double dx, double dy, double dz,
                        const int32_t *k_top, const double *grad_elev);

/* Soil (Sec. 1, Eqs. 2-4; Sec. 3.2, Eq. 5 for layered sets).  params (host)
 * holds nlayer rows {theta_r, theta_s, alpha [1/m], n, Ks [m/s], S [1/m]}.
 * layer_of_cell (host, N bytes) selects a row per cell, NULL = row 0.
 * ln_ks_offset (host, N doubles) scales Ks per cell by exp(offset), NULL =
 * none.  model RF_GARDNER uses K = Ks exp(alpha h), theta = theta_r +
 * (theta_s - theta_r) exp(alpha h) (Appendix A, Eq. A6). */
rf_status rf_set_soil(rf_ctx *ctx, int model, int nlayer, const double *params,
                      const uint8_t *layer_of_cell, const double *ln_ks_offset);

/* Boundary condition of one face of the domain box (Sec. 3.1, 3.2, App. A,
 * App. B): RF_NOFLOW; RF_DIRICHLET with head `value` [m] (face conductivity
 * K(value), half-cell distance); RF_FLUX with `value` [m/s] positive into the
 * domain; RF_FREE_DRAINAGE (zero pressure gradient, gravity outflow).  On a
 * masked grid RF_ZMAX applies to the top face of each column's highest
 * active cell; faces towards inactive cells are no-flow. */
rf_status rf_set_bc(rf_ctx *ctx, int face, int type, double value);

/* Time-varying flux on an RF_FLUX face (Sec. 3.2): nseg piecewise-constant
 * segments starting at t_start[s] (host, increasing) with flux[s] [m/s].
 * Before t_start[0] the rf_set_bc value applies.  rf_run never lets a step
 * straddle a segment start.  nseg = 0 clears the table. */
rf_status rf_set_forcing(rf_ctx *ctx, int face, int nseg, const double *t_start,
                         const double *flux);

/* RF_ERR_ARG for an out-of-range field (the options are then unchanged).
 * A different `precision` on a bound context unbinds its workspace. */
rf_status rf_set_options(rf_ctx *ctx, const rf_options *opt);

/* Device workspace the caller must provide for the current grid, soil
 * layering and precision option. */
rf_status rf_workspace_bytes(const rf_ctx *ctx, size_t *bytes);
/* Binds `bytes` bytes of device memory at dev_ptr (256-byte aligned) as the
 * workspace; uploads grid and soil tables into it. */
rf_status rf_bind_workspace(rf_ctx *ctx, void *dev_ptr, size_t bytes);

/* Size of the library's static workspace (rf_bind_static_workspace). */
#define RF_STATIC_WORKSPACE_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): rf_bind_workspace
 * with the library's own static workspace, a device array of
 * RF_STATIC_WORKSPACE_BYTES (64 MiB) that each GPU holds from the library's
 * load until the process ends.  Calls no hipMalloc or other allocating
 * routine.  RF_ERR_NOMEM when the grid needs more than that (as
 * rf_workspace_bytes says: about 144 bytes per cell in FP64, so up to about
 * 4.4e5 cells).  Every context bound this way on one GPU shares that GPU's
 * array: binding clears what must start at zero, but work of two such
 * contexts that overlaps in time on one GPU races, and a context's state is
 * lost when another one binds; rf_set_state again after any other context
 * has bound it. */
rf_status rf_bind_static_workspace(rf_ctx *ctx);

/* Sets h^n from h_dev (device, N doubles) at time t; resets the water-balance
 * accumulators and the EBATS state.  RF_ERR_NONFINITE if an active cell of
 * h_dev is not finite (the state is then unchanged). */
rf_status rf_set_state(rf_ctx *ctx, const double *h_dev, double t);
/* Copies h^n into h_dev (device, N doubles, may be NULL) and the time into
 * *t (may be NULL). */
rf_status rf_get_state(const rf_ctx *ctx, double *h_dev, double *t);

/* One backward-Euler step of size dt with the Picard loop (Sec. 2.2, 2.3).
 * h_guess_dev (device, N doubles) is the first Picard iterate; NULL = h^n.
 * On RF_ERR_NOT_CONVERGED / RF_ERR_LINEAR / RF_ERR_NONFINITE the state is
 * left bitwise as before the call.  *out (may be NULL) receives the stats. */
rf_status rf_step(rf_ctx *ctx, double dt, const double *h_guess_dev, rf_step_stats *out);

/* Advances to t_end with fixed dt0 steps (ebats = 0) or EBATS (Sec. 2.2):
 * a step that fails or needs more than max_iters Picard iterations is rerun
 * with dt/factor; after inc_after consecutive accepted steps with at most
 * few_iters iterations dt grows by factor, up to dt_max.  Returns
 * RF_ERR_NOT_CONVERGED if dt falls below dt_min (state at the last accepted
 * step).  *out (may be NULL) receives the totals.  The next step is enqueued
 * before the current one is waited for whenever its dt does not depend on
 * how the current one goes; the results are those of the same steps taken
 * one rf_step at a time.  Nothing is left in flight on return. */
rf_status rf_run(rf_ctx *ctx, double t_end, rf_run_stats *out);

/* rf_run that also stops after max_steps (>= 1) accepted steps: the same
 * steps, in the same way, as rf_run up to that point (EBATS state, run-ahead,
 * statistics); a later rf_run or rf_run_steps continues from there.  Lets a
 * caller take a fixed number of adaptive steps (Sec. 2.2, EBATS), e.g. to
 * time them.  RF_ERR_ARG when max_steps < 1. */
rf_status rf_run_steps(rf_ctx *ctx, double t_end, long max_steps, rf_run_stats *out);

/* Water balance since rf_set_state: storage sum V theta~(h) (Eq. 2 plus
 * S*max(h,0)) and the boundary inflow of every accepted step, evaluated with
 * the converged iterate. */
rf_status rf_mass_balance(const rf_ctx *ctx, rf_mass *out);

/* --- building blocks of one Picard iteration, for inspection and tests --- */

/* theta~(h), C(h) and K(h) (Eqs. 2-4) of every cell at h_dev (device, N);
 * any output pointer may be NULL.  Inactive cells are not written. */
rf_status rf_eval_soil(rf_ctx *ctx, const double *h_dev, double *theta_dev, double *C_dev,
                       double *K_dev);

/* Assembles the Picard system of iterate hm_dev (device, N) for the step
 * h^n -> h^n + dt (Sec. 2.2) and keeps it as the current operator; writes the
 * matrix diagonal A_cc and right-hand side b_c (device, N each, may be NULL)
 * of active cells. */
rf_status rf_assemble(rf_ctx *ctx, const double *hm_dev, double dt, double *diag_dev,
                      double *rhs_dev);
/* y = A x with the operator of the last rf_assemble (device, N each). */
rf_status rf_apply_operator(rf_ctx *ctx, const double *x_dev, double *y_dev);
/* z = M^-1 r with the preconditioner of the last rf_assemble (device, N). */
rf_status rf_apply_precond(rf_ctx *ctx, const double *r_dev, double *z_dev);

/* --- measurement ------------------------------------------------------- */

#define RF_NKERNELS 8
typedef struct {
    const char *name[RF_NKERNELS];  /* "coeff", "resid", "spmv", "update", "apply_h", "accept", "misc" */
    long launches[RF_NKERNELS];     /* launches that did work, timed with HIP events */
    double ms[RF_NKERNELS];         /* summed event time of those launches */
    long idle_launches[RF_NKERNELS];/* PCG launches enqueued past convergence (return at once) */
    double idle_ms[RF_NKERNELS];
    long cells;                     /* active cells of the grid */
} rf_timing;

/* Times the launches of kernel k when bit k of `mask` is set (k indexes
 * rf_timing.name; mask 0xff times every kernel, 0 turns timing off): the
 * launch carries two HIP events in its own dispatch, which record when the
 * kernel starts and ends.  A timed launch costs some overhead (about 2 % of a
 * step when one kernel of the 1 M-cell hillslope is timed).  Waits for the
 * stream and resets the counters. */
rf_status rf_set_timing(rf_ctx *ctx, int mask);
/* Changes which kernels are timed (mask as in rf_set_timing) and in which
 * steps: the first step planned from now on and every `every`-th one after
 * it (every >= 1; 1 = every step), keeping the counters gathered so far;
 * does not wait.  Lets a caller time a sample of the steps of a long run.
 * RF_ERR_ARG when every < 1. */
rf_status rf_select_timing(rf_ctx *ctx, int mask, int every);
rf_status rf_get_timing(rf_ctx *ctx, rf_timing *out);

#ifdef __cplusplus
}
#endif
#endif /* RF_H */
