/*
 * rf_ensemble.h -- C ABI of the column ensemble: many independent 1-D
 * vertical soil columns advanced together on one MI355X (gfx950).
 *
 * Each column is the Richards equation of rf.h (Orgogozo et al.,
 * arXiv:1809.10895, Sec. 1, Eqs. 1-4) on a 1 m x 1 m x (len * dz) stack of
 * cells with its own van Genuchten-Mualem parameters, discretised exactly as
 * the 3-D solver does it (Sec. 2.2: backward Euler, classical or modified
 * Picard, arithmetic-mean face conductivity, explicit gravity; Sec. 2.3: the
 * Picard exit test over the column; EBATS per column, Sec. 2.2).  On a
 * column the 7-point operator is tridiagonal, and the paper's DIC-PCG
 * (Sec. 2.2) converges in one iteration to its exact LDL^T solve; the
 * ensemble solves that factorisation directly.
 *
 * Conventions (as in rf.h): SI units, z upward, k = 0 the bottom cell.  The
 * state of all columns is one packed device array: column c occupies
 * elements [off_c, off_c + len_c) with off_c = len_0 + ... + len_{c-1}.
 * Host pointers are copied during the call; device pointers belong to the
 * caller; the library never allocates device memory (the caller binds a
 * workspace) and enqueues all work on the stream given to rf_ens_create.
 * Every call returns an rf_status; rf_ens_last_error() explains the last
 * failure.  Order: rf_ens_create -> rf_ens_setup -> rf_ens_bind_workspace ->
 * rf_ens_set_state -> rf_ens_run.  Boundary conditions, options and the tile
 * may change at any time after rf_ens_setup (a change of `precision` needs
 * no new workspace here).
 */
#ifndef RF_ENSEMBLE_H
#define RF_ENSEMBLE_H

#include "rf.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RF_ENS_MAX_LEN 448   /* cells per column: 7 per lane of a 64-lane wavefront */

typedef struct rf_ens rf_ens;

/* Launch shape of the persistent kernel: waves_per_block wavefronts per
 * workgroup (one column per wavefront at a time, taken from a shared queue
 * in order of decreasing length) and blocks_per_cu workgroups per compute
 * unit.  rf_ens_autotune picks one by timing. */
typedef struct {
    int waves_per_block;   /* 1, 2, 4 or 8 */
    int blocks_per_cu;     /* 1 .. 16 */
} rf_ens_tile;

/* Per-column record (rf_ens_get_columns). */
typedef struct {
    int status;            /* RF_OK, RF_ERR_NOT_CONVERGED (fixed dt: Picard limit;
                              EBATS: dt fell below dt_min) or RF_ERR_NONFINITE */
    int accepted, rejected;
    int easy;              /* EBATS count of consecutive easy steps */
    long picard_total;     /* Picard iterations, rejected steps included */
    double t;              /* time the column has reached [s] */
    double dt_next;        /* step EBATS will try next [s] */
    double storage0;       /* sum of dz * theta~(h) at rf_ens_set_state [m] */
    double storage;        /* the same now [m] */
    double inflow_top;     /* water entered through the top since rf_ens_set_state [m] */
    double inflow_bottom;  /* the same through the base (negative = drainage) [m] */
} rf_ens_column;

/* Totals of one rf_ens_run. */
typedef struct {
    long accepted, rejected, picard_total;
    long cell_steps;       /* sum over columns of len * accepted steps */
    int failed;            /* columns whose status is not RF_OK */
    double t_min;          /* smallest time reached by a column [s] */
    double max_balance_error;  /* max over columns of |storage - storage0 - inflows| [m] */
    double kernel_ms;      /* duration of the persistent kernel (HIP events) [ms] */
} rf_ens_summary;

rf_status rf_ens_create(rf_ens **out, int hip_device, void *hip_stream);
rf_status rf_ens_destroy(rf_ens *e);
const char *rf_ens_last_error(const rf_ens *e);

/* ncol >= 1 columns; len[c] in [1, RF_ENS_MAX_LEN] cells of height dz > 0;
 * soil[6c .. 6c+5] = theta_r, theta_s, alpha [1/m], n (> 1), Ks [m/s],
 * S [1/m] of column c (host).  model: RF_VGM (Eqs. 2-4) or RF_GARDNER
 * (App. A).  RF_ERR_ARG on an out-of-range value. */
rf_status rf_ens_setup(rf_ens *e, int ncol, const int32_t *len, double dz, int model,
                       const double *soil);
/* Boundary condition shared by every column, face RF_ZMIN or RF_ZMAX, types
 * as in rf_set_bc (Sec. 3.1, App. A).  Defaults: no flow. */
rf_status rf_ens_set_bc(rf_ens *e, int face, int type, double value);
/* Uses tol_picard, max_picard, chord_eps, dt0, dt_max, dt_min, ebats,
 * inc_after, few_iters, max_iters, factor, precision and picard_variant of
 * rf_options (rf_default_options gives the defaults).  RF_PREC_MIXED solves
 * each Picard increment's tridiagonal system in FP32; coefficients, the
 * residual and h stay FP64 (the Picard loop refines the FP32 solve). */
rf_status rf_ens_set_options(rf_ens *e, const rf_options *o);
rf_status rf_ens_set_tile(rf_ens *e, const rf_ens_tile *t);
/* Bounds of one rf_ens_run: at most max_steps steps (accepted + rejected)
 * per column, and max_seconds of wall clock for the launch, after which
 * every column stops at its last accepted state and rf_ens_run reports
 * RF_ERR_NOT_CONVERGED (a later call continues).  Defaults: 1e8 steps, 60 s. */
rf_status rf_ens_set_limits(rf_ens *e, long max_steps, double max_seconds);
rf_status rf_ens_get_tile(const rf_ens *e, rf_ens_tile *t);

/* Total cells of the packed state. */
rf_status rf_ens_cells(const rf_ens *e, long *ncell);
rf_status rf_ens_workspace_bytes(const rf_ens *e, size_t *bytes);
/* Binds `bytes` of device memory at dev (256-byte aligned) as the workspace
 * and uploads the column table. */
rf_status rf_ens_bind_workspace(rf_ens *e, void *dev, size_t bytes);

/* Sets every column's head from h_dev (device, packed, rf_ens_cells doubles)
 * at time t, resets the per-column EBATS state (dt = dt0), counters and
 * water-balance accumulators.  RF_ERR_NONFINITE if a value is not finite. */
rf_status rf_ens_set_state(rf_ens *e, const double *h_dev, double t);
rf_status rf_ens_get_state(const rf_ens *e, double *h_dev);

/* Advances every column from its own time to t_end in ONE persistent kernel
 * launch: each wavefront takes a column from the queue and runs its whole
 * time loop (steps, Picard iterations, EBATS) with the column held in
 * registers.  A column that fails keeps its last accepted state and its
 * status; the others go on.  Returns
 * RF_ERR_NOT_CONVERGED or RF_ERR_NONFINITE if any column failed (the
 * summary says how many), RF_OK otherwise.  *out may be NULL.
 * Currently switched off: returns RF_ERR_STATE (rf_ens_last_error says why)
 * without launching anything, as does rf_ens_autotune. */
rf_status rf_ens_run(rf_ens *e, double t_end, rf_ens_summary *out);

/* Copies the ncol per-column records to host memory out[ncol]. */
rf_status rf_ens_get_columns(const rf_ens *e, rf_ens_column *out);

/* Times rf_ens_run over t_span seconds for each launch shape of a fixed
 * candidate set (wavefronts per block x blocks per CU), restoring the state
 * after each trial; keeps and returns the fastest in *best (may be NULL).
 * The state, counters and balances are as before the call. */
rf_status rf_ens_autotune(rf_ens *e, double t_span, rf_ens_tile *best);

#ifdef __cplusplus
}
#endif

#endif /* RF_ENSEMBLE_H */
