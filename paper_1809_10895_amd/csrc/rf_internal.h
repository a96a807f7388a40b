// Internal declarations shared by the HIP kernels (rf_kernels.hip) and the
// host orchestrator (rf_host.cpp) of the MI355X Richards-equation library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rf.h"

namespace rf {

constexpr int kWave = 64;           // CDNA wavefront
constexpr int kWavesPerBlock = 8;   // one column per wave at a time
constexpr int kThreads = kWave * kWavesPerBlock;
constexpr int kPartialsMax = 512;   // partials every block of a consumer kernel may combine
constexpr int kRunsPerWave = 12;     // runs of active cells per wave of k_coeff / k_accept on large grids
constexpr int kRedSlots = 8;        // values per block partial
constexpr int kTileX = 8;           // tiled stencil kernels: interior columns of a tile along x
                                    // (one per wave); along y: Geo::tile_y (2 or 4)

// Per-layer van Genuchten parameters (Ks is per cell).
struct Layer {
    double tr, ts, a, n, m, S;
};

struct Soil {
    int model;
    int nlayer;
    Layer L[RF_MAX_LAYERS];
};

// Geometry and launch shapes of one grid.  Kernels that write block
// partials use nblk blocks of cpb columns, or, for the tiled stencil kernels,
// nblk_t blocks of one tile each.  Every consumer combines np partials at
// offset foff (in values of the partial set): the producer's own partials
// (np = nblk, foff = 0) when every producer has the same kPartialsMax or
// fewer blocks; otherwise a one-block fold kernel after each producer
// combines them into the slot foff (np = 1).  Kernels without a reduction
// use nblk_w blocks of cpb_w columns (one column per wave).
struct Geo {
    int nx, ny, nz, ncol;
    int nblk, cpb;          // kernels that write block partials
    int np;                 // partials a consumer combines: nblk, or 1 after a fold kernel
    int foff;               // where they start, in values of nv: 0, or the fold output slot
    int nblk_w, cpb_w;
    int block_map;          // 0 identity, 1 one slab per XCD, 2 slabs entered at staggered points
    int tiled;              // stencil kernels stage kTileX x kTileY tiles with halo in LDS
    int tile_y;             // interior columns of a tile along y (2 or 4)
    int ntx;                // tiles along x
    int nblk_t;             // tiled kernels: blocks (one tile each)
    int nchunk;             // runs of kWave consecutive active cells (column order)
    int nblk_r;             // blocks of the kernels over those runs (k_coeff, k_accept)
    long nact;              // active cells
    double V;               // cell volume
    double A[3];            // face areas normal to x, y, z
    double Tk[3];           // A / distance between centres, per unit K
    double g[3];            // grad of elevation
};

// Boundary conditions of the six faces at the current time.
struct Bc {
    int type[6];
    double value[6];        // Dirichlet head or flux (already resolved at time t)
};

// Scalars kept on the device across the kernels of one time step.  Every
// field is written by thread 0 of block 0 only, and never read back by the
// other blocks of the kernel that writes it except where all blocks take the
// same decision anyway, so no inter-block fence or atomic is needed: values
// reach other blocks at the next kernel boundary.
struct Scalars {
    // PCG of the current Picard iteration
    double rho[2];    // r.z of iteration j kept in slot j & 1
    double resmax;    // max |r / diag| seen by the last direction update
    double pq;
    double alpha;     // alpha of the last direction update; the next spmv kernel (or, after
                      // the solve's last update, k_apply_h) adds alpha p to e
    int iters;        // PCG updates completed (written by the update kernel)
    int plast;        // direction buffer the last spmv kernel that went on wrote (0: p0, 1: p1;
                      // the host's parity of an iteration need not follow the device's count)
    int jcur;         // index of the direction update in flight (spmv kernel)
    int done;         // PCG finished (converged, hit max_cg or failed)
    int fail;         // 1 breakdown (p.q <= 0), 2 max_cg reached, 3 non-finite
    int final_iters;  // PCG iterations of the finished solve
    // Picard control of the step
    int stall;        // PCG of iteration stall_m not finished within the enqueued chunk
    int stall_m;
    int picard_done;  // an update met tol_picard (decided by the next coefficient kernel)
    int picard_m;     // Picard iteration whose update met tol_picard
    int accepted;     // the step was accepted
    int accept_m;
    int cur_m;        // Picard iteration whose residual was formed last
    int accepted_serial;  // host serial of the last step accepted (written by k_accept only)
    int pad;
    double tol_eff;   // PCG exit tolerance of the current solve (absolute, or relative in FP32)
    int cg_log[RF_MAX_PICARD_LOG];       // PCG iterations of each Picard iteration
    double delta_log[RF_MAX_PICARD_LOG]; // max |h^{m+1} - h^m| of each Picard iteration
};

// The arrays one PCG solve works on, in the precision T of that solve: the
// FP64 arrays, or (mixed precision) FP32 copies of the operator and
// preconditioner with FP32 vectors.
template <typename T>
struct CgVec {
    T *K, *Dd, *diag, *tz, *rdp, *r, *p0, *p1, *q, *e, *z;
};

// Device arrays inside the bound workspace.  The Picard iterate h^m (m >= 1)
// lives in hb[m & 1], h^0 at h0m; iteration m writes h^{m+1} into
// hb[(m + 1) & 1].
struct Arrays {
    double *hn, *thn, *hb0, *hb1, *K, *Dd, *bst, *diag, *r, *p0, *p1, *q, *e, *z, *Ks;
    const double *h0m;        // iterate of Picard iteration 0: hn when the step starts
                              // from h^n, else hb0 (filled by k_step_begin)
    double *dh;               // last accepted increment h^n - h^{n-1} (extrapolated first iterate)
    double *tz;               // z-line: coupling of cell k with k+1 (A_z K_f / dz)
    double *rdp;              // z-line: reciprocal pivots
    uint8_t *layer;           // may be null
    int32_t *ktop;
    const int4 *chunk;        // per run q of kWave active cells (cells kWave q .. in column
                              // order): x = column of its first cell, y = that cell's k,
                              // z = lane bounds l1 | l2 << 8 | l3 << 16 where the run moves
                              // to columns x+1, x+2, x+3 (65: not within the run)
    double *pr;               // block partials of (r.z, max|r/diag|)  [(nblk + 1) * 2]
    double *pq;               // block partials of p.q                 [nblk + 1]
    double *pd;               // block partials of (max|e|, non-finite) [(nblk + 1) * 2]
    double *ps;               // block partials of host-side sums       [(nblk + 1) * kRedSlots]
    double *ks_layer;         // Ks of each layer                           [RF_MAX_LAYERS]
    double *krb;              // K(h_b)/Ks of each Dirichlet face and layer [6 * RF_MAX_LAYERS]
    Layer *layers;            // van Genuchten parameters of each layer     [RF_MAX_LAYERS]
    double *bt;               // boundary coefficients of each face          [6 * 4]
    CgVec<float> f;           // FP32 PCG arrays (mixed precision only; null otherwise)
    Scalars *sc;
};

// Kernel identifiers for timing.
enum KernelId { K_COEFF = 0, K_RESID, K_SPMV, K_UPDATE, K_APPLYH, K_ACCEPT, K_DECIDE, K_BEGIN };

// Launchers (rf_kernels.hip).  All enqueue on `s` and return the launch status.
//
// Timing: after arm_launch_events(a, b) the next kernel that a launcher
// enqueues on this thread carries the two events in its own dispatch, so a
// records when that kernel starts and b when it ends (the fold kernel a
// launcher may add after it is not included).  disarm_launch_events()
// clears them and says whether they were still unused.
void arm_launch_events(hipEvent_t start, hipEvent_t stop);
bool disarm_launch_events();
hipError_t launch_init_ks(const Geo &g, const Soil &so, const Arrays &a, hipStream_t s);
hipError_t launch_check_finite(const Geo &g, const Arrays &a, const double *h, hipStream_t s);
hipError_t launch_set_state(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            hipStream_t s);
// Step flags and boundary tables; with h0 (not null) also hb0 = h0 + ratio *
// dh (ratio 0: a copy of h0), for a.h0m = hb0.  Without h0 the step starts
// from h^n (a.h0m = hn) and one block does the rest.  gate >= 0: only if the
// step with that serial has been accepted; otherwise nothing is done and the
// step's later kernels are held (stall raised with stall_m = -1).
hipError_t launch_step_begin(const Geo &g, const Soil &so, const Bc &bc, const Arrays &a,
                             const double *h0, double ratio, int gate, hipStream_t s);
hipError_t launch_decide(const Geo &g, const Arrays &a, int m, double tol_picard, hipStream_t s);
hipError_t launch_coeff(const Geo &g, const Soil &so, const Arrays &a, int m, double dt,
                        double chord_eps, int variant, hipStream_t s);
// PCG tolerances of one solve: exit when max|r/diag| <= max(tol_cg,
// rel * (its value at the start)); rel = 0 in FP64.
struct CgTol {
    double tol_cg, rel;
    int max_cg;
};

// refactor: compute (and store) the z-line factors of this iteration's matrix;
// otherwise the stored ones are used.  The residual and update launchers add,
// when consumers read folded partials, a one-block fold that also takes the
// next spmv kernel's exit decision with the tolerances t.
hipError_t launch_resid(const Geo &g, const Arrays &a, int precond, int m, double *bout,
                        bool mixed, bool refactor, const CgTol &t, hipStream_t s);
hipError_t launch_spmv(const Geo &g, const Arrays &a, int precond, bool mixed, int parity,
                       const CgTol &t, hipStream_t s);
// factors_current: the z-line factors are this Picard iteration's (the
// diagonal is then rebuilt from them instead of read).
hipError_t launch_update(const Geo &g, const Arrays &a, int precond, bool mixed, int parity,
                         bool factors_current, const CgTol &t, hipStream_t s);
hipError_t launch_apply_h(const Geo &g, const Arrays &a, int m, bool mixed, const CgTol &t,
                          hipStream_t s);
// track: also dh = h^{n+1} - h^n.  serial: the host's tag of the step,
// recorded on acceptance.
hipError_t launch_accept(const Geo &g, const Soil &so, const Arrays &a, bool track, int serial,
                         hipStream_t s);
hipError_t launch_eval_soil(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            double *theta, double *C, double *K, hipStream_t s);
hipError_t launch_operator(const Geo &g, const Arrays &a, const double *x, double *y,
                           hipStream_t s);
hipError_t launch_precond(const Geo &g, const Arrays &a, int precond, const double *r, double *z,
                          hipStream_t s);
// Folds the nprod (default g.nblk) partials of nv values (max where bit i of
// maxmask is set) of the last producer into the slot P[g.foff*nv ..] when
// consumers read a folded total (g.np == 1, g.foff > 0); no-op otherwise.
// The fold reads only block partials, so folding again after a producer
// that returned early gives the same total.
hipError_t launch_fold(const Geo &g, double *P, int nv, unsigned maxmask, hipStream_t s,
                       int nprod = -1);
hipError_t launch_copy_active(const Geo &g, const Arrays &a, const double *src, double *dst,
                              hipStream_t s);
// Zeroes `bytes` (a multiple of 4) at device address p with a kernel.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);

// Host-side entry points shared by the C ABI's source files (rf_host.cpp).
// The device of a context, and the binding of a device workspace of `bytes`
// at dev_ptr (what rf_bind_workspace does after its argument checks).
int ctx_device(const rf_ctx *c);
rf_status ctx_bind(rf_ctx *c, void *dev_ptr, size_t bytes);

}  // namespace rf
