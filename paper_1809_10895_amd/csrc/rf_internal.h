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
constexpr int kMaxBlocks = 512;     // 2 per CU on 256 CUs; one partial per thread when combined
constexpr int kRedSlots = 8;        // values per block partial

// Per-layer van Genuchten parameters (Ks is per cell).
struct Layer {
    double tr, ts, a, n, m, S;
};

struct Soil {
    int model;
    int nlayer;
    Layer L[RF_MAX_LAYERS];
};

// Geometry and launch shape of one grid.
struct Geo {
    int nx, ny, nz, ncol;
    int nblk;               // blocks launched (multiple of 8 when >= 8)
    int cpb;                // columns per logical block
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

// Scalars kept on the device between kernels of the PCG loop.  Every field
// is written by thread 0 of block 0 only, and never read by the other blocks
// of the kernel that writes it (results reach them at the next kernel
// boundary), so no inter-block fence or atomic is needed.
struct Scalars {
    double rho[2];    // r.z of iteration j kept in slot j & 1
    double resmax;    // max |r / diag| seen by the last direction update
    double pq;
    int iters;        // PCG updates completed (written by the update kernel)
    int jcur;         // index of the direction update in flight (spmv kernel)
    int done;         // PCG finished (converged, hit max_cg or failed)
    int fail;         // 1 breakdown (p.q <= 0), 2 max_cg reached, 3 non-finite
    int applied;      // Picard update h^{m+1} = h^m + e written
    int final_iters;  // PCG iterations of the finished solve
    int pad[2];
};

// Device arrays inside the bound workspace.
struct Arrays {
    double *hn, *thn, *hm, *hnew, *K, *Dd, *bst, *diag, *r, *p0, *p1, *q, *e, *z, *Ks;
    double *tz;               // z-line: coupling of cell k with k+1 (A_z K_f / dz)
    double *rdp;              // z-line: reciprocal pivots
    uint8_t *layer;           // may be null
    int32_t *ktop;
    double *pr;               // block partials of (r.z, max|r/diag|)      [kMaxBlocks * 2]
    double *pq;               // block partials of p.q                     [kMaxBlocks]
    double *pd;               // block partials of (max|e|, non-finite)     [kMaxBlocks * 2]
    double *ps;               // block partials of host-side sums           [kMaxBlocks * kRedSlots]
    double *ks_layer;         // Ks of each layer                           [RF_MAX_LAYERS]
    Scalars *sc;
};

// Kernel identifiers for timing.
enum KernelId { K_COEFF = 0, K_RESID, K_SPMV, K_UPDATE, K_APPLYH, K_ACCEPT, K_MISC, K_COUNT };

// Launchers (rf_kernels.hip).  All enqueue on `s` and return the launch status.
hipError_t launch_init_ks(const Geo &g, const Soil &so, const Arrays &a, hipStream_t s);
hipError_t launch_check_finite(const Geo &g, const Arrays &a, const double *h, hipStream_t s);
hipError_t launch_set_state(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            hipStream_t s);
hipError_t launch_coeff(const Geo &g, const Soil &so, const Bc &bc, const Arrays &a, double dt,
                        double chord_eps, hipStream_t s);
hipError_t launch_resid(const Geo &g, const Arrays &a, int precond, double *bout, hipStream_t s);
hipError_t launch_spmv(const Geo &g, const Arrays &a, int precond, const double *p_in,
                       double *p_out, double tol_cg, int max_cg, hipStream_t s);
hipError_t launch_update(const Geo &g, const Arrays &a, int precond, const double *p, hipStream_t s);
hipError_t launch_apply_h(const Geo &g, const Arrays &a, double tol_cg, int max_cg, hipStream_t s);
hipError_t launch_accept(const Geo &g, const Soil &so, const Bc &bc, const Arrays &a,
                         hipStream_t s);
hipError_t launch_eval_soil(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            double *theta, double *C, double *K, hipStream_t s);
hipError_t launch_operator(const Geo &g, const Arrays &a, const double *x, double *y,
                           hipStream_t s);
hipError_t launch_precond(const Geo &g, const Arrays &a, int precond, const double *r, double *z,
                          hipStream_t s);
hipError_t launch_copy_active(const Geo &g, const Arrays &a, const double *src, double *dst,
                              hipStream_t s);

}  // namespace rf
