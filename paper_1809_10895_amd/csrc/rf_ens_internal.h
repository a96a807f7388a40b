// Internal declarations shared by the column-ensemble kernels
// (rf_ensemble.hip) and their host side (rf_ensemble_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rf_ensemble.h"
#include "rf_internal.h"

namespace rf {

constexpr int kEnsMaxP = 7;   // cells per lane: RF_ENS_MAX_LEN = 64 * kEnsMaxP
static_assert(RF_ENS_MAX_LEN == kWave * kEnsMaxP, "column length limit");

// Per-column soil: the van Genuchten-Mualem layer (m = 1 - 1/n) and Ks.
struct EnsSoil {
    Layer L;
    double ks;
    double pad;
};

// Options of the time loop, as kernel arguments.
struct EnsOpt {
    double tol_picard, chord_eps, dt0, dt_max, dt_min, factor, dz;
    int max_picard, ebats, inc_after, few_iters, max_iters, variant, model;
    int bc_type[2];         // [0] base (RF_ZMIN), [1] top (RF_ZMAX)
    double bc_value[2];
};

// Bounds of one run (kernel arguments).
struct EnsRunParams {
    double t_end;
    long long max_steps;    // accepted + rejected steps per column and run
    long long max_ticks;    // wall-clock budget of the run, in wall_clock64 ticks
};

// Device arrays in the bound workspace.
struct EnsArrays {
    double *h;              // packed heads
    EnsSoil *soil;          // [ncol]
    int32_t *len;           // [ncol]
    int64_t *off;           // [ncol]
    int32_t *order;         // [ncol] queue order (decreasing length)
    rf_ens_column *col;     // [ncol] per-column state and counters
    rf_ens_summary *sum;    // totals of the last run
    unsigned int *queue;    // next queue position
    double *h_bak;          // autotuner: copy of h
    rf_ens_column *col_bak; // autotuner: copy of the column records
};

hipError_t launch_ens_init(const EnsArrays &a, int ncol, const EnsOpt &o, double t, hipStream_t s);
hipError_t launch_ens_check(const EnsArrays &a, long ncell, hipStream_t s);
hipError_t launch_ens_reset(const EnsArrays &a, hipStream_t s);
hipError_t launch_ens_run(const EnsArrays &a, int ncol, const EnsOpt &o, const EnsRunParams &rp,
                          bool mixed, int nblocks, int waves_per_block, hipStream_t s);
hipError_t launch_ens_summary(const EnsArrays &a, int ncol, hipStream_t s);
// Largest dynamic occupancy (blocks per CU) of the run kernel for a block size.
int ens_max_blocks_per_cu(bool mixed, int waves_per_block);

}  // namespace rf
