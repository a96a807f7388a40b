// Host orchestrator and C ABI of the MI355X Richards-equation library.
//
// The host owns only control flow: the Picard loop of one backward-Euler
// step (Sec. 2.2), the global exit test (Sec. 2.3), the EBATS time loop
// (Sec. 2.2), forcing lookup and the water-balance accumulators.  All
// per-cell arithmetic runs in the HIP kernels of rf_kernels.hip, enqueued on
// the caller's stream; the host reads back a few scalars once per PCG poll.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "rf_internal.h"

using namespace rf;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kArraySkew = 4352;   // 17 x 256 B

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct EvPair {
    hipEvent_t a, b;
    int kernel;
    int serial; // step of the launch
    int m;      // Picard iteration of the launch (-1: none)
    int j;      // PCG iteration of an spmv/update launch, launch count of apply_h/accept
};

// One step as the host enqueued it: where it starts, what its first kernel
// needs, how much Picard and PCG work went in, and where its scalars and
// acceptance partials are read back.
struct StepRec {
    int serial = 0;             // tag the acceptance kernel leaves on the device
    int slot = 0;               // readback slot (pinned host mirrors and event)
    int timing = 0;             // kernels timed in this step
    double t = 0.0, dt = 0.0;   // start time and time step
    double ratio = 0.0;         // first iterate h^n + ratio (h^n - h^{n-1})
    const double *guess = nullptr;
    const double *h0m = nullptr;   // where Picard iteration 0 reads h^0
    int max_picard = 1;
    int M = 0;                  // Picard iterations enqueued
    int naccept = 0;            // acceptance launches enqueued
    rf::Bc bc{};
    int pairs_enq[RF_MAX_PICARD_LOG];   // PCG iterations enqueued per Picard iteration
    int apply_enq[RF_MAX_PICARD_LOG];   // Picard-update launches per Picard iteration
};

}  // namespace

struct rf_ctx {
    int device = 0;
    int n_cu = 0;             // compute units of the device
    hipStream_t stream = nullptr;
    char err[512] = {0};

    bool have_grid = false, have_soil = false, have_ws = false, have_state = false;
    int nx = 0, ny = 0, nz = 0;
    double dx = 0, dy = 0, dz = 0;
    double gvec[3] = {0, 0, 1};
    std::vector<int32_t> ktop;
    std::vector<int32_t> chunk;            // active-cell runs, 4 ints each (Arrays::chunk)
    long active = 0;

    int model = RF_VGM;
    int nlayer = 0;
    double params[RF_MAX_LAYERS][6];
    std::vector<uint8_t> layer;
    std::vector<double> lnks;

    int bc_type[6] = {0, 0, 0, 0, 0, 0};
    double bc_value[6] = {0, 0, 0, 0, 0, 0};
    std::vector<double> seg_t[6], seg_q[6];

    rf_options opt;

    void *ws = nullptr;
    size_t ws_bytes = 0;
    Arrays A{};
    Geo G{};
    Soil S{};

    double t = 0.0, dt_cur = 1.0;
    int easy = 0;
    double dt_prev = 0.0;                  // last accepted dt with dh tracked (0: none)
    double storage0 = 0.0, storage = 0.0, inflow[6] = {0, 0, 0, 0, 0, 0};
    int pred_picard = 3;                   // Picard iterations enqueued up front
    int pred_cg[RF_MAX_PICARD_LOG];        // PCG iterations enqueued per Picard iteration
    int serial = 0;                        // last step serial handed out
    StepRec rec[2];                        // steps in flight (two when rf_run runs ahead)

    Scalars *hsc = nullptr;   // pinned host mirrors of the device scalars, one per slot
    double *hpart = nullptr;  // pinned host copies of block partials, one area per slot
    hipEvent_t done_ev[2] = {nullptr, nullptr};   // recorded after each slot's readback
    bool assembled = false;

    int timing = 0;           // bit k: time kernel k
    int timing_every = 1;     // in every timing_every-th step
    long timing_count = 0;    // steps planned since the selection
    std::vector<EvPair> pending;
    std::vector<EvPair> freelist;
    rf_timing tm{};
};

static const char *kKernelNames[RF_NKERNELS] = {"coeff", "resid", "spmv", "update",
                                                "apply_h", "accept", "decide", "begin"};

static rf_status fail(rf_ctx *c, rf_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, RF_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// timing helpers
// ---------------------------------------------------------------------------

static void timed_begin(rf_ctx *c, const StepRec &r, int kernel, int m, int j, EvPair &p)
{
    p.kernel = -1;
    if (!((r.timing >> kernel) & 1)) return;
    if (c->freelist.empty()) {
        // timing-only events: no system-scope fence (no L2 writeback and
        // invalidate) at each record, so they do not slow the kernels they
        // bracket and time those rather than the fences
        EvPair q;
        (void)hipEventCreateWithFlags(&q.a, hipEventDisableSystemFence);
        (void)hipEventCreateWithFlags(&q.b, hipEventDisableSystemFence);
        c->freelist.push_back(q);
    }
    p = c->freelist.back();
    c->freelist.pop_back();
    p.kernel = kernel;
    p.serial = r.serial;
    p.m = m;
    p.j = j;
    arm_launch_events(p.a, p.b);
}

// The launcher's kernel took the events; should none have (no launch), both
// are recorded here, an empty interval.
static void timed_end(rf_ctx *c, EvPair &p)
{
    if (p.kernel < 0) return;
    if (disarm_launch_events()) {
        (void)hipEventRecord(p.a, c->stream);
        (void)hipEventRecord(p.b, c->stream);
    }
    c->pending.push_back(p);
}

// After step `serial`: a launch did work iff the device logs say so (kernels
// enqueued speculatively past the end of a PCG solve or of the Picard loop
// return at once).  last_m: last Picard iteration that ran; cg[m]: PCG
// iterations of iteration m; napply[m] / naccept: launches of the kind.
// Events of other steps stay pending.
static void timed_collect(rf_ctx *c, int serial, int last_m, const int *cg, const int *napply,
                          int naccept)
{
    if (c->pending.empty()) return;
    std::vector<int> seen_apply(RF_MAX_PICARD_LOG, 0);
    int seen_accept = 0;
    std::vector<EvPair> other;
    for (auto &p : c->pending) {
        if (p.serial != serial) {
            other.push_back(p);
            continue;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        bool work = true;
        const int m = p.m;
        const bool logged = m >= 0 && m < RF_MAX_PICARD_LOG;
        switch (p.kernel) {
        case K_COEFF: case K_RESID: case K_DECIDE:
            work = m <= last_m;
            break;
        case K_SPMV: case K_UPDATE:
            work = logged && m <= last_m && p.j < cg[m];
            break;
        case K_APPLYH:
            work = logged && m <= last_m && ++seen_apply[m] == napply[m];
            break;
        case K_ACCEPT:
            work = ++seen_accept == naccept;
            break;
        default:
            break;
        }
        if (work) {
            c->tm.launches[p.kernel]++;
            c->tm.ms[p.kernel] += ms;
        } else {
            c->tm.idle_launches[p.kernel]++;
            c->tm.idle_ms[p.kernel] += ms;
        }
        c->freelist.push_back(p);
    }
    c->pending.swap(other);
}

// Returns the events of one step (serial >= 0) or of every step to the pool.
static void timed_drop(rf_ctx *c, int serial = -1)
{
    std::vector<EvPair> other;
    for (auto &p : c->pending) {
        if (serial < 0 || p.serial == serial) c->freelist.push_back(p);
        else other.push_back(p);
    }
    c->pending.swap(other);
}

#define TIMED(ctx, rec, kid, m, j, call)                                \
    do {                                                                \
        EvPair ev_;                                                     \
        timed_begin(ctx, rec, kid, m, j, ev_);                          \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) {                                         \
            disarm_launch_events();                                     \
            if (ev_.kernel >= 0) ctx->freelist.push_back(ev_);          \
            return fail(ctx, RF_ERR_HIP, "launch %s: %s", kKernelNames[kid], \
                        hipGetErrorString(e_));                         \
        }                                                               \
        timed_end(ctx, ev_);                                            \
    } while (0)

// ---------------------------------------------------------------------------
// layout
// ---------------------------------------------------------------------------

static size_t max_partial_blocks(const rf_ctx *c)
{
    const size_t ncol = (size_t)c->nx * c->ny;
    size_t nb = (ncol + kWavesPerBlock - 1) / kWavesPerBlock;
    if (nb >= 8) nb = (nb + 7) / 8 * 8;
    // tiled stencil kernels: one block per tile of kTileX x 2 or more columns
    size_t nt = (size_t)((c->nx + kTileX - 1) / kTileX) * ((c->ny + 1) / 2);
    nt = std::min<size_t>(nt, (size_t)1 << 22);
    return std::max(nb, nt);
}

static size_t layout(const rf_ctx *c, char *base, Arrays *A)
{
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    const size_t ncol = (size_t)c->nx * c->ny;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    Arrays a{};
    double **dbl[] = {&a.hn, &a.thn, &a.hb0, &a.hb1, &a.K, &a.Dd, &a.bst, &a.diag, &a.r,
                      &a.p0, &a.p1, &a.q, &a.e, &a.z, &a.Ks, &a.tz, &a.rdp, &a.dh};
    // Per-cell arrays are often a power of two in size; a kernel streams several
    // of them at the same index, so successive arrays are skewed by a few KiB
    // plus a fraction of a DRAM page to keep those streams on different
    // channels.
    int ia = 0;
    for (double **p : dbl) *p = (double *)take(N * sizeof(double) + kArraySkew * (size_t)(++ia % 8));
    if (c->opt.precision == RF_PREC_MIXED) {
        CgVec<float> &f = a.f;
        float **flt[] = {&f.K, &f.Dd, &f.diag, &f.tz, &f.rdp, &f.r, &f.p0, &f.p1, &f.q, &f.e, &f.z};
        for (float **p : flt) *p = (float *)take(N * sizeof(float) + kArraySkew * (size_t)(++ia % 8));
    }
    a.layer = c->layer.empty() ? nullptr : (uint8_t *)take(N);
    a.ktop = (int32_t *)take(ncol * sizeof(int32_t));
    a.chunk = (const int4 *)take(std::max<size_t>(c->chunk.size(), 4) * sizeof(int32_t));
    const size_t nb1 = max_partial_blocks(c) + 1;
    a.pr = (double *)take(nb1 * 2 * sizeof(double));
    a.pq = (double *)take(nb1 * sizeof(double));
    a.pd = (double *)take(nb1 * 2 * sizeof(double));
    a.ps = (double *)take(nb1 * kRedSlots * sizeof(double));
    a.ks_layer = (double *)take(RF_MAX_LAYERS * sizeof(double));
    a.krb = (double *)take(6 * RF_MAX_LAYERS * sizeof(double));
    a.layers = (Layer *)take(RF_MAX_LAYERS * sizeof(Layer));
    a.bt = (double *)take(24 * sizeof(double));
    a.sc = (Scalars *)take(sizeof(Scalars));
    a.h0m = a.hb0;
    if (A) *A = a;
    return off;
}

// Launch shapes of the grid (see Geo).  Partial arrays are sized for one
// column per wave, so changing the shape never changes the workspace layout.
// The runs of kWave consecutive active cells (in column order, columns of
// no active cell skipped) that the per-cell kernels give one wavefront each:
// for run q, its first cell (column, k) and the lanes where it enters each
// of the next three columns, l1 <= l2 <= l3 (65 when the run ends first);
// lanes from l3 on walk the active lengths themselves.
static void build_chunks(rf_ctx *c)
{
    const size_t ncol = c->ktop.size();
    const long nchunk = (c->active + kWave - 1) / kWave;
    c->chunk.assign((size_t)nchunk * 4, 0);
    size_t col = 0;
    int k = 0;
    for (long q = 0; q < nchunk; q++) {
        while (col < ncol && k >= c->ktop[col]) {
            k = 0;
            col++;
        }
        int l[3];
        int lane = c->ktop[col] - k;             // where the run leaves column col
        size_t nc = col;
        for (int t = 0; t < 3; t++) {
            l[t] = std::min(lane, kWave + 1);
            nc++;
            if (lane <= kWave) lane += (nc < ncol) ? c->ktop[nc] : kWave + 1;
        }
        int32_t *r = &c->chunk[(size_t)q * 4];
        r[0] = (int32_t)col;
        r[1] = k;
        r[2] = l[0] | (l[1] << 8) | (l[2] << 16);
        r[3] = 0;
        // advance kWave active cells
        int left = kWave;
        while (left > 0 && col < ncol) {
            const int room = c->ktop[col] - k;
            if (room > left) {
                k += left;
                left = 0;
            } else {
                left -= room;
                col++;
                k = 0;
            }
        }
    }
}

static void set_shapes(rf_ctx *c)
{
    Geo &G = c->G;
    const size_t ncol = (size_t)c->nx * c->ny;
    // kernels without block partials: one column per wave
    size_t nw = (ncol + kWavesPerBlock - 1) / kWavesPerBlock;
    nw = std::min<size_t>(nw, (size_t)1 << 20);
    if (nw >= 8) nw = (nw + 7) / 8 * 8;
    G.nblk_w = (int)nw;
    G.cpb_w = (int)((ncol + nw - 1) / nw);
    // kernels with block partials: cols_per_wave columns per wave (latency
    // hiding needs many waves; a large grid pays one fold kernel per reduction)
    const int cpw = std::max(1, c->opt.cols_per_wave > 0 ? c->opt.cols_per_wave : 4);
    size_t nb = (ncol + (size_t)kWavesPerBlock * cpw - 1) / ((size_t)kWavesPerBlock * cpw);
    nb = std::min<size_t>(nb, (size_t)1 << 20);
    if (nb >= 8) nb = (nb + 7) / 8 * 8;
    G.nblk = (int)nb;
    G.cpb = (int)((ncol + nb - 1) / nb);

    // When the whole grid of the reducing kernels is resident at once (two
    // blocks per CU), give each XCD one slab of consecutive columns: the
    // +-y neighbour columns of a block then sit in its own XCD's L2 instead
    // of being fetched again by another XCD (spmv moved 1.5x its algorithmic
    // bytes with the identity map).  Larger grids stream through in launch
    // order, where the identity map measured faster.
    G.block_map = (c->n_cu > 0 && G.nblk <= 2 * c->n_cu) ? 1 : 0;
    // tiled stencil kernels (columns of at most one wave, grids of at least
    // one tile): one block per tile, their own partial count
    // tile height (a taller tile reads fewer halo columns from L2 or HBM
    // but takes more LDS per block, and fewer blocks fit a CU); one block
    // per tile, on grids of at most 2^22 tiles
    G.tile_y = (c->opt.tile_rows > 0) ? c->opt.tile_rows : 2;
    G.ntx = (c->nx + kTileX - 1) / kTileX;
    const long ntiles = (long)G.ntx * ((c->ny + G.tile_y - 1) / G.tile_y);
    G.nblk_t = (int)std::min<long>(ntiles, 1L << 22);
    // tiles where the column kernels' own grid already needs fold kernels
    // (large grids); on smaller grids both measure alike and tiles would add
    // folds
    const bool want = c->opt.stencil == RF_STENCIL_TILES ||
                      (c->opt.stencil == RF_STENCIL_AUTO && G.nblk > kPartialsMax);
    G.tiled = want && c->nz <= kWave && c->nx >= kTileX && c->ny >= G.tile_y &&
              ntiles <= (1L << 22);
    // what consumers of block partials read (see Geo): the producers' own
    // partials if they all have the same, few enough blocks; else a folded
    // total in the slot after the largest producer's partials
    const int nprod = std::max(G.nblk, G.tiled ? G.nblk_t : 0);
    const bool same = !G.tiled || G.nblk_t == G.nblk;
    if (nprod <= 1) {
        G.np = 1;
        G.foff = 0;
    } else if (nprod > kPartialsMax || !same) {
        G.np = 1;
        G.foff = nprod;
    } else {
        G.np = G.nblk;
        G.foff = 0;
    }
    // k_coeff and k_accept walk runs of active cells, FP64-ALU bound: where
    // their partials are folded anyway (large grids), a grid of kRunsPerWave
    // runs per wave pays each wave's start-up (the record and the soil table)
    // over several runs; elsewhere they take the reducing kernels' grid,
    // whose partials the host reads as written
    G.nblk_r = G.nblk;
    if (G.np == 1 && G.foff != 0) {
        const long per = (long)kWavesPerBlock * kRunsPerWave;
        G.nblk_r = (int)std::max<long>(8, std::min<long>(G.nblk, (G.nchunk + per - 1) / per));
    }
}


static Bc bc_at(const rf_ctx *c, double t)
{
    Bc b;
    for (int f = 0; f < 6; f++) {
        b.type[f] = c->bc_type[f];
        b.value[f] = c->bc_value[f];
        const auto &ts = c->seg_t[f];
        if (c->bc_type[f] == RF_FLUX && !ts.empty() && t >= ts[0]) {
            size_t s = 0;
            while (s + 1 < ts.size() && ts[s + 1] <= t) s++;
            b.value[f] = c->seg_q[f][s];
        }
    }
    return b;
}

static double next_forcing_change(const rf_ctx *c, double t)
{
    double tn = INFINITY;
    for (int f = 0; f < 6; f++) {
        if (c->bc_type[f] != RF_FLUX) continue;
        for (double s : c->seg_t[f])
            if (s > t * (1.0 + 1e-15) + 1e-12 && s < tn) tn = s;
    }
    return tn;
}

constexpr size_t kSlotPartials = (size_t)kPartialsMax * kRedSlots;

// Enqueues the copy of the nv-valued block partials of the last kernel into
// readback slot `slot` (combine_partials reads them after a wait).
static rf_status copy_partials(rf_ctx *c, const double *dev, int nv, int slot = 0)
{
    HIPCHK(c, hipMemcpyAsync(c->hpart + slot * kSlotPartials, dev + (size_t)c->G.foff * nv,
                             (size_t)c->G.np * nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return RF_OK;
}

// Combines copied partials on the host in block order (sum, or max where
// bit i of maxmask is set).
static void combine_partials(const rf_ctx *c, int nv, unsigned maxmask, double *tot, int slot = 0)
{
    const double *hp = c->hpart + slot * kSlotPartials;
    for (int i = 0; i < nv; i++) tot[i] = 0.0;
    for (int b = 0; b < c->G.np; b++)
        for (int i = 0; i < nv; i++) {
            const double x = hp[(size_t)b * nv + i];
            tot[i] = ((maxmask >> i) & 1u) ? std::max(tot[i], x) : tot[i] + x;
        }
}

// A step's readback: the device scalars and the acceptance kernel's
// partials (storage, face inflows) into the step's slot, then the slot's
// event.  The partials are only used when the scalars say the step was
// accepted, and then the acceptance kernel was the last one to write them.
constexpr int kAcceptSlots = 7;
static rf_status enqueue_readback(rf_ctx *c, const StepRec &r)
{
    HIPCHK(c, hipMemcpyAsync(c->hsc + r.slot, c->A.sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                             c->stream));
    rf_status s = copy_partials(c, c->A.ps, kAcceptSlots, r.slot);
    if (s) return s;
    HIPCHK(c, hipEventRecord(c->done_ev[r.slot], c->stream));
    return RF_OK;
}

// Waits for the last readback of a slot.  last: nothing is enqueued behind
// it, so the stream itself can be polled.
static rf_status wait_readback(rf_ctx *c, int slot, bool last)
{
    if (c->opt.host_wait == RF_WAIT_BLOCK) {
        HIPCHK(c, hipEventSynchronize(c->done_ev[slot]));
        return RF_OK;
    }
    // polled until the work has completed or failed
    for (;;) {
        const hipError_t q = last ? hipStreamQuery(c->stream) : hipEventQuery(c->done_ev[slot]);
        if (q == hipSuccess) return RF_OK;
        if (q != hipErrorNotReady) HIPCHK(c, q);
    }
}

// Copies the nv-valued block partials of the last kernel, waits, and
// combines them.
static rf_status host_reduce(rf_ctx *c, const double *dev, int nv, unsigned maxmask, double *tot)
{
    rf_status s = copy_partials(c, dev, nv);
    if (s) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    combine_partials(c, nv, maxmask, tot);
    return RF_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void rf_default_options(rf_options *o)
{
    if (!o) return;
    o->tol_picard = 1e-6;
    o->tol_cg = 1e-8;
    o->max_picard = 50;
    o->max_cg = 10000;
    o->chord_eps = 1e-9;
    o->precond = RF_PRECOND_ZLINE;
    o->check_every = 8;
    o->dt0 = 1.0;
    o->dt_max = 3600.0;
    o->dt_min = 1e-6;
    o->ebats = 1;
    o->inc_after = 10;
    o->few_iters = 3;
    o->max_iters = 8;
    o->factor = 1.3;
    o->cols_per_wave = 0;
    o->precision = RF_PREC_FP64;
    o->cg_rel_tol = 0.0;
    o->picard_variant = RF_PICARD_CHORD;
    o->first_iterate = RF_FIRST_PREVIOUS;
    o->zline_refactor = RF_REFACTOR_EVERY;
    o->host_wait = RF_WAIT_SPIN;
    o->stencil = RF_STENCIL_AUTO;
    o->tile_rows = 0;
}

rf_status rf_create(rf_ctx **out, int hip_device, void *hip_stream)
{
    if (!out) return RF_ERR_ARG;
    *out = nullptr;
    rf_ctx *c = new (std::nothrow) rf_ctx();
    if (!c) return RF_ERR_NOMEM;
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    rf_default_options(&c->opt);
    c->dt_cur = c->opt.dt0;
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipHostMalloc((void **)&c->hsc, 2 * sizeof(Scalars), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->hpart, 2 * kSlotPartials * sizeof(double),
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->done_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->done_ev[1], hipEventDisableTiming) != hipSuccess) {
        if (c->hsc) (void)hipHostFree(c->hsc);
        if (c->hpart) (void)hipHostFree(c->hpart);
        if (c->done_ev[0]) (void)hipEventDestroy(c->done_ev[0]);
        delete c;
        return RF_ERR_HIP;
    }
    memset(c->hsc, 0, 2 * sizeof(Scalars));
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess)
        c->n_cu = 0;
    c->tm.cells = 0;
    for (int k = 0; k < RF_NKERNELS; k++) c->tm.name[k] = kKernelNames[k];
    for (int m = 0; m < RF_MAX_PICARD_LOG; m++) c->pred_cg[m] = 2;
    *out = c;
    return RF_OK;
}

void rf_destroy(rf_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto &p : c->freelist) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    if (c->hsc) (void)hipHostFree(c->hsc);
    if (c->hpart) (void)hipHostFree(c->hpart);
    for (hipEvent_t ev : c->done_ev)
        if (ev) (void)hipEventDestroy(ev);
    delete c;
}

const char *rf_last_error(const rf_ctx *c) { return c ? c->err : "null context"; }

rf_status rf_setup_grid(rf_ctx *c, int nx, int ny, int nz, double dx, double dy, double dz,
                        const int32_t *k_top, const double *grad_elev)
{
    if (!c) return RF_ERR_ARG;
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !(dy > 0) || !(dz > 0) ||
        (double)nx * ny > 2e9 || (double)nx * ny * nz > 4e10)
        return fail(c, RF_ERR_ARG, "invalid grid %d x %d x %d / %g %g %g", nx, ny, nz, dx, dy, dz);
    c->nx = nx; c->ny = ny; c->nz = nz;
    c->dx = dx; c->dy = dy; c->dz = dz;
    c->gvec[0] = grad_elev ? grad_elev[0] : 0.0;
    c->gvec[1] = grad_elev ? grad_elev[1] : 0.0;
    c->gvec[2] = grad_elev ? grad_elev[2] : 1.0;
    const size_t ncol = (size_t)nx * ny;
    c->ktop.assign(ncol, nz);
    c->active = 0;
    for (size_t i = 0; i < ncol; i++) {
        int kt = k_top ? k_top[i] : nz;
        kt = std::max(0, std::min(nz, kt));
        c->ktop[i] = kt;
        c->active += kt;
    }
    build_chunks(c);
    Geo &G = c->G;
    G.nx = nx; G.ny = ny; G.nz = nz;
    G.ncol = (int)ncol;
    G.nact = c->active;
    G.nchunk = (int)(c->chunk.size() / 4);
    set_shapes(c);
    G.V = dx * dy * dz;
    G.A[0] = dy * dz; G.A[1] = dx * dz; G.A[2] = dx * dy;
    G.Tk[0] = G.A[0] / dx; G.Tk[1] = G.A[1] / dy; G.Tk[2] = G.A[2] / dz;
    for (int i = 0; i < 3; i++) G.g[i] = c->gvec[i];
    c->have_grid = true;
    c->have_soil = false;
    c->have_ws = false;
    c->have_state = false;
    c->assembled = false;
    c->layer.clear();
    c->lnks.clear();
    c->tm.cells = c->active;
    return RF_OK;
}

static rf_status upload_soil(rf_ctx *c)
{
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    Arrays &A = c->A;
    if (!c->layer.empty() && !A.layer)
        return fail(c, RF_ERR_STATE, "layer table added after binding: bind the workspace again");
    if (A.layer) HIPCHK(c, hipMemcpyAsync(A.layer, c->layer.data(), N, hipMemcpyHostToDevice, c->stream));
    if (!c->lnks.empty())
        HIPCHK(c, hipMemcpyAsync(A.Ks, c->lnks.data(), N * sizeof(double), hipMemcpyHostToDevice,
                                 c->stream));
    else
        HIPCHK(c, launch_zero(A.Ks, N * sizeof(double), c->stream));
    double ksl[RF_MAX_LAYERS];
    for (int l = 0; l < c->nlayer; l++) ksl[l] = c->params[l][4];
    HIPCHK(c, hipMemcpyAsync(A.ks_layer, ksl, sizeof(ksl), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(A.layers, c->S.L, sizeof(c->S.L), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_init_ks(c->G, c->S, A, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RF_OK;
}

rf_status rf_set_soil(rf_ctx *c, int model, int nlayer, const double *params,
                      const uint8_t *layer_of_cell, const double *ln_ks_offset)
{
    if (!c) return RF_ERR_ARG;
    if (!c->have_grid) return fail(c, RF_ERR_STATE, "rf_set_soil before rf_setup_grid");
    if (!params || nlayer < 1 || nlayer > RF_MAX_LAYERS || (model != RF_VGM && model != RF_GARDNER))
        return fail(c, RF_ERR_ARG, "invalid soil arguments");
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    for (int l = 0; l < nlayer; l++) {
        const double *p = params + 6 * l;
        if (!(p[0] >= 0) || !(p[1] > p[0]) || !(p[2] > 0) || !(p[4] > 0) || !(p[5] >= 0) ||
            (model == RF_VGM && !(p[3] > 1.0)))
            return fail(c, RF_ERR_ARG, "invalid soil parameters in layer %d", l);
    }
    if (layer_of_cell)
        for (size_t i = 0; i < N; i++)
            if (layer_of_cell[i] >= nlayer) return fail(c, RF_ERR_ARG, "layer index out of range");
    const bool had_layer = !c->layer.empty();
    c->model = model;
    c->nlayer = nlayer;
    for (int l = 0; l < nlayer; l++) memcpy(c->params[l], params + 6 * l, 6 * sizeof(double));
    if (layer_of_cell) c->layer.assign(layer_of_cell, layer_of_cell + N); else c->layer.clear();
    if (ln_ks_offset) c->lnks.assign(ln_ks_offset, ln_ks_offset + N); else c->lnks.clear();
    Soil &S = c->S;
    S.model = model;
    S.nlayer = nlayer;
    for (int l = 0; l < nlayer; l++) {
        const double *p = params + 6 * l;
        S.L[l].tr = p[0]; S.L[l].ts = p[1]; S.L[l].a = p[2]; S.L[l].n = p[3];
        S.L[l].m = (model == RF_VGM) ? 1.0 - 1.0 / p[3] : 0.0;
        S.L[l].S = p[5];
    }
    c->have_soil = true;
    if (c->have_ws) {
        if (had_layer != !c->layer.empty()) {
            c->have_ws = false;   // layout changes: the caller must bind again
            c->have_state = false;
            return RF_OK;
        }
        rf_status s = upload_soil(c);
        if (s) return s;
        c->have_state = false;
    }
    return RF_OK;
}

rf_status rf_set_bc(rf_ctx *c, int face, int type, double value)
{
    if (!c) return RF_ERR_ARG;
    if (!c->have_grid) return fail(c, RF_ERR_STATE, "rf_set_bc before rf_setup_grid");
    if (face < 0 || face > 5 || type < 0 || type > 3 || !std::isfinite(value))
        return fail(c, RF_ERR_ARG, "invalid boundary condition");
    c->bc_type[face] = type;
    c->bc_value[face] = value;
    return RF_OK;
}

rf_status rf_set_forcing(rf_ctx *c, int face, int nseg, const double *t_start, const double *flux)
{
    if (!c) return RF_ERR_ARG;
    if (!c->have_grid) return fail(c, RF_ERR_STATE, "rf_set_forcing before rf_setup_grid");
    if (face < 0 || face > 5 || nseg < 0 || (nseg > 0 && (!t_start || !flux)))
        return fail(c, RF_ERR_ARG, "invalid forcing");
    for (int s = 1; s < nseg; s++)
        if (!(t_start[s] > t_start[s - 1])) return fail(c, RF_ERR_ARG, "forcing times must increase");
    c->seg_t[face].assign(t_start, t_start + nseg);
    c->seg_q[face].assign(flux, flux + nseg);
    return RF_OK;
}

rf_status rf_set_options(rf_ctx *c, const rf_options *o)
{
    if (!c || !o) return RF_ERR_ARG;
    if (!(o->tol_picard > 0) || !(o->tol_cg > 0) || o->max_picard < 1 || o->max_cg < 1 ||
        !(o->chord_eps >= 0) || (o->precond != RF_PRECOND_JACOBI && o->precond != RF_PRECOND_ZLINE) ||
        o->check_every < 1 || !(o->dt0 > 0) || !(o->dt_max > 0) || !(o->dt_min > 0) ||
        o->inc_after < 1 || o->few_iters < 1 || o->max_iters < 1 || !(o->factor > 1.0) ||
        o->cols_per_wave < 0 || (o->precision != RF_PREC_FP64 && o->precision != RF_PREC_MIXED) ||
        !(o->cg_rel_tol >= 0.0 && o->cg_rel_tol < 1.0) ||
        (o->picard_variant != RF_PICARD_CHORD && o->picard_variant != RF_PICARD_MODIFIED) ||
        (o->first_iterate != RF_FIRST_PREVIOUS && o->first_iterate != RF_FIRST_EXTRAPOLATE) ||
        (o->zline_refactor != RF_REFACTOR_EVERY && o->zline_refactor != RF_REFACTOR_STEP) ||
        (o->host_wait != RF_WAIT_SPIN && o->host_wait != RF_WAIT_BLOCK) ||
        (o->stencil != RF_STENCIL_COLUMNS && o->stencil != RF_STENCIL_TILES &&
         o->stencil != RF_STENCIL_AUTO) ||
        (o->tile_rows != 0 && o->tile_rows != 2 && o->tile_rows != 4))
        return fail(c, RF_ERR_ARG, "invalid options");
    if (c->have_ws && o->precision != c->opt.precision) {
        // the FP32 arrays exist only in a workspace laid out for them
        c->have_ws = false;
        c->have_state = false;
        c->assembled = false;
    }
    c->opt = *o;
    c->dt_cur = o->dt0;
    c->easy = 0;
    c->dt_prev = 0.0;
    if (c->have_grid) set_shapes(c);
    return RF_OK;
}

rf_status rf_workspace_bytes(const rf_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return RF_ERR_ARG;
    if (!c->have_grid || !c->have_soil) return RF_ERR_STATE;
    *bytes = layout(c, nullptr, nullptr);
    return RF_OK;
}

}  // extern "C"

int rf::ctx_device(const rf_ctx *c) { return c->device; }

// Binds `bytes` of device memory at dev_ptr as the workspace: lays out the
// arrays, uploads the grid and soil tables and clears the device scalars.
// Allocates nothing.
rf_status rf::ctx_bind(rf_ctx *c, void *dev_ptr, size_t bytes)
{
    if (!c->have_grid || !c->have_soil)
        return fail(c, RF_ERR_STATE, "workspace bound before grid and soil");
    if (!dev_ptr || ((uintptr_t)dev_ptr % kAlign) != 0)
        return fail(c, RF_ERR_ARG, "workspace must be a 256-byte aligned device pointer");
    const size_t need = layout(c, nullptr, nullptr);
    if (bytes < need)
        return fail(c, RF_ERR_NOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
    HIPCHK(c, hipSetDevice(c->device));
    layout(c, (char *)dev_ptr, &c->A);
    c->ws = dev_ptr;
    c->ws_bytes = bytes;
    HIPCHK(c, hipMemcpyAsync(c->A.ktop, c->ktop.data(), c->ktop.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
    if (!c->chunk.empty())
        HIPCHK(c, hipMemcpyAsync((void *)c->A.chunk, c->chunk.data(), c->chunk.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_zero(c->A.sc, sizeof(Scalars), c->stream));
    rf_status s = upload_soil(c);
    if (s) return s;
    c->have_ws = true;
    c->have_state = false;
    c->assembled = false;
    return RF_OK;
}

extern "C" {

rf_status rf_bind_workspace(rf_ctx *c, void *dev_ptr, size_t bytes)
{
    if (!c) return RF_ERR_ARG;
    return ctx_bind(c, dev_ptr, bytes);
}

rf_status rf_set_state(rf_ctx *c, const double *h_dev, double t)
{
    if (!c || !h_dev) return RF_ERR_ARG;
    if (!c->have_ws) return fail(c, RF_ERR_STATE, "rf_set_state before rf_bind_workspace");
    if (!std::isfinite(t)) return fail(c, RF_ERR_ARG, "non-finite time");
    HIPCHK(c, launch_check_finite(c->G, c->A, h_dev, c->stream));
    double bad = 0.0;
    rf_status s = host_reduce(c, c->A.ps, 1, 0u, &bad);
    if (s) return s;
    if (bad != 0.0)
        return fail(c, RF_ERR_NONFINITE, "%.0f non-finite active cells in the state", bad);
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    // inactive cells are carried unchanged: take the whole array first
    HIPCHK(c, hipMemcpyAsync(c->A.hn, h_dev, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, launch_set_state(c->G, c->S, c->A, h_dev, c->stream));
    double st = 0.0;
    s = host_reduce(c, c->A.ps, 1, 0u, &st);
    if (s) return s;
    c->storage0 = c->storage = st;
    for (int f = 0; f < 6; f++) c->inflow[f] = 0.0;
    c->t = t;
    c->dt_cur = c->opt.dt0;
    c->easy = 0;
    c->dt_prev = 0.0;
    c->have_state = true;
    return RF_OK;
}

rf_status rf_get_state(const rf_ctx *cc, double *h_dev, double *t)
{
    rf_ctx *c = const_cast<rf_ctx *>(cc);
    if (!c) return RF_ERR_ARG;
    if (!c->have_state) return fail(c, RF_ERR_STATE, "rf_get_state before rf_set_state");
    if (h_dev) {
        const size_t N = (size_t)c->nx * c->ny * c->nz;
        HIPCHK(c, hipMemcpyAsync(h_dev, c->A.hn, N * sizeof(double), hipMemcpyDeviceToDevice,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (t) *t = c->t;
    return RF_OK;
}

static bool mixed(const rf_ctx *c) { return c->opt.precision == RF_PREC_MIXED; }

static CgTol cg_tol(const rf_ctx *c) { return CgTol{c->opt.tol_cg, c->opt.cg_rel_tol, c->opt.max_cg}; }

// Enqueues n more PCG iterations of Picard iteration m of step r (the
// direction buffers alternate with the iteration count).
static rf_status enqueue_pairs(rf_ctx *c, StepRec &r, int m, int n)
{
    c->A.h0m = r.h0m;
    Arrays &A = c->A;
    const int pc = c->opt.precond;
    const int mi = std::min(m, RF_MAX_PICARD_LOG - 1);
    for (int i = 0; i < n; i++) {
        const int j = r.pairs_enq[mi]++;
        TIMED(c, r, K_SPMV, m, j, launch_spmv(c->G, A, pc, mixed(c), j & 1, cg_tol(c), c->stream));
        const bool current = (m == 0) || c->opt.zline_refactor == RF_REFACTOR_EVERY;
        TIMED(c, r, K_UPDATE, m, j,
              launch_update(c->G, A, pc, mixed(c), j & 1, current, cg_tol(c), c->stream));
    }
    return RF_OK;
}

static rf_status enqueue_apply(rf_ctx *c, StepRec &r, int m)
{
    c->A.h0m = r.h0m;
    const int mi = std::min(m, RF_MAX_PICARD_LOG - 1);
    TIMED(c, r, K_APPLYH, m, r.apply_enq[mi]++,
          launch_apply_h(c->G, c->A, m, mixed(c), cg_tol(c), c->stream));
    return RF_OK;
}

// Picard iteration m: exit test of iteration m-1, coefficients, residual,
// a predicted number of PCG iterations, Picard update.  Every kernel returns
// at once when an earlier one has ended the step.
static rf_status enqueue_iteration(rf_ctx *c, StepRec &r, int m)
{
    c->A.h0m = r.h0m;
    const Geo &G = c->G;
    Arrays &A = c->A;
    const int mi = std::min(m, RF_MAX_PICARD_LOG - 1);
    if (m > 0) TIMED(c, r, K_DECIDE, m, -1, launch_decide(G, A, m, c->opt.tol_picard, c->stream));
    TIMED(c, r, K_COEFF, m, -1, launch_coeff(G, c->S, A, m, r.dt, c->opt.chord_eps,
                                             c->opt.picard_variant, c->stream));
    const bool refactor = (m == 0) || c->opt.zline_refactor == RF_REFACTOR_EVERY;
    TIMED(c, r, K_RESID, m, -1,
          launch_resid(G, A, c->opt.precond, m, nullptr, mixed(c), refactor, cg_tol(c), c->stream));
    rf_status s = enqueue_pairs(c, r, m, std::max(1, c->pred_cg[mi]));
    if (s) return s;
    return enqueue_apply(c, r, m);
}

static bool extrapolating(const rf_ctx *c) { return c->opt.first_iterate == RF_FIRST_EXTRAPOLATE; }

// Exit test of the last enqueued iteration, acceptance, readback.
static rf_status enqueue_accept(rf_ctx *c, StepRec &r)
{
    c->A.h0m = r.h0m;
    TIMED(c, r, K_DECIDE, r.M, -1, launch_decide(c->G, c->A, r.M, c->opt.tol_picard, c->stream));
    TIMED(c, r, K_ACCEPT, r.M, r.naccept,
          launch_accept(c->G, c->S, c->A, extrapolating(c), r.serial, c->stream));
    r.naccept++;
    return enqueue_readback(c, r);
}

// Fills the record of a step from time t with dt.  dt_prev: the step before
// it, for the extrapolated first iterate (0: none).
static void plan_step(rf_ctx *c, StepRec &r, int slot, double t, double dt, double dt_prev,
                      const double *guess, int max_picard)
{
    r.serial = ++c->serial;
    if (r.serial <= 0) r.serial = c->serial = 1;
    r.slot = slot;
    r.timing = (c->timing && (c->timing_count++ % c->timing_every) == 0) ? c->timing : 0;
    r.t = t;
    r.dt = dt;
    r.ratio = (!guess && extrapolating(c) && dt_prev > 0.0) ? dt / dt_prev : 0.0;
    r.guess = guess;
    // a step from h^n reads it in place; a guess or an extrapolated start is
    // formed in hb0 by k_step_begin
    r.h0m = (guess || r.ratio != 0.0) ? c->A.hb0 : c->A.hn;
    r.max_picard = max_picard;
    r.M = 0;
    r.naccept = 0;
    r.bc = bc_at(c, t);
    for (int m = 0; m < RF_MAX_PICARD_LOG; m++) r.pairs_enq[m] = r.apply_enq[m] = 0;
}

// Enqueues a whole step speculatively: as many Picard iterations and PCG
// iterations as the last step needed, acceptance and readback; the device
// decides, after every update, whether to go on.  gate >= 0: the step only
// starts if the step with that serial was accepted (enqueued ahead of it).
static rf_status enqueue_step(rf_ctx *c, StepRec &r, int gate)
{
    c->A.h0m = r.h0m;
    const double *h0 = (r.h0m == c->A.hn) ? nullptr : (r.guess ? r.guess : c->A.hn);
    TIMED(c, r, K_BEGIN, -1, -1,
          launch_step_begin(c->G, c->S, r.bc, c->A, h0, r.ratio, gate, c->stream));
    r.M = std::max(1, std::min(r.max_picard, c->pred_picard));
    for (int m = 0; m < r.M; m++) {
        rf_status s = enqueue_iteration(c, r, m);
        if (s) return s;
    }
    return enqueue_accept(c, r);
}

// Waits for step r and completes it: if the enqueued work fell short (a PCG
// solve not finished, or the Picard test not yet met) enqueues more from
// where the device stopped, until the step is accepted, fails or runs out of
// Picard iterations; then the statistics and the host-side bookkeeping.
// last: nothing is enqueued behind the step's readback.  first_batch: the
// step was accepted by the work enqueued up front (a step enqueued behind it
// with this step's serial as gate has then run).
static rf_status finish_step(rf_ctx *c, StepRec &r, bool last, rf_step_stats *st, bool *first_batch)
{
    memset(st, 0, sizeof(*st));
    st->dt = r.dt;
    st->t = r.t;
    Arrays &A = c->A;
    *first_batch = true;
    rf_status status = RF_OK;
    for (;;) {
        rf_status s = wait_readback(c, r.slot, last);
        if (s) return s;
        const Scalars &h = c->hsc[r.slot];
        if (h.accepted) break;
        if (h.fail) {
            status = (h.fail == 3) ? RF_ERR_NONFINITE : RF_ERR_LINEAR;
            break;
        }
        if (!h.stall && r.M >= r.max_picard) {
            status = RF_ERR_NOT_CONVERGED;
            break;
        }
        // more work for this step, behind everything enqueued so far; the
        // stall flag (raised by this step's PCG, or by a step enqueued behind
        // this one that found it not accepted) is cleared first
        *first_batch = false;
        last = true;
        HIPCHK(c, launch_zero(&A.sc->stall, sizeof(int), c->stream));
        if (h.stall) {
            // PCG of iteration ms needs more iterations than were enqueued
            const int ms = h.stall_m;
            s = enqueue_pairs(c, r, ms, std::max(1, c->opt.check_every / 2));
            if (s) return s;
            s = enqueue_apply(c, r, ms);
            if (s) return s;
            for (int m = ms + 1; m < r.M; m++) {
                s = enqueue_iteration(c, r, m);
                if (s) return s;
            }
        } else {
            const int M2 = std::min(r.max_picard, r.M + std::max(1, r.M / 2));
            for (int m = r.M; m < M2; m++) {
                s = enqueue_iteration(c, r, m);
                if (s) return s;
            }
            r.M = M2;
        }
        s = enqueue_accept(c, r);
        if (s) return s;
    }
    const Scalars h = c->hsc[r.slot];
    const int M = r.M;
    const int last_m = h.accepted ? h.accept_m : (status == RF_ERR_NOT_CONVERGED ? M - 1 : h.cur_m);
    st->picard_iters = last_m + 1;
    for (int m = 0; m <= last_m && m < RF_MAX_PICARD_LOG; m++) {
        const bool solved = m < last_m || h.accepted || status == RF_ERR_NOT_CONVERGED;
        st->cg_iters[m] = solved ? h.cg_log[m] : h.final_iters;
        st->delta[m] = solved ? h.delta_log[m] : 0.0;
        st->cg_iters_total += st->cg_iters[m];
    }
    int cgl[RF_MAX_PICARD_LOG], napp[RF_MAX_PICARD_LOG];
    for (int m = 0; m < RF_MAX_PICARD_LOG; m++) {
        cgl[m] = (m <= last_m) ? st->cg_iters[m] : 0;
        napp[m] = r.apply_enq[m];
    }
    timed_collect(c, r.serial, last_m, cgl, napp, h.accepted ? r.naccept : -1);
    if (status != RF_OK) {
        if (status == RF_ERR_NOT_CONVERGED)
            fail(c, status, "Picard did not converge in %d iterations (dt %g)", r.max_picard, r.dt);
        else
            fail(c, status, "PCG %s in Picard iteration %d after %d iterations",
                 h.fail == 1 ? "breakdown" : h.fail == 2 ? "hit max_cg" : "produced NaN/Inf",
                 h.cur_m, h.final_iters);
        return status;
    }
    // prediction for the next step
    c->pred_picard = last_m + 1;
    for (int m = 0; m <= last_m && m < RF_MAX_PICARD_LOG; m++) c->pred_cg[m] = std::max(1, st->cg_iters[m]);
    double sums[kAcceptSlots];
    combine_partials(c, kAcceptSlots, 0u, sums, r.slot);   // read back with the scalars
    c->storage = sums[0];
    for (int f = 0; f < 6; f++) c->inflow[f] += r.dt * sums[1 + f];
    c->t = r.t + r.dt;
    c->dt_prev = extrapolating(c) ? r.dt : 0.0;
    st->converged = 1;
    st->t = c->t;
    return RF_OK;
}

// One backward-Euler step from c->t, enqueued and completed on its own.
static rf_status picard_step(rf_ctx *c, double dt, const double *guess, int max_picard,
                             rf_step_stats *st)
{
    StepRec &r = c->rec[0];
    plan_step(c, r, 0, c->t, dt, c->dt_prev, guess, max_picard);
    rf_status s = enqueue_step(c, r, -1);
    if (s) return s;
    bool first = true;
    return finish_step(c, r, true, st, &first);
}

rf_status rf_step(rf_ctx *c, double dt, const double *h_guess_dev, rf_step_stats *out)
{
    if (!c) return RF_ERR_ARG;
    if (!c->have_state) return fail(c, RF_ERR_STATE, "rf_step before rf_set_state");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, RF_ERR_ARG, "invalid dt %g", dt);
    timed_drop(c);   // events of a step that ended in an error
    rf_step_stats st;
    rf_status s = picard_step(c, dt, h_guess_dev, c->opt.max_picard, &st);
    if (out) *out = st;
    return s;
}

static bool before(double t, double t_end) { return t < t_end * (1.0 - 1e-15) - 1e-12; }

// Step from t: dt0 clipped at the next change of the forcing and at t_end.
static double fixed_dt(const rf_ctx *c, double t, double t_end, bool *clipped = nullptr)
{
    double dt = c->opt.dt0;
    bool cl = false;
    const double tf = next_forcing_change(c, t);
    if (t + dt > tf) { dt = tf - t; cl = true; }
    if (t + dt > t_end) { dt = t_end - t; cl = true; }
    if (clipped) *clipped = cl;
    return dt;
}

// Fixed steps.  The next step does not depend on how this one went (it is
// this step's end, with dt0), so it is enqueued before this one is waited
// for, gated on this step's acceptance: the device goes from one step to the
// next without waiting for the host.  If this step needed more work than was
// enqueued up front, the next one found it not accepted, did nothing, and is
// enqueued again behind that work.
static rf_status run_fixed(rf_ctx *c, double t_end, long max_acc, rf_run_stats &rs)
{
    if (!before(c->t, t_end)) return RF_OK;
    StepRec *cur = &c->rec[0], *nxt = &c->rec[1];
    plan_step(c, *cur, 0, c->t, fixed_dt(c, c->t, t_end), c->dt_prev, nullptr, c->opt.max_picard);
    rf_status s = enqueue_step(c, *cur, -1);
    if (s) return s;
    for (;;) {
        const double tn = cur->t + cur->dt;
        const bool ahead = before(tn, t_end) && rs.accepted + 1 < max_acc;
        const double dt_prev = extrapolating(c) ? cur->dt : 0.0;
        if (ahead) {
            plan_step(c, *nxt, cur->slot ^ 1, tn, fixed_dt(c, tn, t_end), dt_prev, nullptr,
                      c->opt.max_picard);
            s = enqueue_step(c, *nxt, cur->serial);
            if (s) return s;
        }
        rf_step_stats st;
        bool first = true;
        s = finish_step(c, *cur, !ahead, &st, &first);
        rs.picard_total += st.picard_iters;
        rs.cg_total += st.cg_iters_total;
        if (s != RF_OK) {
            if (s != RF_ERR_HIP) rs.rejected++;
            if (ahead && s != RF_ERR_HIP) {
                // the step behind found this one not accepted and did nothing
                const rf_status w = wait_readback(c, nxt->slot, true);
                if (w) return w;
                timed_drop(c, nxt->serial);
            }
            return s;
        }
        rs.accepted++;
        if (!ahead) return RF_OK;
        if (!first) {
            timed_drop(c, nxt->serial);
            plan_step(c, *nxt, nxt->slot, tn, nxt->dt, dt_prev, nullptr, c->opt.max_picard);
            s = enqueue_step(c, *nxt, -1);
            if (s) return s;
        }
        std::swap(cur, nxt);
    }
}

// EBATS (Sec. 2.2).  The next step's dt depends on how this one goes only
// through acceptance (a rejected step is rerun with dt / factor) and when
// this step could complete a run of inc_after easy steps (dt then grows).
// Otherwise the next step is enqueued ahead, as with fixed steps, with the
// dt it will have if this one is accepted; if it is not, the step behind
// found it not accepted and did nothing.
static rf_status run_ebats(rf_ctx *c, double t_end, long max_acc, rf_run_stats &rs)
{
    if (!before(c->t, t_end)) return RF_OK;
    auto plan_at = [&](StepRec &r, int slot, double t, double dt, double dt_prev, bool &clipped) {
        clipped = false;
        const double tf = next_forcing_change(c, t);
        if (t + dt > tf) { dt = tf - t; clipped = true; }
        if (t + dt > t_end) { dt = t_end - t; clipped = true; }
        plan_step(c, r, slot, t, dt, dt_prev, nullptr, c->opt.max_iters);
    };
    StepRec *cur = &c->rec[0], *nxt = &c->rec[1];
    bool clipped = false, clipped_nxt = false;
    plan_at(*cur, 0, c->t, c->dt_cur, c->dt_prev, clipped);
    rf_status s = enqueue_step(c, *cur, -1);
    if (s) return s;
    for (;;) {
        const double tn = cur->t + cur->dt;
        const bool ahead = before(tn, t_end) && c->easy + 1 < c->opt.inc_after &&
                           rs.accepted + 1 < max_acc;
        if (ahead) {
            // dt_cur after this step if it is accepted (no growth possible here)
            const double dt_next = clipped ? c->dt_cur : cur->dt;
            plan_at(*nxt, cur->slot ^ 1, tn, dt_next, extrapolating(c) ? cur->dt : 0.0,
                    clipped_nxt);
            s = enqueue_step(c, *nxt, cur->serial);
            if (s) return s;
        }
        rf_step_stats st;
        bool first = true;
        s = finish_step(c, *cur, !ahead, &st, &first);
        rs.picard_total += st.picard_iters;
        rs.cg_total += st.cg_iters_total;
        if (s == RF_ERR_HIP || s == RF_ERR_ARG || s == RF_ERR_STATE) return s;
        if (s != RF_OK) {
            rs.rejected++;
            if (ahead) {
                // the step behind found this one not accepted and did nothing
                const rf_status w = wait_readback(c, nxt->slot, true);
                if (w) return w;
                timed_drop(c, nxt->serial);
            }
            c->dt_cur = cur->dt / c->opt.factor;
            c->easy = 0;
            if (c->dt_cur < c->opt.dt_min)
                return fail(c, RF_ERR_NOT_CONVERGED, "EBATS: dt %g fell below dt_min %g", c->dt_cur,
                            c->opt.dt_min);
            plan_at(*cur, cur->slot, cur->t, c->dt_cur, c->dt_prev, clipped);
            s = enqueue_step(c, *cur, -1);
            if (s) return s;
            continue;
        }
        rs.accepted++;
        if (!clipped) c->dt_cur = cur->dt;
        if (st.picard_iters <= c->opt.few_iters) {
            if (++c->easy >= c->opt.inc_after) {
                c->dt_cur = std::min(c->dt_cur * c->opt.factor, c->opt.dt_max);
                c->easy = 0;
            }
        } else {
            c->easy = 0;
        }
        if (!before(tn, t_end) || rs.accepted >= max_acc) return RF_OK;
        if (!ahead || !first) {
            // the next step was not enqueued, or did nothing: enqueue it now
            if (ahead) timed_drop(c, nxt->serial);
            plan_at(*nxt, cur->slot ^ 1, tn, c->dt_cur, c->dt_prev, clipped_nxt);
            s = enqueue_step(c, *nxt, -1);
            if (s) return s;
        }
        std::swap(cur, nxt);
        clipped = clipped_nxt;
    }
}

static rf_status run_capped(rf_ctx *c, double t_end, long max_acc, rf_run_stats *out)
{
    rf_run_stats rs;
    memset(&rs, 0, sizeof(rs));
    timed_drop(c);
    const rf_status ret = c->opt.ebats ? run_ebats(c, t_end, max_acc, rs)
                                       : run_fixed(c, t_end, max_acc, rs);
    rs.t = c->t;
    rs.dt_last = c->opt.ebats ? c->dt_cur : c->opt.dt0;
    if (out) *out = rs;
    return ret;
}

rf_status rf_run(rf_ctx *c, double t_end, rf_run_stats *out)
{
    if (!c) return RF_ERR_ARG;
    if (!c->have_state) return fail(c, RF_ERR_STATE, "rf_run before rf_set_state");
    return run_capped(c, t_end, LONG_MAX, out);
}

rf_status rf_run_steps(rf_ctx *c, double t_end, long max_steps, rf_run_stats *out)
{
    if (!c) return RF_ERR_ARG;
    if (!c->have_state) return fail(c, RF_ERR_STATE, "rf_run_steps before rf_set_state");
    if (max_steps < 1) return fail(c, RF_ERR_ARG, "max_steps %ld < 1", max_steps);
    return run_capped(c, t_end, max_steps, out);
}

rf_status rf_mass_balance(const rf_ctx *c, rf_mass *out)
{
    if (!c || !out) return RF_ERR_ARG;
    if (!c->have_state) return RF_ERR_STATE;
    out->storage = c->storage;
    out->storage0 = c->storage0;
    double in = 0.0;
    for (int f = 0; f < 6; f++) {
        out->inflow[f] = c->inflow[f];
        in += c->inflow[f];
    }
    out->error = c->storage - c->storage0 - in;
    return RF_OK;
}

rf_status rf_eval_soil(rf_ctx *c, const double *h_dev, double *theta_dev, double *C_dev,
                       double *K_dev)
{
    if (!c || !h_dev) return RF_ERR_ARG;
    if (!c->have_ws) return fail(c, RF_ERR_STATE, "rf_eval_soil before rf_bind_workspace");
    HIPCHK(c, launch_eval_soil(c->G, c->S, c->A, h_dev, theta_dev, C_dev, K_dev, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RF_OK;
}

rf_status rf_assemble(rf_ctx *c, const double *hm_dev, double dt, double *diag_dev,
                      double *rhs_dev)
{
    if (!c || !hm_dev) return RF_ERR_ARG;
    if (!c->have_state) return fail(c, RF_ERR_STATE, "rf_assemble before rf_set_state");
    if (!(dt > 0)) return fail(c, RF_ERR_ARG, "invalid dt");
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    const Bc bc = bc_at(c, c->t);
    (void)N;
    c->A.h0m = c->A.hb0;
    HIPCHK(c, launch_step_begin(c->G, c->S, bc, c->A, hm_dev, 0.0, -1, c->stream));
    HIPCHK(c, launch_coeff(c->G, c->S, c->A, 0, dt, c->opt.chord_eps, c->opt.picard_variant,
                           c->stream));
    HIPCHK(c, launch_resid(c->G, c->A, c->opt.precond, 0, rhs_dev, false, true, cg_tol(c), c->stream));
    if (diag_dev) HIPCHK(c, launch_copy_active(c->G, c->A, c->A.diag, diag_dev, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->assembled = true;
    return RF_OK;
}

rf_status rf_apply_operator(rf_ctx *c, const double *x_dev, double *y_dev)
{
    if (!c || !x_dev || !y_dev) return RF_ERR_ARG;
    if (!c->assembled) return fail(c, RF_ERR_STATE, "rf_apply_operator before rf_assemble");
    HIPCHK(c, launch_operator(c->G, c->A, x_dev, y_dev, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RF_OK;
}

rf_status rf_apply_precond(rf_ctx *c, const double *r_dev, double *z_dev)
{
    if (!c || !r_dev || !z_dev) return RF_ERR_ARG;
    if (!c->assembled) return fail(c, RF_ERR_STATE, "rf_apply_precond before rf_assemble");
    HIPCHK(c, launch_precond(c->G, c->A, c->opt.precond, r_dev, z_dev, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RF_OK;
}

rf_status rf_set_timing(rf_ctx *c, int mask)
{
    if (!c) return RF_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    timed_drop(c);
    c->timing = mask & 0xff;
    c->timing_every = 1;
    c->timing_count = 0;
    const long cells = c->active;
    memset(&c->tm, 0, sizeof(c->tm));
    for (int k = 0; k < RF_NKERNELS; k++) c->tm.name[k] = kKernelNames[k];
    c->tm.cells = cells;
    return RF_OK;
}

rf_status rf_select_timing(rf_ctx *c, int mask, int every)
{
    if (!c || every < 1) return RF_ERR_ARG;
    c->timing = mask & 0xff;
    c->timing_every = every;
    c->timing_count = 0;
    return RF_OK;
}

rf_status rf_get_timing(rf_ctx *c, rf_timing *out)
{
    if (!c || !out) return RF_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *out = c->tm;
    return RF_OK;
}

}  // extern "C"
