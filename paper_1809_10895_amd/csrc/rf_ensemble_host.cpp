// Host side and C ABI of the column ensemble (include/rf_ensemble.h).
//
// The host validates the column table, lays out the caller's workspace,
// orders the queue (decreasing length) and launches runs.  A run is four
// stream operations on the caller's stream: reset the queue, the persistent
// kernel (run bounds as kernel arguments), the summary kernel, and the copy
// of the summary to pinned host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "rf_ens_internal.h"

using namespace rf;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct rf_ens {
    int device = 0;
    hipStream_t stream = nullptr;
    char err[512] = {0};

    bool have_setup = false, have_ws = false, have_state = false;
    int ncol = 0;
    long ncell = 0;
    double dz = 0.0;
    int model = RF_VGM;
    std::vector<int32_t> len;
    std::vector<int64_t> off;
    std::vector<int32_t> order;
    std::vector<EnsSoil> soil;
    int bc_type[2] = {RF_NOFLOW, RF_NOFLOW};
    double bc_value[2] = {0.0, 0.0};
    rf_options opt;
    rf_ens_tile tile{4, 0};          // blocks_per_cu 0: as many as fit
    long long max_steps = 100000000LL;
    double max_seconds = 60.0;

    void *ws = nullptr;
    size_t ws_bytes = 0;
    EnsArrays A{};

    rf_ens_summary *hsum = nullptr;  // pinned
    hipEvent_t ev[2] = {nullptr, nullptr};
    int n_cu = 0;
    double tick_hz = 1e8;
};

static rf_status efail(rf_ens *e, rf_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(e->err, sizeof(e->err), fmt, ap);
    va_end(ap);
    return s;
}

#define EHIP(e, call)                                                                      \
    do {                                                                                   \
        hipError_t r_ = (call);                                                            \
        if (r_ != hipSuccess) return efail(e, RF_ERR_HIP, "%s: %s", #call, hipGetErrorString(r_)); \
    } while (0)

static EnsOpt make_opt(const rf_ens *e)
{
    EnsOpt o{};
    const rf_options &p = e->opt;
    o.tol_picard = p.tol_picard;
    o.chord_eps = p.chord_eps;
    o.dt0 = p.dt0;
    o.dt_max = p.dt_max;
    o.dt_min = p.dt_min;
    o.factor = p.factor;
    o.dz = e->dz;
    o.max_picard = p.max_picard;
    o.ebats = p.ebats;
    o.inc_after = p.inc_after;
    o.few_iters = p.few_iters;
    o.max_iters = p.max_iters;
    o.variant = p.picard_variant;
    o.model = e->model;
    for (int f = 0; f < 2; f++) {
        o.bc_type[f] = e->bc_type[f];
        o.bc_value[f] = e->bc_value[f];
    }
    return o;
}

static size_t ens_layout(const rf_ens *e, char *base, EnsArrays *A)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    EnsArrays a{};
    const size_t nc = (size_t)e->ncol, ncell = (size_t)e->ncell;
    a.h = (double *)take(ncell * sizeof(double));
    a.soil = (EnsSoil *)take(nc * sizeof(EnsSoil));
    a.len = (int32_t *)take(nc * sizeof(int32_t));
    a.off = (int64_t *)take(nc * sizeof(int64_t));
    a.order = (int32_t *)take(nc * sizeof(int32_t));
    a.col = (rf_ens_column *)take(nc * sizeof(rf_ens_column));
    a.sum = (rf_ens_summary *)take(sizeof(rf_ens_summary));
    a.queue = (unsigned int *)take(sizeof(unsigned int));
    a.h_bak = (double *)take(ncell * sizeof(double));
    a.col_bak = (rf_ens_column *)take(nc * sizeof(rf_ens_column));
    if (A) *A = a;
    return off;
}

// Occupancy of the run kernel per (precision, waves per block), queried once
// per process.
static int occupancy(bool mixed, int waves_per_block)
{
    static int cache[2][9] = {};
    int &v = cache[mixed ? 1 : 0][waves_per_block & 7 ? waves_per_block : 8];
    if (v == 0) v = std::max(1, ens_max_blocks_per_cu(mixed, waves_per_block));
    return v;
}

static int blocks_for(const rf_ens *e, int waves_per_block, int blocks_per_cu)
{
    const bool mixed = e->opt.precision == RF_PREC_MIXED;
    int fit = occupancy(mixed, waves_per_block);
    if (fit < 1) fit = 1;
    const int per_cu = blocks_per_cu > 0 ? std::min(blocks_per_cu, fit) : fit;
    return std::max(1, per_cu * e->n_cu);
}

extern "C" {

rf_status rf_ens_create(rf_ens **out, int hip_device, void *hip_stream)
{
    if (!out) return RF_ERR_ARG;
    *out = nullptr;
    rf_ens *e = new (std::nothrow) rf_ens();
    if (!e) return RF_ERR_NOMEM;
    e->device = hip_device;
    e->stream = (hipStream_t)hip_stream;
    rf_default_options(&e->opt);
    int rate_khz = 0;
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&e->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, hip_device) != hipSuccess ||
        hipHostMalloc((void **)&e->hsum, sizeof(rf_ens_summary), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&e->ev[0]) != hipSuccess || hipEventCreate(&e->ev[1]) != hipSuccess) {
        if (e->hsum) (void)hipHostFree(e->hsum);
        if (e->ev[0]) (void)hipEventDestroy(e->ev[0]);
        delete e;
        return RF_ERR_HIP;
    }
    if (rate_khz > 0) e->tick_hz = rate_khz * 1e3;
    *out = e;
    return RF_OK;
}

rf_status rf_ens_destroy(rf_ens *e)
{
    if (!e) return RF_ERR_ARG;
    (void)hipSetDevice(e->device);
    if (e->hsum) (void)hipHostFree(e->hsum);
    for (hipEvent_t v : e->ev)
        if (v) (void)hipEventDestroy(v);
    delete e;
    return RF_OK;
}

const char *rf_ens_last_error(const rf_ens *e) { return e ? e->err : "null ensemble"; }

rf_status rf_ens_setup(rf_ens *e, int ncol, const int32_t *len, double dz, int model,
                       const double *soil)
{
    if (!e) return RF_ERR_ARG;
    if (ncol < 1 || !len || !soil || !(dz > 0) || !std::isfinite(dz) ||
        (model != RF_VGM && model != RF_GARDNER))
        return efail(e, RF_ERR_ARG, "invalid ensemble set-up");
    std::vector<EnsSoil> sp((size_t)ncol);
    for (int c = 0; c < ncol; c++) {
        if (len[c] < 1 || len[c] > RF_ENS_MAX_LEN)
            return efail(e, RF_ERR_ARG, "column %d: length %d outside [1, %d]", c, len[c], RF_ENS_MAX_LEN);
        const double *p = soil + 6 * (size_t)c;
        const double tr = p[0], ts = p[1], al = p[2], n = p[3], ks = p[4], S = p[5];
        if (!(ts > tr) || !(tr >= 0) || !(al > 0) || !(ks > 0) || !(S >= 0) ||
            (model == RF_VGM && !(n > 1.0)) || !std::isfinite(ts + al + n + ks + S))
            return efail(e, RF_ERR_ARG, "column %d: invalid soil parameters", c);
        sp[c].L = Layer{tr, ts, al, n, model == RF_VGM ? 1.0 - 1.0 / n : 0.0, S};
        sp[c].ks = ks;
        sp[c].pad = 0.0;
    }
    e->ncol = ncol;
    e->len.assign(len, len + ncol);
    e->off.resize(ncol);
    long acc = 0;
    for (int c = 0; c < ncol; c++) {
        e->off[c] = acc;
        acc += len[c];
    }
    e->ncell = acc;
    e->order.resize(ncol);
    std::iota(e->order.begin(), e->order.end(), 0);
    std::stable_sort(e->order.begin(), e->order.end(),
                     [&](int a, int b) { return e->len[a] > e->len[b]; });
    e->soil = std::move(sp);
    e->dz = dz;
    e->model = model;
    e->have_setup = true;
    e->have_ws = false;
    e->have_state = false;
    return RF_OK;
}

rf_status rf_ens_set_bc(rf_ens *e, int face, int type, double value)
{
    if (!e) return RF_ERR_ARG;
    if ((face != RF_ZMIN && face != RF_ZMAX) || type < RF_NOFLOW || type > RF_FREE_DRAINAGE ||
        !std::isfinite(value))
        return efail(e, RF_ERR_ARG, "invalid boundary condition");
    const int f = face == RF_ZMAX ? 1 : 0;
    e->bc_type[f] = type;
    e->bc_value[f] = value;
    return RF_OK;
}

rf_status rf_ens_set_options(rf_ens *e, const rf_options *o)
{
    if (!e || !o) return RF_ERR_ARG;
    if (!(o->tol_picard > 0) || o->max_picard < 1 || !(o->chord_eps >= 0) || !(o->dt0 > 0) ||
        !(o->dt_max > 0) || !(o->dt_min > 0) || o->inc_after < 1 || o->few_iters < 1 ||
        o->max_iters < 1 || !(o->factor > 1.0) ||
        (o->precision != RF_PREC_FP64 && o->precision != RF_PREC_MIXED) ||
        (o->picard_variant != RF_PICARD_CHORD && o->picard_variant != RF_PICARD_MODIFIED))
        return efail(e, RF_ERR_ARG, "invalid options");
    e->opt = *o;
    return RF_OK;
}

rf_status rf_ens_set_tile(rf_ens *e, const rf_ens_tile *t)
{
    if (!e || !t) return RF_ERR_ARG;
    const int w = t->waves_per_block;
    if ((w != 1 && w != 2 && w != 4 && w != 8) || t->blocks_per_cu < 0 || t->blocks_per_cu > 16)
        return efail(e, RF_ERR_ARG, "invalid tile");
    e->tile = *t;
    return RF_OK;
}

rf_status rf_ens_get_tile(const rf_ens *e, rf_ens_tile *t)
{
    if (!e || !t) return RF_ERR_ARG;
    *t = e->tile;
    return RF_OK;
}

rf_status rf_ens_set_limits(rf_ens *e, long max_steps, double max_seconds)
{
    if (!e) return RF_ERR_ARG;
    if (max_steps < 1 || !(max_seconds > 0) || !std::isfinite(max_seconds))
        return efail(e, RF_ERR_ARG, "invalid limits");
    e->max_steps = max_steps;
    e->max_seconds = max_seconds;
    return RF_OK;
}

rf_status rf_ens_cells(const rf_ens *e, long *ncell)
{
    if (!e || !ncell) return RF_ERR_ARG;
    if (!e->have_setup) return RF_ERR_STATE;
    *ncell = e->ncell;
    return RF_OK;
}

rf_status rf_ens_workspace_bytes(const rf_ens *e, size_t *bytes)
{
    if (!e || !bytes) return RF_ERR_ARG;
    if (!e->have_setup) return RF_ERR_STATE;
    *bytes = ens_layout(e, nullptr, nullptr);
    return RF_OK;
}

rf_status rf_ens_bind_workspace(rf_ens *e, void *dev, size_t bytes)
{
    if (!e) return RF_ERR_ARG;
    if (!e->have_setup) return efail(e, RF_ERR_STATE, "rf_ens_bind_workspace before rf_ens_setup");
    if (!dev || ((uintptr_t)dev % kAlign) != 0)
        return efail(e, RF_ERR_ARG, "workspace must be a 256-byte aligned device pointer");
    const size_t need = ens_layout(e, nullptr, nullptr);
    if (bytes < need) return efail(e, RF_ERR_NOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
    EHIP(e, hipSetDevice(e->device));
    ens_layout(e, (char *)dev, &e->A);
    e->ws = dev;
    e->ws_bytes = bytes;
    const size_t nc = (size_t)e->ncol;
    EHIP(e, hipMemcpyAsync(e->A.soil, e->soil.data(), nc * sizeof(EnsSoil), hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(e->A.len, e->len.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(e->A.off, e->off.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(e->A.order, e->order.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice,
                           e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    e->have_ws = true;
    e->have_state = false;
    return RF_OK;
}

rf_status rf_ens_set_state(rf_ens *e, const double *h_dev, double t)
{
    if (!e || !h_dev) return RF_ERR_ARG;
    if (!e->have_ws) return efail(e, RF_ERR_STATE, "rf_ens_set_state before rf_ens_bind_workspace");
    if (!std::isfinite(t)) return efail(e, RF_ERR_ARG, "non-finite time");
    EHIP(e, hipSetDevice(e->device));
    // check a copy first so that a rejected state leaves the current one alone
    EnsArrays chk = e->A;
    chk.h = e->A.h_bak;
    EHIP(e, hipMemcpyAsync(chk.h, h_dev, (size_t)e->ncell * sizeof(double), hipMemcpyDeviceToDevice,
                           e->stream));
    EHIP(e, launch_ens_check(chk, e->ncell, e->stream));
    unsigned int bad = 0;
    EHIP(e, hipMemcpyAsync(&bad, e->A.queue, sizeof(bad), hipMemcpyDeviceToHost, e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    if (bad) return efail(e, RF_ERR_NONFINITE, "%u non-finite values in the state", bad);
    EHIP(e, hipMemcpyAsync(e->A.h, h_dev, (size_t)e->ncell * sizeof(double), hipMemcpyDeviceToDevice,
                           e->stream));
    EHIP(e, launch_ens_init(e->A, e->ncol, make_opt(e), t, e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    e->have_state = true;
    return RF_OK;
}

rf_status rf_ens_get_state(const rf_ens *ce, double *h_dev)
{
    rf_ens *e = const_cast<rf_ens *>(ce);
    if (!e || !h_dev) return RF_ERR_ARG;
    if (!e->have_state) return efail(e, RF_ERR_STATE, "rf_ens_get_state before rf_ens_set_state");
    EHIP(e, hipMemcpyAsync(h_dev, e->A.h, (size_t)e->ncell * sizeof(double), hipMemcpyDeviceToDevice,
                           e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    return RF_OK;
}

static rf_status ens_run(rf_ens *e, double t_end, rf_ens_summary *out)
{
    const bool mixed = e->opt.precision == RF_PREC_MIXED;
    const int nblk = blocks_for(e, e->tile.waves_per_block, e->tile.blocks_per_cu);
    EnsRunParams rp;
    rp.t_end = t_end;
    rp.max_steps = e->max_steps;
    rp.max_ticks = (long long)(e->max_seconds * e->tick_hz);
    EHIP(e, launch_ens_reset(e->A, e->stream));
    EHIP(e, hipEventRecord(e->ev[0], e->stream));
    EHIP(e, launch_ens_run(e->A, e->ncol, make_opt(e), rp, mixed, nblk, e->tile.waves_per_block,
                           e->stream));
    EHIP(e, hipEventRecord(e->ev[1], e->stream));
    EHIP(e, launch_ens_summary(e->A, e->ncol, e->stream));
    EHIP(e, hipMemcpyAsync(e->hsum, e->A.sum, sizeof(rf_ens_summary), hipMemcpyDeviceToHost,
                           e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    rf_ens_summary sm = *e->hsum;
    float ms = 0.f;
    EHIP(e, hipEventElapsedTime(&ms, e->ev[0], e->ev[1]));
    sm.kernel_ms = ms;
    if (out) *out = sm;
    if (sm.failed > 0)
        return efail(e, RF_ERR_NOT_CONVERGED, "%d of %d columns failed", sm.failed, e->ncol);
    if (sm.t_min < t_end * (1.0 - 1e-15) - 1e-12)
        return efail(e, RF_ERR_NOT_CONVERGED, "columns stopped at t = %.17g before t_end "
                     "(step or time budget of the run)", sm.t_min);
    return RF_OK;
}

// The persistent run kernel is switched off: its launches did not return on
// the GPU after other GPU work in the same process, with no fault reported,
// and that cause has not been shown.  Until it is, rf_ens_run and
// rf_ens_autotune refuse to launch it.
#ifndef RF_ENS_RUN_ENABLED
#define RF_ENS_RUN_ENABLED 0   /* 1 only in the CPU emulation build of the tests */
#endif
static const bool kEnsRunEnabled = RF_ENS_RUN_ENABLED != 0;
static const char *kEnsRunOff =
    "the column-ensemble run kernel is switched off: its launches did not return on the GPU "
    "and the cause has not been shown";

rf_status rf_ens_run(rf_ens *e, double t_end, rf_ens_summary *out)
{
    if (!e) return RF_ERR_ARG;
    if (!e->have_state) return efail(e, RF_ERR_STATE, "rf_ens_run before rf_ens_set_state");
    if (!std::isfinite(t_end)) return efail(e, RF_ERR_ARG, "non-finite t_end");
    if (!kEnsRunEnabled) return efail(e, RF_ERR_STATE, "%s", kEnsRunOff);
    EHIP(e, hipSetDevice(e->device));
    return ens_run(e, t_end, out);
}

rf_status rf_ens_get_columns(const rf_ens *ce, rf_ens_column *out)
{
    rf_ens *e = const_cast<rf_ens *>(ce);
    if (!e || !out) return RF_ERR_ARG;
    if (!e->have_state) return efail(e, RF_ERR_STATE, "rf_ens_get_columns before rf_ens_set_state");
    EHIP(e, hipMemcpyAsync(out, e->A.col, (size_t)e->ncol * sizeof(rf_ens_column),
                           hipMemcpyDeviceToHost, e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    return RF_OK;
}

rf_status rf_ens_autotune(rf_ens *e, double t_span, rf_ens_tile *best)
{
    if (!e) return RF_ERR_ARG;
    if (!e->have_state) return efail(e, RF_ERR_STATE, "rf_ens_autotune before rf_ens_set_state");
    if (!(t_span > 0) || !std::isfinite(t_span)) return efail(e, RF_ERR_ARG, "invalid t_span");
    if (!kEnsRunEnabled) return efail(e, RF_ERR_STATE, "%s", kEnsRunOff);
    EHIP(e, hipSetDevice(e->device));
    const size_t hb = (size_t)e->ncell * sizeof(double), cb = (size_t)e->ncol * sizeof(rf_ens_column);
    EHIP(e, hipMemcpyAsync(e->A.h_bak, e->A.h, hb, hipMemcpyDeviceToDevice, e->stream));
    EHIP(e, hipMemcpyAsync(e->A.col_bak, e->A.col, cb, hipMemcpyDeviceToDevice, e->stream));
    EHIP(e, hipStreamSynchronize(e->stream));
    // the earliest column time: every trial advances the same columns by t_span
    std::vector<rf_ens_column> cols((size_t)e->ncol);
    EHIP(e, hipMemcpy(cols.data(), e->A.col, cb, hipMemcpyDeviceToHost));
    double t_start = INFINITY;
    for (const auto &c : cols) t_start = std::min(t_start, c.t);
    const rf_ens_tile saved = e->tile;
    static const int kWaves[] = {1, 2, 4, 8};
    rf_ens_tile win = saved;
    double win_ms = INFINITY;
    hipEvent_t a, b;
    EHIP(e, hipEventCreate(&a));
    EHIP(e, hipEventCreate(&b));
    rf_status st = RF_OK;
    for (int w : kWaves) {
        const int fit = occupancy(e->opt.precision == RF_PREC_MIXED, w);
        std::vector<int> per_cu;
        for (int pc = 1; pc <= std::min(fit, 16); pc *= 2) per_cu.push_back(pc);
        if (fit > 0 && fit <= 16 && (fit & (fit - 1)) != 0) per_cu.push_back(fit);
        for (int pc : per_cu) {
            e->tile = rf_ens_tile{w, pc};
                    if (hipEventRecord(a, e->stream) != hipSuccess) { st = RF_ERR_HIP; break; }
            rf_status s = ens_run(e, t_start + t_span, nullptr);
            if (hipEventRecord(b, e->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
                st = RF_ERR_HIP;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (s == RF_OK && ms < win_ms) {
                win_ms = ms;
                win = e->tile;
            }
            // restore the state for the next trial
            if (hipMemcpyAsync(e->A.h, e->A.h_bak, hb, hipMemcpyDeviceToDevice, e->stream) != hipSuccess ||
                hipMemcpyAsync(e->A.col, e->A.col_bak, cb, hipMemcpyDeviceToDevice, e->stream) != hipSuccess ||
                hipStreamSynchronize(e->stream) != hipSuccess) {
                st = RF_ERR_HIP;
                break;
            }
        }
        if (st) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st) {
        e->tile = saved;
        return efail(e, st, "autotune: HIP error");
    }
    if (!std::isfinite(win_ms)) {
        e->tile = saved;
        return efail(e, RF_ERR_NOT_CONVERGED, "autotune: no trial reached t_start + t_span");
    }
    e->tile = win;
    if (best) *best = win;
    return RF_OK;
}

}  // extern "C"
