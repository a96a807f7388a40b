// Host side and C ABI of the learned Picard guess (include/rf_guess.h): the
// workspace layout, parameter initialisation and transfer, and the launch
// sequences of prediction, gradient and one Adam step (rf_guess.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <random>
#include <vector>

#include "rf_guess_internal.h"

using namespace rf;

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kLossBlocks = 256;
}  // namespace

struct rf_guess {
    int device = 0;
    hipStream_t stream = nullptr;
    char err[512] = {0};
    bool have_setup = false, have_ws = false;
    NetGeo G{};
    NetArrays A{};
    std::vector<float> init;        // parameters to upload at binding
    double *hloss = nullptr;        // pinned loss partials
    long adam_t = 0;
};

static rf_status gfail(rf_guess *g, rf_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g->err, sizeof(g->err), fmt, ap);
    va_end(ap);
    return s;
}

#define GHIP(g, call)                                                                           \
    do {                                                                                        \
        hipError_t r_ = (call);                                                                 \
        if (r_ != hipSuccess) return gfail(g, RF_ERR_HIP, "%s: %s", #call, hipGetErrorString(r_)); \
    } while (0)

static size_t net_layout(const rf_guess *g, char *base, NetArrays *out)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    const size_t N = (size_t)g->G.ncell;
    NetArrays a{};
    a.feat = (bf16 *)take(N * kFeat * sizeof(bf16));
    for (int l = 0; l < 3; l++) a.act[l] = (bf16 *)take(N * kHid * sizeof(bf16));
    a.y = (float *)take(N * sizeof(float));
    a.dz3 = (bf16 *)take(N * 8 * sizeof(bf16));
    for (int l = 0; l < 2; l++) a.dz[l] = (bf16 *)take(N * kHid * sizeof(bf16));
    a.p = (float *)take(kParams * sizeof(float));
    a.g = (float *)take(kParams * sizeof(float));
    a.m = (float *)take(kParams * sizeof(float));
    a.v = (float *)take(kParams * sizeof(float));
    const int cin_f[kNetLayers] = {8, 32, 32, 32}, cob_f[kNetLayers] = {2, 2, 2, 1};
    const int cin_b[kNetLayers] = {0, 32, 32, 8};
    for (int l = 0; l < kNetLayers; l++) {
        a.wf[l] = (bf16 *)take(packed_size(cin_f[l], cob_f[l]) * sizeof(bf16));
        a.wb[l] = l > 0 ? (bf16 *)take(packed_size(cin_b[l], 2) * sizeof(bf16)) : nullptr;
    }
    a.part = (float *)take((size_t)std::max(g->G.chunks * kTaps * 1024, 256 * 32) * sizeof(float));
    a.lpart = (double *)take(kLossBlocks * sizeof(double));
    a.lblocks = kLossBlocks;
    if (out) *out = a;
    return off;
}

static void init_params(rf_guess *g, unsigned seed)
{
    g->init.assign(kParams, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int l = 0; l < kNetLayers - 1; l++) {   // the output layer starts at zero
        const double sd = std::sqrt(2.0 / (kTaps * kCin[l]));
        const int n = kCout[l] * kTaps * kCin[l];
        for (int e = 0; e < n; e++) g->init[param_w(l) + e] = (float)(sd * nd(rng));
    }
}

static rf_status upload_params(rf_guess *g, const float *host)
{
    GHIP(g, hipMemcpyAsync(g->A.p, host, kParams * sizeof(float), hipMemcpyHostToDevice, g->stream));
    GHIP(g, hipMemsetAsync(g->A.m, 0, kParams * sizeof(float), g->stream));
    GHIP(g, hipMemsetAsync(g->A.v, 0, kParams * sizeof(float), g->stream));
    GHIP(g, net_pack(g->A, g->stream));
    GHIP(g, hipStreamSynchronize(g->stream));
    g->adam_t = 0;
    return RF_OK;
}

static rf_status forward_loss(rf_guess *g, const double *hn, const double *hprev, const double *lnks,
                              double rain, const double *target, double *loss)
{
    GHIP(g, net_features(g->G, g->A, hn, hprev, lnks, rain, g->stream));
    GHIP(g, net_forward(g->G, g->A, g->stream));
    GHIP(g, net_loss(g->G, g->A, hn, hprev, target, g->stream));
    GHIP(g, net_backward(g->G, g->A, g->stream));
    GHIP(g, hipMemcpyAsync(g->hloss, g->A.lpart, kLossBlocks * sizeof(double), hipMemcpyDeviceToHost,
                           g->stream));
    GHIP(g, hipStreamSynchronize(g->stream));
    double s = 0.0;
    for (int b = 0; b < kLossBlocks; b++) s += g->hloss[b];
    if (loss) *loss = s;
    return RF_OK;
}

extern "C" {

size_t rf_guess_param_count(void) { return (size_t)kParams; }

rf_status rf_guess_create(rf_guess **out, int hip_device, void *hip_stream)
{
    if (!out) return RF_ERR_ARG;
    *out = nullptr;
    rf_guess *g = new (std::nothrow) rf_guess();
    if (!g) return RF_ERR_NOMEM;
    g->device = hip_device;
    g->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipHostMalloc((void **)&g->hloss, kLossBlocks * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete g;
        return RF_ERR_HIP;
    }
    *out = g;
    return RF_OK;
}

rf_status rf_guess_destroy(rf_guess *g)
{
    if (!g) return RF_ERR_ARG;
    (void)hipSetDevice(g->device);
    if (g->hloss) (void)hipHostFree(g->hloss);
    delete g;
    return RF_OK;
}

const char *rf_guess_last_error(const rf_guess *g) { return g ? g->err : "null network"; }

rf_status rf_guess_setup(rf_guess *g, int nx, int ny, int nz, unsigned seed)
{
    if (!g) return RF_ERR_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || (long)nx * ny * nz > (1L << 31))
        return gfail(g, RF_ERR_ARG, "invalid grid %d x %d x %d", nx, ny, nz);
    NetGeo &G = g->G;
    G.nx = nx;
    G.ny = ny;
    G.nz = nz;
    G.ncol = nx * ny;
    G.ncell = (long)nx * ny * nz;
    G.zt = (nz + 63) / 64;
    G.units = G.ncol * G.zt;
    G.cols_per_chunk = std::max(16, (G.ncol + 255) / 256);
    G.chunks = (G.ncol + G.cols_per_chunk - 1) / G.cols_per_chunk;
    init_params(g, seed);
    g->have_setup = true;
    g->have_ws = false;
    return RF_OK;
}

rf_status rf_guess_workspace_bytes(const rf_guess *g, size_t *bytes)
{
    if (!g || !bytes) return RF_ERR_ARG;
    if (!g->have_setup) return RF_ERR_STATE;
    *bytes = net_layout(g, nullptr, nullptr);
    return RF_OK;
}

rf_status rf_guess_bind_workspace(rf_guess *g, void *dev, size_t bytes)
{
    if (!g) return RF_ERR_ARG;
    if (!g->have_setup) return gfail(g, RF_ERR_STATE, "rf_guess_bind_workspace before rf_guess_setup");
    if (!dev || ((uintptr_t)dev % kAlign) != 0)
        return gfail(g, RF_ERR_ARG, "workspace must be a 256-byte aligned device pointer");
    const size_t need = net_layout(g, nullptr, nullptr);
    if (bytes < need) return gfail(g, RF_ERR_NOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
    GHIP(g, hipSetDevice(g->device));
    net_layout(g, (char *)dev, &g->A);
    rf_status s = upload_params(g, g->init.data());
    if (s) return s;
    g->have_ws = true;
    return RF_OK;
}

rf_status rf_guess_set_params(rf_guess *g, const float *host)
{
    if (!g || !host) return RF_ERR_ARG;
    if (!g->have_ws) return gfail(g, RF_ERR_STATE, "rf_guess_set_params before rf_guess_bind_workspace");
    for (int e = 0; e < kParams; e++)
        if (!std::isfinite(host[e])) return gfail(g, RF_ERR_NONFINITE, "parameter %d is not finite", e);
    g->init.assign(host, host + kParams);
    return upload_params(g, host);
}

rf_status rf_guess_get_params(const rf_guess *cg, float *host)
{
    rf_guess *g = const_cast<rf_guess *>(cg);
    if (!g || !host) return RF_ERR_ARG;
    if (!g->have_ws) return gfail(g, RF_ERR_STATE, "rf_guess_get_params before rf_guess_bind_workspace");
    GHIP(g, hipMemcpyAsync(host, g->A.p, kParams * sizeof(float), hipMemcpyDeviceToHost, g->stream));
    GHIP(g, hipStreamSynchronize(g->stream));
    return RF_OK;
}

rf_status rf_guess_predict(rf_guess *g, const double *hn, const double *hprev, const double *lnks,
                           double rain, double *guess_dev)
{
    if (!g || !hn || !hprev || !guess_dev) return RF_ERR_ARG;
    if (!g->have_ws) return gfail(g, RF_ERR_STATE, "rf_guess_predict before rf_guess_bind_workspace");
    if (!std::isfinite(rain)) return gfail(g, RF_ERR_ARG, "non-finite rain");
    GHIP(g, net_features(g->G, g->A, hn, hprev, lnks, rain, g->stream));
    GHIP(g, net_forward(g->G, g->A, g->stream));
    GHIP(g, net_output(g->G, g->A, hn, hprev, guess_dev, g->stream));
    GHIP(g, hipStreamSynchronize(g->stream));
    return RF_OK;
}

rf_status rf_guess_gradient(rf_guess *g, const double *hn, const double *hprev, const double *lnks,
                            double rain, const double *target, double *loss, float *grad_host)
{
    if (!g || !hn || !hprev || !target) return RF_ERR_ARG;
    if (!g->have_ws) return gfail(g, RF_ERR_STATE, "rf_guess_gradient before rf_guess_bind_workspace");
    rf_status s = forward_loss(g, hn, hprev, lnks, rain, target, loss);
    if (s) return s;
    if (grad_host) {
        GHIP(g, hipMemcpyAsync(grad_host, g->A.g, kParams * sizeof(float), hipMemcpyDeviceToHost, g->stream));
        GHIP(g, hipStreamSynchronize(g->stream));
    }
    return RF_OK;
}

rf_status rf_guess_train_step(rf_guess *g, const double *hn, const double *hprev, const double *lnks,
                              double rain, const double *target, double lr, double *loss)
{
    if (!g || !hn || !hprev || !target) return RF_ERR_ARG;
    if (!g->have_ws) return gfail(g, RF_ERR_STATE, "rf_guess_train_step before rf_guess_bind_workspace");
    if (!(lr > 0) || !std::isfinite(lr)) return gfail(g, RF_ERR_ARG, "invalid learning rate");
    double l = 0.0;
    rf_status s = forward_loss(g, hn, hprev, lnks, rain, target, &l);
    if (s) return s;
    if (!std::isfinite(l)) return gfail(g, RF_ERR_NONFINITE, "non-finite loss");
    g->adam_t++;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)g->adam_t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)g->adam_t));
    GHIP(g, net_adam(g->A, (float)lr, bc1, bc2, g->stream));
    GHIP(g, hipStreamSynchronize(g->stream));
    if (loss) *loss = l;
    return RF_OK;
}

}  // extern "C"
