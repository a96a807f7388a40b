// Internal declarations of the learned Picard guess (rf_guess.hip kernels,
// rf_guess_host.cpp host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rf_guess.h"

namespace rf {

typedef __bf16 bf16;

constexpr int kTaps = 27;
constexpr int kHid = 32;          // hidden channels
constexpr int kFeat = 8;          // feature channels as stored (4 used)
constexpr int kNetLayers = 4;
constexpr int kCin[kNetLayers] = {4, 32, 32, 32};
constexpr int kCout[kNetLayers] = {32, 32, 32, 1};
constexpr double kHScale = 10.0;       // h^n feature: h / 10 m
constexpr double kDhScale = 100.0;     // (h^n - h^{n-1}) * 100 / m
constexpr double kRainScale = 1e7;     // rain * 1e7 s/m
constexpr double kOutScale = 0.01;     // h^{n+1,0} = h^n + (h^n - h^{n-1}) + 0.01 m * y

// Offsets of W_l and b_l in the FP32 parameter vector.
constexpr int param_w(int l)
{
    int o = 0;
    for (int i = 0; i < l; i++) o += kCout[i] * kTaps * kCin[i] + kCout[i];
    return o;
}
constexpr int param_b(int l) { return param_w(l) + kCout[l] * kTaps * kCin[l]; }
constexpr int kParams = param_w(kNetLayers);

// Packed BF16 operands of the convolution kernels: a layer's weights in the
// A-operand lane order of v_mfma_f32_16x16x32_bf16 (16 output channels x 32
// reduction values per step; each lane holds 8 consecutive reduction values
// of one output channel).  A step is one tap (32 input channels) or, for
// 8-channel inputs, four taps of 8 channels.
constexpr int packed_steps(int cin_stored) { return cin_stored == 32 ? kTaps : (kTaps + 3) / 4; }
constexpr int packed_size(int cin_stored, int cout_blocks)
{
    return packed_steps(cin_stored) * cout_blocks * 64 * 8;
}

struct NetGeo {
    int nx, ny, nz;
    int ncol;
    long ncell;
    int units;              // (column, 64-cell z-tile) work units
    int zt;                 // z-tiles per column
    int chunks;             // column chunks of the weight-gradient kernel
    int cols_per_chunk;
};

struct NetArrays {
    bf16 *feat;             // [N][8]
    bf16 *act[3];           // a1, a2, a3: [N][32]
    float *y;               // [N]
    bf16 *dz3;              // [N][8] (channel 0)
    bf16 *dz[2];            // [N][32] ping-pong
    float *p, *g, *m, *v;   // parameters, gradient, Adam moments [kParams]
    bf16 *wf[kNetLayers];   // forward packed weights
    bf16 *wb[kNetLayers];   // backward-data packed weights (layers 1..3)
    float *part;            // weight-gradient partials [chunks][27][32][32]
    double *lpart;          // loss block partials
    int lblocks;
};

hipError_t net_pack(const NetArrays &a, hipStream_t s);
hipError_t net_features(const NetGeo &g, const NetArrays &a, const double *hn, const double *hprev,
                        const double *lnks, double rain, hipStream_t s);
hipError_t net_forward(const NetGeo &g, const NetArrays &a, hipStream_t s);
hipError_t net_output(const NetGeo &g, const NetArrays &a, const double *hn, const double *hprev,
                      double *guess, hipStream_t s);
hipError_t net_loss(const NetGeo &g, const NetArrays &a, const double *hn, const double *hprev,
                    const double *target, hipStream_t s);
hipError_t net_backward(const NetGeo &g, const NetArrays &a, hipStream_t s);
hipError_t net_adam(const NetArrays &a, float lr, float bc1, float bc2, hipStream_t s);

}  // namespace rf
