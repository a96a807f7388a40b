// Soil hydraulic functions shared by the device code of the 3-D solver
// (rf_kernels.hip) and of the column ensemble (rf_ensemble.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "rf_internal.h"

namespace rf {

// van Genuchten-Mualem theta~ (Eq. 2 plus S*h above saturation), capacity
// C (Eq. 3) and conductivity K (Eq. 4), or Gardner's exponential forms.
// With u = (alpha |h|)^n and m = 1 - 1/n:  Se = (1+u)^-m,
// 1 - (1 - Se^(1/m))^m = 1 - (u/(1+u))^m = -expm1(-m log(1 + 1/u)), and
// C = (ts-tr) alpha n m (alpha|h|)^(n-1) (1+u)^-(1+m) = (ts-tr) n m Se u / ((1+u)|h|).
// log(1+u) and log(1+1/u) come from one log1p of min(u, 1/u); no branch of
// the formula cancels.  Five transcendentals per cell.
__device__ __forceinline__ void soil_eval(int model, double h, const Layer &L, double ks,
                                          double &th, double &C, double &K)
{
    if (h >= 0.0) {
        th = L.ts + L.S * h;
        C = L.S;
        K = ks;
        return;
    }
    if (model == RF_GARDNER) {
        const double e = exp(L.a * h);
        th = L.tr + (L.ts - L.tr) * e;
        C = L.a * (L.ts - L.tr) * e;
        K = ks * e;
        return;
    }
    const double lu = L.n * log(-L.a * h);     // log u
    const double u = exp(lu);
    const bool small = u <= 1.0;
    const double t = small ? u : 1.0 / u;      // min(u, 1/u)
    const double lp = log1p(t);
    const double l1 = small ? lp : lu + lp;    // log(1 + u)
    const double lq = small ? lp - lu : lp;    // log(1 + 1/u)
    const double sqSe = exp(-0.5 * L.m * l1);  // Se^(1/2)
    const double Se = sqSe * sqSe;
    th = L.tr + (L.ts - L.tr) * Se;
    const double frac = 1.0 / (1.0 + (small ? 1.0 / u : t));   // u / (1 + u)
    C = (L.ts - L.tr) * L.n * L.m * Se * frac / (-h);
    const double w = -expm1(-L.m * lq);
    K = ks * sqSe * w * w;
}

// van Genuchten-Mualem without a branch on the sign of h: a saturated cell
// evaluates the unsaturated forms at h = -1 m and takes the saturated values
// (theta~ = theta_s + S h, C = S, K = Ks).  Unsaturated cells get exactly the
// arithmetic of soil_eval; the straight-line code lets the evaluations of
// several cells interleave.
__device__ __forceinline__ void soil_eval_vgm_flat(double h, const Layer &L, double ks, double &th,
                                                   double &C, double &K)
{
    const bool sat = h >= 0.0;
    const double hu = sat ? -1.0 : h;
    const double lu = L.n * log(-L.a * hu);    // log u
    const double u = exp(lu);
    const bool small = u <= 1.0;
    const double t = small ? u : 1.0 / u;      // min(u, 1/u)
    const double lp = log1p(t);
    const double l1 = small ? lp : lu + lp;    // log(1 + u)
    const double lq = small ? lp - lu : lp;    // log(1 + 1/u)
    const double sqSe = exp(-0.5 * L.m * l1);  // Se^(1/2)
    const double Se = sqSe * sqSe;
    const double frac = 1.0 / (1.0 + (small ? 1.0 / u : t));   // u / (1 + u)
    const double w = -expm1(-L.m * lq);
    th = sat ? L.ts + L.S * h : L.tr + (L.ts - L.tr) * Se;
    C = sat ? L.S : (L.ts - L.tr) * L.n * L.m * Se * frac / (-hu);
    K = sat ? ks : ks * sqSe * w * w;
}

// theta~ of van Genuchten-Mualem without a branch on the sign of h (the
// arithmetic of soil_theta for unsaturated cells).
__device__ __forceinline__ double soil_theta_vgm_flat(double h, const Layer &L)
{
    const bool sat = h >= 0.0;
    const double lu = L.n * log(-L.a * (sat ? -1.0 : h));
    const double th = L.tr + (L.ts - L.tr) * exp(-L.m * log1p(exp(lu)));
    return sat ? L.ts + L.S * h : th;
}

__device__ __forceinline__ double soil_theta(int model, double h, const Layer &L)
{
    if (h >= 0.0) return L.ts + L.S * h;
    if (model == RF_GARDNER) return L.tr + (L.ts - L.tr) * exp(L.a * h);
    const double lu = L.n * log(-L.a * h);
    return L.tr + (L.ts - L.tr) * exp(-L.m * log1p(exp(lu)));
}

__device__ __forceinline__ double soil_K(int model, double h, const Layer &L, double ks)
{
    double th, C, K;
    soil_eval(model, h, L, ks, th, C, K);
    return K;
}

}  // namespace rf
