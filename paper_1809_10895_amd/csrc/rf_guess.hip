// HIP kernels (gfx950 / CDNA4) of the learned Picard guess: a four-layer
// 3x3x3 convolutional network trained and evaluated on the matrix cores.
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16: the
// output tile of one wavefront is 16 output channels x 64 cells (one z-run of
// a column, cells z-fastest as in the solver), the reduction runs over taps
// and input channels, 32 values per instruction (one tap of 32 channels, or
// four taps of an 8-channel input).  Activations are channels-last BF16 (a
// cell's 32 channels are one 64-byte row).  A block stages a 4 x 2 patch of
// columns with a one-cell border (<= 99 KB) and the layer's packed weights
// (<= 55 KB) in LDS once, so every input row crosses L2 about three times
// instead of once per tap.  The backward pass reuses the same kernel
// with transposed, tap-mirrored weights (the gradient with respect to a
// layer's input) and a ReLU-mask epilogue; the weight gradient is a second
// MFMA kernel whose reduction runs over cells, with LDS transposes of the
// two channels-last operands, and per-chunk partials summed in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>

#include "rf_guess_internal.h"

namespace rf {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

enum { EPI_RELU = 0, EPI_MASK = 2 };

// Neighbour of cell (i, j, k) through tap t = 9 (di+1) + 3 (dj+1) + (dk+1);
// false outside the grid (zero padding).
__device__ __forceinline__ bool tap_nbr(const NetGeo &g, int i, int j, int k, int t, long &cell)
{
    const int di = t / 9 - 1, dj = (t / 3) % 3 - 1, dk = t % 3 - 1;
    const int ii = i + di, jj = j + dj, kk = k + dk;
    cell = (long)kk + (long)g.nz * ((long)ii + (long)g.nx * jj);
    return ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
}

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; e++) z[e] = (bf16)0.0f;
    return z;
}

// x of the lane whose index differs in bit 0 / bit 1 (DPP quad_perm, all
// lanes of the quad active).
__device__ __forceinline__ float dpp_quad_xor1(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ float dpp_quad_xor2(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
}

// One convolution layer over one block patch: PX x PY columns and 64 cells
// of z.  The patch's input plus a one-cell border (6 x 4 columns x 66 cells,
// zero outside the grid) is staged in LDS once, with the layer's packed
// weights; each of the eight wavefronts then computes one column, 16 output
// channels x 64 cells per MFMA group, reading every tap's operand from LDS.
// CIN: stored input channels (8 or 32); COB: output blocks of 16 channels (1
// or 2).  EPI_RELU: out = bf16(relu(acc + bias)); EPI_MASK: out = bf16(acc)
// where mask > 0, else 0 (gradient through a ReLU).
//
// The patch is held in LDS as planes of one 16-byte channel chunk over the
// z-run of a column ([column][chunk][z]), so the sixteen lanes that read one
// MFMA operand row (sixteen consecutive cells of one chunk) read 256
// consecutive bytes: no bank conflicts.  (Channels-last order would put them
// 64 bytes apart, a four-way conflict on every operand read.)  Staging issues
// all of a thread's global loads before its first LDS write, so the block
// waits for one memory round trip instead of one per chunk.
constexpr int PX = 4, PY = 2, TX = PX + 2, TY = PY + 2, TZ = 64 + 2;
constexpr int kTileThreads = 64 * PX * PY;

// Patch staging: element e of the patch (chunk fastest, then z, then
// column, i.e. the order of global memory) -> its 16 bytes, zero outside the
// grid; ZT cells of z per tile plus the border (TZ = ZT + 2).  PLANES: LDS
// index in [column][chunk][z] order, else e itself.
template <int CH, bool PLANES, int ZT = 64>
__device__ __forceinline__ void stage_patch(const NetGeo &g, const bf16 *__restrict__ in, int px0,
                                            int py0, int z0, bf16x8 *sT)
{
    constexpr int TZ = ZT + 2;
    constexpr int NST = TX * TY * TZ * CH;
    constexpr int PER = (NST + kTileThreads - 1) / kTileThreads;
    bf16x8 v[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int e = threadIdx.x + u * kTileThreads;
        const int part = e % CH, cz = e / CH;
        const int zl = cz % TZ, cl = cz / TZ;
        const int i = px0 - 1 + cl % TX, j = py0 - 1 + cl / TX, k = z0 - 1 + zl;
        const bool ok = e < NST && i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz;
        const long cell = (long)k + (long)g.nz * ((long)i + (long)g.nx * j);
        v[u] = ok ? *reinterpret_cast<const bf16x8 *>(in + cell * (8 * CH) + 8 * part) : zero8();
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int e = threadIdx.x + u * kTileThreads;
        if (e >= NST) break;
        const int part = e % CH, cz = e / CH;
        const int zl = cz % TZ, cl = cz / TZ;
        sT[PLANES ? (cl * CH + part) * TZ + zl : e] = v[u];
    }
}

template <int CIN, int COB, int EPI>
__global__ void __launch_bounds__(kTileThreads) k_conv(NetGeo g, const bf16 *__restrict__ in,
                                                       const bf16 *__restrict__ wp,
                                                       const float *__restrict__ bias,
                                                       bf16 *__restrict__ out, const bf16 *__restrict__ mask)
{
    constexpr int STEPS = packed_steps(CIN);
    constexpr int NPK = STEPS * COB * 64;
    constexpr int CH = CIN / 8;                    // 16-byte chunks per cell
    __shared__ bf16x8 sW[NPK];
    __shared__ bf16x8 sT[TX * TY * TZ * CH];
    // patch of this block
    const int pxn = (g.nx + PX - 1) / PX, pyn = (g.ny + PY - 1) / PY;
    const int zti = blockIdx.x % g.zt;
    const int pxy = blockIdx.x / g.zt;
    const int px0 = (pxy % pxn) * PX, py0 = (pxy / pxn) * PY, z0 = zti * 64;
    const bf16x8 *wv = reinterpret_cast<const bf16x8 *>(wp);
    {
        constexpr int PW = (NPK + kTileThreads - 1) / kTileThreads;
        bf16x8 w[PW];
#pragma unroll
        for (int u = 0; u < PW; u++) {
            const int e = threadIdx.x + u * kTileThreads;
            w[u] = e < NPK ? wv[e] : zero8();
        }
#pragma unroll
        for (int u = 0; u < PW; u++) {
            const int e = threadIdx.x + u * kTileThreads;
            if (e < NPK) sW[e] = w[u];
        }
    }
    stage_patch<CH, true>(g, in, px0, py0, z0, sT);
    (void)pyn;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, q = lane >> 4;
    const int wave = threadIdx.x >> 6;
    const int cx = wave % PX, cy = wave / PX;
    const int i = px0 + cx, j = py0 + cy;
    if (i >= g.nx || j >= g.ny) return;
    const int col = i + g.nx * j;
    f32x4 acc[COB][4];
#pragma unroll
    for (int b = 0; b < COB; b++)
#pragma unroll
        for (int t = 0; t < 4; t++) acc[b][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the operands of step s + 1 are read from LDS while the MFMAs of step s
    // run (two register sets in turn)
    auto load = [&](int s, bf16x8 (&A)[COB], bf16x8 (&B)[4]) {
#pragma unroll
        for (int b = 0; b < COB; b++) A[b] = sW[(s * COB + b) * 64 + lane];
        const int tap = (CIN == 32) ? s : 4 * s + q;
        const bool tok = tap < kTaps;
        const int tt = tok ? tap : 0;
        const int di = tt / 9 - 1, dj = (tt / 3) % 3 - 1, dk = tt % 3 - 1;
        const int cl = (cx + 1 + di) + TX * (cy + 1 + dj);
        const int part = (CIN == 32) ? q : 0;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int zl = 16 * t + n + 1 + dk;
            B[t] = tok ? sT[(cl * CH + part) * TZ + zl] : zero8();
        }
    };
    auto mfma = [&](const bf16x8 (&A)[COB], const bf16x8 (&B)[4]) {
#pragma unroll
        for (int t = 0; t < 4; t++)
#pragma unroll
            for (int b = 0; b < COB; b++)
                acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[b], B[t], acc[b][t], 0, 0, 0);
    };
    bf16x8 A0[COB], B0[4], A1[COB], B1[4];
    load(0, A0, B0);
    for (int s = 0; s < STEPS; s += 2) {
        if (s + 1 < STEPS) load(s + 1, A1, B1);
        mfma(A0, B0);
        if (s + 1 < STEPS) {
            if (s + 2 < STEPS) load(s + 2, A0, B0);
            mfma(A1, B1);
        }
    }
    // lane holds rows 4q..4q+3 (output channels) of column n (cell)
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int k = z0 + 16 * t + n;
        if (k >= g.nz) continue;
        const long cell = (long)col * g.nz + k;
#pragma unroll
        for (int b = 0; b < COB; b++) {
            const int co0 = 16 * b + 4 * q;
            bf16x4 o;
            if (EPI == EPI_MASK) {
                const bf16x4 mk = *reinterpret_cast<const bf16x4 *>(mask + cell * kHid + co0);
#pragma unroll
                for (int v = 0; v < 4; v++)
                    o[v] = (float)mk[v] > 0.f ? (bf16)acc[b][t][v] : (bf16)0.0f;
            } else {
#pragma unroll
                for (int v = 0; v < 4; v++) o[v] = (bf16)fmaxf(acc[b][t][v] + bias[co0 + v], 0.f);
            }
            *reinterpret_cast<bf16x4 *>(out + cell * kHid + co0) = o;
        }
    }
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// The output layer (32 channels -> 1) is a matrix-vector product per cell: on
// the 16 x 16 MFMA tile it would fill one output row of sixteen.  Here it
// runs on the VALU with packed BF16 dot products (v_dot2_f32_bf16, FP32
// accumulation), from an LDS patch like k_conv's but of kOutZ cells of z (a
// smaller patch, so that two blocks fit a CU and one block's staging overlaps
// another's arithmetic): four adjacent lanes share a cell, lane q taking
// channels 8q..8q+7, so that a wavefront's LDS reads are consecutive 16-byte
// chunks (no bank conflicts) and its weight reads are four-way broadcasts;
// the four partial sums of a cell are added with two quad DPP exchanges.  A
// wavefront covers its column's kOutZ cells in passes of 16.
// outf = sum + bias (FP32).
constexpr int kOutZ = 32;

__global__ void __launch_bounds__(kTileThreads) k_conv_out(NetGeo g, const bf16 *__restrict__ in,
                                                           const bf16 *__restrict__ wp,
                                                           const float *__restrict__ bias,
                                                           float *__restrict__ outf)
{
    constexpr int CIN = kHid, CH = CIN / 8, TZO = kOutZ + 2;
    static_assert(CH == 4, "one lane per 16-byte chunk of a cell, four per cell");
    __shared__ bf16x8 sW[kTaps * CH];
    __shared__ bf16x8 sT[TX * TY * TZO * CH];
    const int pxn = (g.nx + PX - 1) / PX;
    const int zto = (g.nz + kOutZ - 1) / kOutZ;
    const int zti = blockIdx.x % zto;
    const int pxy = blockIdx.x / zto;
    const int px0 = (pxy % pxn) * PX, py0 = (pxy / pxn) * PY, z0 = zti * kOutZ;
    // packed forward weights, one output block: step s, lane 16 q holds
    // channels 8q..8q+7 of output channel 0 at tap s
    const bf16x8 *wv = reinterpret_cast<const bf16x8 *>(wp);
    for (int e = threadIdx.x; e < kTaps * CH; e += kTileThreads) sW[e] = wv[(e / CH) * 64 + 16 * (e % CH)];
    stage_patch<CH, false, kOutZ>(g, in, px0, py0, z0, sT);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int cx = wave % PX, cy = wave / PX;
    const int i = px0 + cx, j = py0 + cy;
    if (i >= g.nx || j >= g.ny) return;            // whole wavefront
    const int q = lane & 3, cc = lane >> 2;
    const float b0 = bias[0];
#pragma unroll
    for (int pass = 0; pass < kOutZ / 16; pass++) {
        const int kl = 16 * pass + cc;              // cell of the column's z-run
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tap = 0; tap < kTaps; tap++) {
            const int di = tap / 9 - 1, dj = (tap / 3) % 3 - 1, dk = tap % 3 - 1;
            const int cl = (cx + 1 + di) + TX * (cy + 1 + dj);
            const bf16x8 x = sT[(cl * TZO + kl + 1 + dk) * CH + q];
            const bf16x8 w = sW[tap * CH + q];
#pragma unroll
            for (int e = 0; e < 8; e += 2)
                acc[e / 2] = __builtin_amdgcn_fdot2_f32_bf16(bf16x2{x[e], x[e + 1]}, bf16x2{w[e], w[e + 1]},
                                                            acc[e / 2], false);
        }
        float sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        sum += dpp_quad_xor1(sum);
        sum += dpp_quad_xor2(sum);
        const int k = z0 + kl;
        if (q == 0 && k < g.nz) outf[(long)(i + g.nx * j) * g.nz + k] = sum + b0;
    }
}

// Weight gradient of one layer, one tap and one chunk of columns per
// wavefront: D[co][ci] += sum over 32 cells of dz[cell][co] x[cell + tap][ci]
// on the matrix cores, both operands transposed through LDS ([channel][cell]
// rows, so that each lane reads 8 consecutive cells of one channel).
// CIN / COUT: stored channels (8 or 32).
template <int CIN, int COUT>
__global__ void __launch_bounds__(64) k_wgrad(NetGeo g, const bf16 *__restrict__ x,
                                              const bf16 *__restrict__ dz, float *__restrict__ part)
{
    constexpr int CB = (COUT == 32) ? 2 : 1;
    constexpr int NB = (CIN == 32) ? 2 : 1;
    constexpr int LD = 40;                    // row stride (bf16): 80 B keeps 16-byte alignment
    __shared__ __attribute__((aligned(16))) bf16 sA[32 * LD];
    __shared__ __attribute__((aligned(16))) bf16 sB[32 * LD];
    const int tap = blockIdx.x % kTaps, chunk = blockIdx.x / kTaps;
    const int lane = threadIdx.x;
    const int n = lane & 15, q = lane >> 4;
    // rows never written below (channels beyond the stored ones) stay zero
    for (int e = lane; e < 32 * LD; e += 64) {
        sA[e] = (bf16)0.0f;
        sB[e] = (bf16)0.0f;
    }
    __syncthreads();
    f32x4 acc[CB][NB];
#pragma unroll
    for (int b = 0; b < CB; b++)
#pragma unroll
        for (int c = 0; c < NB; c++) acc[b][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int c0 = chunk * g.cols_per_chunk;
    const int c1 = min(c0 + g.cols_per_chunk, g.ncol);
    const int zc = lane >> 1, half = lane & 1;
    for (int col = c0; col < c1; col++) {
        const int i = col % g.nx, j = col / g.nx;
        for (int z0 = 0; z0 < g.nz; z0 += 32) {
            const int z = z0 + zc;
            const bool okc = z < g.nz;
            const long cell = (long)col * g.nz + z;
            long nb = 0;
            const bool okn = okc && tap_nbr(g, i, j, z, tap, nb);
            // dz rows: 16 channels per lane (32 stored) or 8 (lane half 0)
            if (COUT == 32) {
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const bf16x8 v = okc ? *reinterpret_cast<const bf16x8 *>(dz + cell * 32 + 16 * half + 8 * h)
                                         : zero8();
#pragma unroll
                    for (int e = 0; e < 8; e++) sA[(16 * half + 8 * h + e) * LD + zc] = v[e];
                }
            } else if (half == 0) {
                const bf16x8 v = okc ? *reinterpret_cast<const bf16x8 *>(dz + cell * 8) : zero8();
#pragma unroll
                for (int e = 0; e < 8; e++) sA[e * LD + zc] = v[e];
            }
            if (CIN == 32) {
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const bf16x8 v = okn ? *reinterpret_cast<const bf16x8 *>(x + nb * 32 + 16 * half + 8 * h)
                                         : zero8();
#pragma unroll
                    for (int e = 0; e < 8; e++) sB[(16 * half + 8 * h + e) * LD + zc] = v[e];
                }
            } else if (half == 0) {
                const bf16x8 v = okn ? *reinterpret_cast<const bf16x8 *>(x + nb * 8) : zero8();
#pragma unroll
                for (int e = 0; e < 8; e++) sB[e * LD + zc] = v[e];
            }
            __syncthreads();
            bf16x8 A[CB], B[NB];
#pragma unroll
            for (int b = 0; b < CB; b++) A[b] = *reinterpret_cast<const bf16x8 *>(&sA[(16 * b + n) * LD + 8 * q]);
#pragma unroll
            for (int c = 0; c < NB; c++) B[c] = *reinterpret_cast<const bf16x8 *>(&sB[(16 * c + n) * LD + 8 * q]);
#pragma unroll
            for (int b = 0; b < CB; b++)
#pragma unroll
                for (int c = 0; c < NB; c++)
                    acc[b][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[b], B[c], acc[b][c], 0, 0, 0);
            __syncthreads();
        }
    }
    float *P = part + ((long)chunk * kTaps + tap) * 1024;
#pragma unroll
    for (int b = 0; b < CB; b++)
#pragma unroll
        for (int c = 0; c < NB; c++)
#pragma unroll
            for (int v = 0; v < 4; v++) P[(16 * b + 4 * q + v) * 32 + 16 * c + n] = acc[b][c][v];
}

// dW of layer l in the parameter layout, summing the chunk partials in order.
__global__ void k_wreduce(NetGeo g, const float *__restrict__ part, float *__restrict__ grad, int woff,
                          int cin, int cout)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = cout * kTaps * cin;
    if (e >= n) return;
    const int ci = e % cin, tap = (e / cin) % kTaps, co = e / (cin * kTaps);
    float s = 0.f;
    for (int ch = 0; ch < g.chunks; ch++) s += part[((long)ch * kTaps + tap) * 1024 + co * 32 + ci];
    grad[woff + e] = s;
}

// Bias gradient partials: block b sums its cells for every channel.
template <int COUT>
__global__ void __launch_bounds__(256) k_bgrad(NetGeo g, const bf16 *__restrict__ dz,
                                               float *__restrict__ bpart)
{
    __shared__ float s[256];
    const int ch = threadIdx.x & 31, sub = threadIdx.x >> 5;   // 8 cell lanes per channel
    float acc = 0.f;
    if (ch < COUT)
        for (long c = (long)blockIdx.x * 8 + sub; c < g.ncell; c += (long)gridDim.x * 8)
            acc += (float)dz[c * COUT + ch];
    s[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 32) {
        float t = 0.f;
        for (int k = 0; k < 8; k++) t += s[k * 32 + threadIdx.x];
        bpart[blockIdx.x * 32 + threadIdx.x] = t;
    }
}

__global__ void k_breduce(const float *__restrict__ bpart, int nblk, float *__restrict__ grad, int boff,
                          int cout)
{
    const int co = threadIdx.x;
    if (co >= cout) return;
    float t = 0.f;
    for (int b = 0; b < nblk; b++) t += bpart[b * 32 + co];
    grad[boff + co] = t;
}

// Features of every cell (channels 4..7 zero).
__global__ void k_features(NetGeo g, const double *__restrict__ hn, const double *__restrict__ hp,
                           const double *__restrict__ lnks, double rain, bf16 *__restrict__ feat)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    bf16x8 f = zero8();
    f[0] = (bf16)(float)(hn[c] / kHScale);
    f[1] = (bf16)(float)((hn[c] - hp[c]) * kDhScale);
    f[2] = (bf16)(float)(lnks ? lnks[c] : 0.0);
    f[3] = (bf16)(float)(rain * kRainScale);
    *reinterpret_cast<bf16x8 *>(feat + c * kFeat) = f;
}

// The network predicts a correction to the linear extrapolation in time:
// h^{n+1,0} = h^n + (h^n - h^{n-1}) + 0.01 m y.
__device__ __forceinline__ double guess_of(double hn, double hp, float y)
{
    return hn + (hn - hp) + kOutScale * (double)y;
}

__global__ void k_output(NetGeo g, const float *__restrict__ y, const double *__restrict__ hn,
                         const double *__restrict__ hp, double *__restrict__ guess)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    guess[c] = guess_of(hn[c], hp[c], y[c]);
}

// r = (h^{n+1,0} - target) / 0.01 m (the error in units of the output
// scale, so that gradients stay well above Adam's epsilon); loss partials of
// 0.5 r^2 / N; dz3 = dL/dy = r / N.
__global__ void __launch_bounds__(256) k_loss(NetGeo g, const float *__restrict__ y,
                                              const double *__restrict__ hn,
                                              const double *__restrict__ hp,
                                              const double *__restrict__ target, bf16 *__restrict__ dz3,
                                              double *__restrict__ lpart)
{
    __shared__ double s[256];
    const double inv = 1.0 / (double)g.ncell;
    double acc = 0.0;
    for (long c = (long)blockIdx.x * 256 + threadIdx.x; c < g.ncell; c += (long)gridDim.x * 256) {
        const double r = (guess_of(hn[c], hp[c], y[c]) - target[c]) / kOutScale;
        acc += 0.5 * r * r * inv;
        bf16x8 d = zero8();
        d[0] = (bf16)(float)(r * inv);
        *reinterpret_cast<bf16x8 *>(dz3 + c * 8) = d;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = s[0];
}

// Packed BF16 operand of layer l (see packed_size).  Forward: A[m][k] =
// W_l[oc = 16 b + m][tap][ic]; backward (gradient with respect to the layer
// input): the transposed, tap-mirrored W_l[co = ic][26 - tap][ci = oc].
__global__ void k_pack(const float *__restrict__ p, bf16 *__restrict__ dst, int l, int backward,
                       int cin_stored, int cob)
{
    const int steps = (cin_stored == 32) ? kTaps : (kTaps + 3) / 4;
    const int total = steps * cob * 64 * 8;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int jj = e % 8, lane = (e / 8) % 64, b = (e / 512) % cob, s = e / (512 * cob);
    const int m = lane % 16, kq = lane / 16;
    const int oc = 16 * b + m;
    int tap, ic;
    if (cin_stored == 32) {
        tap = s;
        ic = 8 * kq + jj;
    } else {
        tap = 4 * s + kq;
        ic = jj;
    }
    float w = 0.f;
    const int cin = kCin[l], cout = kCout[l];
    if (tap < kTaps) {
        if (!backward) {
            if (oc < cout && ic < cin) w = p[param_w(l) + (oc * kTaps + tap) * cin + ic];
        } else {
            if (ic < cout && oc < cin) w = p[param_w(l) + (ic * kTaps + (kTaps - 1 - tap)) * cin + oc];
        }
    }
    dst[e] = (bf16)w;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float bc1, float bc2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = 0.9f * m[e] + 0.1f * gi;
    const float vi = 0.999f * v[e] + 0.001f * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// One block per patch of PX x PY columns and 64 cells of z (kOutZ for the
// output layer).
int conv_grid(const NetGeo &g)
{
    return ((g.nx + PX - 1) / PX) * ((g.ny + PY - 1) / PY) * g.zt;
}

int conv_out_grid(const NetGeo &g)
{
    return ((g.nx + PX - 1) / PX) * ((g.ny + PY - 1) / PY) * ((g.nz + kOutZ - 1) / kOutZ);
}

}  // namespace

hipError_t net_pack(const NetArrays &a, hipStream_t s)
{
    const int cin_f[kNetLayers] = {8, 32, 32, 32}, cob_f[kNetLayers] = {2, 2, 2, 1};
    const int cin_b[kNetLayers] = {0, 32, 32, 8};
    for (int l = 0; l < kNetLayers; l++) {
        int total = packed_size(cin_f[l], cob_f[l]);
        hipLaunchKernelGGL(k_pack, dim3((total + 255) / 256), dim3(256), 0, s, a.p, a.wf[l], l, 0,
                           cin_f[l], cob_f[l]);
        if (l > 0) {
            total = packed_size(cin_b[l], 2);
            hipLaunchKernelGGL(k_pack, dim3((total + 255) / 256), dim3(256), 0, s, a.p, a.wb[l], l, 1,
                               cin_b[l], 2);
        }
    }
    return hipGetLastError();
}

hipError_t net_features(const NetGeo &g, const NetArrays &a, const double *hn, const double *hprev,
                        const double *lnks, double rain, hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3((unsigned)((g.ncell + 255) / 256)), dim3(256), 0, s, g, hn, hprev,
                       lnks, rain, a.feat);
    return hipGetLastError();
}

hipError_t net_forward(const NetGeo &g, const NetArrays &a, hipStream_t s)
{
    const dim3 grid(conv_grid(g)), block(kTileThreads);
    hipLaunchKernelGGL((k_conv<8, 2, EPI_RELU>), grid, block, 0, s, g, a.feat, a.wf[0], a.p + param_b(0),
                       a.act[0], nullptr);
    hipLaunchKernelGGL((k_conv<32, 2, EPI_RELU>), grid, block, 0, s, g, a.act[0], a.wf[1],
                       a.p + param_b(1), a.act[1], nullptr);
    hipLaunchKernelGGL((k_conv<32, 2, EPI_RELU>), grid, block, 0, s, g, a.act[1], a.wf[2],
                       a.p + param_b(2), a.act[2], nullptr);
    hipLaunchKernelGGL(k_conv_out, dim3(conv_out_grid(g)), block, 0, s, g, a.act[2], a.wf[3],
                       a.p + param_b(3), a.y);
    return hipGetLastError();
}

hipError_t net_output(const NetGeo &g, const NetArrays &a, const double *hn, const double *hprev,
                      double *guess, hipStream_t s)
{
    hipLaunchKernelGGL(k_output, dim3((unsigned)((g.ncell + 255) / 256)), dim3(256), 0, s, g, a.y, hn,
                       hprev, guess);
    return hipGetLastError();
}

hipError_t net_loss(const NetGeo &g, const NetArrays &a, const double *hn, const double *hprev,
                    const double *target, hipStream_t s)
{
    hipLaunchKernelGGL(k_loss, dim3(a.lblocks), dim3(256), 0, s, g, a.y, hn, hprev, target, a.dz3,
                       a.lpart);
    return hipGetLastError();
}

static hipError_t grads_of_layer(const NetGeo &g, const NetArrays &a, int l, const bf16 *x,
                                 const bf16 *dz, hipStream_t s)
{
    const dim3 wg(g.chunks * kTaps);
    if (l == 0)
        hipLaunchKernelGGL((k_wgrad<8, 32>), wg, dim3(64), 0, s, g, x, dz, a.part);
    else if (l == 3)
        hipLaunchKernelGGL((k_wgrad<32, 8>), wg, dim3(64), 0, s, g, x, dz, a.part);
    else
        hipLaunchKernelGGL((k_wgrad<32, 32>), wg, dim3(64), 0, s, g, x, dz, a.part);
    const int nw = kCout[l] * kTaps * kCin[l];
    hipLaunchKernelGGL(k_wreduce, dim3((nw + 255) / 256), dim3(256), 0, s, g, a.part, a.g, param_w(l),
                       kCin[l], kCout[l]);
    constexpr int kBBlocks = 256;
    float *bpart = a.part;   // reused after the weight reduction
    if (l == 3)
        hipLaunchKernelGGL((k_bgrad<8>), dim3(kBBlocks), dim3(256), 0, s, g, dz, bpart);
    else
        hipLaunchKernelGGL((k_bgrad<32>), dim3(kBBlocks), dim3(256), 0, s, g, dz, bpart);
    hipLaunchKernelGGL(k_breduce, dim3(1), dim3(32), 0, s, bpart, kBBlocks, a.g, param_b(l), kCout[l]);
    return hipGetLastError();
}

hipError_t net_backward(const NetGeo &g, const NetArrays &a, hipStream_t s)
{
    const dim3 grid(conv_grid(g)), block(kTileThreads);
    hipError_t e;
    // layer 4 (index 3): input a3, output gradient dz3
    if ((e = grads_of_layer(g, a, 3, a.act[2], a.dz3, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_conv<8, 2, EPI_MASK>), grid, block, 0, s, g, a.dz3, a.wb[3], nullptr, a.dz[0],
                       a.act[2]);
    // layer 3 (index 2): input a2, output gradient dz[0]
    if ((e = grads_of_layer(g, a, 2, a.act[1], a.dz[0], s)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_conv<32, 2, EPI_MASK>), grid, block, 0, s, g, a.dz[0], a.wb[2], nullptr,
                       a.dz[1], a.act[1]);
    // layer 2 (index 1): input a1, output gradient dz[1]
    if ((e = grads_of_layer(g, a, 1, a.act[0], a.dz[1], s)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_conv<32, 2, EPI_MASK>), grid, block, 0, s, g, a.dz[1], a.wb[1], nullptr,
                       a.dz[0], a.act[0]);
    // layer 1 (index 0): input features, output gradient dz[0]
    return grads_of_layer(g, a, 0, a.feat, a.dz[0], s);
}

hipError_t net_adam(const NetArrays &a, float lr, float bc1, float bc2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, a.p, a.g, a.m, a.v, kParams,
                       lr, bc1, bc2);
    return net_pack(a, s);
}

}  // namespace rf
