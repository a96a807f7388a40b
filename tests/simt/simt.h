// SIMT emulation of the HIP device and host API used by the library (3-D
// solver and column ensemble), for running its unmodified kernel and host
// sources on the CPU under
// AddressSanitizer / UndefinedBehaviorSanitizer (test infrastructure only).
//
// Every GPU thread is a fiber of one OS thread (own stack, switched by a
// few instructions of assembly).  A block's
// fibers run round-robin; a cross-lane operation (shuffle, readfirstlane,
// the wave's clock) parks the lane until every live lane of its 64-lane wave
// has reached a cross-lane operation, which must be the same one, and then
// hands each lane its result; __syncthreads parks until every live thread of
// the block has arrived.  Any other state -- lanes of one wave parked at
// different cross-lane operations, a lane reading a lane that has exited, a
// barrier some threads never reach -- is reported as divergence and aborts.
// Blocks run one after another.  Device memory is host memory.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct __attribute__((aligned(16))) int4 {
    int x, y, z, w;
};

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace simt {

enum LaneOp { kShflUp = 1, kShflDown, kShflXor, kShflIdx, kReadFirst, kClock, kReadLane, kDpp };

dim3 thread_idx();
dim3 block_idx();
dim3 block_dim();
dim3 grid_dim();
uint64_t lane_op(int kind, uint64_t bits, int param, int width);
void sync_block();
void launch(dim3 grid, dim3 block, std::function<void()> body);
// lane operations resolved so far (the emulated clock advances with them)
unsigned long long ops_resolved();

template <class T>
inline uint64_t to_bits(T v)
{
    uint64_t b = 0;
    memcpy(&b, &v, sizeof(T));
    return b;
}
template <class T>
inline T from_bits(uint64_t b)
{
    T v;
    memcpy(&v, &b, sizeof(T));
    return v;
}

}  // namespace simt

#define threadIdx (::simt::thread_idx())
#define blockIdx (::simt::block_idx())
#define blockDim (::simt::block_dim())
#define gridDim (::simt::grid_dim())

template <class T>
inline T __shfl_up(T v, unsigned d, int w = 64)
{
    return simt::from_bits<T>(simt::lane_op(simt::kShflUp, simt::to_bits(v), (int)d, w));
}
template <class T>
inline T __shfl_down(T v, unsigned d, int w = 64)
{
    return simt::from_bits<T>(simt::lane_op(simt::kShflDown, simt::to_bits(v), (int)d, w));
}
template <class T>
inline T __shfl_xor(T v, int m, int w = 64)
{
    return simt::from_bits<T>(simt::lane_op(simt::kShflXor, simt::to_bits(v), m, w));
}
template <class T>
inline T __shfl(T v, int src, int w = 64)
{
    return simt::from_bits<T>(simt::lane_op(simt::kShflIdx, simt::to_bits(v), src, w));
}
inline int __builtin_amdgcn_readfirstlane(int v)
{
    return simt::from_bits<int>(simt::lane_op(simt::kReadFirst, simt::to_bits(v), 0, 64));
}
inline int __builtin_amdgcn_readlane(int v, int l)
{
    return simt::from_bits<int>(simt::lane_op(simt::kReadLane, simt::to_bits(v), l, 64));
}
// DPP move (GFX9 controls row_shl/row_shr 1-15, wave_shl1, wave_shr1,
// row_bcast15; all banks enabled): a lane whose row is not in row_mask keeps
// `old`; a lane whose source lies outside its row (or the wave) keeps `old`,
// or gets 0 with bound_ctrl (zero fill, only with all rows enabled)
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                                       bool bound_ctrl)
{
    if (row_mask < 1 || row_mask > 0xF || bank_mask != 0xF || (bound_ctrl && row_mask != 0xF)) abort();
    const uint64_t packed = ((uint64_t)(uint32_t)old << 32) | (uint32_t)src;
    return simt::from_bits<int>(simt::lane_op(simt::kDpp, packed,
                                              ctrl | (row_mask << 16) | ((int)bound_ctrl << 20), 64));
}
// exponent e with |x| in [2^(e-1), 2^e) (v_frexp_exp_i32_f64 / _f32: 0 for 0, inf, NaN)
inline int __builtin_amdgcn_frexp_exp(double x)
{
    if (x == 0.0 || !std::isfinite(x)) return 0;
    int e = 0;
    std::frexp(x, &e);
    return e;
}
inline int __builtin_amdgcn_frexp_expf(float x)
{
    if (x == 0.0f || !std::isfinite(x)) return 0;
    int e = 0;
    std::frexp(x, &e);
    return e;
}
inline int __float_as_int(float f) { return simt::from_bits<int>(simt::to_bits(f)); }
inline float __int_as_float(int i) { return simt::from_bits<float>(simt::to_bits(i)); }
inline long long __double_as_longlong(double d) { return simt::from_bits<long long>(simt::to_bits(d)); }
inline double __longlong_as_double(long long l) { return simt::from_bits<double>(simt::to_bits(l)); }
inline long long wall_clock64()
{
    return (long long)simt::lane_op(simt::kClock, 0, 0, 64);
}
inline unsigned int atomicAdd(unsigned int *p, unsigned int v)
{
    const unsigned int o = *p;   // fibers of one OS thread never interleave inside
    *p = o + v;
    return o;
}
inline void __syncthreads() { simt::sync_block(); }
inline int __double2loint(double d) { return (int)(uint32_t)simt::to_bits(d); }
inline int __double2hiint(double d) { return (int)(uint32_t)(simt::to_bits(d) >> 32); }
inline double __hiloint2double(int hi, int lo)
{
    return simt::from_bits<double>(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
using std::isfinite;
using std::max;
using std::min;

// ---- host API ---------------------------------------------------------
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidDevice = 101, hipErrorNotReady = 600,
       hipErrorInvalidSymbol = 13 };
typedef void *hipStream_t;
struct simt_event;
typedef simt_event *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeWallClockRate };
#define hipHostMallocDefault 0u
#define hipEventDisableTiming 0u
#define hipEventDisableSystemFence 0u

hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int *d);
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int d);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags);
hipError_t hipHostFree(void *p);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipGetLastError();
hipError_t hipStreamQuery(hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
#define HIP_SYMBOL(x) (&(x))
template <class T>
inline hipError_t hipGetSymbolAddress(void **p, const T *sym)
{
    *p = (void *)sym;
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t e);
template <class F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, F, int, size_t)
{
    *n = 1;
    return hipSuccess;
}
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) \
    ::simt::launch(dim3(g), dim3(b), [=]() { k(__VA_ARGS__); })
#define hipExtLaunchKernelGGL(k, g, b, sh, st, ea, eb, fl, ...)                   \
    do {                                                                        \
        hipEventRecord(ea, st);                                                 \
        ::simt::launch(dim3(g), dim3(b), [=]() { k(__VA_ARGS__); });            \
        hipEventRecord(eb, st);                                                 \
    } while (0)
