// Cross-lane primitives of a 64-lane wavefront on gfx950 (GFX9 DPP).
//
// The column recurrences of the solver (vertical neighbours, the z-line
// forward/backward sweeps and the tridiagonal pivots) need shifts and
// prefix scans across the lanes of one wave.  Written with __shfl_* they
// compile to ds_bpermute, a round trip through the LDS crossbar per 32-bit
// value and scan step.  Here the shifts use DPP modifiers (executed by the
// VALU): row_shr/row_shl move data inside each 16-lane row, wave_shr/wave_shl
// move the whole wave by one lane, and the four rows of a scan are chained
// through v_readlane (the row ends become wave-uniform values).
//
// Every function must be called with all 64 lanes active (wave-uniform
// control flow): a DPP source lane that is switched off is not read.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

namespace rf {

// DPP control codes (GFX9 encoding).
enum : int {
    kDppRowShl = 0x100,   // + k: lane i of a row reads lane i + k of the same row
    kDppRowShr = 0x110,   // + k: lane i of a row reads lane i - k of the same row
    kDppWaveShl1 = 0x130, // lane i reads lane i + 1 (lane 63: no source)
    kDppWaveShr1 = 0x138, // lane i reads lane i - 1 (lane 0: no source)
    kDppRowBcast15 = 0x142, // every lane of row r >= 1 reads lane 16 r - 1
};

// x moved by the DPP pattern CTRL; lanes without a source lane get `old`.
template <int CTRL>
__device__ __forceinline__ float dpp(float x, float old)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL,
                                                      0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x, double old)
{
    const long long xi = __double_as_longlong(x), oi = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)xi, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(xi >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) |
                                            (unsigned int)lo));
}

// x moved by CTRL; lanes without a source lane get 0 (the zero fill of DPP,
// BOUND_CTRL = 1, so no register has to be set to the fill value first).
template <int CTRL>
__device__ __forceinline__ float dpp0(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp0(double x)
{
    const long long xi = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)xi, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(xi >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) |
                                            (unsigned int)lo));
}

// x moved by CTRL; lanes without a source lane get 1 (the low word of 1.0 is
// the zero fill, only the high word is set first).
template <int CTRL>
__device__ __forceinline__ float dpp1(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0x3F800000, __float_as_int(x), CTRL, 0xF, 0xF,
                                                      false));
}

template <int CTRL>
__device__ __forceinline__ double dpp1(double x)
{
    const long long xi = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)xi, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0x3FF00000, (int)(xi >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) |
                                            (unsigned int)lo));
}

// The same in the rows named by ROWS (bit r: row r) only; the other rows get
// `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows(float x, float old)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL,
                                                      ROWS, 0xF, false));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double x, double old)
{
    const long long xi = __double_as_longlong(x), oi = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)xi, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(xi >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) |
                                            (unsigned int)lo));
}

// Value of lane L (wave-uniform result).
template <int L>
__device__ __forceinline__ float lane_value(float x)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), L));
}

template <int L>
__device__ __forceinline__ double lane_value(double x)
{
    const long long xi = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)xi, L);
    const int hi = __builtin_amdgcn_readlane((int)(xi >> 32), L);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) |
                                            (unsigned int)lo));
}

// x of lane i - 1 (lane 0 gets `edge`) and of lane i + 1 (lane 63 gets `edge`).
template <typename T>
__device__ __forceinline__ T from_below(T x, T edge) { return dpp<kDppWaveShr1>(x, edge); }
template <typename T>
__device__ __forceinline__ T from_above(T x, T edge) { return dpp<kDppWaveShl1>(x, edge); }
// The same with edge 0.
template <typename T>
__device__ __forceinline__ T from_below0(T x) { return dpp0<kDppWaveShr1>(x); }
template <typename T>
__device__ __forceinline__ T from_above0(T x) { return dpp0<kDppWaveShl1>(x); }

// Inclusive upward scan of affine maps x_k = a_k x_{k-1} + c_k over the
// wave (k = lane); returns x_k for x_{-1} = carry.  Inside each 16-lane row
// the maps are composed in four doubling steps (a lane whose partner lies
// below its row composes with the identity); the rows are then chained from
// the values at lanes 15, 31 and 47.
template <typename T>
__device__ __forceinline__ T scan_affine_up(T a, T c, T carry, int lane)
{
#define RF_UP_STEP(K)                                          \
    {                                                          \
        const T ao = dpp1<kDppRowShr + (K)>(a);                \
        const T co = dpp0<kDppRowShr + (K)>(c);                \
        c = a * co + c;                                        \
        a = a * ao;                                            \
    }
    RF_UP_STEP(1) RF_UP_STEP(2) RF_UP_STEP(4) RF_UP_STEP(8)
#undef RF_UP_STEP
    const T y0 = lane_value<15>(a) * carry + lane_value<15>(c);
    const T y1 = lane_value<31>(a) * y0 + lane_value<31>(c);
    const T y2 = lane_value<47>(a) * y1 + lane_value<47>(c);
    const int row = lane >> 4;
    const T cin = (row == 0) ? carry : (row == 1) ? y0 : (row == 2) ? y1 : y2;
    return a * cin + c;
}

// Inclusive downward scan of x_k = b_k x_{k+1} + c_k; x_64 = carry.  Rows
// are chained from the values at lanes 48, 32 and 16.
template <typename T>
__device__ __forceinline__ T scan_affine_down(T b, T c, T carry, int lane)
{
#define RF_DOWN_STEP(K)                                        \
    {                                                          \
        const T bo = dpp1<kDppRowShl + (K)>(b);                \
        const T co = dpp0<kDppRowShl + (K)>(c);                \
        c = b * co + c;                                        \
        b = b * bo;                                            \
    }
    RF_DOWN_STEP(1) RF_DOWN_STEP(2) RF_DOWN_STEP(4) RF_DOWN_STEP(8)
#undef RF_DOWN_STEP
    const T y3 = lane_value<48>(b) * carry + lane_value<48>(c);
    const T y2 = lane_value<32>(b) * y3 + lane_value<32>(c);
    const T y1 = lane_value<16>(b) * y2 + lane_value<16>(c);
    const int row = lane >> 4;
    const T cin = (row == 3) ? carry : (row == 2) ? y3 : (row == 1) ? y2 : y1;
    return b * cin + c;
}

// Exponent e of a finite x with |x| in [2^(e-1), 2^e) (v_frexp_exp_i32_f64;
// 0 for x = 0).
__device__ __forceinline__ int frexp_exponent(double x) { return __builtin_amdgcn_frexp_exp(x); }
__device__ __forceinline__ int frexp_exponent(float x) { return __builtin_amdgcn_frexp_expf(x); }

// Scales (m00, m01, m10, m11) by the power of two that brings the largest
// magnitude into [1, 2) (exact; zero stays zero).
__device__ __forceinline__ void rescale4(double &m00, double &m01, double &m10, double &m11)
{
    const double sc = fmax(fmax(fabs(m00), fabs(m01)), fmax(fabs(m10), fabs(m11)));
    const int ex = 1 - frexp_exponent(sc);
    m00 = ldexp(m00, ex); m01 = ldexp(m01, ex); m10 = ldexp(m10, ex); m11 = ldexp(m11, ex);
}

__device__ __forceinline__ void rescale2(double &v0, double &v1)
{
    const double sc = fmax(fabs(v0), fabs(v1));
    const int ex = 1 - frexp_exponent(sc);
    v0 = ldexp(v0, ex);
    v1 = ldexp(v1, ex);
}

// Pivots of a column tridiagonal T (diagonal diag_k, off-diagonal t_{k-1}
// below and above): d_k = diag_k - t_{k-1}^2 / d_{k-1}.  The leading minors
// obey P_k = diag_k P_{k-1} - t_{k-1}^2 P_{k-2}, so (P_k, P_{k-1}) is the
// prefix product of the 2x2 matrices [[diag_k, -t_{k-1}^2], [1, 0]] applied
// to (P_{k0-1}, P_{k0-2}); d_k = P_k / P_{k-1}.  Products are rescaled by
// powers of two after every step (only ratios matter).  carry = d_{k0-1}
// (0 for the first cells of the column, where (P_{-1}, P_{-2}) = (1, 0)).
__device__ __forceinline__ double scan_pivots(double diag, double tprev2, double carry, int lane)
{
    double m00 = diag, m01 = -tprev2, m10 = 1.0, m11 = 0.0;
#define RF_PIV_STEP(K)                                                      \
    {                                                                       \
        const double o00 = dpp1<kDppRowShr + (K)>(m00);                     \
        const double o01 = dpp0<kDppRowShr + (K)>(m01);                     \
        const double o10 = dpp0<kDppRowShr + (K)>(m10);                     \
        const double o11 = dpp1<kDppRowShr + (K)>(m11);                     \
        const double n00 = m00 * o00 + m01 * o10;                           \
        const double n01 = m00 * o01 + m01 * o11;                           \
        const double n10 = m10 * o00 + m11 * o10;                           \
        const double n11 = m10 * o01 + m11 * o11;                           \
        m00 = n00; m01 = n01; m10 = n10; m11 = n11;                         \
        rescale4(m00, m01, m10, m11);                                       \
    }
    RF_PIV_STEP(1) RF_PIV_STEP(2) RF_PIV_STEP(4) RF_PIV_STEP(8)
#undef RF_PIV_STEP
    // (P, P_prev) entering each row: carry vector, then through the row ends
    double u0 = (carry != 0.0) ? carry : 1.0, u1 = (carry != 0.0) ? 1.0 : 0.0;
    double r0[4] = {u0, 0, 0, 0}, r1[4] = {u1, 0, 0, 0};
#define RF_PIV_ROW(L, R)                                                        \
    {                                                                           \
        const double a00 = lane_value<L>(m00), a01 = lane_value<L>(m01);        \
        const double a10 = lane_value<L>(m10), a11 = lane_value<L>(m11);        \
        double w0 = a00 * u0 + a01 * u1, w1 = a10 * u0 + a11 * u1;              \
        rescale2(w0, w1);                                                       \
        u0 = w0; u1 = w1;                                                       \
        r0[R] = u0; r1[R] = u1;                                                 \
    }
    RF_PIV_ROW(15, 1) RF_PIV_ROW(31, 2) RF_PIV_ROW(47, 3)
#undef RF_PIV_ROW
    const int row = lane >> 4;
    const double v0 = (row == 0) ? r0[0] : (row == 1) ? r0[1] : (row == 2) ? r0[2] : r0[3];
    const double v1 = (row == 0) ? r1[0] : (row == 1) ? r1[1] : (row == 2) ? r1[2] : r1[3];
    return (m00 * v0 + m01 * v1) / (m10 * v0 + m11 * v1);
}

// ---------------------------------------------------------------------------
// Two columns per wave: column h in lanes 32h .. 32h + 31, each lane carrying
// the composite of its consecutive cells.  The scans below run over the 32
// lanes of each half: four doubling steps inside each 16-lane row, then the
// second row of each half composes with its first row's total (row_bcast:15
// into rows 1 and 3 for the upward scans; lanes 16 and 48 read back into rows
// 0 and 2 for the downward one).
// ---------------------------------------------------------------------------

// Inclusive upward scan of affine maps x -> a x + c within each half:
// (a, c) of lane l becomes the composite of the maps of lanes 32h .. l, the
// later lanes applied last.
template <typename T>
__device__ __forceinline__ void scan_affine_up_half(T &a, T &c)
{
#define RF_UP_STEP(K)                                          \
    {                                                          \
        const T ao = dpp1<kDppRowShr + (K)>(a);                \
        const T co = dpp0<kDppRowShr + (K)>(c);                \
        c = a * co + c;                                        \
        a = a * ao;                                            \
    }
    RF_UP_STEP(1) RF_UP_STEP(2) RF_UP_STEP(4) RF_UP_STEP(8)
#undef RF_UP_STEP
    const T ao = dpp_rows<kDppRowBcast15, 0xA>(a, T(1));
    const T co = dpp_rows<kDppRowBcast15, 0xA>(c, T(0));
    c = a * co + c;
    a = a * ao;
}

// Inclusive downward scan of maps x -> b x + c within each half: (b, c) of
// lane l becomes the composite of the maps of lanes l .. 32h + 31, the lower
// lanes applied last.
template <typename T>
__device__ __forceinline__ void scan_affine_down_half(T &b, T &c, int lane)
{
#define RF_DOWN_STEP(K)                                        \
    {                                                          \
        const T bo = dpp1<kDppRowShl + (K)>(b);                \
        const T co = dpp0<kDppRowShl + (K)>(c);                \
        c = b * co + c;                                        \
        b = b * bo;                                            \
    }
    RF_DOWN_STEP(1) RF_DOWN_STEP(2) RF_DOWN_STEP(4) RF_DOWN_STEP(8)
#undef RF_DOWN_STEP
    const T b16 = lane_value<16>(b), c16 = lane_value<16>(c);
    const T b48 = lane_value<48>(b), c48 = lane_value<48>(c);
    const int row = lane >> 4;
    const T bo = (row == 0) ? b16 : (row == 2) ? b48 : T(1);
    const T co = (row == 0) ? c16 : (row == 2) ? c48 : T(0);
    c = b * co + c;
    b = b * bo;
}

// Inclusive upward scan of 2x2 matrices within each half: m of lane l
// becomes the product of the matrices of lanes 32h .. l, the later lanes on
// the left, rescaled by a power of two after every step (only ratios of its
// entries are used).
__device__ __forceinline__ void scan_matrix_up_half(double &m00, double &m01, double &m10,
                                                    double &m11)
{
#define RF_MAT_MUL                                                              \
    {                                                                           \
        const double n00 = m00 * o00 + m01 * o10;                               \
        const double n01 = m00 * o01 + m01 * o11;                               \
        const double n10 = m10 * o00 + m11 * o10;                               \
        const double n11 = m10 * o01 + m11 * o11;                               \
        m00 = n00; m01 = n01; m10 = n10; m11 = n11;                             \
        rescale4(m00, m01, m10, m11);                                           \
    }
#define RF_MAT_STEP(K)                                                          \
    {                                                                           \
        const double o00 = dpp1<kDppRowShr + (K)>(m00);                         \
        const double o01 = dpp0<kDppRowShr + (K)>(m01);                         \
        const double o10 = dpp0<kDppRowShr + (K)>(m10);                         \
        const double o11 = dpp1<kDppRowShr + (K)>(m11);                         \
        RF_MAT_MUL                                                              \
    }
    RF_MAT_STEP(1) RF_MAT_STEP(2) RF_MAT_STEP(4) RF_MAT_STEP(8)
    {
        const double o00 = dpp_rows<kDppRowBcast15, 0xA>(m00, 1.0);
        const double o01 = dpp_rows<kDppRowBcast15, 0xA>(m01, 0.0);
        const double o10 = dpp_rows<kDppRowBcast15, 0xA>(m10, 0.0);
        const double o11 = dpp_rows<kDppRowBcast15, 0xA>(m11, 1.0);
        RF_MAT_MUL
    }
#undef RF_MAT_STEP
#undef RF_MAT_MUL
}

}  // namespace rf
