// HIP kernels (gfx950 / CDNA4) of the column ensemble: many independent 1-D
// Richards columns, each advanced through its whole time loop by one
// wavefront in one persistent launch.
//
// A column of L <= 448 cells is held in registers for the whole run: lane l
// owns the P = ceil(L / 64) consecutive cells [l P, l P + P) (P is a compile-
// time constant of one of seven instantiations).  Every Picard iteration
// evaluates Eqs. 2-4 for its cells, assembles the column's tridiagonal
// system (Sec. 2.2: backward Euler, chord or modified Picard, arithmetic-mean
// face K, explicit gravity) and solves it exactly -- the LDL^T solve that
// DIC-PCG reaches in one iteration on a tridiagonal matrix -- as three
// blocked scans: each lane composes its P cells sequentially, the 64 lane
// summaries are combined by a shuffle scan, and each lane finishes its
// cells sequentially.  The pivots d_k = a_k - t_{k-1}^2 / d_{k-1} compose as
// 2x2 matrices (rescaled by powers of two), the two substitutions as affine
// maps.  HBM sees the state once at the start and once at the end of the run;
// the kernel is bound by FP64 arithmetic (five transcendentals per cell and
// iteration), not by memory.  Wavefronts take columns from a shared queue in
// order of decreasing length, so unequal columns balance themselves.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "rf_ens_internal.h"
#include "rf_soil.h"

namespace rf {
namespace {

constexpr int kEnsThreadsMax = 512;

// The value of lane 0, marked wave-uniform for the compiler (scalar
// registers, uniform branches).
__device__ __forceinline__ double uni(double x)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double ens_wave_max(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
    return uni(x);
}

__device__ __forceinline__ double ens_wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return uni(x);
}

// 2x2 matrix [[x00, x01], [x10, x11]] scaled by a power of two so that its
// largest entry lies in [0.5, 1): exact, and keeps long products finite.
template <typename T>
struct Mat2 {
    T x00, x01, x10, x11;
};

template <typename T>
__device__ __forceinline__ void rescale(Mat2<T> &m)
{
    const T s = fmax(fmax(fabs(m.x00), fabs(m.x01)), fmax(fabs(m.x10), fabs(m.x11)));
    if (s > T(0) && isfinite(s)) {
        int ex;
        (void)frexp(s, &ex);
        const T f = ldexp(T(1), -ex);
        m.x00 *= f;
        m.x01 *= f;
        m.x10 *= f;
        m.x11 *= f;
    }
}

// a * b (apply b first, then a)
template <typename T>
__device__ __forceinline__ Mat2<T> mmul(const Mat2<T> &a, const Mat2<T> &b)
{
    return Mat2<T>{a.x00 * b.x00 + a.x01 * b.x10, a.x00 * b.x01 + a.x01 * b.x11,
                   a.x10 * b.x00 + a.x11 * b.x10, a.x10 * b.x01 + a.x11 * b.x11};
}

template <typename T>
__device__ __forceinline__ Mat2<T> shfl_up_m(const Mat2<T> &m, int off)
{
    return Mat2<T>{__shfl_up(m.x00, off, kWave), __shfl_up(m.x01, off, kWave),
                   __shfl_up(m.x10, off, kWave), __shfl_up(m.x11, off, kWave)};
}

// Solves the symmetric tridiagonal system with diagonal dg and coupling
// -tu[k] between cells k and k+1 (tu = 0 above the top active cell; inactive
// cells are identity rows) for the right-hand side x, in place, over the
// blocked layout described at the top of the file.
template <int P, typename T>
__device__ __forceinline__ void tri_solve(const T (&dg)[P], const T (&tu)[P], T (&x)[P], int lane)
{
    // coupling of each cell with the one below it: tl(i)
    T tlb = __shfl_up(tu[P - 1], 1, kWave);
    if (lane == 0) tlb = T(0);
#define TL(i) ((i) > 0 ? tu[(i) > 0 ? (i) - 1 : 0] : tlb)
    // pivots: (p_k, q_k) = M_k (p_{k-1}, q_{k-1}), M_k = [[dg_k, -tl_k^2], [1, 0]],
    // d_k = p_k / q_k; the lane's product, then a scan over the lanes
    Mat2<T> m{T(1), T(0), T(0), T(1)};
#pragma unroll
    for (int i = 0; i < P; i++) {
        const T t2 = TL(i) * TL(i);
        m = Mat2<T>{dg[i] * m.x00 - t2 * m.x10, dg[i] * m.x01 - t2 * m.x11, m.x00, m.x01};
        rescale(m);
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const Mat2<T> o = shfl_up_m(m, off);
        if (lane >= off) {
            m = mmul(m, o);
            rescale(m);
        }
    }
    Mat2<T> y = shfl_up_m(m, 1);
    // 1 / d of the cell below the lane's first cell (0 below the column)
    T rdprev = (lane == 0) ? T(0) : y.x10 / y.x00;
    T rd[P];
#pragma unroll
    for (int i = 0; i < P; i++) {
        rd[i] = T(1) / (dg[i] - TL(i) * TL(i) * rdprev);
        rdprev = rd[i];
    }
    // forward substitution w_k = rd_k (x_k + tl_k w_{k-1}) as affine maps
    T A = T(1), C = T(0);
#pragma unroll
    for (int i = 0; i < P; i++) {
        const T ak = TL(i) * rd[i];
        C = ak * C + x[i] * rd[i];
        A = ak * A;
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const T ao = __shfl_up(A, off, kWave), co = __shfl_up(C, off, kWave);
        if (lane >= off) {
            C = A * co + C;
            A = A * ao;
        }
    }
    T wprev = __shfl_up(C, 1, kWave);
    if (lane == 0) wprev = T(0);
#pragma unroll
    for (int i = 0; i < P; i++) {
        x[i] = TL(i) * rd[i] * wprev + x[i] * rd[i];
        wprev = x[i];
    }
    // backward substitution e_k = w_k + (tu_k rd_k) e_{k+1}, from the top
    A = T(1);
    C = T(0);
#pragma unroll
    for (int i = P - 1; i >= 0; i--) {
        const T bk = tu[i] * rd[i];
        C = bk * C + x[i];
        A = bk * A;
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const T ao = __shfl_down(A, off, kWave), co = __shfl_down(C, off, kWave);
        if (lane + off < kWave) {
            C = A * co + C;
            A = A * ao;
        }
    }
    T enext = __shfl_down(C, 1, kWave);
    if (lane == kWave - 1) enext = T(0);
#pragma unroll
    for (int i = P - 1; i >= 0; i--) {
        x[i] = tu[i] * rd[i] * enext + x[i];
        enext = x[i];
    }
#undef TL
}

// Inflow [m^3/s per m^2] through the base (dir = 0) or the top (dir = 1) of a
// column whose end cell has head h and conductivity K (Sec. 3.1, App. A).
__device__ __forceinline__ double ens_inflow(const EnsOpt &o, int dir, double Kb, double h, double K)
{
    const double gn = dir ? 1.0 : -1.0;
    switch (o.bc_type[dir]) {
    case RF_DIRICHLET: return Kb / (0.5 * o.dz) * (o.bc_value[dir] - h) + Kb * gn;
    case RF_FLUX: return o.bc_value[dir];
    case RF_FREE_DRAINAGE: return K * gn;
    default: return 0.0;
    }
}

// The whole time loop of column c (P cells per lane, solve in precision TS).
template <int P, typename TS>
__device__ void run_column(const EnsArrays &a, const EnsOpt &o, const EnsRunParams &rp,
                           long long t0, int c, int lane)
{
    rf_ens_column st = a.col[c];
    if (st.status != RF_OK) return;   // a failed column keeps its last accepted state
    const int L = a.len[c];
    const size_t off = (size_t)a.off[c];
    const EnsSoil sp = a.soil[c];
    const int k0 = lane * P;
    const double dz = o.dz, rdz = 1.0 / o.dz;
    bool act[P];
    double hn[P], thn[P];
#pragma unroll
    for (int i = 0; i < P; i++) {
        act[i] = k0 + i < L;
        hn[i] = act[i] ? a.h[off + k0 + i] : 0.0;
        thn[i] = act[i] ? soil_theta(o.model, hn[i], sp.L) : 0.0;
    }
    const double Kb0 = (o.bc_type[0] == RF_DIRICHLET) ? soil_K(o.model, o.bc_value[0], sp.L, sp.ks) : 0.0;
    const double Kb1 = (o.bc_type[1] == RF_DIRICHLET) ? soil_K(o.model, o.bc_value[1], sp.L, sp.ks) : 0.0;
    const int top_lane = (L - 1) / P, top_i = (L - 1) % P;
    double t = st.t, dt_cur = st.dt_next;
    int easy = st.easy;
    long long steps = 0;
    while (t < rp.t_end * (1.0 - 1e-15) - 1e-12) {
        if (steps >= rp.max_steps || wall_clock64() - t0 > rp.max_ticks) break;
        steps++;
        double dt = o.ebats ? dt_cur : o.dt0;
        bool clipped = false;
        if (t + dt > rp.t_end) {
            dt = rp.t_end - t;
            clipped = true;
        }
        const int maxp = o.ebats ? o.max_iters : o.max_picard;
        const double vdt = dz / dt;
        double hm[P];
#pragma unroll
        for (int i = 0; i < P; i++) hm[i] = hn[i];
        int status = RF_ERR_NOT_CONVERGED, its = 0;
        double Kbot = 0.0, Ktop = 0.0;   // K^m of the end cells (free-drainage inflow)
        for (int m = 0; m < maxp; m++) {
            its++;
            TS dgs[P], tus[P], xs[P];
            {
                // coefficients at h^m: K, storage diagonal and right-hand side
                double K[P], D[P], bs[P];
#pragma unroll
                for (int i = 0; i < P; i++) {
                    double th = 0.0, Cp = 0.0, Ki = 0.0;
                    if (act[i]) soil_eval(o.model, hm[i], sp.L, sp.ks, th, Cp, Ki);
                    K[i] = Ki;
                    if (o.variant == RF_PICARD_MODIFIED) {
                        D[i] = vdt * Cp;
                        bs[i] = vdt * (Cp * hm[i] - (th - thn[i]));
                    } else {
                        const double dh = hm[i] - hn[i];
                        const double Cc = (fabs(dh) >= o.chord_eps) ? (th - thn[i]) / dh : Cp;
                        D[i] = vdt * Cc;
                        bs[i] = D[i] * hn[i];
                    }
                }
                Kbot = K[0];
#pragma unroll
                for (int i = 0; i < P; i++)
                    if (i == top_i) Ktop = K[i];
                // face with the cell above: K_f (face area 1 m^2, distance dz)
                double kfu[P];
                {
                    const double Kn = __shfl_down(K[0], 1, kWave);
#pragma unroll
                    for (int i = 0; i < P; i++) {
                        const double Ka = (i + 1 < P) ? K[i + 1] : Kn;
                        kfu[i] = (k0 + i + 1 < L) ? 0.5 * (K[i] + Ka) : 0.0;
                    }
                }
                // rows: diagonal, right-hand side with explicit gravity, and
                // the residual b - A h^m
                const double kfb = __shfl_up(kfu[P - 1], 1, kWave);
                const double hb = __shfl_up(hm[P - 1], 1, kWave), ha = __shfl_down(hm[0], 1, kWave);
#pragma unroll
                for (int i = 0; i < P; i++) {
                    const double kfd = (i > 0) ? kfu[i - 1] : (lane == 0 ? 0.0 : kfb);
                    const double tu = kfu[i] * rdz, td = kfd * rdz;
                    const double hup = (i + 1 < P) ? hm[i + 1] : ha;
                    const double hdn = (i > 0) ? hm[i - 1] : hb;
                    double dg = D[i] + tu + td;
                    double b = bs[i] + kfu[i] - kfd;
                    const int k = k0 + i;
                    if (k == 0) {
                        if (o.bc_type[0] == RF_DIRICHLET) {
                            const double T = Kb0 / (0.5 * dz);
                            dg += T;
                            b += T * o.bc_value[0] - Kb0;
                        } else if (o.bc_type[0] == RF_FLUX) {
                            b += o.bc_value[0];
                        } else if (o.bc_type[0] == RF_FREE_DRAINAGE) {
                            b -= K[i];
                        }
                    }
                    if (k == L - 1) {
                        if (o.bc_type[1] == RF_DIRICHLET) {
                            const double T = Kb1 / (0.5 * dz);
                            dg += T;
                            b += T * o.bc_value[1] + Kb1;
                        } else if (o.bc_type[1] == RF_FLUX) {
                            b += o.bc_value[1];
                        } else if (o.bc_type[1] == RF_FREE_DRAINAGE) {
                            b += K[i];
                        }
                    }
                    const double r = b - (dg * hm[i] - tu * hup - td * hdn);
                    dgs[i] = act[i] ? (TS)dg : TS(1);
                    tus[i] = act[i] ? (TS)tu : TS(0);
                    xs[i] = act[i] ? (TS)r : TS(0);
                }
            }
            tri_solve<P, TS>(dgs, tus, xs, lane);
            double dmax = 0.0;
            bool finite = true;
#pragma unroll
            for (int i = 0; i < P; i++) {
                if (!act[i]) continue;
                const double e = (double)xs[i];
                hm[i] += e;
                dmax = fmax(dmax, fabs(e));
                finite = finite && isfinite(hm[i]);
            }
            const double delta = ens_wave_max(finite ? dmax : INFINITY);
            if (!(delta == delta) || isinf(delta)) {
                status = RF_ERR_NONFINITE;
                break;
            }
            if (delta < o.tol_picard) {
                status = RF_OK;
                break;
            }
        }
        st.picard_total += its;
        if (status == RF_OK) {
            // inflows with the converged h and the conductivity of the last assembly
            const double qb = uni(ens_inflow(o, 0, Kb0, hm[0], Kbot));
            double qt_l = 0.0;
#pragma unroll
            for (int i = 0; i < P; i++)
                if (i == top_i) qt_l = ens_inflow(o, 1, Kb1, hm[i], Ktop);
            const double qt = uni(__shfl(qt_l, top_lane, kWave));
            st.inflow_bottom += dt * qb;
            st.inflow_top += dt * qt;
#pragma unroll
            for (int i = 0; i < P; i++) {
                hn[i] = hm[i];
                thn[i] = act[i] ? soil_theta(o.model, hn[i], sp.L) : 0.0;
            }
            t += dt;
            st.accepted++;
            if (o.ebats) {
                if (!clipped) dt_cur = dt;
                if (its <= o.few_iters) {
                    if (++easy >= o.inc_after) {
                        dt_cur = fmin(dt_cur * o.factor, o.dt_max);
                        easy = 0;
                    }
                } else {
                    easy = 0;
                }
            }
        } else {
            st.rejected++;
            if (!o.ebats) {
                st.status = status;
                break;
            }
            dt_cur = dt / o.factor;
            easy = 0;
            if (dt_cur < o.dt_min) {
                st.status = RF_ERR_NOT_CONVERGED;
                break;
            }
        }
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < P; i++) {
        if (!act[i]) continue;
        a.h[off + k0 + i] = hn[i];
        s += dz * thn[i];
    }
    st.storage = ens_wave_sum(s);
    st.t = t;
    st.dt_next = o.ebats ? dt_cur : o.dt0;
    st.easy = easy;
    if (lane == 0) a.col[c] = st;
}

template <typename TS>
__global__ void __launch_bounds__(kEnsThreadsMax) k_ens_run(EnsArrays a, int ncol, EnsOpt o,
                                                            EnsRunParams rp)
{
    const int lane = threadIdx.x & (kWave - 1);
    // the run's wall-clock budget counts from this wavefront's start (the
    // persistent grid is sized to be resident at once)
    const long long t0 = wall_clock64();
    for (;;) {
        unsigned int q = 0;
        if (lane == 0) q = atomicAdd(a.queue, 1u);
        q = (unsigned int)__builtin_amdgcn_readfirstlane((int)q);
        if (q >= (unsigned int)ncol) break;
        const int c = a.order[q];
        const int P = (a.len[c] + kWave - 1) / kWave;
        switch (P) {
        case 1: run_column<1, TS>(a, o, rp, t0, c, lane); break;
        case 2: run_column<2, TS>(a, o, rp, t0, c, lane); break;
        case 3: run_column<3, TS>(a, o, rp, t0, c, lane); break;
        case 4: run_column<4, TS>(a, o, rp, t0, c, lane); break;
        case 5: run_column<5, TS>(a, o, rp, t0, c, lane); break;
        case 6: run_column<6, TS>(a, o, rp, t0, c, lane); break;
        default: run_column<7, TS>(a, o, rp, t0, c, lane); break;
        }
    }
}

// Per column (one wavefront each): the record at the start of a run of the
// state now in a.h: storage0 = storage = sum dz theta~, counters cleared.
__global__ void __launch_bounds__(256) k_ens_init(EnsArrays a, int ncol, EnsOpt o, double t)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int c = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (c >= ncol) return;
    const int L = a.len[c];
    const size_t off = (size_t)a.off[c];
    const EnsSoil sp = a.soil[c];
    double s = 0.0;
    for (int k = lane; k < L; k += kWave) s += o.dz * soil_theta(o.model, a.h[off + k], sp.L);
    s = ens_wave_sum(s);
    if (lane == 0) {
        rf_ens_column r;
        r.status = RF_OK;
        r.accepted = 0;
        r.rejected = 0;
        r.easy = 0;
        r.picard_total = 0;
        r.t = t;
        r.dt_next = o.dt0;
        r.storage0 = s;
        r.storage = s;
        r.inflow_top = 0.0;
        r.inflow_bottom = 0.0;
        a.col[c] = r;
    }
}

// Count of non-finite values in the packed state (one block).
__global__ void __launch_bounds__(1024) k_ens_check(EnsArrays a, long ncell)
{
    __shared__ unsigned int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    unsigned int mine = 0;
    for (long i = threadIdx.x; i < ncell; i += blockDim.x) mine += isfinite(a.h[i]) ? 0u : 1u;
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) a.queue[0] = cnt;
}

// Start of a run: queue position 0.
__global__ void k_ens_reset(EnsArrays a)
{
    if (threadIdx.x == 0) a.queue[0] = 0u;
}

// Totals over the column records (one block of 256 threads).
__global__ void __launch_bounds__(256) k_ens_summary(EnsArrays a, int ncol)
{
    __shared__ long long s_acc[256], s_rej[256], s_pic[256], s_cs[256];
    __shared__ int s_fail[256];
    __shared__ double s_tmin[256], s_err[256];
    long long acc = 0, rej = 0, pic = 0, cs = 0;
    int fail = 0;
    double tmin = INFINITY, err = 0.0;
    for (int c = threadIdx.x; c < ncol; c += 256) {
        const rf_ens_column r = a.col[c];
        acc += r.accepted;
        rej += r.rejected;
        pic += r.picard_total;
        cs += (long long)r.accepted * a.len[c];
        fail += (r.status != RF_OK);
        tmin = fmin(tmin, r.t);
        err = fmax(err, fabs(r.storage - r.storage0 - r.inflow_top - r.inflow_bottom));
    }
    const int i = threadIdx.x;
    s_acc[i] = acc;
    s_rej[i] = rej;
    s_pic[i] = pic;
    s_cs[i] = cs;
    s_fail[i] = fail;
    s_tmin[i] = tmin;
    s_err[i] = err;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (i < w) {
            s_acc[i] += s_acc[i + w];
            s_rej[i] += s_rej[i + w];
            s_pic[i] += s_pic[i + w];
            s_cs[i] += s_cs[i + w];
            s_fail[i] += s_fail[i + w];
            s_tmin[i] = fmin(s_tmin[i], s_tmin[i + w]);
            s_err[i] = fmax(s_err[i], s_err[i + w]);
        }
        __syncthreads();
    }
    if (i == 0) {
        rf_ens_summary r;
        r.accepted = s_acc[0];
        r.rejected = s_rej[0];
        r.picard_total = s_pic[0];
        r.cell_steps = s_cs[0];
        r.failed = s_fail[0];
        r.t_min = s_tmin[0];
        r.max_balance_error = s_err[0];
        r.kernel_ms = 0.0;
        a.sum[0] = r;
    }
}

}  // namespace

hipError_t launch_ens_init(const EnsArrays &a, int ncol, const EnsOpt &o, double t, hipStream_t s)
{
    const int per = 256 / kWave;
    hipLaunchKernelGGL(k_ens_init, dim3((ncol + per - 1) / per), dim3(256), 0, s, a, ncol, o, t);
    return hipGetLastError();
}

hipError_t launch_ens_check(const EnsArrays &a, long ncell, hipStream_t s)
{
    hipLaunchKernelGGL(k_ens_check, dim3(1), dim3(1024), 0, s, a, ncell);
    return hipGetLastError();
}

hipError_t launch_ens_reset(const EnsArrays &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ens_reset, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ens_run(const EnsArrays &a, int ncol, const EnsOpt &o, const EnsRunParams &rp,
                          bool mixed, int nblocks, int waves_per_block, hipStream_t s)
{
    if (waves_per_block < 1 || waves_per_block * kWave > kEnsThreadsMax || nblocks < 1)
        return hipErrorInvalidValue;
    const dim3 grid(nblocks), block(waves_per_block * kWave);
    if (mixed)
        hipLaunchKernelGGL(k_ens_run<float>, grid, block, 0, s, a, ncol, o, rp);
    else
        hipLaunchKernelGGL(k_ens_run<double>, grid, block, 0, s, a, ncol, o, rp);
    return hipGetLastError();
}

hipError_t launch_ens_summary(const EnsArrays &a, int ncol, hipStream_t s)
{
    hipLaunchKernelGGL(k_ens_summary, dim3(1), dim3(256), 0, s, a, ncol);
    return hipGetLastError();
}

int ens_max_blocks_per_cu(bool mixed, int waves_per_block)
{
    int n = 0;
    const int threads = waves_per_block * kWave;
    hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ens_run<float>, threads, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ens_run<double>, threads, 0);
    return (e == hipSuccess) ? n : 0;
}

}  // namespace rf
