// HIP kernels (gfx950 / CDNA4) of the Richards-equation Picard / PCG loop.
//
// Work decomposition: one wavefront owns one z-column at a time; lane k of
// the wave holds cell k of the column (columns longer than 64 cells are
// walked in chunks of 64).  With z the fastest index every column is one
// contiguous run of doubles, so each chunk is a single coalesced 512-byte
// access per array, the vertical coupling stays inside the wave (shuffles),
// and the lateral neighbours are the adjacent columns.  Blocks of 4 waves
// take contiguous runs of columns; the block -> columns map is XCD-aware
// (the hardware deals workgroups round-robin over the 8 XCDs, so logical
// block (b % 8) * (G / 8) + b / 8 gives each XCD one contiguous slab of the
// grid and keeps lateral reuse inside one L2).
//
// Global reductions are two-stage, deterministic and fence-free: every block
// writes one partial per value, and the consumer -- every block of the next
// kernel, or the host -- combines the (at most 512) partials in block order.
// Cross-block visibility therefore only ever relies on kernel boundaries: an
// agent-scope fence per block would write back the whole L2 of its XCD, and a
// single ticket counter would serialise every block of the grid.  Scalars
// such as alpha and beta never leave the device during the PCG loop.
#include <hip/hip_runtime.h>
#include <math.h>

#include "rf_internal.h"

namespace rf {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void block_columns(const Geo &g, int &cb, int &ce)
{
    const int b = blockIdx.x, G = gridDim.x;
    const int lb = (G >= 8 && (G & 7) == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
    cb = lb * g.cpb;
    ce = min(cb + g.cpb, g.ncol);
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
    return x;
}

// Block-level reduction of NV values (bit i of MAXMASK set = max, else sum)
// in a fixed order; thread 0 stores the block's partials at out[b*NV + i].
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void block_partial(double (&v)[NV], double *out)
{
    __shared__ double sh[kWavesPerBlock][NV];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < NV; i++) v[i] = ((MAXMASK >> i) & 1u) ? wave_max(v[i]) : wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; i++) sh[w][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; i++) {
            double a = sh[0][i];
            for (int ww = 1; ww < kWavesPerBlock; ww++)
                a = ((MAXMASK >> i) & 1u) ? fmax(a, sh[ww][i]) : a + sh[ww][i];
            out[(size_t)blockIdx.x * NV + i] = a;
        }
    }
}

// Combines the nblk block partials written by the previous kernel, in the
// same fixed order in every block; all threads receive the totals.
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void reduce_partials(const double *P, int nblk, double (&tot)[NV])
{
    __shared__ double sh[kWavesPerBlock][NV];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; i++) v[i] = 0.0;   // identity of sums and of max over |x|
    for (int b = threadIdx.x; b < nblk; b += kThreads)
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const double x = P[(size_t)b * NV + i];
            v[i] = ((MAXMASK >> i) & 1u) ? fmax(v[i], x) : v[i] + x;
        }
#pragma unroll
    for (int i = 0; i < NV; i++) v[i] = ((MAXMASK >> i) & 1u) ? wave_max(v[i]) : wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; i++) sh[w][i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; i++) {
        double a = sh[0][i];
        for (int ww = 1; ww < kWavesPerBlock; ww++)
            a = ((MAXMASK >> i) & 1u) ? fmax(a, sh[ww][i]) : a + sh[ww][i];
        tot[i] = a;
    }
}

__device__ __forceinline__ bool lead_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }

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

// Cell neighbourhood inside a column chunk.  Direction d: 0 -x, 1 +x, 2 -y,
// 3 +y, 4 -z, 5 +z.  nb[d]: neighbour active; bnd[d]: the face is on the
// domain boundary (the +z boundary is the top of the column's active run).
struct Cell {
    size_t idx;
    size_t off[6];
    bool nb[6];
    bool bnd[6];
};

__device__ __forceinline__ void cell_setup(const Geo &g, const int32_t *ktop, int col, int kt,
                                           int k, Cell &c)
{
    const int i = col % g.nx, j = col / g.nx;
    c.idx = (size_t)col * g.nz + k;
    const size_t sx = (size_t)g.nz, sy = (size_t)g.nz * g.nx;
    c.off[0] = c.idx - sx; c.off[1] = c.idx + sx;
    c.off[2] = c.idx - sy; c.off[3] = c.idx + sy;
    c.off[4] = c.idx - 1;  c.off[5] = c.idx + 1;
    c.bnd[0] = (i == 0);          c.nb[0] = !c.bnd[0] && k < ktop[col - 1];
    c.bnd[1] = (i == g.nx - 1);   c.nb[1] = !c.bnd[1] && k < ktop[col + 1];
    c.bnd[2] = (j == 0);          c.nb[2] = !c.bnd[2] && k < ktop[col - g.nx];
    c.bnd[3] = (j == g.ny - 1);   c.nb[3] = !c.bnd[3] && k < ktop[col + g.nx];
    c.bnd[4] = (k == 0);          c.nb[4] = !c.bnd[4];
    c.bnd[5] = (k == kt - 1);     c.nb[5] = !c.bnd[5];
}

__device__ __forceinline__ double gdot(const Geo &g, int d)
{
    const double s = (d & 1) ? 1.0 : -1.0;
    return s * g.g[d >> 1];
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------

// Ks per cell = Ks(layer) * exp(ln_ks_offset); Ks holds the offsets on entry
// (zeros when none were given).
__global__ void __launch_bounds__(kThreads) k_init_ks(Geo g, Soil so, Arrays a, const double *ks_layer)
{
    const size_t N = (size_t)g.ncol * g.nz;
    for (size_t c = (size_t)blockIdx.x * kThreads + threadIdx.x; c < N;
         c += (size_t)gridDim.x * kThreads) {
        const int l = a.layer ? a.layer[c] : 0;
        a.Ks[c] = ks_layer[l] * exp(a.Ks[c]);
    }
}

// Counts non-finite active values of h (sums[0]).
__global__ void __launch_bounds__(kThreads) k_check_finite(Geo g, Arrays a, const double *h)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[1] = {0.0};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k < kt && !isfinite(h[(size_t)col * g.nz + k])) v[0] += 1.0;
        }
    }
    block_partial<1, 0u>(v, a.ps);
}

// h^n <- h, theta~^n <- theta~(h), storage (sums[0]).
__global__ void __launch_bounds__(kThreads) k_set_state(Geo g, Soil so, Arrays a, const double *h)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[1] = {0.0};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < g.nz; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= g.nz) continue;
            const size_t idx = (size_t)col * g.nz + k;
            const double hv = h[idx];
            a.hn[idx] = hv;
            if (k < kt) {
                const Layer &L = so.L[a.layer ? a.layer[idx] : 0];
                const double th = soil_theta(so.model, hv, L);
                a.thn[idx] = th;
                v[0] += g.V * th;
            }
        }
    }
    block_partial<1, 0u>(v, a.ps);
}

// ---------------------------------------------------------------------------
// Picard iteration: coefficients (row a1 of the loop) and boundary terms
// ---------------------------------------------------------------------------

// Per active cell: K = K(h^m); chord capacity C = (theta~(h^m) -
// theta~(h^n)) / (h^m - h^n), or Eq. 3 when |h^m - h^n| < chord_eps;
// Dd = V C / dt + sum of Dirichlet transmissibilities; bst = V C h^n / dt +
// every boundary term of the cell (Dirichlet T h_b + A K(h_b) g.n, flux A q,
// free drainage A K(h^m) g.n).  Interior-face terms are added in k_resid.
__global__ void __launch_bounds__(kThreads) k_coeff(Geo g, Soil so, Bc bc, Arrays a, double dt,
                                                    double chord_eps)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const double dist[3] = {g.A[0] / g.Tk[0], g.A[1] / g.Tk[1], g.A[2] / g.Tk[2]};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            Cell c;
            cell_setup(g, a.ktop, col, kt, k, c);
            const size_t idx = c.idx;
            const Layer &L = so.L[a.layer ? a.layer[idx] : 0];
            const double ks = a.Ks[idx];
            const double hm = a.hm[idx], hn = a.hn[idx];
            double th, C, K;
            soil_eval(so.model, hm, L, ks, th, C, K);
            const double dh = hm - hn;
            const double Cc = (fabs(dh) >= chord_eps) ? (th - a.thn[idx]) / dh : C;
            double D = g.V * Cc / dt;
            double b = D * hn;
#pragma unroll
            for (int d = 0; d < 6; d++) {
                if (!c.bnd[d]) continue;
                const int f = d;                  // direction d crosses face d
                const int ax = d >> 1;
                const double gn = gdot(g, d);
                const int type = bc.type[f];
                if (type == RF_DIRICHLET) {
                    const double hb = bc.value[f];
                    const double Kb = soil_K(so.model, hb, L, ks);
                    const double T = g.A[ax] * Kb / (0.5 * dist[ax]);
                    D += T;
                    b += T * hb + g.A[ax] * Kb * gn;
                } else if (type == RF_FLUX) {
                    b += g.A[ax] * bc.value[f];
                } else if (type == RF_FREE_DRAINAGE) {
                    b += g.A[ax] * K * gn;
                }
            }
            a.K[idx] = K;
            a.Dd[idx] = D;
            a.bst[idx] = b;
        }
    }
}

// ---------------------------------------------------------------------------
// z-line preconditioner pieces (exact LDL^T of each column's vertical part)
// ---------------------------------------------------------------------------

// Inclusive upward scan of affine maps x_k = a_k x_{k-1} + c_k over the
// wave; returns x_k for the given carry x_{k0-1}.
__device__ __forceinline__ double scan_affine_up(double a, double c, double carry, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double ao = __shfl_up(a, off, kWave);
        const double co = __shfl_up(c, off, kWave);
        if (lane >= off) {
            c = a * co + c;
            a = a * ao;
        }
    }
    return a * carry + c;
}

// Inclusive downward scan of x_k = b_k x_{k+1} + c_k.
__device__ __forceinline__ double scan_affine_down(double b, double c, double carry, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double bo = __shfl_down(b, off, kWave);
        const double co = __shfl_down(c, off, kWave);
        if (lane + off < kWave) {
            c = b * co + c;
            b = b * bo;
        }
    }
    return b * carry + c;
}

// Pivots of the column tridiagonal T: d_k = diag_k - t_{k-1}^2 / d_{k-1}.
// With P_k = diag_k P_{k-1} - t_{k-1}^2 P_{k-2} (leading minors), d_k =
// P_k / P_{k-1}; (P_k, P_{k-1}) is a prefix product of 2x2 matrices, scanned
// across the wave with a per-step rescaling (only ratios matter).  carry =
// d_{k0-1} (0 for the first chunk).  Returns d_k.
__device__ __forceinline__ double scan_pivots(double diag, double tprev2, double carry, int lane)
{
    // M = [[m00, m01], [m10, m11]] = [[diag, -tprev2], [1, 0]]
    double m00 = diag, m01 = -tprev2, m10 = 1.0, m11 = 0.0;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double o00 = __shfl_up(m00, off, kWave);
        const double o01 = __shfl_up(m01, off, kWave);
        const double o10 = __shfl_up(m10, off, kWave);
        const double o11 = __shfl_up(m11, off, kWave);
        if (lane >= off) {
            const double n00 = m00 * o00 + m01 * o10;
            const double n01 = m00 * o01 + m01 * o11;
            const double n10 = m10 * o00 + m11 * o10;
            const double n11 = m10 * o01 + m11 * o11;
            const double s = fmax(fmax(fabs(n00), fabs(n01)), fmax(fabs(n10), fabs(n11)));
            const double rs = (s > 0.0) ? 1.0 / s : 1.0;
            m00 = n00 * rs; m01 = n01 * rs; m10 = n10 * rs; m11 = n11 * rs;
        }
    }
    // start vector (P_{k0-1}, P_{k0-2}) ~ (carry, 1), or (1, 0) on the first chunk
    const double v0 = (carry != 0.0) ? carry : 1.0;
    const double v1 = (carry != 0.0) ? 1.0 : 0.0;
    return (m00 * v0 + m01 * v1) / (m10 * v0 + m11 * v1);
}

// z = M^-1 r for one column with reciprocal pivots rdp and couplings t
// (t_k couples k and k+1, zero at the top active cell).  Columns of up to 64
// cells stay in registers; longer columns keep the forward sweep in z.
template <bool ONE_CHUNK>
__device__ __forceinline__ void zline_solve_column(const double *r, const double *rdp,
                                                   const double *tz, double *zout, size_t base,
                                                   int kt, int lane, double &z_reg)
{
    // forward: w_k = (r_k + t_{k-1} w_{k-1}) rdp_k
    double carry = 0.0, wlast = 0.0;
    for (int k0 = 0; k0 < kt; k0 += kWave) {
        const int k = k0 + lane;
        const bool act = k < kt;
        const double rk = act ? r[base + k] : 0.0;
        const double rd = act ? rdp[base + k] : 0.0;
        const double tp = (act && k > 0) ? tz[base + k - 1] : 0.0;
        const double wk = scan_affine_up(tp * rd, rk * rd, carry, lane);
        carry = __shfl(wk, kWave - 1, kWave);
        if (ONE_CHUNK) wlast = wk;
        else if (act) zout[base + k] = wk;
    }
    // backward: z_k = w_k + t_k rdp_k z_{k+1}
    carry = 0.0;
    const int nch = (kt + kWave - 1) / kWave;
    for (int ch = nch - 1; ch >= 0; ch--) {
        const int k = ch * kWave + lane;
        const bool act = k < kt;
        const double wk = ONE_CHUNK ? wlast : (act ? zout[base + k] : 0.0);
        const double bk = (act && k + 1 < kt) ? tz[base + k] * rdp[base + k] : 0.0;
        const double zk = scan_affine_down(bk, act ? wk : 0.0, carry, lane);
        carry = __shfl(zk, 0, kWave);
        if (act) zout[base + k] = zk;
        if (ONE_CHUNK) z_reg = zk;
    }
}

// ---------------------------------------------------------------------------
// Residual of the Picard system and PCG start (rows a2, a3, a5)
// ---------------------------------------------------------------------------

// Adds the interior faces: diag = Dd + sum T_f, b = bst + sum A_f K_f g.n_f
// with K_f = (K_P + K_N)/2 and T_f = A_f K_f / d_f; r = b - A h^m (the
// right-hand side of the increment system A e = r, e0 = 0); e = 0.
// Jacobi: z = r / diag.  z-line: t_k (vertical couplings) and reciprocal
// pivots of each column, z = M^-1 r.  Reduces rho = r.z and max|r/diag|.
template <int PRECOND>
__global__ void __launch_bounds__(kThreads) k_resid(Geo g, Arrays a, double *bout)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[2] = {0.0, 0.0};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        const size_t base = (size_t)col * g.nz;
        // carries between chunks of a long column (z-line only)
        double t_carry = 0.0, d_carry = 0.0, w_carry = 0.0;
        double r = 0.0, tup = 0.0, rdp = 0.0, wk = 0.0;
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            const bool act = k < kt;
            double diag = 1.0;
            r = 0.0;
            tup = 0.0;
            if (act) {
                Cell c;
                cell_setup(g, a.ktop, col, kt, k, c);
                const double Kp = a.K[c.idx], hp = a.hm[c.idx];
                diag = a.Dd[c.idx];
                double Ap = diag * hp, b = a.bst[c.idx];
#pragma unroll
                for (int d = 0; d < 6; d++) {
                    if (!c.nb[d]) continue;
                    const double Kf = 0.5 * (Kp + a.K[c.off[d]]);
                    const double T = g.Tk[d >> 1] * Kf;
                    diag += T;
                    Ap += T * (hp - a.hm[c.off[d]]);
                    b += g.A[d >> 1] * Kf * gdot(g, d);
                    if (d == 5) tup = T;
                }
                r = b - Ap;
                if (bout) bout[c.idx] = b;
                a.r[c.idx] = r;
                a.e[c.idx] = 0.0;
                a.diag[c.idx] = diag;
                v[1] = fmax(v[1], fabs(r / diag));
                if (PRECOND == RF_PRECOND_JACOBI) v[0] += r * (r / diag);
            }
            if (PRECOND == RF_PRECOND_ZLINE) {
                // couplings and pivots of the column tridiagonal, in registers
                double tprev = __shfl_up(tup, 1, kWave);
                if (lane == 0) tprev = t_carry;
                const double dpiv = scan_pivots(act ? diag : 1.0, act ? tprev * tprev : 0.0,
                                                d_carry, lane);
                rdp = act ? 1.0 / dpiv : 0.0;
                wk = scan_affine_up(tprev * rdp, r * rdp, w_carry, lane);
                t_carry = __shfl(tup, kWave - 1, kWave);
                d_carry = __shfl(dpiv, kWave - 1, kWave);
                w_carry = __shfl(wk, kWave - 1, kWave);
                if (act) {
                    a.tz[base + k] = tup;
                    a.rdp[base + k] = rdp;
                    if (kt > kWave) a.z[base + k] = wk;   // forward sweep, re-read by this lane
                }
            }
        }
        if (PRECOND == RF_PRECOND_ZLINE && kt > 0) {
            // backward sweep z_k = w_k + t_k rdp_k z_{k+1}
            if (kt <= kWave) {
                const bool act = lane < kt;
                const double zk = scan_affine_down(act ? tup * rdp : 0.0, act ? wk : 0.0, 0.0, lane);
                if (act) {
                    a.z[base + lane] = zk;
                    v[0] += r * zk;
                }
            } else {
                double carry = 0.0;
                for (int ch = (kt - 1) / kWave; ch >= 0; ch--) {
                    const int k = ch * kWave + lane;
                    const bool act = k < kt;
                    const double wv = act ? a.z[base + k] : 0.0;
                    const double bk = act ? a.tz[base + k] * a.rdp[base + k] : 0.0;
                    const double zk = scan_affine_down(bk, wv, carry, lane);
                    carry = __shfl(zk, 0, kWave);
                    if (act) {
                        a.z[base + k] = zk;
                        v[0] += a.r[base + k] * zk;
                    }
                }
            }
        }
    }
    block_partial<2, 2u>(v, a.pr);
    if (lead_thread()) {
        Scalars *s = a.sc;
        s->rho[0] = 0.0;
        s->rho[1] = 1.0;     // beta of the first direction multiplies nothing
        s->resmax = 0.0;
        s->pq = 0.0;
        s->iters = 0;
        s->jcur = 0;
        s->done = 0;
        s->fail = 0;
        s->applied = 0;
        s->final_iters = 0;
    }
}

// ---------------------------------------------------------------------------
// PCG iteration (row a4): kernel A = direction update + SpMV + p.q
// ---------------------------------------------------------------------------

template <int PRECOND>
__device__ __forceinline__ double pnew_at(const Arrays &a, size_t i, double beta, bool first,
                                          const double *p_in)
{
    const double z = (PRECOND == RF_PRECOND_JACOBI) ? a.r[i] / a.diag[i] : a.z[i];
    return first ? z : z + beta * p_in[i];
}

// Starts PCG iteration j = (updates done so far).  Every block combines the
// (r.z, max|r/diag|) partials of the last update and takes the same exit
// decision; otherwise p = z + beta p_old (z = M^-1 r) at the cell and its
// neighbours, q = A p with A = Dd + sum_f T_f (I - shift_f) rebuilt from
// (K, Dd); writes p, q and the block partials of p.q.
template <int PRECOND>
__global__ void __launch_bounds__(kThreads) k_spmv(Geo g, Arrays a, const double *p_in, double *p_out,
                                                   double tol_cg, int max_cg)
{
    Scalars *s = a.sc;
    if (s->done) return;
    const int j = s->iters;
    double tot[2];
    reduce_partials<2, 2u>(a.pr, gridDim.x, tot);
    const double rho = tot[0], resmax = tot[1];
    const bool bad = !isfinite(rho) || !isfinite(resmax);
    const bool done = bad || resmax <= tol_cg || j >= max_cg;
    if (lead_thread()) {
        s->rho[j & 1] = rho;
        s->resmax = resmax;
        s->jcur = j;
        if (done) {
            s->done = 1;
            s->final_iters = j;
            if (bad) s->fail = 3;
            else if (resmax > tol_cg) s->fail = 2;
        }
    }
    if (done) return;
    const bool first = (j == 0);
    const double beta = first ? 0.0 : rho / s->rho[(j + 1) & 1];
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[1] = {0.0};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            Cell c;
            cell_setup(g, a.ktop, col, kt, k, c);
            const double Kp = a.K[c.idx];
            const double pp = pnew_at<PRECOND>(a, c.idx, beta, first, p_in);
            double q = a.Dd[c.idx] * pp;
#pragma unroll
            for (int d = 0; d < 6; d++) {
                if (!c.nb[d]) continue;
                const double T = g.Tk[d >> 1] * 0.5 * (Kp + a.K[c.off[d]]);
                q += T * (pp - pnew_at<PRECOND>(a, c.off[d], beta, first, p_in));
            }
            p_out[c.idx] = pp;
            a.q[c.idx] = q;
            v[0] += pp * q;
        }
    }
    block_partial<1, 0u>(v, a.pq);
}

// ---------------------------------------------------------------------------
// PCG iteration: kernel B = e += alpha p, r -= alpha q, z = M^-1 r, r.z
// ---------------------------------------------------------------------------

// alpha = rho_j / p.q (every block combines the p.q partials); e += alpha p,
// r -= alpha q, z = M^-1 r; block partials of (r.z, max|r/diag|).
template <int PRECOND>
__global__ void __launch_bounds__(kThreads) k_update(Geo g, Arrays a, const double *p)
{
    Scalars *s = a.sc;
    if (s->done) return;
    const int j = s->jcur;
    double tot[1];
    reduce_partials<1, 0u>(a.pq, gridDim.x, tot);
    const double pq = tot[0];
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (lead_thread()) {
            s->pq = pq;
            s->fail = 1;
            s->done = 1;
            s->final_iters = j;
        }
        return;
    }
    const double alpha = s->rho[j & 1] / pq;
    if (lead_thread()) {
        s->pq = pq;
        s->iters = j + 1;
    }
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[2] = {0.0, 0.0};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        const size_t base = (size_t)col * g.nz;
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            const size_t i = base + k;
            a.e[i] += alpha * p[i];
            const double r = a.r[i] - alpha * a.q[i];
            a.r[i] = r;
            const double dg = a.diag[i];
            if (PRECOND == RF_PRECOND_JACOBI) v[0] += r * (r / dg);
            v[1] = fmax(v[1], fabs(r / dg));
        }
        if (PRECOND == RF_PRECOND_ZLINE && kt > 0) {
            double zr;
            if (kt <= kWave) zline_solve_column<true>(a.r, a.rdp, a.tz, a.z, base, kt, lane, zr);
            else zline_solve_column<false>(a.r, a.rdp, a.tz, a.z, base, kt, lane, zr);
            for (int k0 = 0; k0 < kt; k0 += kWave) {
                const int k = k0 + lane;
                if (k < kt) v[0] += a.r[base + k] * a.z[base + k];
            }
        }
    }
    block_partial<2, 2u>(v, a.pr);
}

// ---------------------------------------------------------------------------
// Picard update and exit test (row a6): h^{m+1} = h^m + e, delta = max|e|
// ---------------------------------------------------------------------------

// Enqueued after every chunk of PCG iterations.  Every block combines the
// last (r.z, max|r/diag|) partials and decides, as the next direction update
// would, whether the solve has finished; if so it writes hnew = h^m + e
// (idempotent, so a repeated launch changes nothing) and the block partials
// of (max|e|, non-finite count), which the host combines.
__global__ void __launch_bounds__(kThreads) k_apply_h(Geo g, Arrays a, double tol_cg, int max_cg)
{
    Scalars *s = a.sc;
    if (s->fail) return;
    const int j = s->iters;
    double tot[2];
    reduce_partials<2, 2u>(a.pr, gridDim.x, tot);
    const bool finished = s->done || !(tot[1] > tol_cg) || j >= max_cg;
    if (!finished) return;
    if (!isfinite(tot[0]) || !isfinite(tot[1]) || (!s->done && tot[1] > tol_cg)) {
        if (lead_thread()) {   // the next direction update would stop with this status
            s->fail = (!isfinite(tot[0]) || !isfinite(tot[1])) ? 3 : 2;
            s->final_iters = j;
        }
        return;
    }
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[2] = {0.0, 0.0};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            const size_t i = (size_t)col * g.nz + k;
            const double e = a.e[i];
            const double h = a.hm[i] + e;
            a.hnew[i] = h;
            v[0] = fmax(v[0], fabs(e));
            if (!isfinite(h)) v[1] += 1.0;
        }
    }
    block_partial<2, 1u>(v, a.pd);
    if (lead_thread()) {
        s->applied = 1;
        s->final_iters = j;
    }
}

// ---------------------------------------------------------------------------
// Step acceptance (row a7): h^n <- h^{m+1}, theta~^n, storage, face inflows
// ---------------------------------------------------------------------------

// Block partials: [0] storage sum V theta~(h); [1+f] inflow rate through
// face f with h = h^{m+1} and K = K(h^m) (the converged system).
__global__ void __launch_bounds__(kThreads) k_accept(Geo g, Soil so, Bc bc, Arrays a)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const double dist[3] = {g.A[0] / g.Tk[0], g.A[1] / g.Tk[1], g.A[2] / g.Tk[2]};
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            Cell c;
            cell_setup(g, a.ktop, col, kt, k, c);
            const size_t idx = c.idx;
            const Layer &L = so.L[a.layer ? a.layer[idx] : 0];
            const double h = a.hm[idx];
            a.hn[idx] = h;
            const double th = soil_theta(so.model, h, L);
            a.thn[idx] = th;
            v[0] += g.V * th;
#pragma unroll
            for (int d = 0; d < 6; d++) {
                if (!c.bnd[d]) continue;
                const int ax = d >> 1;
                const double gn = gdot(g, d);
                const int type = bc.type[d];
                double q = 0.0;
                if (type == RF_DIRICHLET) {
                    const double hb = bc.value[d];
                    const double Kb = soil_K(so.model, hb, L, a.Ks[idx]);
                    q = g.A[ax] * Kb / (0.5 * dist[ax]) * (hb - h) + g.A[ax] * Kb * gn;
                } else if (type == RF_FLUX) {
                    q = g.A[ax] * bc.value[d];
                } else if (type == RF_FREE_DRAINAGE) {
                    q = g.A[ax] * a.K[idx] * gn;
                }
                v[1 + d] += q;
            }
        }
    }
    block_partial<7, 0u>(v, a.ps);
}

// ---------------------------------------------------------------------------
// inspection kernels
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kThreads) k_eval_soil(Geo g, Soil so, Arrays a, const double *h,
                                                        double *theta, double *Cout, double *Kout)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            const size_t idx = (size_t)col * g.nz + k;
            const Layer &L = so.L[a.layer ? a.layer[idx] : 0];
            double th, C, K;
            soil_eval(so.model, h[idx], L, a.Ks[idx], th, C, K);
            if (theta) theta[idx] = th;
            if (Cout) Cout[idx] = C;
            if (Kout) Kout[idx] = K;
        }
    }
}

// y = A x with the operator (K, Dd) of the last assembly.
__global__ void __launch_bounds__(kThreads) k_operator(Geo g, Arrays a, const double *x, double *y)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            Cell c;
            cell_setup(g, a.ktop, col, kt, k, c);
            const double Kp = a.K[c.idx], xp = x[c.idx];
            double q = a.Dd[c.idx] * xp;
#pragma unroll
            for (int d = 0; d < 6; d++) {
                if (!c.nb[d]) continue;
                const double T = g.Tk[d >> 1] * 0.5 * (Kp + a.K[c.off[d]]);
                q += T * (xp - x[c.off[d]]);
            }
            y[c.idx] = q;
        }
    }
}

template <int PRECOND>
__global__ void __launch_bounds__(kThreads) k_precond(Geo g, Arrays a, const double *r, double *z)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        const size_t base = (size_t)col * g.nz;
        if (PRECOND == RF_PRECOND_JACOBI) {
            for (int k0 = 0; k0 < kt; k0 += kWave) {
                const int k = k0 + lane;
                if (k < kt) z[base + k] = r[base + k] / a.diag[base + k];
            }
        } else if (kt > 0) {
            double zr;
            if (kt <= kWave) zline_solve_column<true>(r, a.rdp, a.tz, z, base, kt, lane, zr);
            else zline_solve_column<false>(r, a.rdp, a.tz, z, base, kt, lane, zr);
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_copy_active(Geo g, Arrays a, const double *src, double *dst)
{
    int cb, ce;
    block_columns(g, cb, ce);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k < kt) dst[(size_t)col * g.nz + k] = src[(size_t)col * g.nz + k];
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define RF_LAUNCH(kern, ...)                                                            \
    do {                                                                                \
        hipLaunchKernelGGL(kern, dim3(g.nblk), dim3(kThreads), 0, s, __VA_ARGS__);     \
        return hipGetLastError();                                                       \
    } while (0)

hipError_t launch_init_ks(const Geo &g, const Soil &so, const Arrays &a, hipStream_t s)
{
    RF_LAUNCH(k_init_ks, g, so, a, (const double *)a.ks_layer);
}

hipError_t launch_check_finite(const Geo &g, const Arrays &a, const double *h, hipStream_t s)
{
    RF_LAUNCH(k_check_finite, g, a, h);
}

hipError_t launch_set_state(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            hipStream_t s)
{
    RF_LAUNCH(k_set_state, g, so, a, h);
}

hipError_t launch_coeff(const Geo &g, const Soil &so, const Bc &bc, const Arrays &a, double dt,
                        double chord_eps, hipStream_t s)
{
    RF_LAUNCH(k_coeff, g, so, bc, a, dt, chord_eps);
}

hipError_t launch_resid(const Geo &g, const Arrays &a, int precond, double *bout, hipStream_t s)
{
    if (precond == RF_PRECOND_ZLINE) RF_LAUNCH(k_resid<RF_PRECOND_ZLINE>, g, a, bout);
    RF_LAUNCH(k_resid<RF_PRECOND_JACOBI>, g, a, bout);
}

hipError_t launch_spmv(const Geo &g, const Arrays &a, int precond, const double *p_in,
                       double *p_out, double tol_cg, int max_cg, hipStream_t s)
{
    if (precond == RF_PRECOND_ZLINE)
        RF_LAUNCH(k_spmv<RF_PRECOND_ZLINE>, g, a, p_in, p_out, tol_cg, max_cg);
    RF_LAUNCH(k_spmv<RF_PRECOND_JACOBI>, g, a, p_in, p_out, tol_cg, max_cg);
}

hipError_t launch_update(const Geo &g, const Arrays &a, int precond, const double *p, hipStream_t s)
{
    if (precond == RF_PRECOND_ZLINE) RF_LAUNCH(k_update<RF_PRECOND_ZLINE>, g, a, p);
    RF_LAUNCH(k_update<RF_PRECOND_JACOBI>, g, a, p);
}

hipError_t launch_apply_h(const Geo &g, const Arrays &a, double tol_cg, int max_cg, hipStream_t s)
{
    RF_LAUNCH(k_apply_h, g, a, tol_cg, max_cg);
}

hipError_t launch_accept(const Geo &g, const Soil &so, const Bc &bc, const Arrays &a,
                         hipStream_t s)
{
    RF_LAUNCH(k_accept, g, so, bc, a);
}

hipError_t launch_eval_soil(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            double *theta, double *C, double *K, hipStream_t s)
{
    RF_LAUNCH(k_eval_soil, g, so, a, h, theta, C, K);
}

hipError_t launch_operator(const Geo &g, const Arrays &a, const double *x, double *y,
                           hipStream_t s)
{
    RF_LAUNCH(k_operator, g, a, x, y);
}

hipError_t launch_precond(const Geo &g, const Arrays &a, int precond, const double *r, double *z,
                          hipStream_t s)
{
    if (precond == RF_PRECOND_ZLINE) RF_LAUNCH(k_precond<RF_PRECOND_ZLINE>, g, a, r, z);
    RF_LAUNCH(k_precond<RF_PRECOND_JACOBI>, g, a, r, z);
}

hipError_t launch_copy_active(const Geo &g, const Arrays &a, const double *src, double *dst,
                              hipStream_t s)
{
    RF_LAUNCH(k_copy_active, g, a, src, dst);
}

}  // namespace rf
