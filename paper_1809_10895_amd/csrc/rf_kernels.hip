// HIP kernels (gfx950 / CDNA4) of the Richards-equation Picard / PCG loop.
//
// Work decomposition: one wavefront owns one z-column at a time; lane k of
// the wave holds cell k of the column (columns longer than 64 cells are
// walked in chunks of 64).  With z the fastest index every column is one
// contiguous run of doubles, so each chunk is a single coalesced 512-byte
// access per array, the vertical coupling stays inside the wave (DPP lane
// shifts and scans, rf_wave.h), and the lateral neighbours are the adjacent
// columns.  Blocks of 8 waves take contiguous runs of columns (optionally
// remapped per XCD, see block_columns).  The PCG kernels are templated on
// the precision of their vectors: FP64, or FP32 under FP64 Picard refinement
// (mixed precision); their reductions are FP64 in both.
//
// Global reductions are two-stage, deterministic and fence-free: every block
// writes one partial per value, and the consumer -- every block of the next
// kernel, or the host -- combines the partials in block order (large grids
// first fold them with a one-block kernel).
// Cross-block visibility therefore only ever relies on kernel boundaries: an
// agent-scope fence per block would write back the whole L2 of its XCD, and a
// single ticket counter would serialise every block of the grid.  Scalars
// such as alpha and beta never leave the device during the PCG loop.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "rf_internal.h"
#include "rf_soil.h"
#include "rf_wave.h"

namespace rf {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Columns [cb, ce) of this block: logical block lb takes cpb consecutive
// columns.  The hardware deals workgroups round-robin over the 8 XCDs
// (block b runs on XCD b % 8); map 1 undoes that so each XCD works through
// one contiguous slab (lateral neighbours stay in one L2), and map 2 also
// starts each XCD at a different point of its slab, so that the eight
// streams are not a power-of-two stride apart at every instant.
__device__ __forceinline__ void block_columns(const Geo &g, int cpb, int &cb, int &ce)
{
    const int b = blockIdx.x, G = gridDim.x;
    int lb = b;
    if (g.block_map != 0 && G >= 8 && (G & 7) == 0) {
        const int per = G >> 3, x = b & 7;
        int r = b >> 3;
        if (g.block_map == 2) r = (r + (x * per) / 8) % per;
        lb = x * per + r;
    }
    cb = lb * cpb;
    ce = min(cb + cpb, g.ncol);
}

// Sum / max over the wave, the same value in every lane: an in-row scan
// with DPP shifts leaves each 16-lane row's total in its last lane; the four
// row totals are combined in a fixed order.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp<kDppRowShr + 1>(x, 0.0);
    x += dpp<kDppRowShr + 2>(x, 0.0);
    x += dpp<kDppRowShr + 4>(x, 0.0);
    x += dpp<kDppRowShr + 8>(x, 0.0);
    return (lane_value<15>(x) + lane_value<31>(x)) + (lane_value<47>(x) + lane_value<63>(x));
}

// (A lane without a partner compares with itself.)
__device__ __forceinline__ double wave_max(double x)
{
    x = fmax(x, dpp<kDppRowShr + 1>(x, x));
    x = fmax(x, dpp<kDppRowShr + 2>(x, x));
    x = fmax(x, dpp<kDppRowShr + 4>(x, x));
    x = fmax(x, dpp<kDppRowShr + 8>(x, x));
    return fmax(fmax(lane_value<15>(x), lane_value<31>(x)), fmax(lane_value<47>(x), lane_value<63>(x)));
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

// First half of reduce_partials: this thread's share of the nblk block
// partials (blocks threadIdx.x, + kThreads, ...), so that their loads can be
// issued early and combined later with combine_partials.  The loads of eight
// partials are issued before any is added (one round trip per eight instead
// of one per partial, which is what a one-block fold over thousands of
// partials waits on); they are added in block order, as one at a time.
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void gather_partials(const double *P, int nblk, double (&v)[NV])
{
    constexpr int U = 8;
#pragma unroll
    for (int i = 0; i < NV; i++) v[i] = 0.0;   // identity of sums and of max over |x|
    int b = threadIdx.x;
    for (; b + (U - 1) * kThreads < nblk; b += U * kThreads) {
        double x[U][NV];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int i = 0; i < NV; i++) x[u][i] = P[(size_t)(b + u * kThreads) * NV + i];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int i = 0; i < NV; i++)
                v[i] = ((MAXMASK >> i) & 1u) ? fmax(v[i], x[u][i]) : v[i] + x[u][i];
    }
    for (; b < nblk; b += kThreads)
#pragma unroll
        for (int i = 0; i < NV; i++) {
            const double x = P[(size_t)b * NV + i];
            v[i] = ((MAXMASK >> i) & 1u) ? fmax(v[i], x) : v[i] + x;
        }
}

// Second half: the gathered shares combined over the block in a fixed order;
// all threads receive the totals.  Call from every thread.
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void combine_partials(double (&v)[NV], double (&tot)[NV])
{
    __shared__ double sh[kWavesPerBlock][NV];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
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

// Combines the nblk block partials written by the previous kernel, in the
// same fixed order in every block; all threads receive the totals.
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void reduce_partials(const double *P, int nblk, double (&tot)[NV])
{
    __shared__ double sh[kWavesPerBlock][NV];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double v[NV];
    gather_partials<NV, MAXMASK>(P, nblk, v);
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

// Columns of one wave processed together in the short-column paths (columns
// of at most 64 cells), so that their loads are in flight at the same time:
// every kernel there first gathers all values of the group with branch-free
// loads, then computes.  Lanes without a cell read their own column's first
// cell (no extra cache lines) and are masked at the stores.
constexpr int kColGroup = 4;

struct ColSlot {
    int col;      // column (clamped into the block's range)
    int kt;       // active cells (0 if the slot is past the block's columns)
    bool act;     // this lane holds an active cell
    size_t base;  // first cell of the column
    size_t i;     // this lane's cell (always inside the column, active or not)
};

// Addresses do not wait for k_top: every lane of a column reads its own cell
// (masked cells are valid memory), so the data loads and the k_top loads of
// a group are all in flight together; the masks apply to the results.
__device__ __forceinline__ ColSlot col_slot(const Geo &g, const int32_t *__restrict__ ktop, int col,
                                            int ce, int lane)
{
    ColSlot c;
    const bool valid = col < ce;
    c.col = valid ? col : ce - 1;
    c.base = (size_t)c.col * g.nz;
    c.i = c.base + min(lane, g.nz - 1);
    const int kt = ktop[c.col];
    c.kt = valid ? kt : 0;
    c.act = lane < c.kt;
    return c;
}

// Lateral neighbours (0 -x, 1 +x, 2 -y, 3 +y) of a slot: whether the
// neighbour cell is active, and its index (this cell's index where the
// domain ends).
__device__ __forceinline__ void lateral(const Geo &g, const int32_t *__restrict__ ktop,
                                        const ColSlot &c, int lane, bool (&nb)[4], size_t (&in)[4])
{
    const int i = c.col % g.nx, j = c.col / g.nx;
    const size_t sx = (size_t)g.nz, sy = (size_t)g.nz * g.nx;
    const bool has[4] = {i > 0, i < g.nx - 1, j > 0, j < g.ny - 1};
    const int cn[4] = {has[0] ? c.col - 1 : c.col, has[1] ? c.col + 1 : c.col,
                       has[2] ? c.col - g.nx : c.col, has[3] ? c.col + g.nx : c.col};
    int ktn[4];
#pragma unroll
    for (int d = 0; d < 4; d++) ktn[d] = ktop[cn[d]];      // unconditional: all in flight
#pragma unroll
    for (int d = 0; d < 4; d++) {
        const size_t off = (d < 2) ? sx : sy;
        in[d] = has[d] ? ((d & 1) ? c.i + off : c.i - off) : c.i;
        nb[d] = c.act & has[d] & (lane < ktn[d]);            // no short-circuit branches
    }
}

// Tiles of the tiled stencil kernels: block b owns the kTileX x TY columns
// of tile (b % ntx, b / ntx); with its one-column halo they form a
// (kTileX + 2) x (TY + 2) array of slots (the four corners unused), slot
// (sx, sy) = sx + SX sy.  Wave w owns the TY interior columns at sx = w + 1.
template <int TY>
struct Tile {
    static constexpr int SX = kTileX + 2, SY = TY + 2, NS = SX * SY;
    static constexpr int NH = 2 * kTileX + 2 * TY;                           // halo slots
    static_assert(kTileX == kWavesPerBlock, "one tile row along x per wave");

    // Column of slot sl of the tile whose slot (0, 0) is the grid column
    // (i0, j0), or -1 (a corner, or outside the grid).
    __device__ static __forceinline__ int column(const Geo &g, int i0, int j0, int sl)
    {
        const int sx = sl % SX, sy = sl / SX;
        const int gi = i0 + sx, gj = j0 + sy;
        const bool corner = (sx == 0 || sx == SX - 1) && (sy == 0 || sy == SY - 1);
        const bool in = sl < NS && !corner && gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny;
        return in ? gi + g.nx * gj : -1;
    }
    // slot of wave w's interior column t
    __device__ static __forceinline__ int own(int w, int t) { return (w + 1) + SX * (t + 1); }
};

// Which slots of a Tile<TY> wave w loads (its u-th: slot(w, u), or NS for
// none).  OWN_FIRST = false: slots w, w + 8, ... (neighbouring waves load
// neighbouring columns).  OWN_FIRST = true: its own TY interior columns
// first, so that it holds their values itself, then its share of the halo
// (dealt w, w + 8, ...: the first row, the two ends of each interior row,
// the last row).
template <int TY, bool OWN_FIRST>
struct TileSlots {
    using Tl = Tile<TY>;
    static constexpr int PER = OWN_FIRST ? TY + (Tl::NH + kWavesPerBlock - 1) / kWavesPerBlock
                                         : (Tl::NS + kWavesPerBlock - 1) / kWavesPerBlock;

    __device__ static __forceinline__ int slot(int w, int u)
    {
        if (!OWN_FIRST) return w + u * kWavesPerBlock;
        if (u < TY) return Tl::own(w, u);
        int h = w + (u - TY) * kWavesPerBlock;
        if (h >= Tl::NH) return Tl::NS;
        if (h < kTileX) return 1 + h;
        h -= kTileX;
        if (h < 2 * TY) return (h & 1) * (Tl::SX - 1) + Tl::SX * (1 + (h >> 1));
        h -= 2 * TY;
        return 1 + h + Tl::SX * (Tl::SY - 1);
    }
};

// The columns and active lengths one wave needs for tile `tile` (-1: none):
// its share of the slots (TileSlots) and its own TY interior columns.  The
// active lengths are scalar loads, issued together.
template <int TY, bool OWN_FIRST>
struct TileCols {
    using Sl = TileSlots<TY, OWN_FIRST>;
    int col[Sl::PER], kt[Sl::PER], oc[TY], okt[TY];

    __device__ __forceinline__ void fetch(const Geo &g, const int32_t *__restrict__ ktop, int tile,
                                          int w)
    {
        using Tl = Tile<TY>;
        const int i0 = (tile % g.ntx) * kTileX - 1, j0 = (tile / g.ntx) * TY - 1;
#pragma unroll
        for (int u = 0; u < Sl::PER; u++) {
            col[u] = (tile >= 0) ? Tl::column(g, i0, j0, Sl::slot(w, u)) : -1;
            kt[u] = (col[u] >= 0) ? ktop[col[u]] : 0;
        }
#pragma unroll
        for (int t = 0; t < TY; t++) {
            oc[t] = (tile >= 0) ? Tl::column(g, i0, j0, Tl::own(w, t)) : -1;
            okt[t] = (oc[t] >= 0) ? ktop[oc[t]] : 0;
        }
    }
};

__device__ __forceinline__ bool lead_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }

// Boundary terms of a cell with face f on the domain boundary, in terms of
// the face conductivity Kb = Ks * krb[f][layer] and the cell's K (Sec. 3.1,
// 3.2, App. A, App. B):  diagonal += cD Kb;  right-hand side += cKb Kb +
// cK K + c0, where Dirichlet h_b gives cD = 2 A/d (half-cell distance),
// cKb = cD h_b + A g.n; flux q gives c0 = A q; free drainage gives cK = A g.n;
// no-flow gives nothing.  The inflow through the face at head h is
// (cKb - cD h) Kb + cK K + c0.
struct FaceTab {
    double cD, cKb, cK, c0;
};

// Stages the face table and the Dirichlet relative conductivities in LDS.
__device__ __forceinline__ void stage_bc(const Arrays &a, FaceTab *sBT, double *sKR)
{
    const double *src = a.bt;
    double *d = reinterpret_cast<double *>(sBT);
    for (int i = threadIdx.x; i < 24; i += kThreads) d[i] = src[i];
    for (int i = threadIdx.x; i < 6 * RF_MAX_LAYERS; i += kThreads) sKR[i] = a.krb[i];
}

// Copies the layer table into LDS (cells index it with their own layer, so
// it must not stay in kernel arguments, which live in scalar registers).
// Call from every thread of the block.
__device__ __forceinline__ void stage_layers(const Arrays &a, int nlayer, Layer *sL)
{
    double *d = reinterpret_cast<double *>(sL);
    const double *src = reinterpret_cast<const double *>(a.layers);
    for (int i = threadIdx.x; i < nlayer * 6; i += kThreads) d[i] = src[i];
    __syncthreads();
}

// Cell neighbourhood inside a column chunk.  Direction d: 0 -x, 1 +x, 2 -y,
// 3 +y, 4 -z, 5 +z.  nb[d]: neighbour active; bnd[d]: the face is on the
// domain boundary (the +z boundary is the top of the column's active run).
// The cell of one lane in run q of kWave consecutive active cells (see
// Arrays::chunk; rec is the run's record, read once per wavefront): column,
// k, whether it exists (runs past the last active cell are short) and
// whether it is its column's top cell.  Lanes past the third column of the
// run walk the active lengths (columns shorter than a run only).
struct RunCell {
    int col, k;
    bool act, top;
    size_t i;       // cell index (0 for a lane without a cell)
};

__device__ __forceinline__ RunCell run_cell(const Geo &g, const int32_t *__restrict__ ktop,
                                            const int4 &rec, int q, int lane)
{
    const int l1 = rec.z & 255, l2 = (rec.z >> 8) & 255, l3 = (rec.z >> 16) & 255;
    RunCell r;
    r.act = (long)q * kWave + lane < g.nact;
    if (lane < l1) {
        r.col = rec.x;
        r.k = rec.y + lane;
        r.top = lane == l1 - 1;
    } else if (lane < l2) {
        r.col = rec.x + 1;
        r.k = lane - l1;
        r.top = lane == l2 - 1;
    } else if (lane < l3) {
        r.col = rec.x + 2;
        r.k = lane - l2;
        r.top = lane == l3 - 1;
    } else {
        int col = rec.x + 3, k = lane - l3, kt = 0;
        if (r.act) {
            kt = ktop[col];
            while (k >= kt) {
                k -= kt;
                col++;
                kt = ktop[col];
            }
        }
        r.col = col;
        r.k = k;
        r.top = k == kt - 1;
    }
    if (!r.act) {
        r.col = 0;
        r.k = 0;
        r.top = false;
    }
    r.i = (size_t)r.col * g.nz + r.k;
    return r;
}

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

#define RF_WAVE_IDS                                                     \
    const int lane = threadIdx.x & (kWave - 1);                         \
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave)

// Ks per cell = Ks(layer) * exp(ln_ks_offset); Ks holds the offsets on entry
// (zeros when none were given).
__global__ void __launch_bounds__(kThreads) k_init_ks(Geo g, Arrays a)
{
    const size_t N = (size_t)g.ncol * g.nz;
    for (size_t c = (size_t)blockIdx.x * kThreads + threadIdx.x; c < N;
         c += (size_t)gridDim.x * kThreads) {
        const int l = a.layer ? a.layer[c] : 0;
        a.Ks[c] = a.ks_layer[l] * exp(a.Ks[c]);
    }
}

// Block partials (ps) of the number of non-finite active values of h.
__global__ void __launch_bounds__(kThreads) k_check_finite(Geo g, Arrays a, const double *h)
{
    int cb, ce;
    block_columns(g, g.cpb, cb, ce);
    RF_WAVE_IDS;
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

// h^n <- h (every cell), theta~^n <- theta~(h) and block partials of the
// storage sum V theta~ (active cells).
__global__ void __launch_bounds__(kThreads) k_set_state(Geo g, Soil so, Arrays a, const double *h)
{
    __shared__ Layer sL[RF_MAX_LAYERS];
    stage_layers(a, so.nlayer, sL);
    int cb, ce;
    block_columns(g, g.cpb, cb, ce);
    RF_WAVE_IDS;
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
                const Layer &L = sL[a.layer ? a.layer[idx] : 0];
                const double th = soil_theta(so.model, hv, L);
                a.thn[idx] = th;
                v[0] += g.V * th;
            }
        }
    }
    block_partial<1, 0u>(v, a.ps);
}

// ---------------------------------------------------------------------------
// Step control
// ---------------------------------------------------------------------------

// First Picard iterate h^0 = h0 (h^n or a caller's guess) into hb[0]; resets
// the step flags; block 0 tabulates the relative conductivity K(h_b)/Ks of
// every Dirichlet face for every layer (the face conductivity of a cell is
// its own Ks times that entry).
__global__ void __launch_bounds__(kThreads) k_step_begin(Geo g, Soil so, Bc bc, Arrays a,
                                                         const double *h0, double ratio, int gate)
{
    if (gate >= 0 && a.sc->accepted_serial != gate) {
        // enqueued behind a step that its own work did not accept: nothing
        // is done, and the stall flag holds every later kernel of this step
        // (no block of this kernel writes accepted_serial, so all blocks
        // take the same branch)
        if (lead_thread() && !a.sc->stall) {
            a.sc->stall = 1;
            a.sc->stall_m = -1;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x < 6 * RF_MAX_LAYERS) {
        const int f = threadIdx.x / RF_MAX_LAYERS, l = threadIdx.x % RF_MAX_LAYERS;
        double kr = 0.0;
        if (bc.type[f] == RF_DIRICHLET && l < so.nlayer)
            kr = soil_K(so.model, bc.value[f], a.layers[l], 1.0);
        a.krb[threadIdx.x] = kr;
        if (threadIdx.x < 6) {
            const int ff = threadIdx.x, ax = ff >> 1;
            const double gn = ((ff & 1) ? 1.0 : -1.0) * g.g[ax];
            const double Tb = 2.0 * g.Tk[ax];
            double cD = 0.0, cKb = 0.0, cK = 0.0, c0 = 0.0;
            if (bc.type[ff] == RF_DIRICHLET) {
                cD = Tb;
                cKb = Tb * bc.value[ff] + g.A[ax] * gn;
            } else if (bc.type[ff] == RF_FLUX) {
                c0 = g.A[ax] * bc.value[ff];
            } else if (bc.type[ff] == RF_FREE_DRAINAGE) {
                cK = g.A[ax] * gn;
            }
            a.bt[4 * ff + 0] = cD;
            a.bt[4 * ff + 1] = cKb;
            a.bt[4 * ff + 2] = cK;
            a.bt[4 * ff + 3] = c0;
        }
    }
    int cb, ce;
    block_columns(g, g.cpb_w, cb, ce);
    RF_WAVE_IDS;
    if (h0)
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            const size_t i = (size_t)col * g.nz + k;
            a.hb0[i] = (ratio != 0.0) ? h0[i] + ratio * a.dh[i] : h0[i];
        }
    }
    if (lead_thread()) {
        Scalars *s = a.sc;
        s->done = 0;
        s->fail = 0;
        s->iters = 0;
        s->final_iters = 0;
        s->stall = 0;
        s->stall_m = 0;
        s->picard_done = 0;
        s->picard_m = 0;
        s->accepted = 0;
        s->accept_m = 0;
    }
}

// Global Picard exit test (Sec. 2.3) of the update written by iteration m-1:
// one block combines the (max|e|, non-finite) partials; converged when
// max |h^m - h^{m-1}| < tol_picard.
__global__ void __launch_bounds__(kThreads) k_decide(Geo g, Arrays a, int m, double tol_picard)
{
    Scalars *s = a.sc;
    if (s->fail || s->stall || s->picard_done) return;
    // the nblk partials of k_apply_h as it wrote them (no fold kernel: this
    // one-block kernel is their only reader; a max and a count combine alike
    // in any order)
    double tot[2];
    reduce_partials<2, 1u>(a.pd, g.nblk, tot);
    if (threadIdx.x == 0) {
        if (m - 1 < RF_MAX_PICARD_LOG) s->delta_log[m - 1] = tot[0];
        if (tot[1] > 0.0 || !isfinite(tot[0])) {
            s->fail = 3;
            s->done = 1;
        } else if (tot[0] < tol_picard) {
            s->picard_done = 1;
            s->picard_m = m - 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Picard iteration: coefficients and boundary terms
// ---------------------------------------------------------------------------

// Per active cell of h^m: K = K(h^m); chord capacity C = (theta~(h^m) -
// theta~(h^n)) / (h^m - h^n), or Eq. 3 when |h^m - h^n| < chord_eps;
// Dd = V C / dt + the boundary diagonal terms; bst = V C h^n / dt + the
// boundary right-hand-side terms (see FaceTab).  Modified Picard: C = Eq. 3
// at h^m and bst = V (C h^m - (theta~(h^m) - theta~^n)) / dt + boundary
// terms.  Interior-face terms are added in k_resid.
//
// Diagonal and right-hand side of one active cell from theta~, C, K at h^m;
// bnd: its faces on the domain boundary.
__device__ __forceinline__ void coeff_terms(const FaceTab *sBT, const double *sKR,
                                            int lay, const bool (&bnd)[6], double hm, double hn,
                                            double thn, double ks, double th, double C, double K,
                                            double vdt, double chord_eps, int variant, double &D,
                                            double &b)
{
    if (variant == RF_PICARD_MODIFIED) {
        D = vdt * C;
        b = vdt * (C * hm - (th - thn));
    } else {
        const double dh = hm - hn;
        const double Cc = (fabs(dh) >= chord_eps) ? (th - thn) / dh : C;
        D = vdt * Cc;
        b = D * hn;
    }
#pragma unroll
    for (int d = 0; d < 6; d++) {
        if (!bnd[d]) continue;
        const double Kb = ks * sKR[d * RF_MAX_LAYERS + lay];
        D += sBT[d].cD * Kb;
        b += sBT[d].cKb * Kb + sBT[d].cK * K + sBT[d].c0;
    }
}

// The soil model is a template parameter.  A wavefront evaluates runs of
// kWave consecutive active cells (Arrays::chunk), so no lane works on a cell
// above its column's top, whatever the active lengths; the loads of a run are
// issued together, and van Genuchten-Mualem is evaluated branch-free.  At
// most 128 VGPRs (four waves per SIMD, two 512-thread blocks per CU): a
// second run's loads in flight during the evaluation spilled registers and
// measured slower.
template <int MODEL, bool FLAT>
__global__ void __launch_bounds__(kThreads, 4) k_coeff(Geo g, Soil so, Arrays a, int m, double dt,
                                                    double chord_eps, int variant)
{
    Scalars *s = a.sc;
    if (s->fail || s->stall || s->picard_done) return;
    __shared__ Layer sL[RF_MAX_LAYERS];
    __shared__ FaceTab sBT[6];
    __shared__ double sKR[6 * RF_MAX_LAYERS];
    stage_bc(a, sBT, sKR);
    stage_layers(a, so.nlayer, sL);
    const double *hmv = (m == 0) ? a.h0m : (m & 1) ? a.hb1 : a.hb0;
    const double vdt = g.V / dt;
    RF_WAVE_IDS;
    // one run of kWave active cells per wavefront at a time
    const int qs = gridDim.x * kWavesPerBlock;
    int q = blockIdx.x * kWavesPerBlock + w;
    int4 rec_next = (q < g.nchunk) ? a.chunk[q] : int4{0, 0, 0, 0};
    for (; q < g.nchunk; q += qs) {
        // the next run's record is read while this run is evaluated
        const int4 rec = rec_next;
        if (q + qs < g.nchunk) rec_next = a.chunk[q + qs];
        const RunCell rc = run_cell(g, a.ktop, rec, q, lane);
        const size_t i = rc.i;
        const int lay = a.layer ? a.layer[i] : 0;
        const double ks = a.Ks[i], hm = hmv[i], hn = a.hn[i], thn = a.thn[i];
        double th, C, K;
        if (FLAT) {
            soil_eval_vgm_flat(hm, sL[lay], ks, th, C, K);
        } else {
            soil_eval(MODEL, hm, sL[lay], ks, th, C, K);
        }
        if (!rc.act) continue;
        const int ci = rc.col % g.nx, cj = rc.col / g.nx;
        const bool bnd[6] = {ci == 0, ci == g.nx - 1, cj == 0, cj == g.ny - 1, rc.k == 0, rc.top};
        double D, b;
        coeff_terms(sBT, sKR, lay, bnd, hm, hn, thn, ks, th, C, K, vdt, chord_eps, variant, D, b);
        a.K[i] = K;
        a.Dd[i] = D;
        a.bst[i] = b;
    }
}

// ---------------------------------------------------------------------------
// z-line preconditioner pieces (exact LDL^T of each column's vertical part)
// ---------------------------------------------------------------------------

// z = M^-1 r for a column longer than one wave, from memory: forward sweep
// w_k = (r_k + t_{k-1} w_{k-1}) rdp_k into zout, backward sweep
// z_k = w_k + t_k rdp_k z_{k+1}.  Every lane re-reads only what it wrote.
template <typename T>
__device__ __forceinline__ void zline_solve_long(const T *r, const T *rdp, const T *tz, T *zout,
                                                 size_t base, int kt, int lane)
{
    T carry = 0;
    for (int k0 = 0; k0 < kt; k0 += kWave) {
        const int k = k0 + lane;
        const bool act = k < kt;
        const T rk = act ? r[base + k] : T(0);
        const T rd = act ? rdp[base + k] : T(0);
        const T tp = (act && k > 0) ? tz[base + k - 1] : T(0);
        const T wk = scan_affine_up<T>(tp * rd, rk * rd, carry, lane);
        carry = lane_value<kWave - 1>(wk);
        if (act) zout[base + k] = wk;
    }
    carry = 0;
    for (int ch = (kt - 1) / kWave; ch >= 0; ch--) {
        const int k = ch * kWave + lane;
        const bool act = k < kt;
        const T wk = act ? zout[base + k] : T(0);
        const T bk = act ? tz[base + k] * rdp[base + k] : T(0);
        const T zk = scan_affine_down<T>(bk, wk, carry, lane);
        carry = lane_value<0>(zk);
        if (act) zout[base + k] = zk;
    }
}

// The same for a column of at most 64 cells, entirely in registers: r, rdp
// and t of lane k; returns z_k.
template <typename T>
__device__ __forceinline__ T zline_solve_short(T r, T rd, T t, int lane)
{
    const T tp = from_below0<T>(t);
    const T wk = scan_affine_up<T>(tp * rd, r * rd, T(0), lane);
    return scan_affine_down<T>(t * rd, wk, T(0), lane);
}

// The same for two columns at once, one per half-wave, two cells per lane
// (cells k0 = 2 (lane & 31) and k0 + 1): r, rdp and t of the lane's two
// cells (zero above the column's top); returns their z.  Each lane composes
// the affine maps of its two cells, the composites are scanned over the
// half, and the lane's cells are finished from its neighbour lane's prefix.
template <typename T>
__device__ __forceinline__ void zline_solve_pair(const T (&r)[2], const T (&rd)[2], const T (&t)[2],
                                                 int lane, T (&z)[2])
{
    const bool first = (lane & 31) == 0, last = (lane & 31) == 31;
    // forward sweep w_k = (r_k + t_{k-1} w_{k-1}) rdp_k
    const T A0 = from_below0<T>(t[1]) * rd[0], B0 = r[0] * rd[0];
    const T A1 = t[0] * rd[1], B1 = r[1] * rd[1];
    T fa = A1 * A0, fc = A1 * B0 + B1;
    scan_affine_up_half<T>(fa, fc);
    T wb = from_below0<T>(fc);
    if (first) wb = T(0);
    const T w0 = A0 * wb + B0, w1 = A1 * w0 + B1;
    // backward sweep z_k = w_k + t_k rdp_k z_{k+1}
    const T C0 = t[0] * rd[0], C1 = t[1] * rd[1];
    T bb = C0 * C1, bc = C0 * w1 + w0;
    scan_affine_down_half<T>(bb, bc, lane);
    T za = from_above0<T>(bc);
    if (last) za = T(0);
    z[1] = C1 * za + w1;
    z[0] = C0 * z[1] + w0;
}

// ---------------------------------------------------------------------------
// Residual of the Picard system and PCG start
// ---------------------------------------------------------------------------

// max(m, |a_c| / d_c) over the lane's active cells c (d_c > 0) with one
// division: with d_c = 2^-e_c c_c, c_c in [1, 2) (exact scalings, so that no
// product over- or underflows where the quotients do not),
// |a_c| / d_c = 2^e_c |a_c| c_other / (c_0 c_1).
template <typename T>
__device__ __forceinline__ double max_ratio_pair(double m, T a0, T d0, bool act0, T a1, T d1,
                                                 bool act1)
{
    const int e0 = 1 - frexp_exponent((double)d0), e1 = 1 - frexp_exponent((double)d1);
    const double c0 = ldexp((double)d0, e0), c1 = ldexp((double)d1, e1);
    const double n0 = act0 ? ldexp(fabs((double)a0) * c1, e0) : 0.0;
    const double n1 = act1 ? ldexp(fabs((double)a1) * c0, e1) : 0.0;
    return (act0 || act1) ? fmax(m, fmax(n0, n1) / (c0 * c1)) : m;
}

// Two columns of at most 64 cells at once, one per half-wave, two cells per
// lane: cells k0 = 2 (lane & 31) and k0 + 1 of this half's column (active
// length kt, first cell i0 = its index of k0): the interior faces, the
// residual r = b - A h^m of the increment system, diag (stored only where a
// later kernel reads it: Jacobi, factors kept from an earlier iteration, or
// the assembly for the caller; the update kernel otherwise rebuilds it from
// this iteration's factors), the z-line factors (refactor) and z = M^-1 r,
// and the block-partial contributions v = (r.z, max|r/diag|); the PCG
// iterate e needs no clearing (the first spmv kernel to add to it writes
// it).  The z-line pivots and sweeps first compose each lane's two
// cells and then scan over the 32 lanes of the half (half the scan steps per
// cell, and no chaining across four rows).  Kp, hp, Dp, bp, tzs, rds: the two
// cells' values; Kn, hn, nb: their lateral neighbours.
template <int PRECOND, typename T>
__device__ __forceinline__ void resid_pair(const Geo &g, const CgVec<T> &cv, double *bout,
                                           int refactor, int kt, size_t i0, int k0, int lane,
                                           const double (&Kp)[2], const double (&hp)[2],
                                           const double (&Dp)[2], const double (&bp)[2],
                                           const double (&Kn)[2][4], const double (&hn)[2][4],
                                           const bool (&nb)[2][4], const double (&tzs)[2],
                                           const double (&rds)[2], double (&v)[2])
{
    constexpr bool kCopyKD = !std::is_same<T, double>::value;
    const double gz[2] = {gdot(g, 4), gdot(g, 5)};
    // below the first cell lies the lower lane's second, above the second
    // cell the upper lane's first (masked by k > 0 and k + 1 < kt)
    const double Kd[2] = {from_below0(Kp[1]), Kp[0]}, hd[2] = {from_below0(hp[1]), hp[0]};
    const double Ku[2] = {Kp[1], from_above0(Kp[0])}, hu[2] = {hp[1], from_above0(hp[0])};
    const bool keep_diag = PRECOND == RF_PRECOND_JACOBI || !refactor || bout != nullptr;
    double diag[2], r[2], tup[2];
    T rs[2];
    bool act[2];
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const int k = k0 + c;
        act[c] = k < kt;
        double dg = act[c] ? Dp[c] : 1.0, Ap = Dp[c] * hp[c], b = bp[c], tu = 0.0;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            if (!nb[c][d]) continue;
            const double Kf = 0.5 * (Kp[c] + Kn[c][d]);
            const double Tf = g.Tk[d >> 1] * Kf;
            dg += Tf;
            Ap += Tf * (hp[c] - hn[c][d]);
            b += g.A[d >> 1] * Kf * gdot(g, d);
        }
        if (act[c] && k > 0) {
            const double Kf = 0.5 * (Kp[c] + Kd[c]);
            const double Tf = g.Tk[2] * Kf;
            dg += Tf;
            Ap += Tf * (hp[c] - hd[c]);
            b += g.A[2] * Kf * gz[0];
        }
        if (act[c] && k + 1 < kt) {
            const double Kf = 0.5 * (Kp[c] + Ku[c]);
            tu = g.Tk[2] * Kf;
            dg += tu;
            Ap += tu * (hp[c] - hu[c]);
            b += g.A[2] * Kf * gz[1];
        }
        diag[c] = dg;
        tup[c] = tu;
        r[c] = act[c] ? b - Ap : 0.0;
        rs[c] = (T)r[c];
        if (act[c]) {
            const size_t i = i0 + c;
            if (bout) bout[i] = b;
            cv.r[i] = rs[c];
            if (keep_diag) cv.diag[i] = (T)dg;
            if (kCopyKD) {
                cv.K[i] = (T)Kp[c];
                cv.Dd[i] = (T)Dp[c];
            }
            if (PRECOND == RF_PRECOND_JACOBI) v[0] += (double)rs[c] * (double)(rs[c] / (T)dg);
        }
    }
    v[1] = max_ratio_pair<double>(v[1], r[0], diag[0], act[0], r[1], diag[1], act[1]);
    if (PRECOND == RF_PRECOND_ZLINE) {
        double tzv[2], rdp[2];
        if (refactor) {
            // leading minors P_k = diag_k P_{k-1} - t_{k-1}^2 P_{k-2}: the lane's
            // two-cell matrix, scanned over the half, then the lower lane's
            // prefix (P_{k0-1}, P_{k0-2}) carried through the lane's cells
            const double tb = from_below0(tup[1]);
            const double q0 = act[0] ? tb * tb : 0.0, q1 = act[1] ? tup[0] * tup[0] : 0.0;
            double m00 = diag[1] * diag[0] - q1, m01 = -(diag[1] * q0), m10 = diag[0], m11 = -q0;
            rescale4(m00, m01, m10, m11);
            scan_matrix_up_half(m00, m01, m10, m11);
            double u0 = from_below0(m00), u1 = from_below0(m10);
            if ((lane & 31) == 0) {
                u0 = 1.0;
                u1 = 0.0;
            }
            const double P0 = diag[0] * u0 - q0 * u1;
            const double P1 = diag[1] * P0 - q1 * u0;
            // 1/d_k = P_{k-1} / P_k for both cells from one division, with
            // P_c = 2^-s_c p_c, p_c in [1, 2) (exact scalings: no product of
            // two minors can over- or underflow)
            const int s0 = 1 - frexp_exponent(P0), s1 = 1 - frexp_exponent(P1);
            const double p0 = ldexp(P0, s0), p1 = ldexp(P1, s1);
            const double inv = 1.0 / (p0 * p1);
            rdp[0] = act[0] ? ldexp(u0 * p1 * inv, s0) : 0.0;        // u0 / P0
            rdp[1] = act[1] ? ldexp(p0 * p0 * inv, s1 - s0) : 0.0;   // P0 / P1
            tzv[0] = tup[0];
            tzv[1] = tup[1];
        } else {
#pragma unroll
            for (int c = 0; c < 2; c++) {
                tzv[c] = act[c] ? tzs[c] : 0.0;
                rdp[c] = act[c] ? rds[c] : 0.0;
            }
        }
        double z[2];
        zline_solve_pair<double>(r, rdp, tzv, lane, z);
#pragma unroll
        for (int c = 0; c < 2; c++) {
            if (!act[c]) continue;
            const size_t i = i0 + c;
            const T zs = (T)z[c];
            if (refactor) {
                cv.tz[i] = (T)tup[c];
                cv.rdp[i] = (T)rdp[c];
            }
            cv.z[i] = zs;
            v[0] += (double)rs[c] * (double)zs;
        }
    }
}

// The residual kernel's PCG start (every kernel of the solve reads them):
// written by the lead thread only.
__device__ __forceinline__ void resid_reset_scalars(Scalars *s, int m)
{
    s->rho[0] = 0.0;
    s->rho[1] = 1.0;
    s->resmax = 0.0;
    s->pq = 0.0;
    s->iters = 0;
    s->jcur = 0;
    s->done = 0;
    s->fail = 0;
    s->final_iters = 0;
    s->cur_m = m;
}

// Adds the interior faces: diag = Dd + sum T_f, b = bst + sum A_f K_f g.n_f
// with K_f = (K_P + K_N)/2 and T_f = A_f K_f / d_f; r = b - A h^m (the
// right-hand side of the increment system A e = r, e0 = 0; e itself is
// written by the first spmv kernel that adds to it).  Jacobi: z = r / diag.
// z-line: t_k (vertical couplings) and reciprocal pivots of each column
// (refactor = 1), or those stored by the step's first Picard iteration
// (refactor = 0), and z = M^-1 r with them.  Block partials of (r.z,
// max|r/diag|).
// Everything is computed in FP64; the PCG arrays v receive it in the
// precision T of the solve (FP32 copies of K and Dd as well when T is float).
template <int PRECOND, typename T>
__global__ void __launch_bounds__(kThreads) k_resid(Geo g, Arrays a, CgVec<T> cv, int m, double *bout,
                                                    int refactor)
{
    constexpr bool kCopyKD = !std::is_same<T, double>::value;
    Scalars *s = a.sc;
    if (s->fail || s->stall || s->picard_done) return;
    const double *hmv = (m == 0) ? a.h0m : (m & 1) ? a.hb1 : a.hb0;
    int cb, ce;
    block_columns(g, g.cpb, cb, ce);
    RF_WAVE_IDS;
    double v[2] = {0.0, 0.0};
    if (g.nz <= kWave) {
        // short columns, two at a time (resid_pair): column c0 + 8 h in
        // half-wave h, cells k0 and k0 + 1 in each lane.  K and h^m at the
        // cells and their lateral neighbours are gathered first; a cell at or
        // above its column's top reads a cell of its own column (valid
        // memory, masked afterwards); vertical neighbours come from the
        // adjacent lanes
        const int half = lane >> 5, k0 = 2 * (lane & 31);
        const size_t sx = (size_t)g.nz, sy = (size_t)g.nz * g.nx;
        for (int c0 = cb + w; c0 < ce; c0 += kWavesPerBlock * 2) {
            const int cq = c0 + half * kWavesPerBlock;
            const int col = (cq < ce) ? cq : c0;
            const int kcol = a.ktop[col];
            const int kt = (cq < ce) ? kcol : 0;
            const size_t base = (size_t)col * g.nz;
            const int ci = col % g.nx, cj = col / g.nx;
            const bool has[4] = {ci > 0, ci < g.nx - 1, cj > 0, cj < g.ny - 1};
            const int cn[4] = {has[0] ? col - 1 : col, has[1] ? col + 1 : col,
                               has[2] ? col - g.nx : col, has[3] ? col + g.nx : col};
            int ktn[4];
#pragma unroll
            for (int d = 0; d < 4; d++) ktn[d] = a.ktop[cn[d]];
            double Kp[2], hp[2], Dp[2], bp[2], Kn[2][4], hn[2][4], tzs[2], rds[2];
            bool nb[2][4];
#pragma unroll
            for (int c = 0; c < 2; c++) {
                const int k = k0 + c;
                const size_t i = base + min(k, g.nz - 1);
                Kp[c] = a.K[i];
                hp[c] = hmv[i];
                Dp[c] = a.Dd[i];
                bp[c] = a.bst[i];
                tzs[c] = rds[c] = 0.0;
                if (PRECOND == RF_PRECOND_ZLINE && !refactor) {
                    tzs[c] = (double)cv.tz[i];
                    rds[c] = (double)cv.rdp[i];
                }
#pragma unroll
                for (int d = 0; d < 4; d++) {
                    const size_t off = (d < 2) ? sx : sy;
                    const size_t in = has[d] ? ((d & 1) ? i + off : i - off) : i;
                    nb[c][d] = (k < kt) & has[d] & (k < ktn[d]);   // no short-circuit branches
                    Kn[c][d] = a.K[in];
                    hn[c][d] = hmv[in];
                }
            }
            resid_pair<PRECOND, T>(g, cv, bout, refactor, kt, base + k0, k0, lane, Kp, hp, Dp, bp,
                                   Kn, hn, nb, tzs, rds, v);
        }
    } else
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        const size_t base = (size_t)col * g.nz;
        // carries between chunks of a long column (z-line only)
        double t_carry = 0.0, d_carry = 0.0, w_carry = 0.0;
        double r = 0.0, tup = 0.0, tzv = 0.0, rdp = 0.0, wk = 0.0;
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            const bool act = k < kt;
            double diag = 1.0;
            r = 0.0;
            tup = 0.0;
            if (act) {
                Cell c;
                cell_setup(g, a.ktop, col, kt, k, c);
                const double Kp = a.K[c.idx], hp = hmv[c.idx];
                diag = a.Dd[c.idx];
                double Ap = diag * hp, b = a.bst[c.idx];
#pragma unroll
                for (int d = 0; d < 6; d++) {
                    if (!c.nb[d]) continue;
                    const double Kf = 0.5 * (Kp + a.K[c.off[d]]);
                    const double Tf = g.Tk[d >> 1] * Kf;
                    diag += Tf;
                    Ap += Tf * (hp - hmv[c.off[d]]);
                    b += g.A[d >> 1] * Kf * gdot(g, d);
                    if (d == 5) tup = Tf;
                }
                r = b - Ap;
                if (bout) bout[c.idx] = b;
                cv.r[c.idx] = (T)r;
                cv.diag[c.idx] = (T)diag;
                if (kCopyKD) {
                    cv.K[c.idx] = (T)Kp;
                    cv.Dd[c.idx] = (T)a.Dd[c.idx];
                }
                v[1] = fmax(v[1], fabs(r / diag));
                if (PRECOND == RF_PRECOND_JACOBI) v[0] += (double)(T)r * (double)((T)r / (T)diag);
            }
            if (PRECOND == RF_PRECOND_ZLINE) {
                // couplings and pivots of the column tridiagonal, in registers,
                // or the stored ones of the step's first iteration
                if (refactor) {
                    const double tprev = from_below(tup, t_carry);
                    const double dpiv = scan_pivots(act ? diag : 1.0, act ? tprev * tprev : 0.0,
                                                    d_carry, lane);
                    rdp = act ? 1.0 / dpiv : 0.0;
                    d_carry = lane_value<kWave - 1>(dpiv);
                    tzv = tup;
                } else {
                    tzv = act ? (double)cv.tz[base + k] : 0.0;
                    rdp = act ? (double)cv.rdp[base + k] : 0.0;
                }
                const double tprev = from_below(tzv, t_carry);
                wk = scan_affine_up<double>(tprev * rdp, r * rdp, w_carry, lane);
                t_carry = lane_value<kWave - 1>(tzv);
                w_carry = lane_value<kWave - 1>(wk);
                if (act) {
                    if (refactor) {
                        cv.tz[base + k] = (T)tup;
                        cv.rdp[base + k] = (T)rdp;
                    }
                    if (kt > kWave) cv.z[base + k] = (T)wk;   // forward sweep, re-read by this lane
                }
            }
        }
        if (PRECOND == RF_PRECOND_ZLINE && kt > 0) {
            // backward sweep z_k = w_k + t_k rdp_k z_{k+1}
            if (kt <= kWave) {
                const bool act = lane < kt;
                const double zk = scan_affine_down<double>(act ? tzv * rdp : 0.0, act ? wk : 0.0,
                                                           0.0, lane);
                if (act) {
                    const T zs = (T)zk;
                    cv.z[base + lane] = zs;
                    v[0] += (double)(T)r * (double)zs;
                }
            } else {
                // backward sweep in the precision of the stored sweep values
                T carry = 0;
                for (int ch = (kt - 1) / kWave; ch >= 0; ch--) {
                    const int k = ch * kWave + lane;
                    const bool act = k < kt;
                    const T wv = act ? cv.z[base + k] : T(0);
                    const T bk = act ? cv.tz[base + k] * cv.rdp[base + k] : T(0);
                    const T zk = scan_affine_down<T>(bk, wv, carry, lane);
                    carry = lane_value<0>(zk);
                    if (act) {
                        cv.z[base + k] = zk;
                        v[0] += (double)cv.r[base + k] * (double)zk;
                    }
                }
            }
        }
    }
    block_partial<2, 2u>(v, a.pr);
    if (lead_thread()) resid_reset_scalars(s, m);
}

// The residual kernel with the lateral neighbours staged in LDS (columns of
// at most one wave; the tile layout of Tile<TY>, one tile per block).  Every
// wave reads K and h^m of its share of the tile's slots and Dd, bst of its
// own columns (masked by their active lengths), stages K and h^m in LDS, and
// forms its TY interior columns two at a time with resid_pair (one column
// per half-wave, two cells per lane), whose arithmetic per cell is that of
// k_resid.  The step flags are read first, alone (scalar loads),
// so that each block of a launch past the end of the step ends after that
// one round trip, with no vector load in flight; then the active lengths,
// so that no lane above its column's top loads anything.  Three
// blocks fit a CU (LDS and the register bound), which hides the latency of
// each block's two round trips better than fewer blocks walking several
// tiles (measured).  Writes the (r.z, max|r/diag|) block partials of nblk_t
// blocks into pr.
template <int PRECOND, typename T, int TY>
__global__ void __launch_bounds__(kThreads, 3) k_resid_tile(Geo g, Arrays a, CgVec<T> cv, int m,
                                                            double *bout, int refactor)
{
    using Tl = Tile<TY>;
    Scalars *s = a.sc;
    const int stop = s->fail | s->stall | s->picard_done;
    __shared__ double sH[Tl::NS][kWave];
    __shared__ double sK[Tl::NS][kWave];
    __shared__ int sKt[Tl::NS];
    const double *hmv = (m == 0) ? a.h0m : (m & 1) ? a.hb1 : a.hb0;
    if (stop) return;
    RF_WAVE_IDS;
    TileCols<TY, false> tc;
    using Sl = TileSlots<TY, false>;
    tc.fetch(g, a.ktop, blockIdx.x, w);
    static_assert(TY % 2 == 0, "columns are formed in pairs");
    constexpr int NP = TY / 2;
    // the lane's two cells in column h = lane >> 5 of each pair of own columns
    const int half = lane >> 5, k0 = 2 * (lane & 31);
    double K[Sl::PER], h[Sl::PER], Dp[NP][2], bp[NP][2], tzs[NP][2], rds[NP][2];
#pragma unroll
    for (int u = 0; u < Sl::PER; u++) {
        K[u] = 0.0;
        h[u] = 0.0;
        if (lane < tc.kt[u]) {
            const size_t i = (size_t)tc.col[u] * g.nz + lane;
            K[u] = a.K[i];
            h[u] = hmv[i];
        }
    }
    int okt[NP];
    size_t i0[NP];
#pragma unroll
    for (int p = 0; p < NP; p++) {
        const int oc = half ? tc.oc[2 * p + 1] : tc.oc[2 * p];
        okt[p] = half ? tc.okt[2 * p + 1] : tc.okt[2 * p];
        i0[p] = (size_t)(oc >= 0 ? oc : 0) * g.nz + k0;
#pragma unroll
        for (int c = 0; c < 2; c++) {
            Dp[p][c] = 0.0;
            bp[p][c] = 0.0;
            tzs[p][c] = 0.0;
            rds[p][c] = 0.0;
            if (k0 + c < okt[p]) {
                const size_t i = i0[p] + c;
                Dp[p][c] = a.Dd[i];
                bp[p][c] = a.bst[i];
                if (PRECOND == RF_PRECOND_ZLINE && !refactor) {
                    tzs[p][c] = (double)cv.tz[i];
                    rds[p][c] = (double)cv.rdp[i];
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < Sl::PER; u++) {
        const int sl = Sl::slot(w, u);
        if (sl >= Tl::NS) continue;
        if (lane < tc.kt[u]) {
            sK[sl][lane] = K[u];
            sH[sl][lane] = h[u];
        }
        if (lane == 0) sKt[sl] = tc.kt[u];
    }
    __syncthreads();
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int p = 0; p < NP; p++) {
        const int c0 = Tl::own(w, 2 * p + half);
        const int nbs[4] = {c0 - 1, c0 + 1, c0 - Tl::SX, c0 + Tl::SX};   // -x, +x, -y, +y
        int ktn[4];
#pragma unroll
        for (int d = 0; d < 4; d++) ktn[d] = sKt[nbs[d]];
        double Kp[2], hp[2], Kn[2][4], hn[2][4];
        bool nb[2][4];
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int k = k0 + c;
            const bool act = k < okt[p];
            Kp[c] = act ? sK[c0][k] : 0.0;
            hp[c] = act ? sH[c0][k] : 0.0;
#pragma unroll
            for (int d = 0; d < 4; d++) {
                nb[c][d] = act && k < ktn[d];
                Kn[c][d] = nb[c][d] ? sK[nbs[d]][k] : 0.0;
                hn[c][d] = nb[c][d] ? sH[nbs[d]][k] : 0.0;
            }
        }
        resid_pair<PRECOND, T>(g, cv, bout, refactor, okt[p], i0[p], k0, lane, Kp, hp, Dp[p],
                               bp[p], Kn, hn, nb, tzs[p], rds[p], v);
    }
    block_partial<2, 2u>(v, a.pr);
    if (lead_thread()) resid_reset_scalars(s, m);
}

// ---------------------------------------------------------------------------
// PCG iteration, kernel A: exit test, direction update, SpMV, p.q
// ---------------------------------------------------------------------------

template <int PRECOND, typename T>
__device__ __forceinline__ T pnew_at(const CgVec<T> &cv, size_t i, T beta, bool first, const T *p_in)
{
    const T z = (PRECOND == RF_PRECOND_JACOBI) ? cv.r[i] / cv.diag[i] : cv.z[i];
    return first ? z : z + beta * p_in[i];
}

// Combines the (r.z, max|r/diag|) partials of the last update and takes
// the exit decision of PCG iteration j (max|r/diag| <= tol, with tol =
// max(tol_cg, rel * the value at j = 0) fixed at j = 0).  Called by every
// thread; returns true when the solve goes on, with rho = r.z.
__device__ __forceinline__ bool spmv_continue(const Geo &g, const Arrays &a, Scalars *s, int j,
                                              double tol_cg, double rel, int max_cg, double &rho)
{
    double tot[2];
    reduce_partials<2, 2u>(a.pr + 2 * g.foff, g.np, tot);
    rho = tot[0];
    const double resmax = tot[1];
    const double tol = (j == 0) ? fmax(tol_cg, rel * resmax) : s->tol_eff;
    const bool bad = !isfinite(rho) || !isfinite(resmax);
    const bool done = bad || resmax <= tol || j >= max_cg;
    if (lead_thread()) {
        s->rho[j & 1] = rho;
        s->resmax = resmax;
        s->jcur = j;
        if (j == 0) s->tol_eff = tol;
        if (done) {
            s->done = 1;
            s->final_iters = j;
            if (bad) s->fail = 3;
            else if (resmax > tol) s->fail = 2;
        }
    }
    return !done;
}

// Values of G columns of one wave (and of their lateral neighbours) read by
// the spmv kernel.  Every load is unconditional (first iteration: the old
// direction is read but not used), so all are in flight at once.
template <int PRECOND, typename T, int G>
struct SpmvGroup {
    ColSlot cs[G];
    bool nb[G][4];
    T K[G], D[G], z[G], p[G], e[G], Kn[G][4], zn[G][4], pn[G][4];

    // with_e: also the PCG iterate e at the columns' cells (to add alpha p_old;
    // before the second step e is 0 and is not read)
    __device__ __forceinline__ void load(const Geo &g, const Arrays &a, const CgVec<T> &cv,
                                         const T *__restrict__ p_in, int c0, int ce, bool with_e,
                                         int lane)
    {
        size_t in[G][4];
#pragma unroll
        for (int u = 0; u < G; u++) {
            cs[u] = col_slot(g, a.ktop, c0 + u * kWavesPerBlock, ce, lane);
            lateral(g, a.ktop, cs[u], lane, nb[u], in[u]);
        }
#pragma unroll
        for (int u = 0; u < G; u++) {
            const size_t i = cs[u].i;
            K[u] = cv.K[i];
            D[u] = cv.Dd[i];
            z[u] = (PRECOND == RF_PRECOND_JACOBI) ? cv.r[i] / cv.diag[i] : cv.z[i];
            p[u] = p_in[i];
            e[u] = with_e ? cv.e[i] : T(0);
#pragma unroll
            for (int d = 0; d < 4; d++) {
                const size_t jn = in[u][d];
                Kn[u][d] = cv.K[jn];
                zn[u][d] = (PRECOND == RF_PRECOND_JACOBI) ? cv.r[jn] / cv.diag[jn] : cv.z[jn];
                pn[u][d] = p_in[jn];
            }
        }
    }
};

// Starts PCG iteration j = (updates done so far).  Every block combines the
// (r.z, max|r/diag|) partials of the last update and takes the same exit
// decision (spmv_continue); otherwise p = z + beta p_old (z = M^-1 r) at the
// cell and its neighbours, q = A p with A = Dd + sum_f T_f (I - shift_f)
// rebuilt from (K, Dd), and the last update's step on the iterate, e +=
// alpha_{j-1} p_old (p_old is read anyway; the solve's last such step is
// k_apply_h's); writes p, q, e and the block partials of p.q.  Vector
// arithmetic in T, reductions and the scalars rho, beta in FP64.  The
// direction buffers alternate: parity 0 reads p0 and writes p1.
template <int PRECOND, typename T>
__global__ void __launch_bounds__(kThreads) k_spmv(Geo g, Arrays a, CgVec<T> cv, int parity,
                                                   double tol_cg, double rel, int max_cg)
{
    Scalars *s = a.sc;
    if (s->done || s->fail || s->stall || s->picard_done) return;
    const int j = s->iters;
    const T alpha_prev = (T)s->alpha;     // alpha_{j-1}: e += alpha_{j-1} p_{j-1} here
    const T *__restrict__ p_in = parity ? cv.p1 : cv.p0;
    T *__restrict__ p_out = parity ? cv.p0 : cv.p1;
    const bool first = (j == 0);
    int cb, ce;
    block_columns(g, g.cpb, cb, ce);
    RF_WAVE_IDS;
    const T tz2 = (T)(0.5 * g.Tk[2]);
    const T tx2[2] = {(T)(0.5 * g.Tk[0]), (T)(0.5 * g.Tk[1])};
    double v[1] = {0.0};
    double rho;
    if (g.nz <= kWave) {
        // p_new = z + beta p_old and K at the cell and its lateral
        // neighbours for G2 columns, then the stencil; the vertical
        // neighbours come from the adjacent lanes.  FP64: one column at a
        // time (70 VGPRs, so more waves are resident on large grids; two
        // took 126); FP32: two, whose loads interleave
        constexpr int G2 = std::is_same<T, double>::value ? 1 : 2;
        // FP64: the first group's loads are in flight while the partials are
        // combined (2 % on this kernel; with FP32's two columns it was slower)
        constexpr bool kAhead = std::is_same<T, double>::value;
        SpmvGroup<PRECOND, T, G2> gr;
        if (kAhead && cb + w < ce) gr.load(g, a, cv, p_in, cb + w, ce, j >= 2, lane);
        if (!spmv_continue(g, a, s, j, tol_cg, rel, max_cg, rho)) return;
        if (lead_thread()) s->plast = parity ? 0 : 1;
        const T beta = first ? T(0) : (T)(rho / s->rho[(j + 1) & 1]);
        for (int c0 = cb + w; c0 < ce; c0 += kWavesPerBlock * G2) {
            if (!kAhead || c0 != cb + w) gr.load(g, a, cv, p_in, c0, ce, j >= 2, lane);
            T pp[G2], pn[G2][4];
#pragma unroll
            for (int u = 0; u < G2; u++) {
                pp[u] = first ? gr.z[u] : gr.z[u] + beta * gr.p[u];
#pragma unroll
                for (int d = 0; d < 4; d++) pn[u][d] = first ? gr.zn[u][d] : gr.zn[u][d] + beta * gr.pn[u][d];
            }
#pragma unroll
            for (int u = 0; u < G2; u++) {
                const int kt = gr.cs[u].kt;
                const T Kp = gr.K[u];
                const T Kd = from_below0(Kp), pdn = from_below0(pp[u]);
                const T Ku = from_above0(Kp), pup = from_above0(pp[u]);
                if (!gr.cs[u].act) continue;
                T q = gr.D[u] * pp[u];
#pragma unroll
                for (int d = 0; d < 4; d++)
                    if (gr.nb[u][d]) q += tx2[d >> 1] * (Kp + gr.Kn[u][d]) * (pp[u] - pn[u][d]);
                if (lane > 0) q += tz2 * (Kp + Kd) * (pp[u] - pdn);
                if (lane + 1 < kt) q += tz2 * (Kp + Ku) * (pp[u] - pup);
                p_out[gr.cs[u].i] = pp[u];
                cv.q[gr.cs[u].i] = q;
                if (!first) cv.e[gr.cs[u].i] = gr.e[u] + alpha_prev * gr.p[u];
                v[0] += (double)pp[u] * (double)q;
            }
        }
        block_partial<1, 0u>(v, a.pq);
        return;
    }
    if (!spmv_continue(g, a, s, j, tol_cg, rel, max_cg, rho)) return;
    if (lead_thread()) s->plast = parity ? 0 : 1;
    const T beta = first ? T(0) : (T)(rho / s->rho[(j + 1) & 1]);
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            Cell c;
            cell_setup(g, a.ktop, col, kt, k, c);
            const T Kp = cv.K[c.idx];
            const T pp = pnew_at<PRECOND, T>(cv, c.idx, beta, first, p_in);
            if (j == 1) cv.e[c.idx] = alpha_prev * p_in[c.idx];      // e was 0
            else if (j >= 2) cv.e[c.idx] += alpha_prev * p_in[c.idx];
            T q = cv.Dd[c.idx] * pp;
#pragma unroll
            for (int d = 0; d < 6; d++) {
                if (!c.nb[d]) continue;
                const T tf = (d < 4) ? tx2[d >> 1] : tz2;
                q += tf * (Kp + cv.K[c.off[d]]) * (pp - pnew_at<PRECOND, T>(cv, c.off[d], beta, first, p_in));
            }
            p_out[c.idx] = pp;
            cv.q[c.idx] = q;
            v[0] += (double)pp * (double)q;
        }
    }
    block_partial<1, 0u>(v, a.pq);
}

// The exit decision of PCG iteration j from the combined (r.z, max|r/diag|)
// totals, as spmv_continue takes it; tol_prev is the solve's tolerance read
// from the scalars (used for j > 0).  Returns true when the solve goes on.
__device__ __forceinline__ bool spmv_decide(Scalars *s, int j, const double (&tot)[2],
                                            double tol_prev, double tol_cg, double rel, int max_cg)
{
    const double rho = tot[0], resmax = tot[1];
    const double tol = (j == 0) ? fmax(tol_cg, rel * resmax) : tol_prev;
    const bool bad = !isfinite(rho) || !isfinite(resmax);
    const bool done = bad || resmax <= tol || j >= max_cg;
    if (lead_thread()) {
        s->rho[j & 1] = rho;
        s->resmax = resmax;
        s->jcur = j;
        if (j == 0) s->tol_eff = tol;
        if (done) {
            s->done = 1;
            s->final_iters = j;
            if (bad) s->fail = 3;
            else if (resmax > tol) s->fail = 2;
        }
    }
    return !done;
}

// The same PCG step with the lateral neighbours staged in LDS (columns of at
// most one wave; the tile layout of Tile<TY>, one tile per block).  The tile
// and its one-column halo are read once into LDS as p_new = z + beta p_old
// and K, every wave reading a share of the slots with the loads of all its
// slots in flight together.  The step flags, the iteration count, the rho
// slots and the solve's tolerance are read first, alone (scalar loads): each
// block of a launch past the end of the solve (marked finished by the fold
// after the last update) ends after that one round trip, with no vector load
// in flight.  Then the active lengths and this thread's share of the last
// update's partials, so that no lane above its column's top loads anything.
// Wave w forms q = A p for its TY interior columns from LDS, and e +=
// alpha_{j-1} p_old at them, with the arithmetic per cell of k_spmv.  Three
// blocks fit a CU.  Writes p, q, e and the block partials of p.q (nblk_t
// blocks).
template <int PRECOND, typename T, int TY>
__global__ void __launch_bounds__(kThreads, 3) k_spmv_tile(Geo g, Arrays a, CgVec<T> cv, int parity,
                                                           double tol_cg, double rel, int max_cg)
{
    using Tl = Tile<TY>;
    Scalars *s = a.sc;
    const int stop = s->done | s->fail | s->stall | s->picard_done;
    const int j = s->iters;
    const double rho_slot[2] = {s->rho[0], s->rho[1]};
    const double tol_prev = s->tol_eff;
    const T alpha_prev = (T)s->alpha;     // alpha_{j-1}: e += alpha_{j-1} p_{j-1} here
    __shared__ T sP[Tl::NS][kWave];
    __shared__ T sK[Tl::NS][kWave];
    __shared__ int sKt[Tl::NS];
    const T *__restrict__ p_in = parity ? cv.p1 : cv.p0;
    T *__restrict__ p_out = parity ? cv.p0 : cv.p1;
    if (stop) return;
    RF_WAVE_IDS;
    TileCols<TY, true> tc;
    using Sl = TileSlots<TY, true>;
    tc.fetch(g, a.ktop, blockIdx.x, w);
    double pv[2];
    gather_partials<2, 2u>(a.pr + 2 * g.foff, g.np, pv);
    const bool first = (j == 0);
    T z[Sl::PER], po[Sl::PER], K[Sl::PER], Dd[TY], eo[TY], pw[TY];
#pragma unroll
    for (int u = 0; u < Sl::PER; u++) {
        z[u] = T(0);
        po[u] = T(0);
        K[u] = T(0);
        if (lane < tc.kt[u]) {
            const size_t i = (size_t)tc.col[u] * g.nz + lane;
            z[u] = (PRECOND == RF_PRECOND_JACOBI) ? cv.r[i] / cv.diag[i] : cv.z[i];
            po[u] = p_in[i];
            K[u] = cv.K[i];
        }
    }
#pragma unroll
    for (int t = 0; t < TY; t++) {
        Dd[t] = eo[t] = T(0);
        pw[t] = po[t];                          // own column t is the wave's slot t
        if (lane < tc.okt[t]) {
            const size_t i = (size_t)tc.oc[t] * g.nz + lane;
            Dd[t] = cv.Dd[i];
            if (j >= 2) eo[t] = cv.e[i];        // (e is 0 before the first step)
        }
    }
    double tot[2];
    combine_partials<2, 2u>(pv, tot);
    if (!spmv_decide(s, j, tot, tol_prev, tol_cg, rel, max_cg)) return;
    if (lead_thread()) s->plast = parity ? 0 : 1;
    const T beta = first ? T(0) : (T)(tot[0] / rho_slot[(j + 1) & 1]);
#pragma unroll
    for (int u = 0; u < Sl::PER; u++) {
        const int sl = Sl::slot(w, u);
        if (sl >= Tl::NS) continue;
        if (lane < tc.kt[u]) {
            sP[sl][lane] = first ? z[u] : z[u] + beta * po[u];
            sK[sl][lane] = K[u];
        }
        if (lane == 0) sKt[sl] = tc.kt[u];
    }
    __syncthreads();
    const T tz2 = (T)(0.5 * g.Tk[2]);
    const T tx2[2] = {(T)(0.5 * g.Tk[0]), (T)(0.5 * g.Tk[1])};
    double v[1] = {0.0};
#pragma unroll
    for (int t = 0; t < TY; t++) {
        const int c = Tl::own(w, t);
        const int nbs[4] = {c - 1, c + 1, c - Tl::SX, c + Tl::SX};   // -x, +x, -y, +y
        const bool act = lane < tc.okt[t];
        const T pp = act ? sP[c][lane] : T(0);
        const T Kp = act ? sK[c][lane] : T(0);
        const T Kd = from_below0(Kp), pdn = from_below0(pp);
        const T Ku = from_above0(Kp), pup = from_above0(pp);
        T q = Dd[t] * pp;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const bool nb = act && lane < sKt[nbs[d]];
            if (nb) q += tx2[d >> 1] * (Kp + sK[nbs[d]][lane]) * (pp - sP[nbs[d]][lane]);
        }
        if (act && lane > 0) q += tz2 * (Kp + Kd) * (pp - pdn);
        if (act && lane + 1 < tc.okt[t]) q += tz2 * (Kp + Ku) * (pp - pup);
        if (act) {
            const size_t i = (size_t)tc.oc[t] * g.nz + lane;
            p_out[i] = pp;
            cv.q[i] = q;
            if (!first) cv.e[i] = eo[t] + alpha_prev * pw[t];
            v[0] += (double)pp * (double)q;
        }
    }
    block_partial<1, 0u>(v, a.pq);
}

// ---------------------------------------------------------------------------
// PCG iteration, kernel B: e += alpha p, r -= alpha q, z = M^-1 r, r.z
// ---------------------------------------------------------------------------

// Combines the p.q partials of the spmv kernel: alpha = rho_j / p.q, or a
// breakdown (p.q not positive or not finite) that ends the solve.  Called
// by every thread; returns false on breakdown.
__device__ __forceinline__ bool update_alpha(const Geo &g, const Arrays &a, Scalars *s, int j,
                                             double &alpha)
{
    double tot[1];
    reduce_partials<1, 0u>(a.pq + g.foff, g.np, tot);
    const double pq = tot[0];
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (lead_thread()) {
            s->pq = pq;
            s->fail = 1;
            s->done = 1;
            s->final_iters = j;
        }
        return false;
    }
    alpha = s->rho[j & 1] / pq;
    if (lead_thread()) {
        s->pq = pq;
        s->alpha = alpha;
        s->iters = j + 1;
    }
    return true;
}


// alpha = rho_j / pq from the combined p.q total, or a breakdown (p.q not
// positive or not finite) that ends the solve; rho_j is read by the caller
// beforehand.  Called by every thread; returns false on breakdown.
__device__ __forceinline__ bool update_decide(Scalars *s, int j, double pq, double rho_j,
                                              double &alpha)
{
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (lead_thread()) {
            s->pq = pq;
            s->fail = 1;
            s->done = 1;
            s->final_iters = j;
        }
        return false;
    }
    alpha = rho_j / pq;
    if (lead_thread()) {
        s->pq = pq;
        s->alpha = alpha;
        s->iters = j + 1;
    }
    return true;
}

// Columns of one group of a wave (G columns, 8 apart) and their active
// lengths: wave-uniform, fetched by scalar loads ahead of the group's data so
// that the data loads can be masked without waiting for them.
template <int G>
struct GroupCols {
    int col[G], kt[G];

    __device__ __forceinline__ void fetch(const int32_t *__restrict__ ktop, int c0, int ce)
    {
#pragma unroll
        for (int u = 0; u < G; u++) {
            const int c = c0 + u * kWavesPerBlock;
            col[u] = (c < ce) ? c : -1;
            kt[u] = (c < ce) ? ktop[c] : 0;
        }
    }
};

// Values the update kernel reads for a group of two columns, one per
// half-wave, two cells per lane (cells k0 = 2 (lane & 31) and k0 + 1),
// loaded by the lanes below each column's active length only: r, q, the
// z-line factors (z-line) and the diagonal, unless it is rebuilt from the
// factors (rebuild: the factors are this iteration's).
template <int PRECOND, typename T>
struct UpdPair {
    int kt;
    size_t i0;
    T r[2], q[2], d[2], rd[2], t[2];

    __device__ __forceinline__ void load(const Geo &g, const CgVec<T> &cv, const GroupCols<2> &gc,
                                         bool rebuild, int lane)
    {
        const int half = lane >> 5, k0 = 2 * (lane & 31);
        const int col = half ? gc.col[1] : gc.col[0];
        kt = half ? gc.kt[1] : gc.kt[0];
        i0 = (size_t)(col >= 0 ? col : 0) * g.nz + k0;
#pragma unroll
        for (int c = 0; c < 2; c++) {
            r[c] = q[c] = rd[c] = t[c] = T(0);
            d[c] = T(1);
            if (k0 + c < kt) {
                const size_t i = i0 + c;
                r[c] = cv.r[i];
                q[c] = cv.q[i];
                if (PRECOND == RF_PRECOND_ZLINE) {
                    rd[c] = cv.rdp[i];
                    t[c] = cv.tz[i];
                }
                if (PRECOND != RF_PRECOND_ZLINE || !rebuild) d[c] = cv.diag[i];
            }
        }
    }
};

// alpha = rho_j / p.q (every block combines the p.q partials; kept in the
// scalars for e += alpha p, which the next spmv kernel applies since it reads
// p anyway, or k_apply_h after the solve's last update); r -= alpha q, z =
// M^-1 r; block partials of (r.z, max|r/diag|).  With the z-line
// preconditioner factored from this iteration's matrix (rebuild), diag is
// rebuilt from the column's pivots d_k = a_k - t_{k-1}^2 / d_{k-1} (rdp =
// 1/d): a_k = 1/rdp_k + t_{k-1}^2 rdp_{k-1}, both terms positive, no
// cancellation; so the kernel reads r, q, rdp, tz and writes r, z.  Short
// columns: two at a time, one per half-wave, two cells per lane
// (zline_solve_pair); the loads of a wave's first group of columns are
// issued before the partials are combined, so the two are in flight
// together, and each further group is loaded while the one before it is
// computed.
template <int PRECOND, typename T>
__global__ void __launch_bounds__(kThreads) k_update(Geo g, Arrays a, CgVec<T> cv, int parity,
                                                     int rebuild)
{
    (void)parity;
    Scalars *s = a.sc;
    int cb, ce;
    block_columns(g, g.cpb, cb, ce);
    RF_WAVE_IDS;
    double v[2] = {0.0, 0.0};
    double alpha_d;
    if (g.nz <= kWave) {
        // short columns: two groups of G columns in turn, the next group's
        // loads in flight while the current one is computed, and the active
        // lengths of the group after it fetched with them; the step flags,
        // rho, the iteration index, the first two groups' active lengths and
        // this thread's share of the p.q partials are read in one round trip
        constexpr int G = 2;
        constexpr int step = kWavesPerBlock * G;
        const int stop = s->done | s->fail | s->stall | s->picard_done;
        const int j = s->jcur;
        const double rho_slot[2] = {s->rho[0], s->rho[1]};
        GroupCols<G> ka, kb;
        ka.fetch(a.ktop, cb + w, ce);
        kb.fetch(a.ktop, cb + w + step, ce);
        double pv[1];
        gather_partials<1, 0u>(a.pq + g.foff, g.np, pv);
        if (stop) return;
        UpdPair<PRECOND, T> ga, gb;
        ga.load(g, cv, ka, rebuild, lane);
        double tot[1];
        combine_partials<1, 0u>(pv, tot);
        if (!update_decide(s, j, tot[0], rho_slot[j & 1], alpha_d)) return;
        const T alpha = (T)alpha_d;
        T *__restrict__ rv = cv.r;
        T *__restrict__ zv = cv.z;
        const int k0 = 2 * (lane & 31);
        auto work = [&](const UpdPair<PRECOND, T> &gr) {
            bool act[2];
            T r[2], dg[2], rd[2], t[2];
#pragma unroll
            for (int c = 0; c < 2; c++) {
                act[c] = k0 + c < gr.kt;
                r[c] = act[c] ? gr.r[c] - alpha * gr.q[c] : T(0);
                rd[c] = act[c] ? gr.rd[c] : T(0);
                t[c] = act[c] ? gr.t[c] : T(0);
                dg[c] = gr.d[c];
            }
            if (PRECOND == RF_PRECOND_ZLINE && rebuild) {
                // a_k = 1/rdp_k + t_{k-1}^2 rdp_{k-1}; the first cell's lower
                // neighbour is the lower lane's second cell
                const T r0 = act[0] ? gr.rd[0] : T(1), r1 = act[1] ? gr.rd[1] : T(1);
                const T rb = from_below0<T>(r1), tb = from_below0<T>(gr.t[1]);
                // 1/r0 and 1/r1 from one division, with r_c = 2^-e_c s_c,
                // s_c in [1, 2) (exact scalings: no overflow of r0 r1 in FP32)
                const int e0 = 1 - frexp_exponent(r0), e1 = 1 - frexp_exponent(r1);
                const T s0 = ldexp(r0, e0), s1 = ldexp(r1, e1);
                const T inv = T(1) / (s0 * s1);
                dg[0] = ldexp(s1 * inv, e0) + tb * tb * rb;
                dg[1] = ldexp(s0 * inv, e1) + gr.t[0] * gr.t[0] * r0;
            }
#pragma unroll
            for (int c = 0; c < 2; c++) {
                if (!act[c]) continue;
                rv[gr.i0 + c] = r[c];
                if (PRECOND == RF_PRECOND_JACOBI) v[0] += (double)r[c] * (double)(r[c] / dg[c]);
            }
            v[1] = max_ratio_pair<T>(v[1], r[0], dg[0], act[0], r[1], dg[1], act[1]);
            if (PRECOND == RF_PRECOND_ZLINE) {
                T z[2];
                zline_solve_pair<T>(r, rd, t, lane, z);
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    if (!act[c]) continue;
                    zv[gr.i0 + c] = z[c];
                    v[0] += (double)r[c] * (double)z[c];
                }
            }
        };
        for (int c0 = cb + w; c0 < ce; c0 += 2 * step) {
            const bool more = c0 + step < ce;
            if (more) {
                gb.load(g, cv, kb, rebuild, lane);
                ka.fetch(a.ktop, c0 + 2 * step, ce);
            }
            work(ga);
            if (!more) break;
            if (c0 + 2 * step < ce) {
                ga.load(g, cv, ka, rebuild, lane);
                kb.fetch(a.ktop, c0 + 3 * step, ce);
            }
            work(gb);
        }
        block_partial<2, 2u>(v, a.pr);
        return;
    }
    if (s->done || s->fail || s->stall || s->picard_done) return;
    const int j = s->jcur;
    if (!update_alpha(g, a, s, j, alpha_d)) return;
    const T alpha = (T)alpha_d;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        const size_t base = (size_t)col * g.nz;
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            const size_t i = base + k;
            const T r = cv.r[i] - alpha * cv.q[i];
            cv.r[i] = r;
            const T dg = cv.diag[i];
            if (PRECOND == RF_PRECOND_JACOBI) v[0] += (double)r * (double)(r / dg);
            v[1] = fmax(v[1], (double)fabs(r / dg));
        }
        if (PRECOND == RF_PRECOND_ZLINE && kt > 0) {
            zline_solve_long<T>(cv.r, cv.rdp, cv.tz, cv.z, base, kt, lane);
            for (int k0 = 0; k0 < kt; k0 += kWave) {
                const int k = k0 + lane;
                if (k < kt) v[0] += (double)cv.r[base + k] * (double)cv.z[base + k];
            }
        }
    }
    block_partial<2, 2u>(v, a.pr);
}

// ---------------------------------------------------------------------------
// Picard update: h^{m+1} = h^m + e + alpha_{J-1} p_{J-1}
// ---------------------------------------------------------------------------

// Enqueued after a chunk of PCG iterations.  Every block combines the last
// (r.z, max|r/diag|) partials and decides, as the next direction update
// would, whether the solve has finished.  If not, the step stalls until the
// host enqueues more iterations; if so, the increment is e plus the last
// update's step alpha_{J-1} p_{J-1} (J updates done; every earlier step was
// added by the spmv kernel after it, and e holds them from J = 2 on; 0 for
// J = 0), hb[(m+1)&1] = hb[m&1] + that, and block
// partials of (max|increment|, non-finite count).  The increment is formed in
// the precision T of the solve; h stays FP64.  p0, p1: the direction buffers.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_apply_h(Geo g, Arrays a, const T *e_in, const T *p0,
                                                      const T *p1, int m, double tol_cg, double rel,
                                                      int max_cg)
{
    Scalars *s = a.sc;
    // the step flags, the solve's state, the first group's active lengths and
    // this thread's share of the last update's partials in one round trip;
    // short columns: the loads of the first group (masked by the active
    // lengths) are in flight while the partials are combined
    const int stop = s->fail | s->stall | s->picard_done;
    const int j = s->iters;
    const int sdone = s->done;
    const double tol_prev = s->tol_eff;
    const T alpha_last = (T)s->alpha;
    const int plast = s->plast;
    const double *__restrict__ hmv = (m == 0) ? a.h0m : (m & 1) ? a.hb1 : a.hb0;
    double *__restrict__ hnext = (m & 1) ? a.hb0 : a.hb1;
    const T *__restrict__ ev = e_in;
    // p_{J-1}: the buffer the last spmv kernel that went on wrote (none when J = 0)
    const T *__restrict__ pl = plast ? p1 : p0;
    const bool step_left = j > 0;
    int cb, ce;
    block_columns(g, g.cpb, cb, ce);
    RF_WAVE_IDS;
    GroupCols<kColGroup> kc;
    if (g.nz <= kWave) kc.fetch(a.ktop, cb + w, ce);
    double pv[2];
    gather_partials<2, 2u>(a.pr + 2 * g.foff, g.np, pv);
    if (stop) return;
    double e[kColGroup], hv[kColGroup];   // e widened to FP64
    auto load = [&]() {
#pragma unroll
        for (int u = 0; u < kColGroup; u++) {
            e[u] = 0.0;
            hv[u] = 0.0;
            if (lane < kc.kt[u]) {
                const size_t i = (size_t)kc.col[u] * g.nz + lane;
                const T et = (j >= 2) ? ev[i] + alpha_last * pl[i] : step_left ? alpha_last * pl[i] : T(0);
                e[u] = (double)et;
                hv[u] = hmv[i];
            }
        }
    };
    if (g.nz <= kWave) load();
    double tot[2];
    combine_partials<2, 2u>(pv, tot);
    // the exit tolerance of this solve (fixed by its first direction update)
    const double tol = (j == 0 && !sdone) ? fmax(tol_cg, rel * tot[1]) : tol_prev;
    const bool bad = !isfinite(tot[0]) || !isfinite(tot[1]);
    const bool finished = sdone || bad || !(tot[1] > tol) || j >= max_cg;
    if (!finished) {
        if (lead_thread()) {
            s->stall = 1;
            s->stall_m = m;
        }
        return;
    }
    if (!sdone && (bad || tot[1] > tol)) {
        if (lead_thread()) {   // the next direction update would stop with this status
            s->fail = bad ? 3 : 2;
            s->done = 1;
            s->final_iters = j;
        }
        return;
    }
    double v[2] = {0.0, 0.0};
    if (g.nz <= kWave) {
        for (int c0 = cb + w; c0 < ce; c0 += kWavesPerBlock * kColGroup) {
            if (c0 != cb + w) {
                kc.fetch(a.ktop, c0, ce);
                load();
            }
#pragma unroll
            for (int u = 0; u < kColGroup; u++) {
                if (lane >= kc.kt[u]) continue;
                const double h = hv[u] + e[u];
                hnext[(size_t)kc.col[u] * g.nz + lane] = h;
                v[0] = fmax(v[0], fabs(e[u]));
                if (!isfinite(h)) v[1] += 1.0;
            }
        }
    } else {
        for (int col = cb + w; col < ce; col += kWavesPerBlock) {
            const int kt = a.ktop[col];
            for (int k0 = 0; k0 < kt; k0 += kWave) {
                const int k = k0 + lane;
                if (k >= kt) continue;
                const size_t i = (size_t)col * g.nz + k;
                const T et = (j >= 2) ? ev[i] + alpha_last * pl[i] : step_left ? alpha_last * pl[i] : T(0);
                const double e = (double)et;
                const double h = hmv[i] + e;
                hnext[i] = h;
                v[0] = fmax(v[0], fabs(e));
                if (!isfinite(h)) v[1] += 1.0;
            }
        }
    }
    block_partial<2, 1u>(v, a.pd);
    if (lead_thread() && m < RF_MAX_PICARD_LOG) s->cg_log[m] = j;
}

// ---------------------------------------------------------------------------
// Step acceptance: h^n <- h^{m+1}, theta~^n, storage, face inflows
// ---------------------------------------------------------------------------

// Runs when the Picard exit test has passed (the flag comes from k_decide).
// TRACK: also dh = h^{n+1} - h^n for the extrapolated first iterate.
// Block partials (ps): [0] storage sum V theta~(h); [1+f] inflow rate through
// face f with h = h^{m+1} and K = K(h^m) (the converged system).
template <bool TRACK, int MODEL, bool FLAT>
__global__ void __launch_bounds__(kThreads, 4) k_accept(Geo g, Soil so, Arrays a, int serial)
{
    Scalars *s = a.sc;
    if (s->fail || s->stall || !s->picard_done) return;
    __shared__ Layer sL[RF_MAX_LAYERS];
    __shared__ FaceTab sBT[6];
    __shared__ double sKR[6 * RF_MAX_LAYERS];
    stage_bc(a, sBT, sKR);
    stage_layers(a, so.nlayer, sL);
    const int mf = s->picard_m;
    const double *hf = ((mf + 1) & 1) ? a.hb1 : a.hb0;
    RF_WAVE_IDS;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    // one run of kWave active cells per wavefront at a time
    const int qs = gridDim.x * kWavesPerBlock;
    int q = blockIdx.x * kWavesPerBlock + w;
    int4 rec_next = (q < g.nchunk) ? a.chunk[q] : int4{0, 0, 0, 0};
    for (; q < g.nchunk; q += qs) {
        // the next run's record is read while this run is evaluated
        const int4 rec = rec_next;
        if (q + qs < g.nchunk) rec_next = a.chunk[q + qs];
        const RunCell rc = run_cell(g, a.ktop, rec, q, lane);
        const size_t i = rc.i;
        const int ci = rc.col % g.nx, cj = rc.col / g.nx;
        const bool bnd[6] = {ci == 0, ci == g.nx - 1, cj == 0, cj == g.ny - 1, rc.k == 0, rc.top};
        // K and Ks enter only the inflow through domain faces
        const bool edge = bnd[0] || bnd[1] || bnd[2] || bnd[3] || bnd[4] || bnd[5];
        const double h = hf[i];
        const double K = edge ? a.K[i] : 0.0, ks = edge ? a.Ks[i] : 0.0;
        const int lay = a.layer ? a.layer[i] : 0;
        double ho = 0.0;
        if (TRACK) ho = a.hn[i];
        const double th = FLAT ? soil_theta_vgm_flat(h, sL[lay]) : soil_theta(MODEL, h, sL[lay]);
        if (!rc.act) continue;
        if (TRACK) a.dh[i] = h - ho;
        a.hn[i] = h;
        a.thn[i] = th;
        v[0] += g.V * th;
#pragma unroll
        for (int d = 0; d < 6; d++) {
            if (!bnd[d]) continue;
            const double Kb = ks * sKR[d * RF_MAX_LAYERS + lay];
            v[1 + d] += (sBT[d].cKb - sBT[d].cD * h) * Kb + sBT[d].cK * K + sBT[d].c0;
        }
    }
    block_partial<7, 0u>(v, a.ps);
    if (lead_thread()) {
        s->accepted = 1;
        s->accept_m = mf;
        s->accepted_serial = serial;
    }
}

// ---------------------------------------------------------------------------
// inspection kernels
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kThreads) k_eval_soil(Geo g, Soil so, Arrays a, const double *h,
                                                        double *theta, double *Cout, double *Kout)
{
    __shared__ Layer sL[RF_MAX_LAYERS];
    stage_layers(a, so.nlayer, sL);
    int cb, ce;
    block_columns(g, g.cpb_w, cb, ce);
    RF_WAVE_IDS;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k >= kt) continue;
            const size_t idx = (size_t)col * g.nz + k;
            const Layer &L = sL[a.layer ? a.layer[idx] : 0];
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
    block_columns(g, g.cpb_w, cb, ce);
    RF_WAVE_IDS;
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
    block_columns(g, g.cpb_w, cb, ce);
    RF_WAVE_IDS;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        const size_t base = (size_t)col * g.nz;
        if (PRECOND == RF_PRECOND_JACOBI) {
            for (int k0 = 0; k0 < kt; k0 += kWave) {
                const int k = k0 + lane;
                if (k < kt) z[base + k] = r[base + k] / a.diag[base + k];
            }
        } else if (kt > kWave) {
            zline_solve_long(r, a.rdp, a.tz, z, base, kt, lane);
        } else if (kt > 0) {
            const bool act = lane < kt;
            const double zk = zline_solve_short(act ? r[base + lane] : 0.0,
                                                act ? a.rdp[base + lane] : 0.0,
                                                act ? a.tz[base + lane] : 0.0, lane);
            if (act) z[base + lane] = zk;
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_copy_active(Geo g, Arrays a, const double *src, double *dst)
{
    int cb, ce;
    block_columns(g, g.cpb_w, cb, ce);
    RF_WAVE_IDS;
    for (int col = cb + w; col < ce; col += kWavesPerBlock) {
        const int kt = a.ktop[col];
        for (int k0 = 0; k0 < kt; k0 += kWave) {
            const int k = k0 + lane;
            if (k < kt) dst[(size_t)col * g.nz + k] = src[(size_t)col * g.nz + k];
        }
    }
}

// Combines the nblk partials of a producer into slot `out` (in values of NV).
// Zeroes n 32-bit words (a kernel rather than a memset, so that the work
// stays a kernel node when a caller captures the stream into a graph).
__global__ void __launch_bounds__(kThreads) k_zero(uint32_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kThreads)
        p[i] = 0u;
}

template <int NV, unsigned MAXMASK>
__global__ void __launch_bounds__(kThreads) k_fold(double *P, int nblk, int out)
{
    double tot[NV];
    reduce_partials<NV, MAXMASK>(P, nblk, tot);
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; i++) P[(size_t)out * NV + i] = tot[i];
}

// The fold of the (r.z, max|r/diag|) partials of a residual or update kernel
// (into the slot `out` the next spmv kernel reads) that also takes that spmv
// kernel's exit decision for PCG iteration j = iters (spmv_decide, with the
// same inputs, so the spmv kernel's own decision repeats it).  A solve that
// has converged is then marked finished before the spmv launch after its last
// iteration starts, and that launch stops at its first read of the flags
// instead of loading its tile.  Nothing is decided when the flags already
// stop the solve (a producer that returned early leaves them as they were).
__global__ void __launch_bounds__(kThreads) k_fold_decide(Arrays a, int nblk, int out, double tol_cg,
                                                          double rel, int max_cg)
{
    double tot[2];
    reduce_partials<2, 2u>(a.pr, nblk, tot);
    if (threadIdx.x == 0) {
        a.pr[(size_t)out * 2] = tot[0];
        a.pr[(size_t)out * 2 + 1] = tot[1];
        Scalars *s = a.sc;
        if (!(s->done | s->fail | s->stall | s->picard_done))
            (void)spmv_decide(s, s->iters, tot, s->tol_eff, tol_cg, rel, max_cg);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
}

void arm_launch_events(hipEvent_t start, hipEvent_t stop)
{
    t_ev_start = start;
    t_ev_stop = stop;
}

bool disarm_launch_events()
{
    const bool unused = t_ev_start != nullptr;
    t_ev_start = t_ev_stop = nullptr;
    return unused;
}

// A launch that takes armed events passes them to the extension launch, which
// stamps them with the kernel's own start and end.
#define RF_LAUNCH_N(nb, kern, ...)                                                      \
    do {                                                                                \
        if (t_ev_start) {                                                               \
            hipEvent_t a_ = t_ev_start, b_ = t_ev_stop;                                 \
            t_ev_start = t_ev_stop = nullptr;                                           \
            hipExtLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), 0, s, a_, b_, 0u,     \
                                  __VA_ARGS__);                                         \
        } else {                                                                        \
            hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), 0, s, __VA_ARGS__);      \
        }                                                                               \
        return hipGetLastError();                                                       \
    } while (0)
// reducing kernels (partials combined later) and wide kernels
#define RF_LAUNCH(kern, ...) RF_LAUNCH_N(g.nblk, kern, __VA_ARGS__)
#define RF_LAUNCH_W(kern, ...) RF_LAUNCH_N(g.nblk_w, kern, __VA_ARGS__)

hipError_t launch_init_ks(const Geo &g, const Soil &so, const Arrays &a, hipStream_t s)
{
    (void)so;
    RF_LAUNCH_W(k_init_ks, g, a);
}

#define RF_LAUNCH_FOLD(P, nv, mask, kern, ...)                                          \
    do {                                                                                \
        const hipError_t e_ = [&]() { RF_LAUNCH_N(g.nblk, kern, __VA_ARGS__); }();        \
        if (e_ != hipSuccess) return e_;                                                \
        return launch_fold(g, P, nv, mask, s);                                          \
    } while (0)

// A kernel over runs of active cells (nblk_r blocks) and the fold of its
// partials.
#define RF_LAUNCH_FOLD_R(P, nv, mask, kern, ...)                                        \
    do {                                                                                \
        const hipError_t e_ = [&]() { RF_LAUNCH_N(g.nblk_r, kern, __VA_ARGS__); }();      \
        if (e_ != hipSuccess) return e_;                                                \
        return launch_fold(g, P, nv, mask, s, g.nblk_r);                                \
    } while (0)

// A tiled kernel (nblk_t blocks) and the fold of its partials.
#define RF_LAUNCH_TILED(P, nv, mask, kern, ...)                                         \
    do {                                                                                \
        const hipError_t e_ = [&]() { RF_LAUNCH_N(g.nblk_t, kern, __VA_ARGS__); }();      \
        if (e_ != hipSuccess) return e_;                                                \
        return launch_fold(g, P, nv, mask, s, g.nblk_t);                                \
    } while (0)

// Folds the (r.z, max|r/diag|) partials of nprod blocks with the next spmv
// kernel's exit decision (k_fold_decide) when consumers read a folded total;
// otherwise the spmv kernel combines the partials and decides itself.
static hipError_t launch_fold_decide(const Geo &g, const Arrays &a, int nprod, const CgTol &t,
                                     hipStream_t s)
{
    if (g.np != 1 || g.foff == 0) return hipSuccess;
    RF_LAUNCH_N(1, k_fold_decide, a, nprod, g.foff, t.tol_cg, t.rel, t.max_cg);
}

// A kernel writing (r.z, max|r/diag|) partials into a.pr from nb blocks, and
// their fold with the decision; RF_LAUNCH_DECIDE_TILED for a tiled kernel.
#define RF_LAUNCH_DECIDE(nb, kern, ...)                                                 \
    do {                                                                                \
        const int nb_ = (nb);                                                           \
        const hipError_t e_ = [&]() { RF_LAUNCH_N(nb_, kern, __VA_ARGS__); }();           \
        if (e_ != hipSuccess) return e_;                                                \
        return launch_fold_decide(g, a, nb_, t, s);                                     \
    } while (0)
#define RF_LAUNCH_DECIDE_TILED(kern, ...) RF_LAUNCH_DECIDE(g.nblk_t, kern, __VA_ARGS__)

hipError_t launch_check_finite(const Geo &g, const Arrays &a, const double *h, hipStream_t s)
{
    RF_LAUNCH_FOLD(a.ps, 1, 0u, k_check_finite, g, a, h);
}

hipError_t launch_set_state(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            hipStream_t s)
{
    RF_LAUNCH_FOLD(a.ps, 1, 0u, k_set_state, g, so, a, h);
}

hipError_t launch_step_begin(const Geo &g, const Soil &so, const Bc &bc, const Arrays &a,
                             const double *h0, double ratio, int gate, hipStream_t s)
{
    if (!h0) RF_LAUNCH_N(1, k_step_begin, g, so, bc, a, h0, ratio, gate);
    RF_LAUNCH_W(k_step_begin, g, so, bc, a, h0, ratio, gate);
}

hipError_t launch_decide(const Geo &g, const Arrays &a, int m, double tol_picard, hipStream_t s)
{
    RF_LAUNCH_N(1, k_decide, g, a, m, tol_picard);
}

hipError_t launch_coeff(const Geo &g, const Soil &so, const Arrays &a, int m, double dt,
                        double chord_eps, int variant, hipStream_t s)
{
    if (so.model == RF_GARDNER)
        RF_LAUNCH_N(g.nblk_r, (k_coeff<RF_GARDNER, false>), g, so, a, m, dt, chord_eps, variant);
    // branch-free van Genuchten-Mualem on columns of at most one wave
    if (g.nz <= kWave) RF_LAUNCH_N(g.nblk_r, (k_coeff<RF_VGM, true>), g, so, a, m, dt, chord_eps, variant);
    RF_LAUNCH_N(g.nblk_r, (k_coeff<RF_VGM, false>), g, so, a, m, dt, chord_eps, variant);
}

// The PCG arrays of the FP64 solve: the workspace arrays themselves.
static CgVec<double> dvec(const Arrays &a)
{
    return CgVec<double>{a.K, a.Dd, a.diag, a.tz, a.rdp, a.r, a.p0, a.p1, a.q, a.e, a.z};
}

hipError_t launch_resid(const Geo &g, const Arrays &a, int precond, int m, double *bout,
                        bool mixed, bool refactor, const CgTol &t, hipStream_t s)
{
    const bool zl = precond == RF_PRECOND_ZLINE;
    const int rf = refactor ? 1 : 0;
    if (g.tiled && g.tile_y == 2) {
        if (mixed && zl)
            RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_ZLINE, float, 2>), g, a, a.f, m, bout, rf);
        if (mixed)
            RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_JACOBI, float, 2>), g, a, a.f, m,
                            bout, rf);
        if (zl)
            RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_ZLINE, double, 2>), g, a, dvec(a), m,
                            bout, rf);
        RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_JACOBI, double, 2>), g, a, dvec(a), m,
                        bout, rf);
    }
    if (g.tiled) {
        if (mixed && zl)
            RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_ZLINE, float, 4>), g, a, a.f, m, bout, rf);
        if (mixed)
            RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_JACOBI, float, 4>), g, a, a.f, m,
                            bout, rf);
        if (zl)
            RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_ZLINE, double, 4>), g, a, dvec(a), m,
                            bout, rf);
        RF_LAUNCH_DECIDE_TILED((k_resid_tile<RF_PRECOND_JACOBI, double, 4>), g, a, dvec(a), m,
                        bout, rf);
    }
    if (mixed && zl)
        RF_LAUNCH_DECIDE(g.nblk, (k_resid<RF_PRECOND_ZLINE, float>), g, a, a.f, m, bout, rf);
    if (mixed) RF_LAUNCH_DECIDE(g.nblk, (k_resid<RF_PRECOND_JACOBI, float>), g, a, a.f, m, bout, rf);
    if (zl) RF_LAUNCH_DECIDE(g.nblk, (k_resid<RF_PRECOND_ZLINE, double>), g, a, dvec(a), m, bout, rf);
    RF_LAUNCH_DECIDE(g.nblk, (k_resid<RF_PRECOND_JACOBI, double>), g, a, dvec(a), m, bout, rf);
}

hipError_t launch_spmv(const Geo &g, const Arrays &a, int precond, bool mixed, int parity,
                       const CgTol &t, hipStream_t s)
{
    const bool zl = precond == RF_PRECOND_ZLINE;
    if (g.tiled && g.tile_y == 2) {
        if (mixed && zl)
            RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_ZLINE, float, 2>), g, a, a.f, parity,
                            t.tol_cg, t.rel, t.max_cg);
        if (mixed)
            RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_JACOBI, float, 2>), g, a, a.f, parity,
                            t.tol_cg, t.rel, t.max_cg);
        if (zl)
            RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_ZLINE, double, 2>), g, a, dvec(a),
                            parity, t.tol_cg, t.rel, t.max_cg);
        RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_JACOBI, double, 2>), g, a, dvec(a),
                        parity, t.tol_cg, t.rel, t.max_cg);
    }
    if (g.tiled) {
        if (mixed && zl)
            RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_ZLINE, float, 4>), g, a, a.f, parity,
                            t.tol_cg, t.rel, t.max_cg);
        if (mixed)
            RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_JACOBI, float, 4>), g, a, a.f, parity,
                            t.tol_cg, t.rel, t.max_cg);
        if (zl)
            RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_ZLINE, double, 4>), g, a, dvec(a),
                            parity, t.tol_cg, t.rel, t.max_cg);
        RF_LAUNCH_TILED(a.pq, 1, 0u, (k_spmv_tile<RF_PRECOND_JACOBI, double, 4>), g, a, dvec(a),
                        parity, t.tol_cg, t.rel, t.max_cg);
    }
    if (mixed && zl)
        RF_LAUNCH_FOLD(a.pq, 1, 0u, (k_spmv<RF_PRECOND_ZLINE, float>), g, a, a.f, parity, t.tol_cg,
                       t.rel, t.max_cg);
    if (mixed)
        RF_LAUNCH_FOLD(a.pq, 1, 0u, (k_spmv<RF_PRECOND_JACOBI, float>), g, a, a.f, parity, t.tol_cg,
                       t.rel, t.max_cg);
    if (zl)
        RF_LAUNCH_FOLD(a.pq, 1, 0u, (k_spmv<RF_PRECOND_ZLINE, double>), g, a, dvec(a), parity,
                       t.tol_cg, t.rel, t.max_cg);
    RF_LAUNCH_FOLD(a.pq, 1, 0u, (k_spmv<RF_PRECOND_JACOBI, double>), g, a, dvec(a), parity, t.tol_cg,
                   t.rel, t.max_cg);
}

hipError_t launch_update(const Geo &g, const Arrays &a, int precond, bool mixed, int parity,
                         bool factors_current, const CgTol &t, hipStream_t s)
{
    const bool zl = precond == RF_PRECOND_ZLINE;
    const int rb = factors_current ? 1 : 0;
    if (mixed && zl)
        RF_LAUNCH_DECIDE(g.nblk, (k_update<RF_PRECOND_ZLINE, float>), g, a, a.f, parity, rb);
    if (mixed) RF_LAUNCH_DECIDE(g.nblk, (k_update<RF_PRECOND_JACOBI, float>), g, a, a.f, parity, rb);
    if (zl) RF_LAUNCH_DECIDE(g.nblk, (k_update<RF_PRECOND_ZLINE, double>), g, a, dvec(a), parity, rb);
    RF_LAUNCH_DECIDE(g.nblk, (k_update<RF_PRECOND_JACOBI, double>), g, a, dvec(a), parity, rb);
}

hipError_t launch_apply_h(const Geo &g, const Arrays &a, int m, bool mixed, const CgTol &t,
                          hipStream_t s)
{
    // its partials are combined by k_decide itself
    if (mixed)
        RF_LAUNCH(k_apply_h<float>, g, a, (const float *)a.f.e, (const float *)a.f.p0,
                  (const float *)a.f.p1, m, t.tol_cg, t.rel, t.max_cg);
    RF_LAUNCH(k_apply_h<double>, g, a, (const double *)a.e, (const double *)a.p0,
              (const double *)a.p1, m, t.tol_cg, t.rel, t.max_cg);
}

hipError_t launch_accept(const Geo &g, const Soil &so, const Arrays &a, bool track, int serial,
                         hipStream_t s)
{
    // van Genuchten-Mualem branch-free on columns of at most one wave (the
    // arithmetic the solver has always used there), branching on taller ones
    const bool vgm = so.model == RF_VGM, flat = vgm && g.nz <= kWave;
    if (track && flat) RF_LAUNCH_FOLD_R(a.ps, 7, 0u, (k_accept<true, RF_VGM, true>), g, so, a, serial);
    if (track && vgm) RF_LAUNCH_FOLD_R(a.ps, 7, 0u, (k_accept<true, RF_VGM, false>), g, so, a, serial);
    if (track) RF_LAUNCH_FOLD_R(a.ps, 7, 0u, (k_accept<true, RF_GARDNER, false>), g, so, a, serial);
    if (flat) RF_LAUNCH_FOLD_R(a.ps, 7, 0u, (k_accept<false, RF_VGM, true>), g, so, a, serial);
    if (vgm) RF_LAUNCH_FOLD_R(a.ps, 7, 0u, (k_accept<false, RF_VGM, false>), g, so, a, serial);
    RF_LAUNCH_FOLD_R(a.ps, 7, 0u, (k_accept<false, RF_GARDNER, false>), g, so, a, serial);
}

hipError_t launch_eval_soil(const Geo &g, const Soil &so, const Arrays &a, const double *h,
                            double *theta, double *C, double *K, hipStream_t s)
{
    RF_LAUNCH_W(k_eval_soil, g, so, a, h, theta, C, K);
}

hipError_t launch_operator(const Geo &g, const Arrays &a, const double *x, double *y,
                           hipStream_t s)
{
    RF_LAUNCH_W(k_operator, g, a, x, y);
}

hipError_t launch_precond(const Geo &g, const Arrays &a, int precond, const double *r, double *z,
                          hipStream_t s)
{
    if (precond == RF_PRECOND_ZLINE) RF_LAUNCH_W(k_precond<RF_PRECOND_ZLINE>, g, a, r, z);
    RF_LAUNCH_W(k_precond<RF_PRECOND_JACOBI>, g, a, r, z);
}

hipError_t launch_fold(const Geo &g, double *P, int nv, unsigned maxmask, hipStream_t s, int nprod)
{
    if (nprod < 0) nprod = g.nblk;
    if (g.np != 1 || g.foff == 0) return hipSuccess;   // partials read as written
    switch (nv * 16 + (int)maxmask) {
    case 1 * 16 + 0: RF_LAUNCH_N(1, (k_fold<1, 0u>), P, nprod, g.foff);
    case 2 * 16 + 1: RF_LAUNCH_N(1, (k_fold<2, 1u>), P, nprod, g.foff);
    case 2 * 16 + 2: RF_LAUNCH_N(1, (k_fold<2, 2u>), P, nprod, g.foff);
    case 7 * 16 + 0: RF_LAUNCH_N(1, (k_fold<7, 0u>), P, nprod, g.foff);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / sizeof(uint32_t);
    if (n == 0) return hipSuccess;
    const size_t nb = std::min<size_t>((n + kThreads - 1) / kThreads, 4096);
    RF_LAUNCH_N(nb, k_zero, (uint32_t *)p, n);
}

hipError_t launch_copy_active(const Geo &g, const Arrays &a, const double *src, double *dst,
                              hipStream_t s)
{
    RF_LAUNCH_W(k_copy_active, g, a, src, dst);
}

}  // namespace rf
