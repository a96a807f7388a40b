// Driver of the CPU emulation build (tests/simt): runs the library's C ABI
// -- with the HIP kernels emulated by simt.h -- on a case read from a text
// file, and prints what the tests compare with the oracle.
//
//   driver ens CASE     column ensemble: rf_ens_run to each stop time
//   driver solver CASE  3-D solver: rf_step with a fixed dt, or rf_run
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/rf.h"
#include "../../include/rf_ensemble.h"

static FILE *in;
static double rd()
{
    double v;
    if (fscanf(in, "%lf", &v) != 1) {
        fprintf(stderr, "driver: bad input\n");
        exit(2);
    }
    return v;
}
static int ri() { return (int)rd(); }
template <class T>
static std::vector<T> rv(size_t n)
{
    std::vector<T> v(n);
    for (size_t i = 0; i < n; i++) v[i] = (T)rd();
    return v;
}
// Device buffers of the case: filled with the byte SIMT_FILL names (default
// 0), so that a run can show whether anything reads memory it never wrote
// (0xFF reads as NaN in every floating-point type).
static void *aligned(size_t n)
{
    void *p = nullptr;
    if (posix_memalign(&p, 256, n ? n : 256)) exit(3);
    const char *f = getenv("SIMT_FILL");
    memset(p, f ? (int)strtol(f, nullptr, 0) : 0, n);
    return p;
}
#define CHK(x)                                                                  \
    do {                                                                        \
        const int s_ = (x);                                                     \
        if (s_ != 0) {                                                          \
            printf("error %d %s\n", s_, #x);                                    \
            return 1;                                                           \
        }                                                                       \
    } while (0)

static int run_ens()
{
    const int ncol = ri();
    const double dz = rd();
    const int model = ri();
    auto len = rv<int32_t>(ncol);
    auto soil = rv<double>(6 * (size_t)ncol);
    rf_ens *e = nullptr;
    CHK(rf_ens_create(&e, 0, nullptr));
    CHK(rf_ens_setup(e, ncol, len.data(), dz, model, soil.data()));
    for (int f = 0; f < 2; f++) {
        const int type = ri();
        const double v = rd();
        CHK(rf_ens_set_bc(e, f == 0 ? RF_ZMIN : RF_ZMAX, type, v));
    }
    rf_options o;
    rf_default_options(&o);
    o.tol_picard = rd();
    o.max_picard = ri();
    o.chord_eps = rd();
    o.dt0 = rd();
    o.dt_max = rd();
    o.dt_min = rd();
    o.ebats = ri();
    o.inc_after = ri();
    o.few_iters = ri();
    o.max_iters = ri();
    o.factor = rd();
    o.precision = ri();
    o.picard_variant = ri();
    CHK(rf_ens_set_options(e, &o));
    const long max_steps = (long)rd();
    const double max_seconds = rd();
    CHK(rf_ens_set_limits(e, max_steps, max_seconds));
    rf_ens_tile tile;
    tile.waves_per_block = ri();
    tile.blocks_per_cu = ri();
    CHK(rf_ens_set_tile(e, &tile));
    const int nrun = ri();
    auto t_end = rv<double>(nrun);
    const int nlim = ri();                      // per-run step budgets (0: the one above)
    auto run_steps = rv<double>(nlim);
    long ncell = 0;
    CHK(rf_ens_cells(e, &ncell));
    auto h0 = rv<double>(ncell);
    size_t bytes = 0;
    CHK(rf_ens_workspace_bytes(e, &bytes));
    void *ws = aligned(bytes);
    CHK(rf_ens_bind_workspace(e, ws, bytes));
    double *hd = (double *)aligned(ncell * sizeof(double));
    memcpy(hd, h0.data(), ncell * sizeof(double));
    CHK(rf_ens_set_state(e, hd, 0.0));
    for (int r = 0; r < nrun; r++) {
        if (r < nlim && run_steps[r] > 0) CHK(rf_ens_set_limits(e, (long)run_steps[r], max_seconds));
        rf_ens_summary sm;
        const int s = rf_ens_run(e, t_end[r], &sm);
        printf("run %d %ld %ld %ld %ld %d %.17g %.17g\n", s, sm.accepted, sm.rejected, sm.picard_total,
               sm.cell_steps, sm.failed, sm.t_min, sm.max_balance_error);
    }
    std::vector<rf_ens_column> cols(ncol);
    CHK(rf_ens_get_columns(e, cols.data()));
    for (int c = 0; c < ncol; c++) {
        const rf_ens_column &r = cols[c];
        printf("col %d %d %d %d %d %ld %.17g %.17g %.17g %.17g %.17g %.17g\n", c, r.status, r.accepted,
               r.rejected, r.easy, r.picard_total, r.t, r.dt_next, r.storage0, r.storage, r.inflow_top,
               r.inflow_bottom);
    }
    CHK(rf_ens_get_state(e, hd));
    printf("h");
    for (long i = 0; i < ncell; i++) printf(" %.17g", hd[i]);
    printf("\n");
    rf_ens_destroy(e);
    free(ws);
    free(hd);
    return 0;
}

static int run_solver()
{
    const int nx = ri(), ny = ri(), nz = ri();
    const double dx = rd(), dy = rd(), dz = rd();
    const size_t N = (size_t)nx * ny * nz, ncol = (size_t)nx * ny;
    std::vector<int32_t> ktop;
    if (ri()) ktop = rv<int32_t>(ncol);
    double g[3] = {rd(), rd(), rd()};
    const int model = ri(), nlayer = ri();
    auto params = rv<double>(6 * (size_t)nlayer);
    std::vector<uint8_t> layer;
    std::vector<double> lnks;
    if (ri()) layer = rv<uint8_t>(N);
    if (ri()) lnks = rv<double>(N);
    rf_ctx *c = nullptr;
    CHK(rf_create(&c, 0, nullptr));
    CHK(rf_setup_grid(c, nx, ny, nz, dx, dy, dz, ktop.empty() ? nullptr : ktop.data(), g));
    CHK(rf_set_soil(c, model, nlayer, params.data(), layer.empty() ? nullptr : layer.data(),
                    lnks.empty() ? nullptr : lnks.data()));
    const int nbc = ri();
    for (int b = 0; b < nbc; b++) {
        const int face = ri(), type = ri();
        const double v = rd();
        CHK(rf_set_bc(c, face, type, v));
    }
    rf_options o;
    rf_default_options(&o);
    o.tol_picard = rd();
    o.tol_cg = rd();
    o.max_picard = ri();
    o.max_cg = ri();
    o.precond = ri();
    o.ebats = ri();
    o.dt0 = rd();
    o.dt_max = rd();
    o.precision = ri();
    o.stencil = ri();
    o.tile_rows = ri();
    o.cols_per_wave = ri();
    o.cg_rel_tol = rd();
    o.zline_refactor = ri();
    CHK(rf_set_options(c, &o));
    const int nsteps = ri();
    const double dt = rd();
    auto h0 = rv<double>(N);
    const int use_static = ri();
    void *ws = nullptr;
    if (use_static) {
        CHK(rf_bind_static_workspace(c));
    } else {
        size_t bytes = 0;
        CHK(rf_workspace_bytes(c, &bytes));
        ws = aligned(bytes);
        CHK(rf_bind_workspace(c, ws, bytes));
    }
    double *hd = (double *)aligned(N * sizeof(double));
    memcpy(hd, h0.data(), N * sizeof(double));
    CHK(rf_set_state(c, hd, 0.0));
    if (nsteps > 0) {
        for (int n = 0; n < nsteps; n++) {
            rf_step_stats st;
            const int s = rf_step(c, dt, nullptr, &st);
            printf("step %d %d %d", s, st.picard_iters, st.cg_iters_total);
            for (int m = 0; m < st.picard_iters && m < RF_MAX_PICARD_LOG; m++) printf(" %.17g", st.delta[m]);
            printf("\n");
            printf("cg");
            for (int m = 0; m < st.picard_iters && m < RF_MAX_PICARD_LOG; m++) printf(" %d", st.cg_iters[m]);
            printf("\n");
            if (s) break;
        }
    } else {
        rf_run_stats rs;
        const int s = rf_run(c, dt, &rs);
        printf("runstats %d %d %d %ld %ld %.17g\n", s, rs.accepted, rs.rejected, rs.picard_total,
               rs.cg_total, rs.t);
    }
    rf_mass m;
    CHK(rf_mass_balance(c, &m));
    printf("mass %.17g %.17g %.17g\n", m.storage, m.storage0, m.error);
    double t = 0.0;
    CHK(rf_get_state(c, hd, &t));
    printf("h");
    for (size_t i = 0; i < N; i++) printf(" %.17g", hd[i]);
    printf("\n");
    rf_destroy(c);
    free(ws);
    free(hd);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: driver ens|solver CASE\n");
        return 2;
    }
    in = fopen(argv[2], "r");
    if (!in) return 2;
    const int r = strcmp(argv[1], "ens") == 0 ? run_ens() : run_solver();
    fclose(in);
    return r;
}
