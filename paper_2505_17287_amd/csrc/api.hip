// C ABI of the ghost-cell IBM projection library (declarations and contracts: include/ibm.h).
// Host-side logic only: argument checks, workspace layout, call-order state, mesh
// validation, multigrid level planning and the solve drivers.  Every step of the method
// runs in the kernels of geometry.hip, sweep.hip, finepass.hip, solver.hip and momentum.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "ibm_impl.hpp"
#include "mesh_check.hpp"

using namespace ibm;

namespace {

// A named host range around each entry point that enqueues device work and around each outer
// iteration of a solve: `rocprofv3 --marker-trace` shows them above the kernels they launch.
// Without a tool attached the calls return at once.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

thread_local std::string t_last_error;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

ibm_status fail(ibm_grid *g, ibm_status st, const std::string &msg) {
    t_last_error = msg;
    if (g) g->err = msg;
    return st;
}

ibm_status hip_fail(ibm_grid *g, hipError_t e, const char *where) {
    return fail(g, IBM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                         \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(g, _e, where); \
    } while (0)

bool finite_increasing(const double *f, int n) {
    for (int i = 0; i <= n; ++i)
        if (!std::isfinite(f[i])) return false;
    for (int i = 0; i < n; ++i)
        if (!(f[i + 1] > f[i])) return false;
    return true;
}

}  // namespace

namespace ibm {

ibm_status report_error(ibm_status st, const std::string &msg) { return fail(nullptr, st, msg); }

// Coarsening by cell width.  Along every axis with at least 4 cells, scanning from the low
// wall, a cell is merged with the next one when their combined width is at most a threshold
// t; every other cell is kept whole.  Level l (built from level l-1) starts from
// t = MERGE_WIDTH x 2^(l-1) h_min (h_min: the smallest cell width of the grid over the axes
// with at least two cells) and raises t by a factor 5/4 until the level holds at most half as
// many cells as level l-1 or every axis is halved outright, so the narrowest cells merge
// first: uniform axes are halved, and in a stretched region cells already wide along one axis
// are kept along it while they are still merged along the others, so coarse cells tend to
// equal widths and point smoothing keeps working.  The plan stops when no axis merges a cell.
// Coarse faces are the fine faces at the start of each coarse cell.
constexpr double MERGE_WIDTH = 3.5;

static int merge_axis(const std::vector<double> &w, double wmax, std::vector<int> &cs) {
    const int n = (int)w.size();
    cs.clear();
    int i = 0;
    while (i < n) {
        cs.push_back(i);
        if (n >= 4 && i + 1 < n && w[i] + w[i + 1] <= wmax)
            i += 2;
        else
            i += 1;
    }
    cs.push_back(n);
    return (int)cs.size() - 1;
}

void plan_levels(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf, LevelHost *lev,
                 int *nlev) {
    LevelHost &L0 = lev[0];
    L0.n[0] = nx;
    L0.n[1] = ny;
    L0.n[2] = nz;
    const double *fs[3] = {xf, yf, zf};
    double hmin = INFINITY;
    for (int d = 0; d < 3; ++d) {
        L0.halved[d] = 0;
        L0.same[d] = 1;
        L0.cs[d].clear();
        L0.f[d].assign(fs[d], fs[d] + L0.n[d] + 1);
        L0.c[d].resize(L0.n[d]);
        L0.w[d].resize(L0.n[d]);
        for (int i = 0; i < L0.n[d]; ++i) {
            L0.c[d][i] = 0.5 * (L0.f[d][i] + L0.f[d][i + 1]);
            L0.w[d][i] = L0.f[d][i + 1] - L0.f[d][i];
        }
        if (L0.n[d] >= 2) hmin = std::min(hmin, *std::min_element(L0.w[d].begin(), L0.w[d].end()));
    }
    int n = 1;
    while (n < MAX_LEVELS) {
        LevelHost &F = lev[n - 1];
        LevelHost &C = lev[n];
        const int64_t nf = F.ncell();
        double wmax = MERGE_WIDTH * std::ldexp(hmin, n - 1);
        bool any = false;
        for (int rise = 0; rise < 64; ++rise, wmax *= 1.25) {
            int64_t nc = 1;
            bool full = true;
            any = false;
            for (int d = 0; d < 3; ++d) {
                C.n[d] = merge_axis(F.w[d], wmax, C.cs[d]);
                nc *= C.n[d];
                any = any || C.n[d] < F.n[d];
                if (F.n[d] >= 4 && C.n[d] != (F.n[d] + 1) / 2) full = false;
            }
            if (2 * nc <= nf || full) break;
        }
        if (!any) break;
        for (int d = 0; d < 3; ++d) {
            C.same[d] = C.n[d] == F.n[d];
            bool uniform = F.n[d] % 2 == 0 && C.n[d] * 2 == F.n[d];
            for (int I = 0; uniform && I <= C.n[d]; ++I) uniform = C.cs[d][I] == 2 * I;
            C.halved[d] = uniform ? 1 : 0;
        }
        for (int d = 0; d < 3; ++d) {
            C.f[d].resize(C.n[d] + 1);
            for (int q = 0; q <= C.n[d]; ++q) C.f[d][q] = F.f[d][C.cs[d][q]];
            C.c[d].resize(C.n[d]);
            C.w[d].resize(C.n[d]);
            for (int i = 0; i < C.n[d]; ++i) {
                C.c[d][i] = 0.5 * (C.f[d][i] + C.f[d][i + 1]);
                C.w[d][i] = C.f[d][i + 1] - C.f[d][i];
            }
        }
        // side rule of the prolongation table (k_prolong_tab) on uniformly halved axes: fine i
        // takes I = i/2 and the coarse neighbour on the side of its centre
        bool sides = true;
        for (int d = 0; d < 3; ++d) {
            if (!C.halved[d]) continue;
            for (int i = 0; i < F.n[d]; ++i) {
                const int I = i / 2, jn = (F.c[d][i] < C.c[d][I]) ? I - 1 : I + 1;
                if (jn >= 0 && jn < C.n[d] && jn != ((i & 1) ? I + 1 : I - 1)) sides = false;
            }
        }
        F.prolong_sides = sides;
        ++n;
    }
    *nlev = n;
}

ChildMap child_map(const LevelHost &C) {
    ChildMap M;
    for (int d = 0; d < 3; ++d) {
        M.cs[d] = C.cs_d[d];
        M.halved[d] = C.halved[d];
        M.same[d] = C.same[d];
    }
    return M;
}

size_t layout(ibm_grid *g, Plan &P, int nx, int ny, int nz, int64_t nv_max, int64_t nt_max, int64_t gmax,
              ibm_precision prec, LevelHost *lev, int nlev) {
    const int64_t N = (int64_t)nx * ny * nz, ncol = (int64_t)nx * ny;
    const int n[3] = {nx, ny, nz};
    ibm_grid tmp;
    ibm_grid *G = g ? g : &tmp;
    G->type = P.take<uint8_t>(N);
    G->inject0 = P.take<uint8_t>(N);
    G->p2 = P.take<double>(N);
    G->frhs = P.take<double>(N);
    G->pz = P.take<double>(N);
    if (prec == IBM_MIXED) {
        G->e32a = P.take<float>(N);
        G->e32b = P.take<float>(N);
        G->r32 = P.take<float>(N);
        G->pz32 = P.take<float>(N);
    } else {
        G->e32a = G->e32b = G->r32 = nullptr;
        G->pz32 = nullptr;
    }
    for (int d = 0; d < 3; ++d) {
        G->faces[d] = P.take<double>(n[d] + 1);
        G->c0[d] = P.take<double>(n[d]);
        G->w0[d] = P.take<double>(n[d]);
        G->dc0[d] = P.take<double>(n[d]);
        G->am0[d] = P.take<double>(n[d]);
        G->ap0[d] = P.take<double>(n[d]);
        G->am0f[d] = P.take<float>(n[d]);
        G->ap0f[d] = P.take<float>(n[d]);
        G->w0f[d] = P.take<float>(n[d]);
    }
    G->verts = P.take<double>(3 * std::max<int64_t>(nv_max, 3));
    G->tris = P.take<int32_t>(3 * std::max<int64_t>(nt_max, 1));
    G->bucket_cnt = P.take<int32_t>(NBUCKET_MAX + 1);
    G->bucket_off = P.take<int32_t>(NBUCKET_MAX + 1);
    G->bucket_ent = P.take<int32_t>(8 * std::max<int64_t>(nt_max, 1) + 16);
    G->col_cnt = P.take<int32_t>(ncol + 1);
    G->col_off = P.take<int32_t>(ncol + 1);
    G->col_fill = P.take<int32_t>(std::max<int64_t>(ncol + 1, NBUCKET_MAX + 1));
    G->cross_cap = 8 * ncol + 4 * std::max<int64_t>(nt_max, 1) + 1024;
    G->crossings = P.take<double>(std::max<int64_t>(G->cross_cap, N / 256 + 1024));
    G->blk_cnt = (int32_t *)P.take<int64_t>(8192);
    G->counters = P.take<int64_t>(16);
    const int64_t gm = std::max<int64_t>(gmax, 1);
    G->g_cell = P.take<int32_t>(gm);
    G->g_st = P.take<int32_t>(8 * gm);
    G->g_flags = P.take<int32_t>(gm);
    G->g_tri = P.take<int32_t>(gm);
    G->g_mask = P.take<uint8_t>(gm);
    G->g_bi = P.take<double>(3 * gm);
    G->g_n = P.take<double>(3 * gm);
    G->g_ip = P.take<double>(3 * gm);
    G->g_beta = P.take<double>(8 * gm);
    G->g_betag = P.take<double>(gm);
    G->g_dl = P.take<double>(gm);
    G->g_h = P.take<double>(gm);
    G->g_data = P.take<double>(gm);
    G->g_scale = P.take<double>(gm);
    G->g_rhs = P.take<double>(gm);
    G->g_betaD = P.take<double>(8 * gm);
    G->g_betaDg = P.take<double>(gm);
    G->g_ubi = P.take<double>(3 * gm);
    G->g_uscr = P.take<double>(3 * gm);
    G->type_prev = P.take<uint8_t>(N);
    G->f_cell = P.take<int32_t>(gm);
    G->f_tri = P.take<int32_t>(gm);
    G->f_st = P.take<int32_t>(8 * gm);
    G->f_flags = P.take<int32_t>(gm);
    G->f_bi = P.take<double>(3 * gm);
    G->f_ip = P.take<double>(3 * gm);
    G->f_beta = P.take<double>(8 * gm);
    G->f_betac = P.take<double>(gm);
    G->f_ubi = P.take<double>(3 * gm);
    G->f_scr = P.take<double>(3 * gm);
    for (int q = 0; q < 10; ++q) G->kv[q] = P.take<double>(N);
    for (int l = 0; l < nlev; ++l) {
        LevelHost &L = lev[l];
        const int64_t NC = L.ncell();
        if (l >= 1) {
            L.active = P.take<uint8_t>(NC);
            for (int d = 0; d < 3; ++d) {
                L.T64[d] = P.take<double>(NC);
                L.T32[d] = P.take<float>(NC);
                L.w64[d] = P.take<double>(L.n[d]);
                L.w32[d] = P.take<float>(L.n[d]);
                L.c64[d] = P.take<double>(2 * L.n[d] + 1);  // centres, then the faces
            }
            for (int d = 0; d < 3; ++d) L.cs_d[d] = P.take<int>(L.n[d] + 1);
            L.e64 = P.take<double>(NC);
            L.R64 = P.take<double>(NC);
            L.e32 = P.take<float>(NC);
            L.R32 = P.take<float>(NC);
            if (sweepC_fused_ok(L.n)) {
                L.e64b = P.take<double>(NC);
                L.e32b = P.take<float>(NC);
            } else {
                L.e64b = nullptr;
                L.e32b = nullptr;
            }
        }
        if (l + 1 < nlev) {
            for (int d = 0; d < 3; ++d) {
                L.plo[d] = P.take<int>(L.n[d]);
                L.phi[d] = P.take<int>(L.n[d]);
                L.pt[d] = P.take<double>(L.n[d]);
            }
        }
    }
    // the largest of: reductions over RED_BLOCKS workgroups (up to 4 sums), the coarsening
    // sums, and one Krylov operator pass (2 sums per z-march workgroup, then 2 per ghost block)
    G->partials = P.take<double>(std::max<int64_t>(
        std::max<int64_t>(4 * RED_BLOCKS, N / 256 + 1024),
        2 * zmarch_partials_max(nx, ny, nz) + 2 * (std::max<int64_t>(gmax, 1) / 256 + 2)));
    G->sc = P.take<Scalars>(1);
    return P.off + 256;
}

}  // namespace ibm


extern "C" {

void ibm_default_opts(ibm_solve_opts *o) {
    if (!o) return;
    o->rel_tol = 1e-10;
    o->max_cycles = 200;
    o->nu1 = 2;
    o->nu2 = 2;
    o->coarsest_sweeps = 16;
    o->precision = IBM_FP64;
    o->use_initial_guess = 0;
    o->fixed_cycles = 0;
    o->method = IBM_BICGSTAB;
    o->srj_sweeps = 16;
    o->breakdown_tol = 1e-12;
}

ibm_status ibm_create_grid(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                           ibm_grid **out) {
    if (!out) return fail(nullptr, IBM_E_ARG, "ibm_create_grid: out is NULL");
    *out = nullptr;
    if (nx < 2 || ny < 2 || nz < 1) return fail(nullptr, IBM_E_ARG, "ibm_create_grid: need nx, ny >= 2 and nz >= 1");
    if ((int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return fail(nullptr, IBM_E_ARG, "ibm_create_grid: more than 2^31 cells");
    if (!xf || !yf || !zf) return fail(nullptr, IBM_E_ARG, "ibm_create_grid: NULL face array");
    if (!finite_increasing(xf, nx) || !finite_increasing(yf, ny) || !finite_increasing(zf, nz))
        return fail(nullptr, IBM_E_ARG, "ibm_create_grid: face coordinates must be finite and strictly increasing");
    ibm_grid *g = new ibm_grid();
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->N = (int64_t)nx * ny * nz;
    g->xf.assign(xf, xf + nx + 1);
    g->yf.assign(yf, yf + ny + 1);
    g->zf.assign(zf, zf + nz + 1);
    plan_levels(nx, ny, nz, xf, yf, zf, g->lev, &g->nlev);
    g->stage = ST_CREATED;
    *out = g;
    return IBM_OK;
}

size_t ibm_workspace_bytes(int nx, int ny, int nz, int64_t nv_max, int64_t nt_max, int64_t max_ghosts,
                           ibm_precision prec) {
    if (nx < 2 || ny < 2 || nz < 1) return 0;
    // Upper bound for any face coordinates: the fine level exactly, plus coarse levels of at
    // most half the previous level's cells each (their sum stays below N) at 61 B per coarse
    // cell, plus per-level 1D arrays and alignment.
    LevelHost lev[1];
    lev[0].n[0] = nx;
    lev[0].n[1] = ny;
    lev[0].n[2] = nz;
    Plan P;
    size_t b = layout(nullptr, P, nx, ny, nz, nv_max, nt_max, max_ghosts, prec, lev, 1);
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t axes = (int64_t)nx + ny + nz;
    return b + (size_t)N * 61 + (size_t)MAX_LEVELS * (size_t)(axes * 64 + 32 * 256) + (1 << 20);
}

size_t ibm_grid_workspace_bytes(const ibm_grid *gc, int64_t nv_max, int64_t nt_max, int64_t max_ghosts,
                                ibm_precision prec) {
    if (!gc) return 0;
    ibm_grid *g = const_cast<ibm_grid *>(gc);
    LevelHost lev[MAX_LEVELS];
    for (int l = 0; l < g->nlev; ++l)
        for (int d = 0; d < 3; ++d) {
            lev[l].n[d] = g->lev[l].n[d];
            lev[l].halved[d] = g->lev[l].halved[d];
        }
    Plan P;
    return layout(nullptr, P, g->nx, g->ny, g->nz, nv_max, nt_max, max_ghosts, prec, lev, g->nlev);
}

ibm_status ibm_bind_workspace(ibm_grid *g, void *device_ptr, size_t bytes, int64_t nv_max, int64_t nt_max,
                              int64_t max_ghosts, ibm_precision prec, void *stream) {
    Range range_("ibm_bind_workspace");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_bind_workspace: NULL handle");
    if (!device_ptr || ((uintptr_t)device_ptr & 255)) return fail(g, IBM_E_ARG, "workspace must be 256-byte aligned");
    if (nv_max < 3 || nt_max < 1 || max_ghosts < 0) return fail(g, IBM_E_ARG, "invalid mesh / ghost capacities");
    size_t need = ibm_grid_workspace_bytes(g, nv_max, nt_max, max_ghosts, prec);
    if (bytes < need)
        return fail(g, IBM_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipGetDevice(&g->device), "hipGetDevice");
    Plan P;
    P.base = (char *)device_ptr;
    std::vector<std::pair<size_t, size_t>> fp_spans;
    if (g->debug_poison) P.fp_spans = &fp_spans;
    layout(g, P, g->nx, g->ny, g->nz, nv_max, nt_max, max_ghosts, prec, g->lev, g->nlev);
    // debug: every floating-point sub-buffer starts as NaN (all bits set), so any value the
    // library reads before writing it propagates into the results
    for (const auto &sp : fp_spans)
        HIP_TRY(hipMemsetAsync((char *)device_ptr + sp.first, 0xFF, sp.second, s), "poison");
    g->ws = (char *)device_ptr;
    g->ws_bytes = bytes;
    g->nv_max = nv_max;
    g->nt_max = nt_max;
    g->ghost_max = max_ghosts;
    g->prec = prec;
    if (!g->sc_host) HIP_TRY(hipHostMalloc((void **)&g->sc_host, sizeof(Scalars), hipHostMallocDefault), "hipHostMalloc");
    const std::vector<double> *fs[3] = {&g->xf, &g->yf, &g->zf};
    for (int d = 0; d < 3; ++d)
        HIP_TRY(hipMemcpyAsync(g->faces[d], fs[d]->data(), sizeof(double) * fs[d]->size(), hipMemcpyHostToDevice, s),
                "upload faces");
    for (int l = 1; l < g->nlev; ++l)
        for (int d = 0; d < 3; ++d) {
            HIP_TRY(hipMemcpyAsync(g->lev[l].c64[d] + g->lev[l].n[d], g->lev[l].f[d].data(),
                                   sizeof(double) * (g->lev[l].n[d] + 1), hipMemcpyHostToDevice, s),
                    "upload coarse faces");
            HIP_TRY(hipMemcpyAsync(g->lev[l].cs_d[d], g->lev[l].cs[d].data(), sizeof(int) * (g->lev[l].n[d] + 1),
                                   hipMemcpyHostToDevice, s),
                    "upload child maps");
        }
    HIP_TRY(hipMemsetAsync(g->sc, 0, sizeof(Scalars), s), "memset scalars");
    HIP_TRY(launch_metrics(g, s), "metrics");
    HIP_TRY(hipStreamSynchronize(s), "bind sync");
    g->stage = ST_BOUND;
    g->ng = 0;
    return IBM_OK;
}

static ibm_status set_geometry_impl(ibm_grid *g, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                                    void *stream, bool known_topology);

ibm_status ibm_set_geometry(ibm_grid *g, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                            void *stream) {
    Range range_("ibm_set_geometry");
    return set_geometry_impl(g, verts, nv, tris, nt, stream, false);
}

static ibm_status set_geometry_impl(ibm_grid *g, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                                    void *stream, bool known_topology) {
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_set_geometry: NULL handle");
    if (g->stage < ST_BOUND) return fail(g, IBM_E_STATE, "ibm_set_geometry before ibm_bind_workspace");
    const double t_in = now_s();
    if (!verts || !tris || nv < 3 || nt < 1) return fail(g, IBM_E_ARG, "ibm_set_geometry: empty mesh");
    if (nv > g->nv_max || nt > g->nt_max) return fail(g, IBM_E_NOMEM, "mesh larger than the bound capacities");
    bool finite = true;  // no early exit: the loops vectorise
    for (int64_t i = 0; i < 3 * nv; ++i) finite &= std::isfinite(verts[i]);
    if (!finite) return fail(g, IBM_E_ARG, "non-finite vertex coordinate");
    // a move that keeps the triangles (the same indices as the last validated mesh, compared
    // exactly) skips the index and closedness checks
    const bool same = known_topology && g->topo_valid && g->topo_nv == nv &&
                      (int64_t)g->topo_tris.size() == 3 * nt &&
                      std::memcmp(g->topo_tris.data(), tris, sizeof(int32_t) * 3 * nt) == 0;
    if (!same) {
        g->topo_valid = false;
        int32_t tmin = tris[0], tmax = tris[0];
        for (int64_t i = 0; i < 3 * nt; ++i) {
            tmin = std::min(tmin, tris[i]);
            tmax = std::max(tmax, tris[i]);
        }
        if (tmin < 0 || tmax >= nv) return fail(g, IBM_E_ARG, "triangle index out of range");
        if (const char *why = mesh_closed_oriented(tris, nt, nv)) return fail(g, IBM_E_GEOMETRY, why);
        g->topo_tris.assign(tris, tris + 3 * nt);
        g->topo_nv = nv;
        g->topo_valid = true;
    }
    // bucket grid over the mesh bounding box: buckets at least as large as the largest
    // triangle extent; each triangle is listed in the bucket of its bounding box's low corner
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, ext[3] = {0, 0, 0};
    for (int64_t t = 0; t < nt; ++t) {
        double tl[3] = {INFINITY, INFINITY, INFINITY}, th[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int q = 0; q < 3; ++q)
            for (int d = 0; d < 3; ++d) {
                double x = verts[3 * tris[3 * t + q] + d];
                tl[d] = std::min(tl[d], x);
                th[d] = std::max(th[d], x);
            }
        for (int d = 0; d < 3; ++d) {
            ext[d] = std::max(ext[d], th[d] - tl[d]);
            lo[d] = std::min(lo[d], tl[d]);
            hi[d] = std::max(hi[d], th[d]);
        }
    }
    double span[3], vol = 1.0;
    for (int d = 0; d < 3; ++d) {
        span[d] = std::max(hi[d] - lo[d], 1e-12);
        vol *= span[d];
    }
    // about eight buckets per triangle over the bounding volume: a search box then spans few
    // triangles beyond those it meets (each triangle is listed once)
    double target = 0.5 * std::cbrt(vol / (double)std::max<int64_t>(nt, 1));
    int64_t total = 1;
    for (int d = 0; d < 3; ++d) {
        double sz = std::max(ext[d], target);
        int nbd = (int)std::max(1.0, std::floor(span[d] / sz));
        g->nb[d] = std::min(nbd, 256);
        total *= g->nb[d];
    }
    while (total > NBUCKET_MAX) {
        for (int d = 0; d < 3; ++d) g->nb[d] = std::max(1, g->nb[d] / 2);
        total = (int64_t)g->nb[0] * g->nb[1] * g->nb[2];
    }
    for (int d = 0; d < 3; ++d) {
        g->bmin[d] = lo[d];
        g->bsize[d] = span[d] / g->nb[d];
        g->bext[d] = ext[d] + 1e-9 * span[d];  // covers the rounding of the extents
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(hipMemcpyAsync(g->verts, verts, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, s), "upload verts");
    HIP_TRY(hipMemcpyAsync(g->tris, tris, sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, s), "upload tris");
    g->nv = nv;
    g->nt = nt;
    HIP_TRY(launch_buckets(g, s), "bucket grid");
    int64_t bucket_overflow = 0;
    HIP_TRY(hipMemcpyAsync(&bucket_overflow, g->counters + 6, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read");
    HIP_TRY(hipStreamSynchronize(s), "set_geometry sync");  // host arrays may be freed after return
    if (bucket_overflow) return fail(g, IBM_E_NOMEM, "triangle bucket grid overflow");
    g->stage = ST_GEOMETRY;
    g->ng = 0;
    g->t_setup = now_s() - t_in;
    return IBM_OK;
}

ibm_status ibm_classify(ibm_grid *g, void *stream, int64_t counts_out[3]) {
    Range range_("ibm_classify");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_classify: NULL handle");
    if (g->stage < ST_GEOMETRY) return fail(g, IBM_E_STATE, "ibm_classify before ibm_set_geometry");
    const double t_in = now_s();
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    int64_t c[4];
    HIP_TRY(launch_classify(g, s, c), "classify");
    int64_t odd = c[3] & (((int64_t)1 << 40) - 1);
    bool overflow = (c[3] >> 40) != 0;
    if (overflow) return fail(g, IBM_E_NOMEM, "too many ray crossings for the workspace");
    g->nfluid = c[0];
    g->nghost_cells = c[1];
    g->ndead = c[2];
    if (counts_out) {
        counts_out[0] = c[0];
        counts_out[1] = c[1];
        counts_out[2] = c[2];
    }
    if (c[1] > g->ghost_max) {
        g->stage = ST_GEOMETRY;
        return fail(g, IBM_E_NOMEM, "ghost cells " + std::to_string(c[1]) + " exceed the bound capacity " +
                                        std::to_string(g->ghost_max));
    }
    if (odd) {
        g->stage = ST_GEOMETRY;
        return fail(g, IBM_E_GEOMETRY, std::to_string(odd) +
                                           " columns with an odd number of ray crossings (mesh not watertight)");
    }
    if (c[0] == 0) return fail(g, IBM_E_GEOMETRY, "no fluid cell");
    g->ng = c[1];
    g->stage = ST_CLASSIFIED;
    g->t_setup += now_s() - t_in;
    return IBM_OK;
}

ibm_status ibm_build_ghost_stencils(ibm_grid *g, void *stream, int64_t *n_ghost_out) {
    Range range_("ibm_build_ghost_stencils");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_build_ghost_stencils: NULL handle");
    if (g->stage < ST_CLASSIFIED) return fail(g, IBM_E_STATE, "ibm_build_ghost_stencils before ibm_classify");
    const double t_in = now_s();
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(hipMemsetAsync(g->counters + 5, 0, sizeof(int64_t), s), "memset");
    HIP_TRY(launch_stencils(g, s), "ghost stencils");
    if (g->ng > 0) HIP_TRY(hipMemsetAsync(g->g_data, 0, sizeof(double) * g->ng, s), "memset neumann");
    if (g->ng > 0) HIP_TRY(hipMemsetAsync(g->g_ubi, 0, sizeof(double) * 3 * g->ng, s), "memset dirichlet");
    HIP_TRY(hipMemsetAsync(g->pz, 0, sizeof(double) * g->N, s), "memset start iterate");
    if (g->pz32) HIP_TRY(hipMemsetAsync(g->pz32, 0, sizeof(float) * g->N, s), "memset start iterate");
    HIP_TRY(launch_ghost_h(g, s), "ghost rhs");
    HIP_TRY(launch_hierarchy(g, s), "hierarchy");
    HIP_TRY(krylov_setup(g, s), "krylov setup");
    int64_t ndeg = 0;
    HIP_TRY(hipMemcpyAsync(&ndeg, g->counters + 5, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read counters");
    HIP_TRY(hipMemcpyAsync(g->sc_host, g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, s), "read scalars");
    HIP_TRY(hipStreamSynchronize(s), "stencils sync");
    g->ndegenerate = ndeg;
    g->vol_fluid = g->sc_host->vol[0];
    for (int l = 0; l < g->nlev; ++l) g->lev[l].vol_active = g->sc_host->vol[l];
    if (n_ghost_out) *n_ghost_out = g->ng;
    g->stage = ST_STENCILS;
    g->t_setup += now_s() - t_in;
    return IBM_OK;
}

ibm_status ibm_get_ghosts(const ibm_grid *gc, void *stream, int32_t *cell, double *bi_xyz, double *n_xyz,
                          double *ip_xyz, int32_t *stencil, double *beta, int32_t *flags) {
    ibm_grid *g = const_cast<ibm_grid *>(gc);
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_get_ghosts: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_get_ghosts before ibm_build_ghost_stencils");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    const int64_t ng = g->ng;
    if (ng > 0) {
        if (cell) HIP_TRY(hipMemcpyAsync(cell, g->g_cell, sizeof(int32_t) * ng, hipMemcpyDeviceToHost, s), "copy");
        if (bi_xyz) HIP_TRY(hipMemcpyAsync(bi_xyz, g->g_bi, sizeof(double) * 3 * ng, hipMemcpyDeviceToHost, s), "copy");
        if (n_xyz) HIP_TRY(hipMemcpyAsync(n_xyz, g->g_n, sizeof(double) * 3 * ng, hipMemcpyDeviceToHost, s), "copy");
        if (ip_xyz) HIP_TRY(hipMemcpyAsync(ip_xyz, g->g_ip, sizeof(double) * 3 * ng, hipMemcpyDeviceToHost, s), "copy");
        if (stencil)
            HIP_TRY(hipMemcpyAsync(stencil, g->g_st, sizeof(int32_t) * 8 * ng, hipMemcpyDeviceToHost, s), "copy");
        if (beta) HIP_TRY(hipMemcpyAsync(beta, g->g_beta, sizeof(double) * 8 * ng, hipMemcpyDeviceToHost, s), "copy");
        if (flags) HIP_TRY(hipMemcpyAsync(flags, g->g_flags, sizeof(int32_t) * ng, hipMemcpyDeviceToHost, s), "copy");
    }
    HIP_TRY(hipStreamSynchronize(s), "get_ghosts sync");
    return IBM_OK;
}

ibm_status ibm_set_neumann_data(ibm_grid *g, const double *dpdn, void *stream) {
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_set_neumann_data: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_set_neumann_data before ibm_build_ghost_stencils");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    if (g->ng > 0) {
        if (dpdn) {
            for (int64_t q = 0; q < g->ng; ++q)
                if (!std::isfinite(dpdn[q])) return fail(g, IBM_E_ARG, "non-finite Neumann data");
            HIP_TRY(hipMemcpyAsync(g->g_data, dpdn, sizeof(double) * g->ng, hipMemcpyHostToDevice, s), "upload");
        } else {
            HIP_TRY(hipMemsetAsync(g->g_data, 0, sizeof(double) * g->ng, s), "memset");
        }
        HIP_TRY(launch_ghost_h(g, s), "ghost rhs");
    }
    HIP_TRY(hipStreamSynchronize(s), "neumann sync");
    return IBM_OK;
}

ibm_status ibm_get_cell_types(const ibm_grid *gc, uint8_t *dst_device, void *stream) {
    ibm_grid *g = const_cast<ibm_grid *>(gc);
    if (!g || !dst_device) return fail(g, IBM_E_ARG, "ibm_get_cell_types: NULL argument");
    if (g->stage < ST_CLASSIFIED) return fail(g, IBM_E_STATE, "ibm_get_cell_types before ibm_classify");
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(hipMemcpyAsync(dst_device, g->type, (size_t)g->N, hipMemcpyDeviceToDevice, (hipStream_t)stream), "copy");
    return IBM_OK;
}

ibm_status ibm_get_levels(const ibm_grid *g, int *n_levels, int *dims) {
    if (!g || !n_levels) return fail(const_cast<ibm_grid *>(g), IBM_E_ARG, "ibm_get_levels: NULL argument");
    *n_levels = g->nlev;
    if (dims)
        for (int l = 0; l < g->nlev; ++l)
            for (int d = 0; d < 3; ++d) dims[3 * l + d] = g->lev[l].n[d];
    return IBM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// solve drivers
// ------------------------------------------------------------------------------------------

ibm_status ibm_get_level_map(const ibm_grid *g, int level, int axis, int *cs) {
    if (!g || !cs) return fail(nullptr, IBM_E_ARG, "ibm_get_level_map: NULL argument");
    if (level < 1 || level >= g->nlev || axis < 0 || axis > 2)
        return fail(const_cast<ibm_grid *>(g), IBM_E_ARG, "ibm_get_level_map: level or axis out of range");
    const std::vector<int> &m = g->lev[level].cs[axis];
    std::copy(m.begin(), m.end(), cs);
    return IBM_OK;
}

static ibm_status check_opts(ibm_grid *g, const ibm_solve_opts *o) {
    if (!o) return fail(g, IBM_E_ARG, "NULL options");
    if (!(o->rel_tol >= 0.0) || o->max_cycles < 1 || o->nu1 < 0 || o->nu2 < 0 || o->coarsest_sweeps < 0 ||
        o->fixed_cycles < 0 || !(o->breakdown_tol >= 0.0 && o->breakdown_tol < 1.0))
        return fail(g, IBM_E_ARG, "invalid solver options");
    if (o->precision == IBM_MIXED && g->prec != IBM_MIXED)
        return fail(g, IBM_E_STATE, "mixed precision needs a workspace bound with IBM_MIXED");
    if (o->precision != IBM_FP64 && o->precision != IBM_MIXED) return fail(g, IBM_E_ARG, "unknown precision");
    if (o->method != IBM_VCYCLE && o->method != IBM_BICGSTAB && o->method != IBM_BICGSTAB_SRJ)
        return fail(g, IBM_E_ARG, "unknown method");
    if (o->method == IBM_BICGSTAB_SRJ) {
        if (o->precision != IBM_FP64) return fail(g, IBM_E_ARG, "the scheduled-Jacobi preconditioner is FP64 only");
        if (o->srj_sweeps < 1 || o->srj_sweeps > IBM_SRJ_MAX) return fail(g, IBM_E_ARG, "srj_sweeps out of range");
        // the schedule of this solve: Chebyshev factors on [1 - cos(pi/m), 1 + cos(pi/m)]
        const int m = o->srj_sweeps;
        g->srj_omega.assign(m, 0.0);
        if (ibm_srj_schedule(std::max(0.0, std::cos(M_PI / m)), m, g->srj_omega.data()) != IBM_OK)
            return fail(g, IBM_E_ARG, "schedule");
    }
    return IBM_OK;
}

// BiCGStab outer iteration (with either preconditioner)
static bool krylov_method(int method) { return method == IBM_BICGSTAB || method == IBM_BICGSTAB_SRJ; }

// enqueue: lambda reset, reference norm, initial iterate + ghost refresh, first residual norm
static hipError_t enqueue_begin(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o, hipStream_t s) {
    hipError_t e;
    if ((e = hipMemsetAsync(g->sc, 0, offsetof(Scalars, mu), s)) != hipSuccess) return e;
    if ((e = ref_norm_pass(g, rhs, s)) != hipSuccess) return e;
    if ((e = init_solution(g, p, g->p2, o->use_initial_guess, s)) != hipSuccess) return e;
    if (krylov_method(o->method)) {
        if ((e = krylov_residual(g, rhs, g->p2, s)) != hipSuccess) return e;
    } else {
        if ((e = norm_pass(g, g->p2, rhs, s, o->precision == IBM_MIXED, true)) != hipSuccess) return e;
    }
    return hipMemcpyAsync(g->sc_host, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, s);
}

// first: the solve's first cycle
static hipError_t enqueue_cycle(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o, int *cur,
                                bool first, hipStream_t s) {
    if (krylov_method(o->method)) {
        *cur = 1;  // the Krylov iterate lives in the second buffer
        return krylov_step(g, g->p2, o, first, s);
    }
    double *bufs[2] = {p, g->p2};
    hipError_t e;
    if (o->precision == IBM_MIXED) e = vcycle_mixed(g, bufs, cur, rhs, s, o);
    else e = vcycle_f64(g, bufs, cur, rhs, s, o);
    if (e != hipSuccess) return e;
    return norm_pass(g, bufs[*cur], rhs, s, o->precision == IBM_MIXED, false);
}

// accumulate the timed smoother launches of the batch that just completed
static void prof_collect(ibm_grid *g) {
    Prof &P = g->prof;
    for (int q = 0; q + 1 < P.used; q += 2) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, P.ev[q], P.ev[q + 1]) == hipSuccess) {
            P.ms[P.kind[q / 2]] += ms;
            P.count[P.kind[q / 2]] += 1;
        }
    }
    P.used = 0;
}

// BiCGStab driver: x lives in the second pressure buffer, the gauged result goes to p
// sync_end: synchronise after the gauge (a caller that enqueues more work on the stream and
// synchronises itself passes false)
static ibm_status solve_krylov(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o,
                               ibm_solve_stats *st, hipStream_t s, bool sync_end) {
    const double t0 = now_s();
    double *x = g->p2;
    HIP_TRY(hipMemsetAsync(g->sc, 0, offsetof(Scalars, mu), s), "memset scalars");
    HIP_TRY(ref_norm_pass(g, rhs, s), "reference norm");
    HIP_TRY(init_solution(g, p, x, o->use_initial_guess, s), "init");
    HIP_TRY(krylov_residual(g, rhs, x, s), "residual");
    Scalars *hs = g->sc_host;
    HIP_TRY(hipMemcpyAsync(hs, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, s), "read");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (hs->bad) return fail(g, IBM_E_NUMERIC, "non-finite right-hand side or initial guess");
    const double r0 = hs->norm;
    if (!(hs->ref > 0.0)) {
        double ref = r0;
        HIP_TRY(hipMemcpyAsync(&g->sc->ref, &ref, sizeof(double), hipMemcpyHostToDevice, s), "set ref");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        hs->ref = ref;
    }
    ibm_status status = IBM_OK;
    int it = 0, restarts = 0;
    double rel = hs->ref > 0.0 ? r0 / hs->ref : 0.0;
    bool have_true = true;  // the scalars describe the true residual of x
    if (hs->ref > 0.0 && (o->fixed_cycles > 0 || rel > o->rel_tol)) {
        const int nit = o->fixed_cycles > 0 ? o->fixed_cycles : o->max_cycles;
        for (it = 1; it <= nit; ++it) {
            Range step_range("bicgstab step");
            HIP_TRY(krylov_step(g, x, o, it == 1, s), "bicgstab step");
            HIP_TRY(hipMemcpyAsync(hs, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, s), "read");
            HIP_TRY(hipStreamSynchronize(s), "step sync");
            if (g->prof.on) prof_collect(g);
            have_true = false;
            rel = hs->rel;
            if (hs->bad || !std::isfinite(hs->norm) || hs->norm > 1e6 * std::max(r0, hs->ref)) {
                status = IBM_E_NUMERIC;
                break;
            }
            if (o->fixed_cycles > 0) {
                if (hs->brk) {
                    HIP_TRY(krylov_restart(g, s), "restart");
                    ++restarts;
                }
                continue;
            }
            if (rel <= o->rel_tol) {
                // confirm with the true residual (this also restarts the recurrences)
                HIP_TRY(krylov_residual(g, rhs, x, s), "true residual");
                HIP_TRY(hipMemcpyAsync(hs, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, s), "read");
                HIP_TRY(hipStreamSynchronize(s), "sync");
                have_true = true;
                rel = hs->rel;
                if (rel <= o->rel_tol) break;
            } else if (hs->brk) {
                HIP_TRY(krylov_restart(g, s), "restart");
                ++restarts;
            }
        }
        if (it > nit) it = nit;
        if (status == IBM_OK && o->fixed_cycles <= 0 && rel > o->rel_tol) status = IBM_NOT_CONVERGED;
    }
    if (!have_true && status != IBM_E_NUMERIC) {
        HIP_TRY(krylov_residual(g, rhs, x, s), "final residual");
        HIP_TRY(hipMemcpyAsync(hs, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, s), "read");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        rel = hs->rel;
    }
    HIP_TRY(gauge_pass(g, x, p, s), "gauge");
    HIP_TRY(ghost_residual_pass(g, p, s), "ghost residual");
    if (sync_end) {
        HIP_TRY(hipMemcpyAsync(&hs->ghost_res, &g->sc->ghost_res, sizeof(double), hipMemcpyDeviceToHost, s), "read");
        HIP_TRY(hipStreamSynchronize(s), "gauge sync");
    }
    if (st) {
        st->cycles = it;
        st->vcycles = 2 * it;
        st->rel_residual = rel;
        st->ghost_residual_max = sync_end ? hs->ghost_res : 0.0;  // else filled by the caller after its sync
        st->lambda = hs->lambda;
        st->div_max = 0.0;
        st->t_setup = g->t_setup;
        st->t_solve = now_s() - t0;
        st->t_correct = 0.0;
        st->restarts = restarts;
    }
    if (status == IBM_E_NUMERIC) return fail(g, status, "non-finite or diverging residual");
    return status;
}

static ibm_status solve_core(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o, ibm_solve_stats *st,
                             hipStream_t s, bool sync_end = true) {
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "solve before ibm_build_ghost_stencils");
    ibm_status cs = check_opts(g, o);
    if (cs != IBM_OK) return cs;
    if (!rhs || !p) return fail(g, IBM_E_ARG, "NULL rhs or p");
    if (krylov_method(o->method)) {
        HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
        return solve_krylov(g, rhs, p, o, st, s, sync_end);
    }
    double t0 = now_s();
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(enqueue_begin(g, rhs, p, o, s), "solve begin");
    HIP_TRY(hipStreamSynchronize(s), "solve sync");
    Scalars *hs = g->sc_host;
    if (hs->bad) return fail(g, IBM_E_NUMERIC, "non-finite right-hand side or initial guess");
    double r0 = hs->norm;
    if (!(hs->ref > 0.0)) {
        // zero-mean-free right-hand side: measure against the initial residual
        double ref = r0;
        HIP_TRY(hipMemcpyAsync(&g->sc->ref, &ref, sizeof(double), hipMemcpyHostToDevice, s), "set ref");
        hs->ref = ref;
    }
    int cur = 1;
    double *bufs[2] = {p, g->p2};
    int cycles = 0;
    ibm_status status = IBM_OK;
    double rel = hs->ref > 0.0 ? r0 / hs->ref : 0.0;
    if (hs->ref > 0.0) {
        const int ncyc = o->fixed_cycles > 0 ? o->fixed_cycles : o->max_cycles;
        for (cycles = 1; cycles <= ncyc; ++cycles) {
            HIP_TRY(enqueue_cycle(g, rhs, p, o, &cur, cycles == 1, s), "cycle");
            HIP_TRY(hipMemcpyAsync(hs, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, s), "read norm");
            HIP_TRY(hipStreamSynchronize(s), "cycle sync");
            if (g->prof.on) prof_collect(g);
            rel = hs->rel;
            if (hs->bad || !std::isfinite(hs->norm)) {
                status = IBM_E_NUMERIC;
                break;
            }
            if (hs->norm > 1e3 * std::max(r0, hs->ref)) {
                status = IBM_E_NUMERIC;
                break;
            }
            if (o->fixed_cycles <= 0 && rel <= o->rel_tol) break;
        }
        if (cycles > ncyc) cycles = ncyc;
        if (status == IBM_OK && o->fixed_cycles <= 0 && rel > o->rel_tol) status = IBM_NOT_CONVERGED;
    }
    HIP_TRY(gauge_pass(g, bufs[cur], p, s), "gauge");
    HIP_TRY(ghost_residual_pass(g, p, s), "ghost residual");
    HIP_TRY(hipMemcpyAsync(&hs->ghost_res, &g->sc->ghost_res, sizeof(double), hipMemcpyDeviceToHost, s), "read");
    HIP_TRY(hipStreamSynchronize(s), "gauge sync");
    if (st) {
        st->cycles = cycles;
        st->vcycles = cycles;
        st->rel_residual = rel;
        st->ghost_residual_max = hs->ghost_res;
        st->lambda = hs->lambda;
        st->div_max = 0.0;
        st->t_setup = g->t_setup;
        st->t_solve = now_s() - t0;
        st->t_correct = 0.0;
        st->restarts = 0;
    }
    if (status == IBM_E_NUMERIC) return fail(g, status, "non-finite or diverging residual");
    return status;
}

extern "C" {

ibm_status ibm_poisson_solve(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o, ibm_solve_stats *s,
                             void *stream) {
    Range range_("ibm_poisson_solve");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_poisson_solve: NULL handle");
    return solve_core(g, rhs, p, o, s, (hipStream_t)stream);
}

ibm_status ibm_project(ibm_grid *g, double *u, double *v, double *w, double dt, double *p, const ibm_solve_opts *o,
                       ibm_solve_stats *st, void *stream) {
    Range range_("ibm_project");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_project: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_project before ibm_build_ghost_stencils");
    if (!u || !v || !w || !p) return fail(g, IBM_E_ARG, "NULL velocity or pressure");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(g, IBM_E_ARG, "dt must be positive and finite");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    double t0 = now_s();
    double *f = g->frhs;
    HIP_TRY(rhs_pass(g, u, v, w, dt, f, s), "rhs");
    ibm_status rs = solve_core(g, f, p, o, st, s, false);  // synchronised after the correction
    if (rs < 0) {
        (void)hipStreamSynchronize(s);  // nothing of the failed solve is left in flight
        return rs;
    }
    double t1 = now_s();
    HIP_TRY(correct_pass(g, u, v, w, p, dt, s), "correct");
    HIP_TRY(divmax_pass(g, u, v, w, s), "divmax");
    HIP_TRY(hipMemcpyAsync(g->sc_host, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, s), "read");
    HIP_TRY(hipStreamSynchronize(s), "project sync");
    if (st) {
        st->div_max = g->sc_host->div_max;
        st->ghost_residual_max = g->sc_host->ghost_res;
        st->t_correct = now_s() - t1;
        (void)t0;
    }
    return rs;
}

// ---- fractional-step composition ---------------------------------------------------------

ibm_status ibm_cell_to_faces(ibm_grid *g, const double *u, const double *v, const double *w, double *uf, double *vf,
                             double *wf, void *stream) {
    Range range_("ibm_cell_to_faces");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_cell_to_faces: NULL handle");
    if (g->stage < ST_BOUND) return fail(g, IBM_E_STATE, "ibm_cell_to_faces before ibm_bind_workspace");
    if (!u || !v || !w || !uf || !vf || !wf) return fail(g, IBM_E_ARG, "ibm_cell_to_faces: NULL field");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(cell_to_faces_pass(g, u, v, w, uf, vf, wf, s), "cell to faces");
    return IBM_OK;
}

ibm_status ibm_correct_cells(ibm_grid *g, double *u, double *v, double *w, const double *p, double dt, void *stream) {
    Range range_("ibm_correct_cells");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_correct_cells: NULL handle");
    if (g->stage < ST_CLASSIFIED) return fail(g, IBM_E_STATE, "ibm_correct_cells before ibm_classify");
    if (!u || !v || !w || !p) return fail(g, IBM_E_ARG, "ibm_correct_cells: NULL field");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(g, IBM_E_ARG, "dt must be positive and finite");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(correct_cells_pass(g, u, v, w, p, dt, s), "correct cells");
    return IBM_OK;
}

// ---- step API --------------------------------------------------------------------------

ibm_status ibm_solve_begin(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o, void *stream) {
    Range range_("ibm_solve_begin");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_solve_begin: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_solve_begin before ibm_build_ghost_stencils");
    ibm_status cs = check_opts(g, o);
    if (cs != IBM_OK) return cs;
    if (!rhs || !p) return fail(g, IBM_E_ARG, "NULL rhs or p");
    if (g->ss.active && !g->ss.done) return fail(g, IBM_E_STATE, "a solve is already in flight on this handle");
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    SolveState &S = g->ss;
    S.active = true;
    S.done = false;
    S.rhs = rhs;
    S.p_user = p;
    S.o = *o;
    S.stream = (hipStream_t)stream;
    S.cycles = 0;
    S.status = IBM_OK;
    S.r0 = -1.0;
    S.cur = 1;
    S.t0 = now_s();
    S.finishing = false;
    S.phase = 0;
    S.restarts = 0;
    if (!S.ev) HIP_TRY(hipEventCreateWithFlags(&S.ev, hipEventDisableTiming), "event");
    HIP_TRY(enqueue_begin(g, rhs, p, o, S.stream), "begin");
    HIP_TRY(hipEventRecord(S.ev, S.stream), "record");
    S.ev_pending = true;
    return IBM_OK;
}

ibm_status ibm_solve_step(ibm_grid *g, int n_cycles) {
    Range range_("ibm_solve_step");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_solve_step: NULL handle");
    SolveState &S = g->ss;
    if (!S.active || S.done) return fail(g, IBM_E_STATE, "no solve in flight");
    if (S.ev_pending || S.finishing) return fail(g, IBM_E_STATE, "previous step not yet polled");
    if (n_cycles < 1) return fail(g, IBM_E_ARG, "n_cycles must be >= 1");
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    const int ncyc = S.o.fixed_cycles > 0 ? S.o.fixed_cycles : S.o.max_cycles;
    for (int q = 0; q < n_cycles && S.cycles < ncyc; ++q) {
        HIP_TRY(enqueue_cycle(g, S.rhs, S.p_user, &S.o, &S.cur, S.cycles == 0, S.stream), "step");
        S.cycles++;
    }
    HIP_TRY(hipMemcpyAsync(g->sc_host, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, S.stream), "read");
    HIP_TRY(hipEventRecord(S.ev, S.stream), "record");
    S.ev_pending = true;
    return IBM_OK;
}

ibm_status ibm_solve_poll(ibm_grid *g, int *done, ibm_solve_stats *st) {
    if (!g || !done) return fail(g, IBM_E_ARG, "ibm_solve_poll: NULL argument");
    SolveState &S = g->ss;
    if (!S.active) return fail(g, IBM_E_STATE, "no solve started");
    if (S.done) {
        *done = 1;
        return (ibm_status)S.status;
    }
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    if (S.ev_pending) {
        hipError_t q = hipEventQuery(S.ev);
        if (q == hipErrorNotReady) {
            *done = 0;
            return IBM_OK;
        }
        if (q != hipSuccess) return hip_fail(g, q, "event query");
        S.ev_pending = false;
        if (g->prof.on) prof_collect(g);
        Scalars *hs = g->sc_host;
        if (S.finishing) {
            S.done = true;
            *done = 1;
            if (st) {
                st->cycles = S.cycles;
                st->vcycles = (krylov_method(S.o.method)) ? 2 * S.cycles : S.cycles;
                st->rel_residual = hs->rel;
                st->ghost_residual_max = hs->ghost_res;
                st->lambda = hs->lambda;
                st->div_max = 0.0;
                st->t_setup = g->t_setup;
                st->restarts = S.restarts;
                st->t_solve = now_s() - S.t0;
                st->t_correct = 0.0;
            }
            return (ibm_status)S.status;
        }
        bool finish = false;
        if (S.r0 < 0.0) {
            S.r0 = hs->norm;
            if (hs->bad) {
                S.status = IBM_E_NUMERIC;
                finish = true;
            } else if (!(hs->ref > 0.0)) {
                double ref = S.r0;
                hs->ref = ref;
                HIP_TRY(hipMemcpyAsync(&g->sc->ref, &g->sc_host->ref, sizeof(double), hipMemcpyHostToDevice, S.stream),
                        "set ref");
                if (!(ref > 0.0)) finish = true;
            }
        } else {
            const int ncyc = S.o.fixed_cycles > 0 ? S.o.fixed_cycles : S.o.max_cycles;
            if (hs->bad || !std::isfinite(hs->norm) || hs->norm > 1e3 * std::max(S.r0, hs->ref)) {
                S.status = IBM_E_NUMERIC;
                finish = true;
            } else if (S.o.fixed_cycles <= 0 && hs->rel <= S.o.rel_tol) {
                if (krylov_method(S.o.method) && S.phase == 0) {
                    // confirm with the true residual before finishing (restarts the recurrences)
                    HIP_TRY(krylov_residual(g, S.rhs, g->p2, S.stream), "true residual");
                    HIP_TRY(hipMemcpyAsync(g->sc_host, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, S.stream),
                            "read");
                    HIP_TRY(hipEventRecord(S.ev, S.stream), "record");
                    S.ev_pending = true;
                    S.phase = 1;
                    *done = 0;
                    return IBM_OK;
                }
                finish = true;
            } else if (S.cycles >= ncyc) {
                if (S.o.fixed_cycles <= 0) S.status = IBM_NOT_CONVERGED;
                finish = true;
            } else if (krylov_method(S.o.method)) {
                S.phase = 0;
                if (hs->brk) {
                    HIP_TRY(krylov_restart(g, S.stream), "restart");
                    ++S.restarts;
                }
            }
        }
        if (finish) {
            double *bufs[2] = {S.p_user, g->p2};
            HIP_TRY(gauge_pass(g, bufs[S.cur], S.p_user, S.stream), "gauge");
            HIP_TRY(ghost_residual_pass(g, S.p_user, S.stream), "ghost residual");
            HIP_TRY(hipMemcpyAsync(g->sc_host, g->sc, offsetof(Scalars, mu), hipMemcpyDeviceToHost, S.stream), "read");
            HIP_TRY(hipEventRecord(S.ev, S.stream), "record");
            S.ev_pending = true;
            S.finishing = true;
            *done = 0;
            return IBM_OK;
        }
        *done = -1;  // idle: waiting for ibm_solve_step
        return IBM_OK;
    }
    *done = S.finishing ? 0 : -1;
    return IBM_OK;
}

// ---- kernel-level hooks -----------------------------------------------------------------

ibm_status ibm_debug_sweep(ibm_grid *g, double *p, const double *rhs, double lambda, int n, int refresh,
                           void *stream) {
    if (!g || !p || !rhs) return fail(g, IBM_E_ARG, "ibm_debug_sweep: NULL argument");
    if (g->stage < ST_CLASSIFIED || (refresh && g->stage < ST_STENCILS))
        return fail(g, IBM_E_STATE, "ibm_debug_sweep before classification / stencils");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(hipMemcpyAsync(&g->sc->lambda, &lambda, sizeof(double), hipMemcpyHostToDevice, s), "set lambda");
    HIP_TRY(hipMemcpyAsync(g->p2, p, sizeof(double) * g->N, hipMemcpyDeviceToDevice, s), "copy");
    double *bufs[2] = {p, g->p2};
    int cur = 0;
    for (int q = 0; q < n; ++q) {
        HIP_TRY(sweep0_f64(g, bufs[cur], bufs[1 - cur], rhs, &g->sc->lambda, s), "sweep");
        if (refresh) HIP_TRY(refresh_f64(g, bufs[cur], bufs[1 - cur], s), "refresh");
        cur = 1 - cur;
    }
    if (cur == 1) HIP_TRY(hipMemcpyAsync(p, g->p2, sizeof(double) * g->N, hipMemcpyDeviceToDevice, s), "copy back");
    HIP_TRY(hipStreamSynchronize(s), "debug sync");
    return IBM_OK;
}

ibm_status ibm_debug_apply(ibm_grid *g, const double *p, double *out, void *stream) {
    if (!g || !p || !out) return fail(g, IBM_E_ARG, "ibm_debug_apply: NULL argument");
    if (g->stage < ST_CLASSIFIED) return fail(g, IBM_E_STATE, "ibm_debug_apply before classification");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(apply0_f64(g, p, out, s), "apply");
    HIP_TRY(hipStreamSynchronize(s), "apply sync");
    return IBM_OK;
}

ibm_status ibm_debug_vector(const ibm_grid *gc, int which, double *dst_device, void *stream) {
    ibm_grid *g = const_cast<ibm_grid *>(gc);
    if (!g || !dst_device) return fail(g, IBM_E_ARG, "ibm_debug_vector: NULL argument");
    if (g->stage < ST_BOUND) return fail(g, IBM_E_STATE, "ibm_debug_vector before ibm_bind_workspace");
    const double *src = nullptr;
    if (which >= 0 && which < 10) src = g->kv[which];
    else if (which == 10) src = g->p2;
    else if (which == 11) src = g->pz;
    else if (which == 12) src = g->frhs;
    if (!src) return fail(g, IBM_E_ARG, "ibm_debug_vector: which must be 0..12");
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(hipMemcpyAsync(dst_device, src, sizeof(double) * g->N, hipMemcpyDeviceToDevice, (hipStream_t)stream),
            "copy");
    return IBM_OK;
}

ibm_status ibm_debug_poison(ibm_grid *g, int on) {
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_debug_poison: NULL handle");
    g->debug_poison = on != 0;
    return IBM_OK;
}

ibm_status ibm_set_profiling(ibm_grid *g, int on) {
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_set_profiling: NULL handle");
    if (on < 0) return fail(g, IBM_E_ARG, "ibm_set_profiling: on must be >= 0");
    Prof &P = g->prof;
    if (on && P.ev.empty()) {
        HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
        P.ev.resize(64);
        P.kind.assign(32, 0);
        for (auto &e : P.ev) HIP_TRY(hipEventCreate(&e), "event create");
    }
    P.on = on != 0;
    P.stride = on > 0 ? on : 1;
    P.seq = 0;
    P.used = 0;
    P.ms[0] = P.ms[1] = 0.0;
    P.count[0] = P.count[1] = 0;
    return IBM_OK;
}

ibm_status ibm_get_profile(const ibm_grid *g, double *ms_fp64, int64_t *n_fp64, double *ms_fp32, int64_t *n_fp32) {
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_get_profile: NULL handle");
    if (ms_fp64) *ms_fp64 = g->prof.ms[0];
    if (n_fp64) *n_fp64 = g->prof.count[0];
    if (ms_fp32) *ms_fp32 = g->prof.ms[1];
    if (n_fp32) *n_fp32 = g->prof.count[1];
    return IBM_OK;
}

// ---- advection-diffusion half-step -------------------------------------------------------

void ibm_default_momentum_opts(ibm_momentum_opts *o) {
    if (!o) return;
    o->nu = 0.0;
    o->dt = 0.0;
    o->first_step = 0;
    o->srj_factors = 8;
    o->omega = nullptr;
    o->rel_tol = 1e-10;
    o->max_cycles = 200;
    o->fixed_cycles = 0;
}

ibm_status ibm_srj_schedule(double rho, int m, double *omega) {
    if (!omega || m < 1 || m > IBM_SRJ_MAX || !(rho >= 0.0 && rho < 1.0))
        return fail(nullptr, IBM_E_ARG, "ibm_srj_schedule: need 0 <= rho < 1, 1 <= m <= IBM_SRJ_MAX");
    // Chebyshev nodes of [1 - rho, 1 + rho]; the factors are their reciprocals
    std::vector<double> w(m);
    for (int k = 1; k <= m; ++k) w[k - 1] = 1.0 / (1.0 + rho * std::cos((2 * k - 1) * M_PI / (2.0 * m)));
    std::sort(w.begin(), w.end(), [](double a, double b) { return a > b; });
    // largest, smallest, second largest, second smallest, ...
    int lo = 0, hi = m - 1, q = 0;
    while (lo <= hi) {
        omega[q++] = w[lo];
        if (lo != hi) omega[q++] = w[hi];
        ++lo;
        --hi;
    }
    return IBM_OK;
}

ibm_status ibm_set_dirichlet_data(ibm_grid *g, const double *ubi, void *stream) {
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_set_dirichlet_data: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_set_dirichlet_data before ibm_build_ghost_stencils");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    if (g->ng > 0) {
        if (ubi) {
            for (int64_t q = 0; q < 3 * g->ng; ++q)
                if (!std::isfinite(ubi[q])) return fail(g, IBM_E_ARG, "non-finite Dirichlet data");
            HIP_TRY(hipMemcpyAsync(g->g_ubi, ubi, sizeof(double) * 3 * g->ng, hipMemcpyHostToDevice, s), "upload");
        } else {
            HIP_TRY(hipMemsetAsync(g->g_ubi, 0, sizeof(double) * 3 * g->ng, s), "memset");
        }
    }
    HIP_TRY(hipStreamSynchronize(s), "dirichlet sync");
    return IBM_OK;
}

ibm_status ibm_get_dirichlet_weights(const ibm_grid *gc, void *stream, double *beta, double *beta_g) {
    ibm_grid *g = const_cast<ibm_grid *>(gc);
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_get_dirichlet_weights: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_get_dirichlet_weights before stencils");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    if (g->ng > 0) {
        if (beta) HIP_TRY(hipMemcpyAsync(beta, g->g_betaD, sizeof(double) * 8 * g->ng, hipMemcpyDeviceToHost, s), "copy");
        if (beta_g) HIP_TRY(hipMemcpyAsync(beta_g, g->g_betaDg, sizeof(double) * g->ng, hipMemcpyDeviceToHost, s), "copy");
    }
    HIP_TRY(hipStreamSynchronize(s), "get_dirichlet sync");
    return IBM_OK;
}

ibm_status ibm_momentum_step(ibm_grid *g, double *u, double *v, double *w, double *hu, double *hv, double *hw,
                             const ibm_momentum_opts *o, ibm_momentum_stats *st, void *stream) {
    Range range_("ibm_momentum_step");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_momentum_step: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_momentum_step before ibm_build_ghost_stencils");
    if (!o) return fail(g, IBM_E_ARG, "NULL options");
    if (!u || !v || !w || !hu || !hv || !hw) return fail(g, IBM_E_ARG, "NULL velocity or convective-term array");
    if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(g, IBM_E_ARG, "dt must be positive and finite");
    if (!(o->nu >= 0.0) || !std::isfinite(o->nu)) return fail(g, IBM_E_ARG, "nu must be non-negative and finite");
    const int m = o->srj_factors;
    if (m < 1 || m > IBM_SRJ_MAX) return fail(g, IBM_E_ARG, "srj_factors out of range");
    if (o->fixed_cycles <= 0 && (o->max_cycles < 1 || !(o->rel_tol > 0.0)))
        return fail(g, IBM_E_ARG, "need max_cycles >= 1 and rel_tol > 0, or fixed_cycles > 0");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    const double t0 = now_s();
    const double a = 0.5 * o->nu * o->dt;
    // the largest diagonal flux sum (separable: the per-axis maxima add up), read once
    if (g->diag_max < 0.0) {
        double dmax = 0.0;
        const int n[3] = {g->nx, g->ny, g->nz};
        for (int d = 0; d < 3; ++d) {
            std::vector<double> am(n[d]), ap(n[d]);
            HIP_TRY(hipMemcpy(am.data(), g->am0[d], sizeof(double) * n[d], hipMemcpyDeviceToHost), "read metrics");
            HIP_TRY(hipMemcpy(ap.data(), g->ap0[d], sizeof(double) * n[d], hipMemcpyDeviceToHost), "read metrics");
            double mx = 0.0;
            for (int i = 0; i < n[d]; ++i) mx = std::max(mx, am[i] + ap[i]);
            dmax += mx;
        }
        g->diag_max = dmax;
    }
    const double rho = (a * g->diag_max) / (1.0 + a * g->diag_max);
    std::vector<double> om(m);
    if (o->omega) {
        for (int k = 0; k < m; ++k) {
            if (!std::isfinite(o->omega[k]) || !(o->omega[k] > 0.0)) return fail(g, IBM_E_ARG, "invalid omega");
            om[k] = o->omega[k];
        }
    } else {
        ibm_status e = ibm_srj_schedule(rho, m, om.data());
        if (e != IBM_OK) return fail(g, e, "schedule");
    }
    double *uvw[3] = {u, v, w}, *hc[3] = {hu, hv, hw};
    double *work[6] = {g->kv[0], g->kv[1], g->kv[2], g->kv[3], g->kv[4], g->kv[5]};
    double *wk[3] = {work[3], work[4], work[5]};
    HIP_TRY(momentum_enqueue_prep(g, uvw, hc, work, o->dt, a, o->first_step ? 1 : 0, s), "momentum rhs");
    double *const *X = uvw;
    double *const *Y = wk;
    const int ncyc = o->fixed_cycles > 0 ? o->fixed_cycles : o->max_cycles;
    Scalars *hs = g->sc_host;
    ibm_status status = IBM_OK;
    int cyc = 0;
    double rel = 0.0;
    for (cyc = 1; cyc <= ncyc; ++cyc) {
        for (int k = 0; k < m; ++k) {
            HIP_TRY(momentum_enqueue_sweep(g, X, Y, work, a, om[k], k == m - 1, s), "srj sweep");
            std::swap(X, Y);
        }
        HIP_TRY(hipMemcpyAsync(&hs->mom_b2, &g->sc->mom_b2, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "read");
        HIP_TRY(hipStreamSynchronize(s), "cycle sync");
        const double bn = std::sqrt(hs->mom_b2);
        rel = bn > 0.0 ? std::sqrt(hs->mom_r2) / bn : 0.0;
        if (!std::isfinite(rel) || !std::isfinite(hs->mom_b2)) {
            status = IBM_E_NUMERIC;
            break;
        }
        if (o->fixed_cycles <= 0 && rel <= o->rel_tol) break;
    }
    if (cyc > ncyc) {
        cyc = ncyc;
        if (o->fixed_cycles <= 0 && status == IBM_OK) status = IBM_NOT_CONVERGED;
    }
    if (X != uvw) {  // the last iterate is in the workspace
        for (int q = 0; q < 3; ++q)
            HIP_TRY(hipMemcpyAsync(uvw[q], X[q], sizeof(double) * g->N, hipMemcpyDeviceToDevice, s), "copy back");
    }
    HIP_TRY(hipStreamSynchronize(s), "momentum sync");
    if (st) {
        st->cycles = cyc;
        st->sweeps = cyc * m;
        st->rel_residual = rel;
        st->rho = rho;
        st->t_step = now_s() - t0;
    }
    if (status == IBM_E_NUMERIC) return fail(g, status, "non-finite residual in the advection-diffusion solve");
    return status;
}

// ---- moving bodies: fresh cells -----------------------------------------------------------

ibm_status ibm_move_geometry(ibm_grid *g, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                             void *stream, int64_t counts_out[3], int64_t *n_fresh_out) {
    Range range_("ibm_move_geometry");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_move_geometry: NULL handle");
    if (g->stage < ST_STENCILS) return fail(g, IBM_E_STATE, "ibm_move_geometry before a first geometry's stencils");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    HIP_TRY(hipMemcpyAsync(g->type_prev, g->type, (size_t)g->N, hipMemcpyDeviceToDevice, s), "save types");
    g->nfresh = 0;
    ibm_status st = set_geometry_impl(g, verts, nv, tris, nt, stream, true);
    if (st != IBM_OK) return st;
    int64_t counts[3];
    if ((st = ibm_classify(g, stream, counts)) != IBM_OK) return st;
    int64_t ng = 0;
    if ((st = ibm_build_ghost_stencils(g, stream, &ng)) != IBM_OK) return st;
    int64_t nf = 0;
    HIP_TRY(launch_fresh(g, s, &nf), "fresh cells");
    if (nf > g->ghost_max)
        return fail(g, IBM_E_NOMEM, "more fresh cells (" + std::to_string(nf) + ") than the ghost capacity " +
                                        std::to_string(g->ghost_max) + ": move in smaller steps or bind more");
    if (nf > 0) HIP_TRY(hipMemsetAsync(g->f_ubi, 0, sizeof(double) * 3 * nf, s), "memset");
    HIP_TRY(hipStreamSynchronize(s), "move sync");
    g->nfresh = nf;
    if (counts_out)
        for (int q = 0; q < 3; ++q) counts_out[q] = counts[q];
    if (n_fresh_out) *n_fresh_out = nf;
    return IBM_OK;
}

ibm_status ibm_get_fresh(const ibm_grid *gc, void *stream, int32_t *cell, double *bi_xyz, double *ip_xyz,
                         int32_t *stencil, double *beta, double *beta_c, int32_t *flags) {
    ibm_grid *g = const_cast<ibm_grid *>(gc);
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_get_fresh: NULL handle");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    const int64_t n = g->nfresh;
    if (n > 0) {
        if (cell) HIP_TRY(hipMemcpyAsync(cell, g->f_cell, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s), "copy");
        if (bi_xyz) HIP_TRY(hipMemcpyAsync(bi_xyz, g->f_bi, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s), "copy");
        if (ip_xyz) HIP_TRY(hipMemcpyAsync(ip_xyz, g->f_ip, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s), "copy");
        if (stencil) HIP_TRY(hipMemcpyAsync(stencil, g->f_st, sizeof(int32_t) * 8 * n, hipMemcpyDeviceToHost, s), "copy");
        if (beta) HIP_TRY(hipMemcpyAsync(beta, g->f_beta, sizeof(double) * 8 * n, hipMemcpyDeviceToHost, s), "copy");
        if (beta_c) HIP_TRY(hipMemcpyAsync(beta_c, g->f_betac, sizeof(double) * n, hipMemcpyDeviceToHost, s), "copy");
        if (flags) HIP_TRY(hipMemcpyAsync(flags, g->f_flags, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s), "copy");
    }
    HIP_TRY(hipStreamSynchronize(s), "get_fresh sync");
    return IBM_OK;
}

ibm_status ibm_fill_fresh(ibm_grid *g, double *u, double *v, double *w, const double *ubi, void *stream) {
    Range range_("ibm_fill_fresh");
    if (!g) return fail(nullptr, IBM_E_ARG, "ibm_fill_fresh: NULL handle");
    if (!u || !v || !w) return fail(g, IBM_E_ARG, "NULL velocity array");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
    const int64_t n = g->nfresh;
    if (n > 0) {
        if (ubi) {
            for (int64_t q = 0; q < 3 * n; ++q)
                if (!std::isfinite(ubi[q])) return fail(g, IBM_E_ARG, "non-finite intercept velocity");
            HIP_TRY(hipMemcpyAsync(g->f_ubi, ubi, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s), "upload");
        } else {
            HIP_TRY(hipMemsetAsync(g->f_ubi, 0, sizeof(double) * 3 * n, s), "memset");
        }
        double *uvw[3] = {u, v, w};
        HIP_TRY(fresh_enqueue_fill(g, uvw, s), "fresh fill");
    }
    HIP_TRY(hipStreamSynchronize(s), "fill sync");
    return IBM_OK;
}

void ibm_destroy_grid(ibm_grid *g) {
    if (!g) return;
    for (auto &e : g->prof.ev) (void)hipEventDestroy(e);
    if (g->ss.ev) (void)hipEventDestroy(g->ss.ev);
    if (g->sc_host) (void)hipHostFree(g->sc_host);
    delete g;
}

const char *ibm_last_error(const ibm_grid *g) {
    if (g) return g->err.c_str();
    return t_last_error.c_str();
}

}  // extern "C"
