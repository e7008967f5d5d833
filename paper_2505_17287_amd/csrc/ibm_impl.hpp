// Internal declarations of the gfx950 ghost-cell IBM projection library.
//
// Data layout in HBM (all inside the caller-owned workspace):
//   level 0 : cell type (uint8), second pressure buffer (FP64), FP32 error / residual
//             buffers for the mixed-precision path; cell fields are [nz][ny][nx].
//   metrics : 1D per-axis arrays (centres, widths, centre distances, flux coefficients),
//             so the 7-point operator of a cell is rebuilt from six scalar loads.
//   geometry: mesh, a uniform triangle bucket grid (closest-point search), per-column ray
//             crossings (classification), and the ghost list in structure-of-arrays form.
//   levels  : per coarse level the error and right-hand side, the active mask and the
//             staircase transmissibilities of each cell's three low faces, plus the
//             per-axis prolongation tables.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/ibm.h"

namespace ibm {

constexpr uint8_t T_FLUID = 0, T_GHOST = 1, T_DEAD = 2;
constexpr int GF_DEGENERATE = 1, GF_CLAMPED = 2, GF_NFALLBACK = 4, GF_SELF = 8;
constexpr int MAX_LEVELS = 24;
constexpr int RED_BLOCKS = 4096;  // fixed block count of the deterministic reductions (enough waves to fill every SIMD)
constexpr int NBUCKET_MAX = 1 << 21;

// ---------------------------------------------------------------------------------------
// device views
// ---------------------------------------------------------------------------------------

template <typename T>
struct AxisCoef {  // per-axis arrays of one level
    const T *am, *ap;  // level 0: per-volume flux coefficients; unused on coarse levels
    const T *w;        // widths
};

template <typename T>
struct Fine {  // level-0 operator view in precision T
    int nx, ny, nz;
    const T *axm, *axp, *aym, *ayp, *azm, *azp;
    const T *wx, *wy, *wz;
    const uint8_t *type;
    const uint8_t *inject;  // 1: fluid cell whose prolongation has an inactive coarse contributor
};

template <typename T>
struct Coarse {  // coarse-level view in precision T
    int n[3];
    const T *w[3];        // widths
    const uint8_t *active;
    const T *Tl[3];       // transmissibility of each cell's low face (integrated form)
    T *e, *R;
    const double *mu;     // compatibility shift per unit volume (device scalar)
};

// fused red-black sweep of level 0 (sweep.hip): pout = one RB-GS sweep of pin; ev0, ev1
// (optional): events recorded when the kernel starts and when it ends
template <typename T>
hipError_t launch_sweep(const Fine<T> &F, const T *pin, T *pout, const T *f, const T *lam, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// the same FP32 sweep writing its result widened to FP64, dead cells zero
hipError_t launch_sweep_widen(const Fine<float> &F, const float *pin, double *pout, const float *f, const float *lam,
                              hipStream_t s);

// fused red-black sweep of a coarse level (sweepc.hip): eout = one RB-GS sweep of L.e, the
// two buffers distinct; for levels of at least SWC_MIN_CELLS cells (sweepC_fused_ok)
bool sweepC_fused_ok(const int n[3]);
template <typename T>
hipError_t launch_sweepC_fused(const Coarse<T> &L, T *eout, hipStream_t s);

// fine index -> (lo, hi, weight of hi) per axis; lo is always the parent (the coarse cell
// holding the fine one)
struct ProlongTab {
    const int *lo[3], *hi[3];
    const double *t[3];
    int halved[3];  // 1: the axis is halved uniformly (fine 2I and 2I+1 make coarse I)
};

// Children of a coarse level (device): coarse index I along axis d holds the finer cells
// cs[d][I] .. cs[d][I+1]-1 (one or two).
struct ChildMap {
    const int *cs[3];
    int halved[3];  // 1: uniform halving along d
    int same[3];    // 1: nothing merged along d (cs[I] = I)
};

// z-march passes of level 0 (finepass.hip).  The reductions write one partial per
// workgroup; *nparts receives their count (at most zmarch_partials_max).
template <typename T>
hipError_t launch_restrict0(const Fine<T> &F, const T *p, const T *f, const T *lam, const Coarse<T> &C,
                            const ChildMap &M, double *partials, int *nparts, hipStream_t s);
template <typename T>
hipError_t launch_prolong0(const Fine<T> &F, const T *pcur, T *pnext, const Coarse<T> &C, const ProlongTab &P,
                           hipStream_t s);
// Krylov operator on fluid rows.  dots 0: w = S y, one sum per workgroup (sum V w).  dots 1
// and 2: w = S y - *mu (device scalar: the image's volume-weighted fluid mean), sums of o w and
// (dots 2) of w w per workgroup, stored with a stride of 1 or 2.  dots 3: the residual
// w = o - S y (o the right-hand side; mu unused), sum V w per workgroup.
hipError_t launch_apply_fluid(const Fine<double> &F, const double *y, double *w, const double *o, const double *mu,
                              int dots, double *partials, int *nparts, hipStream_t s);
hipError_t launch_jacobi0(const Fine<double> &F, const double *y, const double *f, double *out, double omega,
                          hipStream_t s);
int64_t zmarch_partials_max(int nx, int ny, int nz);

// Tiling of the row-wise restrictions (a wave per coarse row: RM_CX coarse columns, RM_W
// coarse rows and kc coarse planes per workgroup of 64 RM_W threads), taken tile by tile
// in a grid-stride loop.  row_tiles picks the z chunks for about per_cu tiles per CU with
// at least kmin coarse planes each (fewer when the level has fewer) and returns the grid:
// a multiple of 8, at most the tile count rounded up and at most cap (a multiple of 8).
constexpr int RM_CX = 32, RM_W = 4, RM_NT = 64 * RM_W;
struct RowTiles {
    int ntx, nty, kc, ntiles;
};
hipError_t row_tiles(const int cn[3], int per_cu, int kmin, int64_t cap, RowTiles *t, int *grid);

struct GhostView {
    int64_t ng;
    const int32_t *cell;
    const int32_t *st;      // 8 per ghost, -1 = unused / own Neumann slot
    const uint8_t *gmask;   // bit m: member m is a ghost cell
    const double *beta;     // 8 per ghost
    const double *h;        // right-hand side of the ghost equation
    const int32_t *flags;
};

// reduction scratch shared by the solver kernels (device)
struct Scalars {
    double lambda;      // current uniform source shift
    double delta;       // lambda_{k+1} - lambda_k (mixed path: FP64)
    float delta32;      // same, FP32 (inner right-hand side shift)
    float pad0;
    double norm;        // ||r - lambda||_2 after the last norm pass
    double rel;         // norm / ref
    double ref;         // reference norm ||f - Vmean(f)||
    double vmean;       // scratch mean
    double div_max;
    double ghost_res;   // max ghost-equation residual of the returned pressure
    int bad;            // non-finite seen
    int pad1;
    // Krylov (BiCGStab) scalars
    double rho, rho_old, alpha, omega, beta;
    double mu_v;        // volume-weighted fluid mean removed from an operator image
    double zero;        // constant 0 (shift of the preconditioner's right-hand side)
    float zero32, pad2;
    double rh2;         // squared norm of the shadow residual (set when it is (re)started)
    int brk;            // near-breakdown seen in the last step: the host restarts the shadow residual
    int pad3;
    double mu[MAX_LEVELS];
    double vol[MAX_LEVELS];   // summed volume of the active cells of each level
    double mom_b2;            // advection-diffusion step: sum of b^2 over fluid rows
    double mom_r2;            // sum of r^2 at the input of the last sweep
};

// ---------------------------------------------------------------------------------------
// host-side state
// ---------------------------------------------------------------------------------------

struct LevelHost {
    int n[3];
    int halved[3];  // uniform halving relative to the next finer level (see plan_levels)
    int same[3];    // nothing merged relative to the next finer level
    std::vector<double> f[3], c[3], w[3];
    std::vector<int> cs[3];  // children starts in the next finer level (levels >= 1)
    int *cs_d[3] = {nullptr, nullptr, nullptr};  // device copy of cs
    int64_t ncell() const { return (int64_t)n[0] * n[1] * n[2]; }
    // device
    uint8_t *active = nullptr;
    double *T64[3] = {nullptr, nullptr, nullptr};
    float *T32[3] = {nullptr, nullptr, nullptr};
    double *w64[3] = {nullptr, nullptr, nullptr};
    float *w32[3] = {nullptr, nullptr, nullptr};
    double *c64[3] = {nullptr, nullptr, nullptr};
    double *e64 = nullptr, *R64 = nullptr;
    float *e32 = nullptr, *R32 = nullptr;
    // second error buffer of the out-of-place coarse sweep (levels that sweepC_fused_ok
    // accepts); swapped with e after each sweep
    double *e64b = nullptr;
    float *e32b = nullptr;
    // prolongation tables of THIS level from the next coarser one
    int *plo[3] = {nullptr, nullptr, nullptr}, *phi[3] = {nullptr, nullptr, nullptr};
    // every halved axis: the second contributor of cell 2I is I-1 and of 2I+1 is I+1 (or none
    // at a wall), which the fully halved prolongation kernel relies on (checked on the host
    // with the arithmetic the device tables use)
    bool prolong_sides = false;
    double *pt[3] = {nullptr, nullptr, nullptr};
    double vol_active = 0.0;  // device-computed, copied back at hierarchy build
};

enum Stage { ST_CREATED = 0, ST_BOUND = 1, ST_GEOMETRY = 2, ST_CLASSIFIED = 3, ST_STENCILS = 4 };

struct SolveState {  // in-flight solve of the step API
    bool active = false, done = true;
    const double *rhs = nullptr;
    double *p_user = nullptr;
    ibm_solve_opts o{};
    hipStream_t stream = nullptr;
    int cycles = 0, status = 0;
    int pending = 0;            // cycles enqueued since the last poll read
    double r0 = 0.0;
    hipEvent_t ev = nullptr;
    bool ev_pending = false;
    int cur = 0;                // which buffer holds the iterate (0 = user p, 1 = workspace)
    bool finishing = false;     // gauge enqueued, waiting for its event
    int phase = 0;              // BiCGStab: 1 while a true-residual confirmation is in flight
    int restarts = 0;           // BiCGStab restarts after a near-breakdown
    double t0 = 0.0;
};

// optional per-launch timing of the level-0 smoother (HIP events on the launch stream)
struct Prof {
    bool on = false;
    int stride = 1;              // time every stride-th level-0 sweep
    long long seq = 0;           // level-0 sweeps launched since profiling was switched on
    std::vector<hipEvent_t> ev;  // start/stop pairs
    std::vector<int> kind;       // per pair: 0 FP64 sweep, 1 FP32 sweep
    int used = 0;
    double ms[2] = {0.0, 0.0};
    long long count[2] = {0, 0};
};

}  // namespace ibm

struct ibm_grid {
    int nx, ny, nz;
    int64_t N;
    std::vector<double> xf, yf, zf;
    int stage = ibm::ST_CREATED;
    std::string err;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t nv_max = 0, nt_max = 0, ghost_max = 0;
    ibm_precision prec = IBM_FP64;
    int device = 0;
    // level-0 device arrays
    uint8_t *type = nullptr;
    uint8_t *inject0 = nullptr;            // per cell: prolongation falls back to injection
    double *p2 = nullptr;                  // second FP64 pressure buffer
    double *frhs = nullptr;                // projection right-hand side
    float *e32a = nullptr, *e32b = nullptr, *r32 = nullptr;
    // start iterate of the Krylov preconditioner's V-cycle: zero except at the ghost cells,
    // whose values are written before each use (cleared whenever the ghost list is rebuilt)
    double *pz = nullptr;
    float *pz32 = nullptr;
    double *faces[3] = {nullptr, nullptr, nullptr};
    double *c0[3] = {nullptr, nullptr, nullptr}, *w0[3] = {nullptr, nullptr, nullptr};
    double *dc0[3] = {nullptr, nullptr, nullptr};
    double *am0[3] = {nullptr, nullptr, nullptr}, *ap0[3] = {nullptr, nullptr, nullptr};
    float *am0f[3] = {nullptr, nullptr, nullptr}, *ap0f[3] = {nullptr, nullptr, nullptr};
    float *w0f[3] = {nullptr, nullptr, nullptr};
    // mesh and geometry scratch
    int64_t nv = 0, nt = 0;
    double *verts = nullptr;
    int32_t *tris = nullptr;
    int32_t *bucket_off = nullptr, *bucket_cnt = nullptr, *bucket_ent = nullptr;
    int nb[3] = {1, 1, 1};
    double bmin[3] = {0, 0, 0}, bsize[3] = {1, 1, 1};
    double bext[3] = {0, 0, 0};  // largest triangle extent per axis (padded for rounding)
    int32_t *col_cnt = nullptr, *col_off = nullptr, *col_fill = nullptr;
    double *crossings = nullptr;
    int64_t cross_cap = 0;
    int32_t *blk_cnt = nullptr;            // per-block counts for compaction / scans
    int64_t *counters = nullptr;           // device counters (fluid, ghost, dead, odd, overflow...)
    // ghosts
    int64_t ng = 0;
    int64_t ndegenerate = 0;
    int32_t *g_cell = nullptr, *g_st = nullptr, *g_flags = nullptr, *g_tri = nullptr;
    uint8_t *g_mask = nullptr;
    double *g_bi = nullptr, *g_n = nullptr, *g_ip = nullptr, *g_beta = nullptr, *g_betag = nullptr;
    double *g_dl = nullptr, *g_h = nullptr, *g_data = nullptr;
    double *g_scale = nullptr;             // diagonal of the flux stencil at each ghost cell
    double *g_rhs = nullptr;               // ghost right-hand sides of a preconditioner call
    double *g_betaD = nullptr;             // 8 per ghost: Dirichlet (velocity) weights
    double *g_betaDg = nullptr;            // per ghost: weight of the intercept value
    double *g_ubi = nullptr;               // 3 per ghost: velocity at the body intercept
    double *g_uscr = nullptr;              // 3 per ghost: held-back ghost values of an in-place pass
    std::vector<int32_t> topo_tris;        // triangle indices of the last validated mesh
    int64_t topo_nv = 0;                   // and its vertex count
    bool topo_valid = false;
    // fresh cells of the last move (capacity ghost_max)
    uint8_t *type_prev = nullptr;          // cell types before the move
    int64_t nfresh = 0;
    int32_t *f_cell = nullptr, *f_tri = nullptr, *f_st = nullptr, *f_flags = nullptr;
    double *f_bi = nullptr, *f_ip = nullptr, *f_beta = nullptr, *f_betac = nullptr, *f_ubi = nullptr,
           *f_scr = nullptr;
    double diag_max = -1.0;                // max over cells of the flux-coefficient sum (< 0: not read yet)
    double t_setup = 0.0;                  // seconds of the last set_geometry + classify + stencils
    std::vector<double> srj_omega;         // relaxation factors of the scheduled-Jacobi preconditioner
    // Krylov vectors (FP64, full grid)
    double *kv[10] = {nullptr};
    // multigrid
    int nlev = 0;
    ibm::LevelHost lev[ibm::MAX_LEVELS];
    double *partials = nullptr;            // RED_BLOCKS * 4 doubles
    ibm::Scalars *sc = nullptr;            // device scalars
    ibm::Scalars *sc_host = nullptr;       // pinned host mirror
    int64_t nfluid = 0, nghost_cells = 0, ndead = 0;
    double vol_fluid = 0.0;
    ibm::SolveState ss;
    ibm::Prof prof;
    // debug: fill every floating-point sub-buffer of the workspace with NaN at bind time
    // (ibm_debug_poison), so a value read before the library wrote it shows up
    bool debug_poison = false;
};

namespace ibm {

// workspace planner: computes offsets (base == nullptr -> sizing only)
struct Plan {
    size_t off = 0;
    char *base = nullptr;
    // optional: (offset, bytes) of every floating-point sub-buffer, for the poisoned bind
    std::vector<std::pair<size_t, size_t>> *fp_spans = nullptr;
    template <typename T>
    T *take(int64_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        const size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
        if (fp_spans && std::is_floating_point<T>::value) fp_spans->emplace_back(off, bytes);
        off += bytes;
        return p;
    }
};

// hierarchy plan on the host (dims + coarse faces), same rule for sizing and binding
// the level's child map (device pointers; level >= 1)
ChildMap child_map(const LevelHost &C);
void plan_levels(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                 LevelHost *lev, int *nlev);
size_t layout(ibm_grid *g, Plan &P, int nx, int ny, int nz, int64_t nv_max, int64_t nt_max, int64_t gmax,
              ibm_precision prec, LevelHost *lev, int nlev);

// classification buffers (geometry.hip): a handle's workspace or the static scratch of the
// no-allocation entry point
struct ClassifyBufs {
    int nx, ny, nz;
    const double *verts;
    const int32_t *tris;
    int64_t nt;
    const double *xc, *yc, *zc;           // cell centres per axis
    int32_t *col_cnt, *col_off, *col_fill;  // ncol + 1 each
    double *crossings;
    int64_t cross_cap;
    int64_t *counters;                    // 8
    int64_t *blk;                         // classify_scan_blocks(ncol + 1)
    int64_t *mark_parts;                  // classify_mark16_parts(nx, ny, nz)
    uint8_t *type;
};
hipError_t launch_classify_cells(const ClassifyBufs &B, hipStream_t s);
int64_t classify_mark16_parts(int nx, int ny, int nz);
int64_t classify_scan_blocks(int64_t n);

// error reporting shared by the entry points (api.hip): sets the thread's last error
ibm_status report_error(ibm_status st, const std::string &msg);

// kernel launchers (geometry.hip)
hipError_t launch_metrics(ibm_grid *g, hipStream_t s);
hipError_t launch_buckets(ibm_grid *g, hipStream_t s);
hipError_t launch_classify(ibm_grid *g, hipStream_t s, int64_t counts[4]);
hipError_t launch_stencils(ibm_grid *g, hipStream_t s);
hipError_t launch_ghost_h(ibm_grid *g, hipStream_t s);
hipError_t launch_hierarchy(ibm_grid *g, hipStream_t s);
hipError_t launch_fresh(ibm_grid *g, hipStream_t s, int64_t *nfresh);

// solver launchers (solver.hip)
hipError_t sweep0_f64(ibm_grid *g, const double *pin, double *pout, const double *f, const double *lambda,
                      hipStream_t s);
hipError_t refresh_f64(ibm_grid *g, const double *src_ghost, double *dst, hipStream_t s);
hipError_t apply0_f64(ibm_grid *g, const double *p, double *out, hipStream_t s);
hipError_t vcycle_f64(ibm_grid *g, double **bufs, int *cur, const double *f, hipStream_t s, const ibm_solve_opts *o);
hipError_t vcycle_mixed(ibm_grid *g, double **bufs, int *cur, const double *f, hipStream_t s,
                        const ibm_solve_opts *o);
hipError_t norm_pass(ibm_grid *g, const double *p, const double *f, hipStream_t s, bool write_r32, bool first);
hipError_t ref_norm_pass(ibm_grid *g, const double *f, hipStream_t s);
hipError_t gauge_pass(ibm_grid *g, const double *pcur, double *pdst, hipStream_t s);
hipError_t ghost_residual_pass(ibm_grid *g, const double *p, hipStream_t s);
hipError_t rhs_pass(ibm_grid *g, const double *u, const double *v, const double *w, double dt, double *f,
                    hipStream_t s);
hipError_t cell_to_faces_pass(ibm_grid *g, const double *u, const double *v, const double *w, double *uf,
                              double *vf, double *wf, hipStream_t s);
hipError_t correct_cells_pass(ibm_grid *g, double *u, double *v, double *w, const double *p, double dt,
                              hipStream_t s);
hipError_t correct_pass(ibm_grid *g, double *u, double *v, double *w, const double *p, double dt,
                        hipStream_t s);
hipError_t divmax_pass(ibm_grid *g, const double *u, const double *v, const double *w, hipStream_t s);
hipError_t init_solution(ibm_grid *g, double *p, double *p2, int use_guess, hipStream_t s);
hipError_t krylov_setup(ibm_grid *g, hipStream_t s);
hipError_t krylov_residual(ibm_grid *g, const double *f, const double *x, hipStream_t s);
// first: the first step after krylov_residual of a new solve (p and v are not read)
hipError_t krylov_step(ibm_grid *g, double *x, const ibm_solve_opts *o, bool first, hipStream_t s);
// the handle's last geometry set-up time is g->t_setup (seconds, host wall clock)
hipError_t krylov_restart(ibm_grid *g, hipStream_t s);

// advection-diffusion half-step launchers (momentum.hip)
hipError_t momentum_enqueue_prep(ibm_grid *g, double *const uvw[3], double *const hc[3], double *const work[6],
                                 double dt, double a, int first, hipStream_t s);
hipError_t momentum_enqueue_sweep(ibm_grid *g, double *const X[3], double *const Y[3], double *const work[6],
                                  double a, double omega, bool sum, hipStream_t s);
hipError_t fresh_enqueue_fill(ibm_grid *g, double *const uvw[3], hipStream_t s);

}  // namespace ibm
