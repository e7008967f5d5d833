/*
 * ibm.h -- C ABI of the MI355X (gfx950) ghost-cell immersed-boundary projection library.
 *
 * The library implements the pressure-projection half of the fractional-step method
 * (Kumar, Seo, Mittal, Romero, Fatica, "A GPU-Accelerated Sharp-Interface Immersed
 * Boundary Solver for Large-Scale Flow Simulations", Section 2.1) with the ghost-cell
 * treatment of an immersed triangulated body (Section 2.2, Eq. 2 and Eq. 3):
 *
 *     classify cells -> ghost-cell stencils -> pressure Poisson solve -> velocity correction
 *
 * Conventions shared by every entry point
 *   - Every function returns ibm_status.  Negative values are errors; positive values are
 *     usable results with a warning (see ibm_solve_stats).  A failed call leaves the handle
 *     usable; ibm_last_error() describes the last failure.
 *   - Cell fields are FP64, contiguous, layout [nz][ny][nx] (x fastest).  Face-normal
 *     velocities use the staggered (MAC) layout u[nz][ny][nx+1], v[nz][ny+1][nx],
 *     w[nz+1][ny][nx].  A grid with nz == 1 is two-dimensional (no z coupling, bilinear
 *     4-cell stencils).
 *   - "host" pointers are read during the call and copied; "device" pointers must point to
 *     device memory of the workspace's device and are only borrowed for the call.
 *   - All GPU work is enqueued on `stream` (a hipStream_t; NULL = the default stream).
 *     The library never allocates device memory: every device buffer it uses lives in the
 *     caller-owned workspace bound by ibm_bind_workspace (small pinned host buffers are
 *     allocated at grid creation for status read-back).
 *   - Call order: create -> bind_workspace -> set_geometry -> classify ->
 *     build_ghost_stencils -> poisson_solve / project.  Out-of-order calls return
 *     IBM_E_STATE; set_geometry invalidates classification and stencils.
 *   - One host thread per handle at a time.  Distinct handles are independent and may run
 *     concurrently on different streams.
 */
#ifndef IBM_H
#define IBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibm_grid ibm_grid; /* opaque: one per problem */

typedef enum {
    IBM_OK = 0,
    IBM_NOT_CONVERGED = 1, /* max_cycles reached; p and stats are valid */
    IBM_E_ARG = -1,        /* invalid argument (sizes, non-monotone or non-finite coordinates) */
    IBM_E_STATE = -2,      /* call out of order */
    IBM_E_GEOMETRY = -3,   /* mesh not closed / not consistently oriented, or no fluid cell */
    IBM_E_NOMEM = -4,      /* workspace too small for this grid / mesh / ghost count */
    IBM_E_DEVICE = -5,     /* HIP error; message in ibm_last_error */
    IBM_E_NUMERIC = -6     /* NaN/Inf or divergence; p holds the last finite iterate */
} ibm_status;

typedef enum { IBM_FP64 = 0, IBM_MIXED = 1 } ibm_precision;

/* Outer iteration of the pressure solve.
   IBM_VCYCLE  : repeated V-cycles (stationary multigrid iteration).
   IBM_BICGSTAB: BiCGStab (the paper's pressure solver family, Section 2.1) right-
                 preconditioned by one V-cycle per preconditioner application.  Ghost rows
                 enter the Krylov operator scaled by the local stencil diagonal, and the
                 fluid part of every residual is projected to zero volume-weighted mean (the
                 uniform source shift lambda).  Both methods converge to the same solution. */
typedef enum { IBM_VCYCLE = 0, IBM_BICGSTAB = 1, IBM_BICGSTAB_SRJ = 2 } ibm_method;
/* IBM_BICGSTAB_SRJ: the paper's own configuration (Section 2.1: BiCGStab with a scheduled
   relaxed Jacobi preconditioner): each preconditioner application is srj_sweeps relaxed
   Jacobi sweeps from zero, with the factors ibm_srj_schedule(max(0, cos(pi / srj_sweeps)),
   srj_sweeps), each sweep followed by the ghost refresh.  FP64 only. */

/* Solver options.  Defaults (ibm_default_opts): rel_tol 1e-10, max_cycles 200, V(2,2),
   16 sweeps on the coarsest level, FP64, zero initial guess, convergence-tested,
   BiCGStab outer iteration, breakdown_tol 1e-12. */
typedef struct {
    double rel_tol;          /* stop when ||r'||_2 <= rel_tol * ||f - Vmean(f)||_2 (fluid rows) */
    int max_cycles;          /* V-cycles (FP64) or refinement steps (mixed) */
    int nu1, nu2;            /* pre- and post-smoothing sweeps per level */
    int coarsest_sweeps;     /* red-black sweeps on the coarsest level */
    ibm_precision precision; /* IBM_MIXED: FP32 V-cycle inside FP64 iterative refinement */
    int use_initial_guess;   /* 1: start from the p passed in */
    int fixed_cycles;        /* > 0: run exactly this many cycles, no convergence test */
    int method;              /* IBM_VCYCLE, IBM_BICGSTAB (default) or IBM_BICGSTAB_SRJ */
    int srj_sweeps;          /* IBM_BICGSTAB_SRJ: sweeps per preconditioner application (16) */
    double breakdown_tol;    /* BiCGStab near-breakdown: an inner product of modulus at most
                                breakdown_tol times its factors' norms (rh.r for rho, rh.A y for
                                alpha), or omega = 0, restarts the shadow residual (1e-12) */
} ibm_solve_opts;

typedef struct {
    int cycles;                /* outer iterations: V-cycles, refinement steps or BiCGStab steps */
    double rel_residual;       /* ||r'||_2 / ||f'||_2 after the last cycle */
    double ghost_residual_max; /* max over ghosts of |p_g - sum_m beta_m p_m - h_g| (degenerate:
                                  |p_g - mean of fluid neighbours|) of the returned p */
    double lambda;             /* uniform source shift making the Neumann system consistent */
    double div_max;            /* projection only: max |D u| over fluid cells after correction */
    double t_setup;            /* seconds of the handle's last geometry set-up (set_geometry,
                                  classify, build_ghost_stencils: host wall clock of the calls) */
    double t_solve, t_correct; /* seconds (host wall clock around the enqueue+sync) */
    int vcycles;               /* V-cycles applied (BiCGStab: 2 per step) */
    int restarts;              /* BiCGStab restarts of the shadow residual after a near-breakdown */
} ibm_solve_stats;

/* Fill `o` with the defaults listed above. */
void ibm_default_opts(ibm_solve_opts *o);

/* Create a handle for an nx x ny x nz cell grid with face coordinates xf[nx+1], yf[ny+1],
   zf[nz+1] (host, strictly increasing, finite; nx, ny >= 2, nz >= 1).  Cell centres,
   widths and the 7-point flux coefficients follow Section 2.1 (central differences on a
   non-uniform Cartesian grid).  No device work is done here. */
ibm_status ibm_create_grid(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                           ibm_grid **out);

/* Bytes of device workspace needed for this grid size, a mesh of at most nv_max vertices
   and nt_max triangles, at most max_ghosts ghost cells, and the given precision.  Needs no
   handle, so it can drive admission decisions. */
size_t ibm_workspace_bytes(int nx, int ny, int nz, int64_t nv_max, int64_t nt_max, int64_t max_ghosts,
                           ibm_precision prec);

/* Exact workspace size for an existing handle (its multigrid plan depends on the face
   coordinates).  ibm_workspace_bytes is an upper bound of this for any coordinates. */
size_t ibm_grid_workspace_bytes(const ibm_grid *g, int64_t nv_max, int64_t nt_max, int64_t max_ghosts,
                                ibm_precision prec);

/* Bind a caller-owned device buffer (>= ibm_workspace_bytes(...) bytes, 256-byte aligned)
   as the handle's workspace and upload the grid metrics.  `prec` = the most demanding
   precision the handle will be used with.  The buffer must outlive every later call. */
ibm_status ibm_bind_workspace(ibm_grid *g, void *device_ptr, size_t bytes, int64_t nv_max, int64_t nt_max,
                              int64_t max_ghosts, ibm_precision prec, void *stream);

/* Set the immersed body: verts[nv][3] (host, FP64), tris[nt][3] (host, int32, outward
   counter-clockwise).  The mesh must be closed and consistently oriented (every directed
   edge once, its reverse once) -> else IBM_E_GEOMETRY.  Several disjoint closed bodies may
   be passed as one mesh.  Uploads the mesh and builds the triangle bucket grid on the GPU. */
ibm_status ibm_set_geometry(ibm_grid *g, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                            void *stream);

/* Classify every cell (Section 2.2, ray tracing): a cell is solid when its centre lies
   strictly inside the body by the parity of crossings of the +z ray through the column
   centre; ghost = solid with a fluid cell among its 26 neighbours; dead = other solid.
   counts_out[3] (host) receives the fluid, ghost and dead counts.  A column whose ray
   crosses the surface an odd number of times (impossible for a closed mesh under the
   edge-ownership rule, so a broken mesh or predicate) -> IBM_E_GEOMETRY with the count in
   the message; the classification is then not usable.  Synchronises `stream`. */
ibm_status ibm_classify(ibm_grid *g, void *stream, int64_t counts_out[3]);

/* ---- classification without a handle: for callers that cannot allocate ---------------
   For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc) and have no handle or workspace: the
   classification of ibm_classify (the same kernels, the same types and counts), with every
   intermediate buffer in a fixed array of IBM_NOALLOC_SCRATCH_MB MiB of device memory that
   the library holds per GPU from its first use until the process ends.  It calls no
   hipMalloc, hipFree or other allocating routine.
     xf[nx+1], yf[ny+1], zf[nz+1]: device, FP64 face coordinates (strictly increasing: not
       checked, the data stay on the device);
     verts[nv][3] FP64, tris[nt][3] int32: device, a closed, consistently oriented mesh (not
       checked: ibm_set_geometry's check needs the mesh on the host);
     type_out[nz][ny][nx]: device, uint8 out (0 fluid, 1 ghost, 2 dead);
     counts_out[3]: host out, fluid, ghost and dead counts.
   Errors: IBM_E_ARG for sizes below 2 x 2 x 1, 2^31 cells or more, NULL pointers or an
   empty mesh; IBM_E_NOMEM when the columns do not fit the scratch (about 1.8 million
   columns at 64 MiB) or the ray crossings overflow it; IBM_E_GEOMETRY when a column has an
   odd number of crossings (type_out is then not valid) or no cell is fluid.  Synchronises
   `stream`.  Every call on one GPU uses that GPU's one scratch array: calls that overlap on
   a GPU (several host threads or streams at once) race and must be serialised by the
   caller. */
#define IBM_NOALLOC_SCRATCH_MB 64
ibm_status ibm_classify_noalloc(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf,
                                const double *verts, int64_t nv, const int32_t *tris, int64_t nt, uint8_t *type_out,
                                int64_t counts_out[3], void *stream);

/* Build the ghost-cell stencils (Section 2.2, Eq. 2 and 3): body intercept = closest mesh
   point, normal, image point = mirror of the ghost centre through the intercept, the 8 (2D:
   4) cells around the image point and the weights of Eq. 2 with the Neumann condition in
   place of the ghost's own value when it belongs to its own box.  Also builds the multigrid
   hierarchy.  n_ghost_out (host) receives the ghost count.  Synchronises `stream`. */
ibm_status ibm_build_ghost_stencils(ibm_grid *g, void *stream, int64_t *n_ghost_out);

/* Copy ghost data to host arrays (any may be NULL): cell[n_G] int32 linear cell index,
   bi_xyz/n_xyz/ip_xyz[3*n_G], stencil[8*n_G] int32 (-1 = unused or the ghost's own
   Neumann slot), beta[8*n_G], flags[n_G] (bit0 degenerate, bit1 clamped image point, bit2
   facet-normal fallback, bit3 ghost in its own box).  Synchronises `stream`. */
ibm_status ibm_get_ghosts(const ibm_grid *g, void *stream, int32_t *cell, double *bi_xyz, double *n_xyz,
                          double *ip_xyz, int32_t *stencil, double *beta, int32_t *flags);

/* Neumann data dp/dn at each body intercept (host, n_G values; NULL = all zero, the
   projection's condition).  Default after build_ghost_stencils: zero. */
ibm_status ibm_set_neumann_data(ibm_grid *g, const double *dpdn, void *stream);

/* Copy the cell types (0 fluid, 1 ghost, 2 dead; uint8 [nz][ny][nx]) to device memory. */
ibm_status ibm_get_cell_types(const ibm_grid *g, uint8_t *dst_device, void *stream);

/* Solve the pressure Poisson equation S p = rhs - lambda on fluid cells with the implicit
   ghost equations, gauge sum_fluid V p = 0 (Section 2.1: the pressure equation of the
   fractional step; the solver is a geometric multigrid V-cycle with red-black Gauss-Seidel
   smoothing).  rhs, p: device, [nz][ny][nx] FP64.  p is overwritten (initial guess read when
   o->use_initial_guess); dead cells are set to 0.  Synchronises `stream` once per cycle. */
ibm_status ibm_poisson_solve(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o,
                             ibm_solve_stats *s, void *stream);

/* Full projection (Section 2.1, fractional step): rhs = (D u*)/dt on fluid cells, solve,
   then u_f -= dt (p_nb - p_c)/d_f on every interior face touching a fluid cell.  u, v, w:
   device MAC arrays, corrected in place; p: device, out. */
ibm_status ibm_project(ibm_grid *g, double *u, double *v, double *w, double dt, double *p,
                       const ibm_solve_opts *o, ibm_solve_stats *s, void *stream);

/* Non-blocking step API: begin enqueues the initial residual, step enqueues n_cycles outer
   iterations plus an asynchronous read-back of the residual norm, and poll never blocks.
   poll sets *done to
     1  finished: converged, failed or out of cycles; the return value is the solve's status
        and s (host, may be NULL) holds its statistics;
     0  work is in flight (the last step, a true-residual confirmation of a BiCGStab
        convergence, or the final gauge): poll again later;
    -1  idle: the previous step has completed and the solve needs more; call ibm_solve_step.
   rhs and p (device) must stay valid until done = 1.  The iterates, step count and result are
   those of ibm_poisson_solve with the same options, bit for bit; the gauge is applied on the
   handle's stream at completion.  ibm_solve_step returns IBM_E_STATE while *done would be 0. */
ibm_status ibm_solve_begin(ibm_grid *g, const double *rhs, double *p, const ibm_solve_opts *o, void *stream);
ibm_status ibm_solve_step(ibm_grid *g, int n_cycles);
ibm_status ibm_solve_poll(ibm_grid *g, int *done, ibm_solve_stats *s);

/* Level count and dims of the multigrid hierarchy (planned at ibm_create_grid from the face
   coordinates alone; host call). */
ibm_status ibm_get_levels(const ibm_grid *g, int *n_levels, int *dims /* 3*n_levels, may be NULL */);

/* Child map of hierarchy level `level` (1 .. n_levels-1) along `axis` (0 x, 1 y, 2 z): coarse
   index I holds the cells cs[I] .. cs[I+1]-1 of level - 1 (one or two).  cs: host, receives
   dims[axis] + 1 ints.  The hierarchy coarsens by cell width (Section 2.1 leaves the solver's
   multigrid to the implementation): level l merges two neighbouring cells of level l-1 along an
   axis with at least 4 cells when their combined width is at most 3.5 x 2^(l-1) h_min (h_min the
   smallest cell width of the grid), scanning from the low wall, and stops when nothing merges or
   the coarse levels would together exceed half the grid's cell count.  Host call. */
ibm_status ibm_get_level_map(const ibm_grid *g, int level, int axis, int *cs);

/* ---- advection-diffusion half-step (Section 2.1) with Dirichlet ghost rows (2.2) ---- */

#define IBM_SRJ_MAX 256 /* most relaxation factors in one scheduled-Jacobi cycle */

/* Options of ibm_momentum_step.  Defaults (ibm_default_momentum_opts): nu = dt = 0 (must be
   set), later steps (first_step 0), 8 relaxation factors of the Chebyshev schedule,
   rel_tol 1e-10, at most 200 cycles, convergence-tested. */
typedef struct {
    double nu;            /* kinematic viscosity (1/Re) */
    double dt;            /* time step */
    int first_step;       /* 1: no previous convective term (H^{n-1} := H^n, forward Euler) */
    int srj_factors;      /* m: sweeps per scheduled-Jacobi cycle, 1..IBM_SRJ_MAX */
    const double *omega;  /* host, m relaxation factors, NULL: ibm_srj_schedule(rho, m) */
    double rel_tol;       /* stop when ||b - A u||_2 <= rel_tol ||b||_2 over fluid rows */
    int max_cycles;       /* cycles of m sweeps */
    int fixed_cycles;     /* > 0: run exactly this many cycles, no convergence test */
} ibm_momentum_opts;

typedef struct {
    int cycles, sweeps;   /* scheduled-Jacobi cycles and sweeps run */
    double rel_residual;  /* fluid-row residual of the input of the last sweep / ||b|| */
    double rho;           /* half-width of the Jacobi-scaled spectrum interval [1-rho, 1+rho] */
    double t_step;        /* seconds (host wall clock around enqueue + sync) */
} ibm_momentum_stats;

void ibm_default_momentum_opts(ibm_momentum_opts *o);

/* Host only.  The m relaxation factors 1/kappa_k, kappa_k = 1 + rho cos((2k-1) pi / (2m)) the
   Chebyshev nodes of [1 - rho, 1 + rho] (the min-max optimal factors for that interval),
   ordered largest, smallest, second largest, ...  omega (host) receives m values.
   IBM_E_ARG unless 0 <= rho < 1 and 1 <= m <= IBM_SRJ_MAX. */
ibm_status ibm_srj_schedule(double rho, int m, double *omega);

/* Velocity at each body intercept for the Dirichlet ghost rows (host, 3*n_G values, x y z
   per ghost; NULL = 0, a stationary no-slip body).  Default after build_ghost_stencils: 0. */
ibm_status ibm_set_dirichlet_data(ibm_grid *g, const double *ubi, void *stream);

/* Dirichlet weights (host out, either may be NULL): beta[8*n_G] on the members listed by
   ibm_get_ghosts' stencil, beta_g[n_G] on the intercept value; ghost row
   u_g + sum_m beta_m u_m = (2 - beta_g) u_BI (BI is the midpoint of the ghost centre and its
   image point).  Zero for degenerate ghosts.  Synchronises `stream`. */
ibm_status ibm_get_dirichlet_weights(const ibm_grid *g, void *stream, double *beta, double *beta_g);

/* One advection-diffusion half-step of the cell-centred velocity (Section 2.1: central
   differences, Adams-Bashforth convection, Crank-Nicolson viscous term solved by scheduled
   relaxed Jacobi; Section 2.2: ghost cells, here with the Dirichlet condition at BI):
     1. the ghost rows are applied once to u^n, in place (dead cells are never read);
     2. H^n = -div(u u) in conservative form (face values by linear interpolation between
        centres; no flux through the box walls), b = u^n + dt (3/2 H^n - 1/2 H^{n-1})
        + (nu dt / 2) L u^n on fluid rows, L the pressure operator's flux Laplacian;
     3. (I - (nu dt / 2) L) u* = b on fluid rows with the ghost rows, by cycles of m relaxed
        Jacobi sweeps (each followed by one pass of the ghost rows), from u^n.
   u, v, w: device [nz][ny][nx] FP64, in u^n, out u* (dead cells 0).  hu, hv, hw: device,
   in H^{n-1} (not read when o->first_step), out H^n (0 off the fluid cells).  Uses six
   N-arrays of the workspace (those of the pressure solver's Krylov vectors): do not overlap
   it with a pressure solve on the same handle.  Synchronises `stream` once per cycle.
   IBM_NOT_CONVERGED when max_cycles is reached (u* is the last iterate). */
ibm_status ibm_momentum_step(ibm_grid *g, double *u, double *v, double *w, double *hu, double *hv, double *hw,
                             const ibm_momentum_opts *o, ibm_momentum_stats *s, void *stream);

/* ---- fractional step: momentum half-step then projection (Section 2.1) ----------------
   The half-step advances cell-centred components and the projection corrects face-normal
   velocities.  A whole step is: ibm_momentum_step (u*), ibm_cell_to_faces (U* on the faces),
   ibm_project (p, corrected U), ibm_correct_cells (the cell-centred u^{n+1}). */

/* Face-normal velocities from cell-centred components: on every interior face the linear
   interpolation between the two centres, (w_b u_a + w_a u_b) / (w_a + w_b) with w the cell
   widths across the face (the interpolation of the convective term); faces on the box walls
   0.  u, v, w: device [nz][ny][nx]; uf [nz][ny][nx+1], vf [nz][ny+1][nx], wf [nz+1][ny][nx]:
   device, out.  Needs a bound workspace.  Enqueued on `stream`, no synchronisation. */
ibm_status ibm_cell_to_faces(ibm_grid *g, const double *u, const double *v, const double *w, double *uf, double *vf,
                             double *wf, void *stream);

/* Cell-centred velocity correction matching the projection's face correction: on fluid
   cells u_c -= (delta_{c-1/2} + delta_{c+1/2}) / 2 along x (v along y, w along z), where
   delta_f = dt (p_b - p_a) / d_f is what ibm_project subtracts on face f (0 on box walls);
   ghost and dead cells unchanged.  u, v, w: device [nz][ny][nx], in place; p: device, the
   projection's pressure.  Needs classification.  Enqueued on `stream`, no synchronisation. */
ibm_status ibm_correct_cells(ibm_grid *g, double *u, double *v, double *w, const double *p, double dt, void *stream);

/* ---- moving bodies: fresh cells (Section 2.2) ---------------------------------------- */

/* Move the body to new vertex positions (host; same conventions and checks as
   ibm_set_geometry) after a previous geometry's stencils: re-classifies, rebuilds the ghost
   stencils and the hierarchy, and lists the fresh cells, the cells that were ghost or dead
   before and are fluid now (increasing linear index).  For each fresh cell c: BI = closest
   point of the moved surface, image point IP = 2 x_c - BI (the centre is the midpoint of BI
   and IP), the 8 (2D: 4) cells around IP with their trilinear weights (Eq. 2), the cell's
   own weight kept apart.  counts_out[3] and n_fresh_out (host) receive the new type counts
   and the fresh count.  IBM_E_NOMEM if there are more fresh cells than the bound ghost
   capacity.  Synchronises `stream`. */
ibm_status ibm_move_geometry(ibm_grid *g, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                             void *stream, int64_t counts_out[3], int64_t *n_fresh_out);

/* Set the fresh cells of three cell-centred fields (device, [nz][ny][nx], in place):
   u_c = (u_BI + sum_{m != c} beta_m u_m) / (2 - beta_c), members read from the fields before
   the pass; degenerate fresh cells (a dead member or no fluid member) take the mean of their
   fluid, non-fresh 26-neighbours.  ubi: host, 3 values per fresh cell (the body velocity at
   its intercept; NULL = 0).  Synchronises `stream`. */
ibm_status ibm_fill_fresh(ibm_grid *g, double *u, double *v, double *w, const double *ubi, void *stream);

/* Copy the fresh-cell data of the last move to host arrays (any may be NULL): cell[n],
   bi_xyz/ip_xyz[3n], stencil[8n] (-1: unused or the cell itself), beta[8n], beta_c[n] (the
   cell's own weight), flags[n] (bit0 degenerate, bit1 clamped image point, bit3 own box). */
ibm_status ibm_get_fresh(const ibm_grid *g, void *stream, int32_t *cell, double *bi_xyz, double *ip_xyz,
                         int32_t *stencil, double *beta, double *beta_c, int32_t *flags);

/* ---- single-step hooks for kernel-level parity tests -------------------------------- */

/* n red-black sweeps of level 0 on p (device, in/out) with right-hand side rhs and shift
   lambda; refresh != 0 follows each sweep with a ghost refresh. */
ibm_status ibm_debug_sweep(ibm_grid *g, double *p, const double *rhs, double lambda, int n, int refresh,
                           void *stream);
/* (S p) on fluid rows, 0 elsewhere (device in/out). */
ibm_status ibm_debug_apply(ibm_grid *g, const double *p, double *out, void *stream);

/* Copy one internal FP64 cell field of the workspace ([nz][ny][nx]) to device memory:
   which 0..9 the Krylov vectors (r, shadow residual, search direction, A y, s, A z,
   preconditioned search directions y and z in two buffers each), 10 the second pressure
   buffer, 11 the preconditioner's start iterate, 12 the projection's right-hand side. */
ibm_status ibm_debug_vector(const ibm_grid *g, int which, double *dst_device, void *stream);

/* Read-before-write check: on != 0 makes every later ibm_bind_workspace of this handle fill
   each floating-point sub-buffer of the workspace with NaN (all bits set) before it writes
   anything.  Results on such a handle equal, bit for bit, those on a handle whose
   workspace held any other content, unless the library reads a value it never wrote.
   Debug only: costs one device memset per sub-buffer at bind. */
ibm_status ibm_debug_poison(ibm_grid *g, int on);

/* Timing of the level-0 smoother.  on = 0: off.  on = n >= 1: every n-th fine-level
   red-black sweep (counted from this call) is timed by two HIP events that the runtime records
   on its launch stream when the kernel starts and when it ends (hipExtLaunchKernel; at most 32
   sweeps between two host synchronisations are timed); a stride above one keeps
   the events' own cost out of the timed run, and a stride coprime to the sweeps of a cycle
   samples every position in it.  on < 0 -> IBM_E_ARG.  get_profile returns the summed
   milliseconds and the number of timed FP64 and FP32 sweeps since profiling was switched on. */
ibm_status ibm_set_profiling(ibm_grid *g, int on);
ibm_status ibm_get_profile(const ibm_grid *g, double *ms_fp64, int64_t *n_fp64, double *ms_fp32, int64_t *n_fp32);

void ibm_destroy_grid(ibm_grid *g);
const char *ibm_last_error(const ibm_grid *g); /* g == NULL: last error of this thread */

#ifdef __cplusplus
}
#endif
#endif /* IBM_H */
