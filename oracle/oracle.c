/*
 * FP64 CPU oracle of the ghost-cell sharp-interface immersed-boundary projection.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code with the HIP path.
 *
 * What it computes (paper: Section 2.1 fractional step and central differences on a
 * non-uniform Cartesian grid; Section 2.2 ghost-cell treatment, Eq. 2 and Eq. 3):
 *   1. grid metrics of a tensor-product grid given by face coordinates;
 *   2. cell classification by ray parity against a closed triangle mesh, ghost cells as
 *      solid cells with a fluid neighbour;
 *   3. per ghost: body intercept (closest surface point), normal, image point, the 8-cell
 *      interpolation box and the weights beta of Eq. 2, found from the Vandermonde system
 *      of Eq. 3 by LU with partial pivoting, with the Neumann condition replacing the row
 *      of the ghost itself when it lies in its own box;
 *   4. the pressure Poisson equation S p = f - lambda on fluid cells plus the implicit
 *      ghost equations, solved by a geometric multigrid V-cycle with red-black
 *      Gauss-Seidel smoothing (multigrid and red-black GS are among the solvers the paper
 *      evaluated, Section 2.1);
 *   5. the divergence right-hand side and the velocity correction of the projection.
 * Everything is plain loops in the order the definitions state; reductions are serial.
 * OpenMP is used only over independent cells of one colour or one elementwise pass.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_STATE (-2)
#define ORC_E_GEOMETRY (-3)
#define ORC_E_NOMEM (-4)
#define ORC_E_NUMERIC (-6)
#define ORC_NOT_CONVERGED 1

#define T_FLUID 0
#define T_GHOST 1
#define T_DEAD 2

#define GF_DEGENERATE 1 /* no fluid member / dead member in the box: neighbour mean */
#define GF_CLAMPED 2    /* image point beyond the outermost cell centres */
#define GF_NFALLBACK 4  /* ghost centre (numerically) on the surface: facet normal */
#define GF_SELF 8       /* ghost is a member of its own box: Neumann row */

#define MAXLEV 32

typedef struct {
    int n[3];
    double *f[3], *c[3], *w[3]; /* faces (n+1), centres, widths */
    int halved[3];              /* some cells merged relative to the next finer level */
    int *cs[3];                 /* coarse index I holds the finer cells cs[I] .. cs[I+1]-1 */
    int *par[3];                /* (finer level) the coarse index holding each cell */
    uint8_t *active;
    double *T[3];               /* integrated transmissibility of each cell's low face */
    double *e, *R, *r;
    double mu;                  /* compatibility shift of R (per unit volume) */
    double vol_active;
    /* prolongation tables from the next coarser level, per axis and per index of this level */
    int *plo[3], *phi[3];
    double *pt[3];
} level_t;

typedef struct {
    double rel_tol;
    int max_cycles, nu1, nu2, coarsest_sweeps, use_initial_guess, fixed_cycles;
    int method; /* 0: V-cycle iteration, 1: BiCGStab preconditioned by one V-cycle,
                   2: BiCGStab preconditioned by srj_m scheduled relaxed Jacobi sweeps */
    int srj_m;                /* method 2: sweeps per preconditioner application */
    const double *srj_omega;  /* method 2: their relaxation factors, in order */
    double breakdown_tol;     /* methods 1, 2: near-breakdown threshold (relative) */
} orc_opts;

typedef struct {
    int cycles, status;
    double rel_residual, ghost_residual_max, lambda, ref_norm, first_norm;
    int restarts;             /* BiCGStab restarts of the shadow residual */
} orc_stats;

typedef struct {
    int nx, ny, nz;
    int64_t ncell;
    double *xf, *yf, *zf;
    double *xc, *yc, *zc, *wx, *wy, *wz;
    double *axm, *axp, *aym, *ayp, *azm, *azp; /* level-0 per-volume coefficients */
    double *dcx, *dcy, *dcz;                   /* centre distance across face i (1..n-1) */
    /* mesh */
    int64_t nv, nt;
    double *verts;
    int32_t *tris;
    int has_mesh;
    /* classification */
    uint8_t *type;
    int classified;
    int64_t nfluid, nghost, ndead, odd_columns;
    int32_t *gcell;
    /* stencils */
    int stencils;
    double *gbi, *gn, *gip, *gbeta, *gbetag, *gdl, *gh, *gdata;
    int32_t *gst, *gflags;
    /* hierarchy */
    int nlev;
    level_t lev[MAXLEV];
    double vol_fluid;
} orc_problem;

/* ------------------------------------------------------------------------------------ */
/* helpers                                                                              */
/* ------------------------------------------------------------------------------------ */

static double *dalloc(int64_t n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }
static int *ialloc(int64_t n) { return (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int)); }

static inline int64_t IDX(const orc_problem *P, int i, int j, int k) {
    return ((int64_t)k * P->ny + j) * P->nx + i;
}

static void axis_metrics(int n, const double *f, double *c, double *w) {
    for (int i = 0; i < n; ++i) {
        c[i] = 0.5 * (f[i] + f[i + 1]);
        w[i] = f[i + 1] - f[i];
    }
}

/* ------------------------------------------------------------------------------------ */
/* grid (Section 2.1: central differences on a non-uniform Cartesian grid)              */
/* ------------------------------------------------------------------------------------ */

static void level0_coeffs(int n, const double *c, const double *w, double *dc, double *am, double *ap) {
    dc[0] = 0.0;
    for (int i = 1; i < n; ++i) dc[i] = c[i] - c[i - 1];
    for (int i = 0; i < n; ++i) {
        /* flux form: (1/w_i) * [ (p_{i+1}-p_i)/dc_{i+1} - (p_i-p_{i-1})/dc_i ];
           walls have zero transmissibility (homogeneous Neumann on the box) */
        am[i] = (i > 0) ? 1.0 / (w[i] * dc[i]) : 0.0;
        ap[i] = (i < n - 1) ? 1.0 / (w[i] * dc[i + 1]) : 0.0;
    }
}

orc_problem *orc_create(int nx, int ny, int nz, const double *xf, const double *yf, const double *zf) {
    if (nx < 2 || ny < 2 || nz < 1) return NULL;
    for (int i = 0; i < nx; ++i) if (!(xf[i + 1] > xf[i])) return NULL;
    for (int i = 0; i < ny; ++i) if (!(yf[i + 1] > yf[i])) return NULL;
    for (int i = 0; i < nz; ++i) if (!(zf[i + 1] > zf[i])) return NULL;
    orc_problem *P = (orc_problem *)calloc(1, sizeof(orc_problem));
    P->nx = nx; P->ny = ny; P->nz = nz;
    P->ncell = (int64_t)nx * ny * nz;
    P->xf = dalloc(nx + 1); memcpy(P->xf, xf, sizeof(double) * (nx + 1));
    P->yf = dalloc(ny + 1); memcpy(P->yf, yf, sizeof(double) * (ny + 1));
    P->zf = dalloc(nz + 1); memcpy(P->zf, zf, sizeof(double) * (nz + 1));
    P->xc = dalloc(nx); P->wx = dalloc(nx);
    P->yc = dalloc(ny); P->wy = dalloc(ny);
    P->zc = dalloc(nz); P->wz = dalloc(nz);
    axis_metrics(nx, P->xf, P->xc, P->wx);
    axis_metrics(ny, P->yf, P->yc, P->wy);
    axis_metrics(nz, P->zf, P->zc, P->wz);
    P->dcx = dalloc(nx); P->axm = dalloc(nx); P->axp = dalloc(nx);
    P->dcy = dalloc(ny); P->aym = dalloc(ny); P->ayp = dalloc(ny);
    P->dcz = dalloc(nz); P->azm = dalloc(nz); P->azp = dalloc(nz);
    level0_coeffs(nx, P->xc, P->wx, P->dcx, P->axm, P->axp);
    level0_coeffs(ny, P->yc, P->wy, P->dcy, P->aym, P->ayp);
    level0_coeffs(nz, P->zc, P->wz, P->dcz, P->azm, P->azp);
    P->type = (uint8_t *)calloc((size_t)P->ncell, 1);
    return P;
}

static void free_hierarchy(orc_problem *P) {
    for (int l = 0; l < P->nlev; ++l) {
        level_t *L = &P->lev[l];
        for (int d = 0; d < 3; ++d) {
            free(L->f[d]); free(L->c[d]); free(L->w[d]); free(L->T[d]);
            free(L->plo[d]); free(L->phi[d]); free(L->pt[d]); free(L->cs[d]); free(L->par[d]);
        }
        free(L->active); free(L->e); free(L->R); free(L->r);
        memset(L, 0, sizeof(*L));
    }
    P->nlev = 0;
}

static void free_stencils(orc_problem *P) {
    free(P->gbi); free(P->gn); free(P->gip); free(P->gbeta); free(P->gbetag); free(P->gdl);
    free(P->gh); free(P->gdata); free(P->gst); free(P->gflags);
    P->gbi = P->gn = P->gip = P->gbeta = P->gbetag = P->gdl = P->gh = P->gdata = NULL;
    P->gst = P->gflags = NULL;
    P->stencils = 0;
}

void orc_destroy(orc_problem *P) {
    if (!P) return;
    free_hierarchy(P);
    free_stencils(P);
    free(P->xf); free(P->yf); free(P->zf); free(P->xc); free(P->yc); free(P->zc);
    free(P->wx); free(P->wy); free(P->wz); free(P->dcx); free(P->dcy); free(P->dcz);
    free(P->axm); free(P->axp); free(P->aym); free(P->ayp); free(P->azm); free(P->azp);
    free(P->verts); free(P->tris); free(P->type); free(P->gcell);
    free(P);
}

void orc_get_metrics(const orc_problem *P, double *xc, double *yc, double *zc, double *axm,
                     double *axp, double *aym, double *ayp, double *azm, double *azp) {
    memcpy(xc, P->xc, sizeof(double) * P->nx);
    memcpy(yc, P->yc, sizeof(double) * P->ny);
    memcpy(zc, P->zc, sizeof(double) * P->nz);
    memcpy(axm, P->axm, sizeof(double) * P->nx); memcpy(axp, P->axp, sizeof(double) * P->nx);
    memcpy(aym, P->aym, sizeof(double) * P->ny); memcpy(ayp, P->ayp, sizeof(double) * P->ny);
    memcpy(azm, P->azm, sizeof(double) * P->nz); memcpy(azp, P->azp, sizeof(double) * P->nz);
}

/* ------------------------------------------------------------------------------------ */
/* mesh                                                                                 */
/* ------------------------------------------------------------------------------------ */

static int cmp_edge(const void *a, const void *b) {
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    return (*x > *y) - (*x < *y);
}

/* closed and consistently oriented: every directed edge occurs once and its reverse once */
int orc_set_mesh(orc_problem *P, const double *verts, int64_t nv, const int32_t *tris, int64_t nt) {
    if (nv < 3 || nt < 1) return ORC_E_ARG;
    for (int64_t t = 0; t < nt; ++t)
        for (int q = 0; q < 3; ++q)
            if (tris[3 * t + q] < 0 || tris[3 * t + q] >= nv) return ORC_E_ARG;
    for (int64_t i = 0; i < 3 * nv; ++i) if (!isfinite(verts[i])) return ORC_E_ARG;
    int64_t ne = 3 * nt;
    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * ne);
    for (int64_t t = 0; t < nt; ++t)
        for (int q = 0; q < 3; ++q) {
            int64_t a = tris[3 * t + q], b = tris[3 * t + (q + 1) % 3];
            e[3 * t + q] = a * nv + b;
        }
    qsort(e, (size_t)ne, sizeof(int64_t), cmp_edge);
    int ok = 1;
    for (int64_t i = 0; i < ne && ok; ++i) {
        if (i + 1 < ne && e[i + 1] == e[i]) ok = 0; /* a directed edge used twice */
        int64_t a = e[i] / nv, b = e[i] % nv;
        if (a == b) ok = 0;
        int64_t rev = b * nv + a;
        if (!bsearch(&rev, e, (size_t)ne, sizeof(int64_t), cmp_edge)) ok = 0;
    }
    free(e);
    if (!ok) return ORC_E_GEOMETRY;
    free(P->verts); free(P->tris);
    P->verts = dalloc(3 * nv); memcpy(P->verts, verts, sizeof(double) * 3 * nv);
    P->tris = (int32_t *)malloc(sizeof(int32_t) * 3 * nt); memcpy(P->tris, tris, sizeof(int32_t) * 3 * nt);
    P->nv = nv; P->nt = nt; P->has_mesh = 1;
    P->classified = 0;
    free_stencils(P);
    free_hierarchy(P);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* classification (Section 2.2: ray tracing marks solid cells; ghost = solid cell with a */
/* fluid neighbour).  Rays run along +z through every column centre (x_i, y_j).         */
/* ------------------------------------------------------------------------------------ */

/* Edge function of the undirected edge {u,v}, always evaluated from the lower vertex
   index, so the two triangles sharing an edge see exactly opposite values. Positive when
   (px,py) lies left of the directed edge u->v. */
static double edge_fn(const double *V, int32_t u, int32_t v, double px, double py) {
    int32_t lo = u < v ? u : v, hi = u < v ? v : u;
    double ax = V[3 * lo], ay = V[3 * lo + 1], bx = V[3 * hi], by = V[3 * hi + 1];
    double e = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
    return (u == lo) ? e : -e;
}

/* top-left ownership of a point lying exactly on a directed edge of a counter-clockwise
   triangle: left edges (going down) and top edges (horizontal, going left) own it */
static int top_left(const double *V, int32_t u, int32_t v) {
    double dx = V[3 * v] - V[3 * u], dy = V[3 * v + 1] - V[3 * u + 1];
    return (dy < 0.0) || (dy == 0.0 && dx < 0.0);
}

/* Does the z-ray through (px,py) cross triangle t?  On success stores the crossing z. */
static int ray_cross(const double *V, const int32_t *tri, double px, double py, double *zout) {
    int32_t a = tri[0], b = tri[1], c = tri[2];
    double area = edge_fn(V, a, b, V[3 * c], V[3 * c + 1]);
    if (area == 0.0) return 0; /* triangle parallel to the ray */
    if (area < 0.0) { int32_t s = b; b = c; c = s; }
    double wab = edge_fn(V, a, b, px, py);
    double wbc = edge_fn(V, b, c, px, py);
    double wca = edge_fn(V, c, a, px, py);
    int in_ab = (wab > 0.0) || (wab == 0.0 && top_left(V, a, b));
    int in_bc = (wbc > 0.0) || (wbc == 0.0 && top_left(V, b, c));
    int in_ca = (wca > 0.0) || (wca == 0.0 && top_left(V, c, a));
    if (!(in_ab && in_bc && in_ca)) return 0;
    /* barycentric interpolation of z: the weight of a vertex is the edge function of the
       opposite edge; written relative to vertex a, so a horizontal facet gives its height
       exactly (a centre on it then lies on the crossing and stays fluid) */
    double za = V[3 * a + 2];
    double num = wca * (V[3 * b + 2] - za);
    num = num + wab * (V[3 * c + 2] - za);
    double den = wbc + wca;
    den = den + wab;
    *zout = za + num / den;
    return 1;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int orc_classify(orc_problem *P, int64_t counts[3]) {
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    uint8_t *solid = (uint8_t *)calloc((size_t)P->ncell, 1);
    int64_t odd = 0;
    if (P->has_mesh) {
        /* pass 1: count crossings per column, pass 2: store them.  A triangle can only be
           crossed by rays whose column centre lies in its xy bounding box. */
        int64_t ncol = (int64_t)nx * ny;
        int64_t *cnt = (int64_t *)calloc((size_t)ncol + 1, sizeof(int64_t));
        for (int pass = 0; pass < 2; ++pass) {
            double *zs = NULL;
            int64_t *fill = NULL;
            if (pass == 1) {
                int64_t tot = 0;
                for (int64_t q = 0; q < ncol; ++q) { int64_t c = cnt[q]; cnt[q] = tot; tot += c; }
                cnt[ncol] = tot;
                zs = dalloc(tot);
                fill = (int64_t *)calloc((size_t)ncol, sizeof(int64_t));
            }
            for (int64_t t = 0; t < P->nt; ++t) {
                const int32_t *tri = P->tris + 3 * t;
                double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
                for (int q = 0; q < 3; ++q) {
                    double x = P->verts[3 * tri[q]], y = P->verts[3 * tri[q] + 1];
                    xmin = fmin(xmin, x); xmax = fmax(xmax, x);
                    ymin = fmin(ymin, y); ymax = fmax(ymax, y);
                }
                for (int j = 0; j < ny; ++j) {
                    if (P->yc[j] < ymin || P->yc[j] > ymax) continue;
                    for (int i = 0; i < nx; ++i) {
                        if (P->xc[i] < xmin || P->xc[i] > xmax) continue;
                        double z;
                        if (!ray_cross(P->verts, tri, P->xc[i], P->yc[j], &z)) continue;
                        int64_t q = (int64_t)j * nx + i;
                        if (pass == 0) cnt[q]++;
                        else zs[cnt[q] + fill[q]++] = z;
                    }
                }
            }
            if (pass == 1) {
                for (int64_t q = 0; q < ncol; ++q) {
                    int64_t b = cnt[q], n = cnt[q + 1] - cnt[q];
                    if (n == 0) continue;
                    qsort(zs + b, (size_t)n, sizeof(double), cmp_double);
                    if (n % 2) { odd++; n -= 1; } /* counted: the call fails below */
                    int i = (int)(q % nx), j = (int)(q / nx);
                    for (int k = 0; k < nz; ++k) {
                        double z = P->zc[k];
                        for (int64_t m = 0; m < n; m += 2)
                            if (z > zs[b + m] && z < zs[b + m + 1]) { solid[IDX(P, i, j, k)] = 1; break; }
                    }
                }
                free(zs); free(fill);
            }
        }
        free(cnt);
    }
    /* ghost: solid with at least one fluid cell in its (in-range) 26-neighbourhood */
    int64_t nf = 0, ng = 0, nd = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (!solid[id]) { P->type[id] = T_FLUID; nf++; continue; }
                int fluid_nb = 0;
                for (int dk = -1; dk <= 1 && !fluid_nb; ++dk)
                    for (int dj = -1; dj <= 1 && !fluid_nb; ++dj)
                        for (int di = -1; di <= 1 && !fluid_nb; ++di) {
                            int ii = i + di, jj = j + dj, kk = k + dk;
                            if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                            if (!solid[IDX(P, ii, jj, kk)]) fluid_nb = 1;
                        }
                if (fluid_nb) { P->type[id] = T_GHOST; ng++; } else { P->type[id] = T_DEAD; nd++; }
            }
    free(solid);
    free(P->gcell);
    P->gcell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ng > 0 ? ng : 1));
    int64_t g = 0;
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] == T_GHOST) P->gcell[g++] = (int32_t)id;
    P->nfluid = nf; P->nghost = ng; P->ndead = nd; P->odd_columns = odd;
    P->classified = 1;
    free_stencils(P);
    free_hierarchy(P);
    if (counts) { counts[0] = nf; counts[1] = ng; counts[2] = nd; }
    /* a closed, consistently oriented mesh crosses every column ray an even number of
       times under the edge-ownership rule; an odd count means a broken mesh or predicate,
       and the classification is refused (the types stay readable for inspection) */
    if (odd) return ORC_E_GEOMETRY;
    return ORC_OK;
}

int64_t orc_odd_columns(const orc_problem *P) { return P->odd_columns; }
int64_t orc_num_ghosts(const orc_problem *P) { return P->nghost; }
void orc_get_types(const orc_problem *P, uint8_t *out) { memcpy(out, P->type, (size_t)P->ncell); }
void orc_get_ghost_cells(const orc_problem *P, int32_t *out) { memcpy(out, P->gcell, sizeof(int32_t) * P->nghost); }

/* ------------------------------------------------------------------------------------ */
/* body intercept: closest point on the mesh (Section 2.2, "closest points on the        */
/* surface ... where a normal can be dropped").  Per triangle the closest point follows  */
/* the Voronoi-region test of Ericson, Real-Time Collision Detection (2005), 5.1.5.      */
/* ------------------------------------------------------------------------------------ */

static void closest_on_triangle(const double *p, const double *a, const double *b, const double *c, double *q) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    for (int d = 0; d < 3; ++d) { ab[d] = b[d] - a[d]; ac[d] = c[d] - a[d]; ap[d] = p[d] - a[d]; }
    double d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
    double d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
    if (d1 <= 0.0 && d2 <= 0.0) { for (int d = 0; d < 3; ++d) q[d] = a[d]; return; }
    for (int d = 0; d < 3; ++d) bp[d] = p[d] - b[d];
    double d3 = ab[0] * bp[0] + ab[1] * bp[1] + ab[2] * bp[2];
    double d4 = ac[0] * bp[0] + ac[1] * bp[1] + ac[2] * bp[2];
    if (d3 >= 0.0 && d4 <= d3) { for (int d = 0; d < 3; ++d) q[d] = b[d]; return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int d = 0; d < 3; ++d) q[d] = a[d] + v * ab[d];
        return;
    }
    for (int d = 0; d < 3; ++d) cp[d] = p[d] - c[d];
    double d5 = ab[0] * cp[0] + ab[1] * cp[1] + ab[2] * cp[2];
    double d6 = ac[0] * cp[0] + ac[1] * cp[1] + ac[2] * cp[2];
    if (d6 >= 0.0 && d5 <= d6) { for (int d = 0; d < 3; ++d) q[d] = c[d]; return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double w = d2 / (d2 - d6);
        for (int d = 0; d < 3; ++d) q[d] = a[d] + w * ac[d];
        return;
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int d = 0; d < 3; ++d) q[d] = b[d] + w * (c[d] - b[d]);
        return;
    }
    double denom = 1.0 / ((va + vb) + vc);
    double v = vb * denom, w = vc * denom;
    for (int d = 0; d < 3; ++d) q[d] = (a[d] + ab[d] * v) + ac[d] * w;
}

/* argmin over triangles of the squared distance; ties go to the lowest triangle index.
   Triangles whose bounding box is farther than `radius` in some axis are skipped; if no
   triangle lies within `radius`, every triangle is searched. */
static int64_t closest_point_mesh(const orc_problem *P, const double *x, double radius, double *bi) {
    for (int pass = 0; pass < 2; ++pass) {
        double best = INFINITY;
        int64_t bt = -1;
        double q[3], bq[3] = {0, 0, 0};
        for (int64_t t = 0; t < P->nt; ++t) {
            const int32_t *tri = P->tris + 3 * t;
            const double *a = P->verts + 3 * tri[0], *b = P->verts + 3 * tri[1], *c = P->verts + 3 * tri[2];
            if (pass == 0) {
                int far = 0;
                for (int d = 0; d < 3 && !far; ++d) {
                    double lo = fmin(a[d], fmin(b[d], c[d])), hi = fmax(a[d], fmax(b[d], c[d]));
                    if (lo > x[d] + radius || hi < x[d] - radius) far = 1;
                }
                if (far) continue;
            }
            closest_on_triangle(x, a, b, c, q);
            double dx = q[0] - x[0], dy = q[1] - x[1], dz = q[2] - x[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < best) { best = d2; bt = t; bq[0] = q[0]; bq[1] = q[1]; bq[2] = q[2]; }
        }
        if (bt >= 0 && (pass == 1 || best <= radius * radius)) {
            bi[0] = bq[0]; bi[1] = bq[1]; bi[2] = bq[2];
            return bt;
        }
    }
    return -1;
}

/* public single-point query (brute force over all triangles) */
int64_t orc_closest_point(const orc_problem *P, const double *x, double *bi) {
    return closest_point_mesh(P, x, INFINITY, bi);
}

/* ------------------------------------------------------------------------------------ */
/* interpolation weights (Eq. 2 and Eq. 3)                                               */
/* ------------------------------------------------------------------------------------ */

/* trilinear monomial basis in local box coordinates: [xyz, xy, yz, xz, x, y, z, 1] */
static void basis3(double x, double y, double z, double *b) {
    b[0] = x * y * z; b[1] = x * y; b[2] = y * z; b[3] = x * z;
    b[4] = x; b[5] = y; b[6] = z; b[7] = 1.0;
}
static void basis3_grad(double x, double y, double z, double *bx, double *by, double *bz) {
    double gx[8] = {y * z, y, 0.0, z, 1.0, 0.0, 0.0, 0.0};
    double gy[8] = {x * z, x, z, 0.0, 0.0, 1.0, 0.0, 0.0};
    double gz[8] = {x * y, 0.0, y, x, 0.0, 0.0, 1.0, 0.0};
    memcpy(bx, gx, sizeof(gx)); memcpy(by, gy, sizeof(gy)); memcpy(bz, gz, sizeof(gz));
}
/* bilinear basis for one-cell-thick (2D) grids: [xy, x, y, 1] */
static void basis2(double x, double y, double *b) { b[0] = x * y; b[1] = x; b[2] = y; b[3] = 1.0; }
static void basis2_grad(double x, double y, double *bx, double *by) {
    bx[0] = y; bx[1] = 1.0; bx[2] = 0.0; bx[3] = 0.0;
    by[0] = x; by[1] = 0.0; by[2] = 1.0; by[3] = 0.0;
}

/* solve A x = rhs (n x n, row-major) by LU with partial pivoting; 0 if singular */
static int lu_solve(int n, double *A, double *rhs) {
    int piv[8];
    for (int k = 0; k < n; ++k) {
        int pr = k;
        double mx = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i) if (fabs(A[i * n + k]) > mx) { mx = fabs(A[i * n + k]); pr = i; }
        if (mx == 0.0) return 0;
        piv[k] = pr;
        if (pr != k) for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[pr * n + j]; A[pr * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            A[i * n + k] /= A[k * n + k];
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= A[i * n + k] * A[k * n + j];
        }
    }
    for (int k = 0; k < n; ++k) if (piv[k] != k) { double t = rhs[k]; rhs[k] = rhs[piv[k]]; rhs[piv[k]] = t; }
    for (int i = 0; i < n; ++i) for (int j = 0; j < i; ++j) rhs[i] -= A[i * n + j] * rhs[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) rhs[i] -= A[i * n + j] * rhs[j];
        rhs[i] /= A[i * n + i];
    }
    return 1;
}

/* largest i in [0, n-2] with c[i] <= x (0 if x < c[0]); n >= 2 */
static int box_lo(const double *c, int n, double x) {
    int lo = 0, hi = n - 2;
    if (x < c[0]) return 0;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (c[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

static double clamp01(double x, int *clamped) {
    if (x < 0.0) { *clamped = 1; return 0.0; }
    if (x > 1.0) { *clamped = 1; return 1.0; }
    return x;
}

int orc_build_stencils(orc_problem *P, int64_t *ng_out) {
    if (!P->classified) return ORC_E_STATE;
    free_stencils(P);
    const int64_t ng = P->nghost;
    const int two_d = (P->nz == 1);
    const int nm = two_d ? 4 : 8;
    P->gbi = dalloc(3 * ng); P->gn = dalloc(3 * ng); P->gip = dalloc(3 * ng);
    P->gbeta = dalloc(8 * ng); P->gbetag = dalloc(ng); P->gdl = dalloc(ng);
    P->gh = dalloc(ng); P->gdata = dalloc(ng);
    P->gst = (int32_t *)malloc(sizeof(int32_t) * 8 * (size_t)(ng > 0 ? ng : 1));
    P->gflags = (int32_t *)calloc((size_t)(ng > 0 ? ng : 1), sizeof(int32_t));
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t g = 0; g < ng; ++g) {
        int64_t id = P->gcell[g];
        int i = (int)(id % P->nx), j = (int)((id / P->nx) % P->ny), k = (int)(id / ((int64_t)P->nx * P->ny));
        double xg[3] = {P->xc[i], P->yc[j], P->zc[k]};
        /* the surface crosses the segment to any fluid neighbour, so the closest point lies
           within the largest centre distance to the 26 neighbours */
        double rx = fmax(i > 0 ? xg[0] - P->xc[i - 1] : 0.0, i < P->nx - 1 ? P->xc[i + 1] - xg[0] : 0.0);
        double ry = fmax(j > 0 ? xg[1] - P->yc[j - 1] : 0.0, j < P->ny - 1 ? P->yc[j + 1] - xg[1] : 0.0);
        double rz = fmax(k > 0 ? xg[2] - P->zc[k - 1] : 0.0, k < P->nz - 1 ? P->zc[k + 1] - xg[2] : 0.0);
        if (two_d) rz = 0.0;
        double radius = sqrt(rx * rx + ry * ry + rz * rz);
        double *bi = P->gbi + 3 * g, *nrm = P->gn + 3 * g, *ip = P->gip + 3 * g;
        int flags = 0;
        int64_t t = -1;
        if (P->has_mesh) t = closest_point_mesh(P, xg, radius, bi);
        if (t < 0) {
#pragma omp atomic write
            err = 1;
            continue;
        }
        if (two_d) bi[2] = xg[2]; /* the body is a prism along z: stay in the cell plane */
        double dvec[3] = {bi[0] - xg[0], bi[1] - xg[1], bi[2] - xg[2]};
        double dist = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
        double hloc = fmin(P->wx[i], P->wy[j]);
        if (!two_d) hloc = fmin(hloc, P->wz[k]);
        const int on_surface = dist <= 1e-12 * hloc;
        if (on_surface) {
            const int32_t *tri = P->tris + 3 * t;
            const double *a = P->verts + 3 * tri[0], *b = P->verts + 3 * tri[1], *c = P->verts + 3 * tri[2];
            double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            double nn[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
            if (two_d) nn[2] = 0.0;
            double ln = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
            for (int d = 0; d < 3; ++d) nrm[d] = nn[d] / ln;
            flags |= GF_NFALLBACK;
            /* the ghost centre is on the surface: it is its own intercept and image point */
            for (int d = 0; d < 3; ++d) bi[d] = xg[d];
            dist = 0.0;
        } else {
            for (int d = 0; d < 3; ++d) nrm[d] = dvec[d] / dist;
        }
        /* image point: mirror of the ghost centre through the body intercept */
        for (int d = 0; d < 3; ++d) ip[d] = (bi[d] + bi[d]) - xg[d];
        double dl = dist + dist;
        P->gdl[g] = dl;
        /* interpolation box: around the image point; for a ghost on the surface (image point
           = the centre itself) the cells on the side the normal points to, so its equation is
           the one-sided normal difference into the fluid */
        int i0, j0, k0;
        if (on_surface) {
            i0 = nrm[0] >= 0.0 ? i : i - 1;
            j0 = nrm[1] >= 0.0 ? j : j - 1;
            k0 = nrm[2] >= 0.0 ? k : k - 1;
            i0 = i0 < 0 ? 0 : (i0 > P->nx - 2 ? P->nx - 2 : i0);
            j0 = j0 < 0 ? 0 : (j0 > P->ny - 2 ? P->ny - 2 : j0);
            k0 = two_d ? 0 : (k0 < 0 ? 0 : (k0 > P->nz - 2 ? P->nz - 2 : k0));
        } else {
            i0 = P->nx > 1 ? box_lo(P->xc, P->nx, ip[0]) : 0;
            j0 = P->ny > 1 ? box_lo(P->yc, P->ny, ip[1]) : 0;
            k0 = P->nz > 1 ? box_lo(P->zc, P->nz, ip[2]) : 0;
        }
        double hx = P->xc[i0 + 1] - P->xc[i0], hy = P->yc[j0 + 1] - P->yc[j0];
        double hz = two_d ? 1.0 : P->zc[k0 + 1] - P->zc[k0];
        int cl = 0;
        double sx = clamp01((ip[0] - P->xc[i0]) / hx, &cl);
        double sy = clamp01((ip[1] - P->yc[j0]) / hy, &cl);
        double sz = two_d ? 0.0 : clamp01((ip[2] - P->zc[k0]) / hz, &cl);
        if (cl) flags |= GF_CLAMPED;
        int32_t mem[8];
        int nfluid = 0, ndead = 0, self = -1;
        for (int m = 0; m < nm; ++m) {
            int a = m & 1, b = (m >> 1) & 1, c = (m >> 2) & 1;
            int64_t mid = IDX(P, i0 + a, j0 + b, k0 + c);
            mem[m] = (int32_t)mid;
            uint8_t ty = P->type[mid];
            if (ty == T_FLUID) nfluid++;
            if (ty == T_DEAD) ndead++;
            if (mid == id) self = m;
        }
        int32_t *st = P->gst + 8 * g;
        double *beta = P->gbeta + 8 * g;
        for (int m = 0; m < 8; ++m) { st[m] = -1; beta[m] = 0.0; }
        P->gbetag[g] = 0.0;
        /* local coordinates of the body intercept in the box */
        double lbx = (bi[0] - P->xc[i0]) / hx, lby = (bi[1] - P->yc[j0]) / hy;
        double lbz = two_d ? 0.0 : (bi[2] - P->zc[k0]) / hz;
        /* The Neumann row replaces the ghost's own value only when the derivative of the
           ghost's own trilinear hat function along n at the intercept is negative, that is
           when the one-sided difference points from the ghost into its box (always so for a
           mirrored image point, whose box holds the intercept); otherwise the row is
           degenerate. */
        int bad_row = 0;
        if (self >= 0) {
            int sa = self & 1, sb = (self >> 1) & 1, sc = (self >> 2) & 1;
            double fx = sa ? lbx : 1.0 - lbx, fy = sb ? lby : 1.0 - lby, fz = sc ? lbz : 1.0 - lbz;
            double dnx = (sa ? 1.0 : -1.0) / hx, dny = (sb ? 1.0 : -1.0) / hy, dnz = (sc ? 1.0 : -1.0) / hz;
            double dn = two_d ? nrm[0] * dnx * fy + nrm[1] * dny * fx
                              : (nrm[0] * dnx * (fy * fz) + nrm[1] * dny * (fx * fz)) + nrm[2] * dnz * (fx * fy);
            if (!(dn < 0.0)) bad_row = 1;
        }
        if (ndead > 0 || nfluid == 0 || bad_row) {
            flags |= GF_DEGENERATE;
            P->gflags[g] = flags;
            continue;
        }
        /* Vandermonde system of Eq. 3: row m is the basis at member m; the ghost's own row
           (when it is in the box) is the normal derivative of the basis at the body
           intercept.  The weights of Eq. 2 are beta = V^{-T} b(image point). */
        double A[64], rhs[8];
        double bx[8], by[8], bz[8];
        for (int m = 0; m < nm; ++m) {
            double row[8];
            int a = m & 1, b = (m >> 1) & 1, c = (m >> 2) & 1;
            if (m == self) {
                if (two_d) {
                    basis2_grad(lbx, lby, bx, by);
                    for (int q = 0; q < 4; ++q) row[q] = nrm[0] * (bx[q] / hx) + nrm[1] * (by[q] / hy);
                } else {
                    basis3_grad(lbx, lby, lbz, bx, by, bz);
                    for (int q = 0; q < 8; ++q)
                        row[q] = (nrm[0] * (bx[q] / hx) + nrm[1] * (by[q] / hy)) + nrm[2] * (bz[q] / hz);
                }
            } else {
                if (two_d) basis2((double)a, (double)b, row);
                else basis3((double)a, (double)b, (double)c, row);
            }
            /* store the transpose: A = V^T */
            for (int q = 0; q < nm; ++q) A[q * nm + m] = row[q];
        }
        if (two_d) basis2(sx, sy, rhs); else basis3(sx, sy, sz, rhs);
        if (!lu_solve(nm, A, rhs)) {
            flags |= GF_DEGENERATE;
            P->gflags[g] = flags;
            continue;
        }
        for (int m = 0; m < nm; ++m) {
            if (m == self) { P->gbetag[g] = rhs[m]; st[m] = -1; beta[m] = rhs[m]; }
            else { st[m] = mem[m]; beta[m] = rhs[m]; }
        }
        if (self >= 0) flags |= GF_SELF;
        P->gflags[g] = flags;
    }
    if (err) { free_stencils(P); return ORC_E_GEOMETRY; }
    for (int64_t g = 0; g < ng; ++g) P->gdata[g] = 0.0;
    /* a degenerate ghost's equation (mean of its fluid neighbours) carries no Neumann term */
    for (int64_t g = 0; g < ng; ++g)
        P->gh[g] = (P->gflags[g] & GF_DEGENERATE) ? 0.0 : (P->gbetag[g] - P->gdl[g]) * P->gdata[g];
    P->stencils = 1;
    free_hierarchy(P);
    if (ng_out) *ng_out = ng;
    return ORC_OK;
}

/* Neumann data g = dp/dn at each body intercept (0 for the projection) */
int orc_set_neumann(orc_problem *P, const double *g) {
    if (!P->stencils) return ORC_E_STATE;
    for (int64_t q = 0; q < P->nghost; ++q) {
        P->gdata[q] = g ? g[q] : 0.0;
        /* ghost row: p_g - sum_{m != g} beta_m p_m = (beta_g - dl) * g_BI */
        P->gh[q] = (P->gflags[q] & GF_DEGENERATE) ? 0.0 : (P->gbetag[q] - P->gdl[q]) * P->gdata[q];
    }
    return ORC_OK;
}

void orc_get_ghosts(const orc_problem *P, double *bi, double *nrm, double *ip, int32_t *st,
                    double *beta, double *betag, double *dl, double *h, int32_t *flags) {
    int64_t ng = P->nghost;
    if (bi) memcpy(bi, P->gbi, sizeof(double) * 3 * ng);
    if (nrm) memcpy(nrm, P->gn, sizeof(double) * 3 * ng);
    if (ip) memcpy(ip, P->gip, sizeof(double) * 3 * ng);
    if (st) memcpy(st, P->gst, sizeof(int32_t) * 8 * ng);
    if (beta) memcpy(beta, P->gbeta, sizeof(double) * 8 * ng);
    if (betag) memcpy(betag, P->gbetag, sizeof(double) * ng);
    if (dl) memcpy(dl, P->gdl, sizeof(double) * ng);
    if (h) memcpy(h, P->gh, sizeof(double) * ng);
    if (flags) memcpy(flags, P->gflags, sizeof(int32_t) * ng);
}

/* ------------------------------------------------------------------------------------ */
/* level-0 operator, smoother and ghost refresh                                         */
/* ------------------------------------------------------------------------------------ */

/* sum of a_f * p_nb over the six faces (wall faces contribute nothing) and the diagonal */
static inline void stencil0(const orc_problem *P, const double *p, int i, int j, int k, double *num, double *diag) {
    int64_t id = IDX(P, i, j, k);
    const int64_t sx = 1, sy = P->nx, sz = (int64_t)P->nx * P->ny;
    double s = 0.0, d = 0.0;
    s = s + (i > 0 ? P->axm[i] * p[id - sx] : 0.0);
    s = s + (i < P->nx - 1 ? P->axp[i] * p[id + sx] : 0.0);
    s = s + (j > 0 ? P->aym[j] * p[id - sy] : 0.0);
    s = s + (j < P->ny - 1 ? P->ayp[j] * p[id + sy] : 0.0);
    s = s + (k > 0 ? P->azm[k] * p[id - sz] : 0.0);
    s = s + (k < P->nz - 1 ? P->azp[k] * p[id + sz] : 0.0);
    d = P->axm[i] + P->axp[i];
    d = d + P->aym[j];
    d = d + P->ayp[j];
    d = d + P->azm[k];
    d = d + P->azp[k];
    *num = s;
    *diag = d;
}

/* (S p)_c on fluid rows (per unit volume), 0 elsewhere */
void orc_apply_S(const orc_problem *P, const double *p, double *out) {
#pragma omp parallel for
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] != T_FLUID) { out[id] = 0.0; continue; }
                double num, diag;
                stencil0(P, p, i, j, k, &num, &diag);
                out[id] = num - diag * p[id];
            }
}

static uint64_t splitmix(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* One red-black Gauss-Seidel sweep over the fluid cells of level 0: every red cell
   ((i+j+k) even), then every black cell, each set to
       p_c = (sum_f a_f p_nb - (f_c - lambda)) / sum_f a_f.
   perm_seed != 0 visits the cells of a colour in a random order (serially); cells of one
   colour never read each other, so the result must not change. */
static void sweep0(const orc_problem *P, double *p, const double *f, double lambda, uint64_t perm_seed) {
    for (int colour = 0; colour < 2; ++colour) {
        if (perm_seed == 0) {
#pragma omp parallel for
            for (int k = 0; k < P->nz; ++k)
                for (int j = 0; j < P->ny; ++j)
                    for (int i = 0; i < P->nx; ++i) {
                        if (((i + j + k) & 1) != colour) continue;
                        int64_t id = IDX(P, i, j, k);
                        if (P->type[id] != T_FLUID) continue;
                        double num, diag;
                        stencil0(P, p, i, j, k, &num, &diag);
                        p[id] = (num - (f[id] - lambda)) / diag;
                    }
        } else {
            int64_t n = 0;
            int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)P->ncell);
            for (int64_t id = 0; id < P->ncell; ++id) {
                int i = (int)(id % P->nx), j = (int)((id / P->nx) % P->ny), k = (int)(id / ((int64_t)P->nx * P->ny));
                if (((i + j + k) & 1) == colour && P->type[id] == T_FLUID) list[n++] = id;
            }
            uint64_t s = perm_seed + (uint64_t)colour;
            for (int64_t q = n - 1; q > 0; --q) {
                int64_t r = (int64_t)(splitmix(&s) % (uint64_t)(q + 1));
                int64_t t = list[q]; list[q] = list[r]; list[r] = t;
            }
            for (int64_t q = 0; q < n; ++q) {
                int64_t id = list[q];
                int i = (int)(id % P->nx), j = (int)((id / P->nx) % P->ny), k = (int)(id / ((int64_t)P->nx * P->ny));
                double num, diag;
                stencil0(P, p, i, j, k, &num, &diag);
                p[id] = (num - (f[id] - lambda)) / diag;
            }
            free(list);
        }
    }
}

/* mean of the fluid cells of the 26-neighbourhood (degenerate ghosts only) */
static double fluid_neighbour_mean(const orc_problem *P, const double *p, int64_t id) {
    int i = (int)(id % P->nx), j = (int)((id / P->nx) % P->ny), k = (int)(id / ((int64_t)P->nx * P->ny));
    double s = 0.0;
    int n = 0;
    for (int dk = -1; dk <= 1; ++dk)
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                int ii = i + di, jj = j + dj, kk = k + dk;
                if (ii < 0 || jj < 0 || kk < 0 || ii >= P->nx || jj >= P->ny || kk >= P->nz) continue;
                int64_t q = IDX(P, ii, jj, kk);
                if (P->type[q] == T_FLUID) { s += p[q]; n++; }
            }
    return n ? s / n : 0.0;
}

/* Ghost values from their implicit equations, all from one snapshot of p (Jacobi over
   the ghosts):  p_g = sum_{m != g} beta_m p_m + h_g, with right-hand sides gh. */
static void ghost_refresh_h(const orc_problem *P, double *p, const double *gh) {
    int64_t ng = P->nghost;
    if (ng == 0) return;
    double *nv = dalloc(ng);
#pragma omp parallel for
    for (int64_t g = 0; g < ng; ++g) {
        if (P->gflags[g] & GF_DEGENERATE) { nv[g] = fluid_neighbour_mean(P, p, P->gcell[g]); continue; }
        const int32_t *st = P->gst + 8 * g;
        const double *beta = P->gbeta + 8 * g;
        double s = 0.0;
        for (int m = 0; m < 8; ++m) if (st[m] >= 0) s = s + beta[m] * p[st[m]];
        nv[g] = s + gh[g];
    }
    for (int64_t g = 0; g < ng; ++g) p[P->gcell[g]] = nv[g];
    free(nv);
}

static void ghost_refresh(const orc_problem *P, double *p) { ghost_refresh_h(P, p, P->gh); }

static double ghost_residual_max(const orc_problem *P, const double *p) {
    double mx = 0.0;
    for (int64_t g = 0; g < P->nghost; ++g) {
        double target;
        if (P->gflags[g] & GF_DEGENERATE) target = fluid_neighbour_mean(P, p, P->gcell[g]);
        else {
            const int32_t *st = P->gst + 8 * g;
            const double *beta = P->gbeta + 8 * g;
            double s = 0.0;
            for (int m = 0; m < 8; ++m) if (st[m] >= 0) s = s + beta[m] * p[st[m]];
            target = s + P->gh[g];
        }
        mx = fmax(mx, fabs(p[P->gcell[g]] - target));
    }
    return mx;
}

/* public debug entry points */
int orc_sweep(orc_problem *P, double *p, const double *f, double lambda, int nsweeps, uint64_t perm_seed, int refresh) {
    if (!P->classified) return ORC_E_STATE;
    if (refresh && P->nghost > 0 && !P->stencils) return ORC_E_STATE;
    for (int s = 0; s < nsweeps; ++s) {
        sweep0(P, p, f, lambda, perm_seed ? perm_seed + 2 * (uint64_t)s : 0);
        if (refresh) ghost_refresh(P, p);
    }
    return ORC_OK;
}
int orc_ghost_refresh(orc_problem *P, double *p) {
    if (!P->stencils) return ORC_E_STATE;
    ghost_refresh(P, p);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* multigrid hierarchy                                                                  */
/* ------------------------------------------------------------------------------------ */

static inline int64_t LIDX(const level_t *L, int i, int j, int k) {
    return ((int64_t)k * L->n[1] + j) * L->n[0] + i;
}
static inline double lvol(const level_t *L, int i, int j, int k) {
    return (L->w[0][i] * L->w[1][j]) * L->w[2][k];
}

static void level_alloc_fields(level_t *L) {
    int64_t nc = (int64_t)L->n[0] * L->n[1] * L->n[2];
    L->active = (uint8_t *)calloc((size_t)nc, 1);
    for (int d = 0; d < 3; ++d) L->T[d] = dalloc(nc);
    L->e = dalloc(nc); L->R = dalloc(nc); L->r = dalloc(nc);
}

static double min_width(const level_t *L, int d) {
    double m = INFINITY;
    for (int i = 0; i < L->n[d]; ++i) m = fmin(m, L->w[d][i]);
    return m;
}

/* Coarsening by cell width.  Along every axis with at least 4 cells, scanning from the low
   wall, a cell is merged with the next one when their combined width is at most a threshold
   t; every other cell is kept whole.  Level l (built from level l-1) starts from
   t = MERGE_WIDTH x 2^(l-1) h_min (h_min: the smallest cell width of the grid over the axes
   with at least two cells) and raises t by a factor 5/4 until the level holds at most half as
   many cells as level l-1 or every axis is halved outright.  So the narrowest cells merge
   first: on a uniform axis this is plain halving, and in a stretched region the cells already
   wide along one axis are kept along it while they are still merged along the others, so
   coarse cells tend to equal widths and point smoothing keeps working.  The hierarchy stops
   when no axis merges a cell or after LEVEL_CAP levels.  merge_axis returns the coarse count
   and fills cs. */
#define LEVEL_CAP 24
#define MERGE_WIDTH 3.5
static int merge_axis(const level_t *F, int d, double wmax, int *cs) {
    const int n = F->n[d];
    int m = 0, i = 0;
    while (i < n) {
        cs[m++] = i;
        if (n >= 4 && i + 1 < n && F->w[d][i] + F->w[d][i + 1] <= wmax) i += 2;
        else i += 1;
    }
    cs[m] = n;
    return m;
}

/* children range of coarse index I along an axis */
static inline void child_range(const int *cs, int I, int *c0, int *c1) {
    *c0 = cs[I];
    *c1 = cs[I + 1] - 1;
}

static int build_hierarchy(orc_problem *P) {
    free_hierarchy(P);
    level_t *L0 = &P->lev[0];
    L0->n[0] = P->nx; L0->n[1] = P->ny; L0->n[2] = P->nz;
    const double *fs[3] = {P->xf, P->yf, P->zf};
    for (int d = 0; d < 3; ++d) {
        L0->f[d] = dalloc(L0->n[d] + 1); memcpy(L0->f[d], fs[d], sizeof(double) * (L0->n[d] + 1));
        L0->c[d] = dalloc(L0->n[d]); L0->w[d] = dalloc(L0->n[d]);
        axis_metrics(L0->n[d], L0->f[d], L0->c[d], L0->w[d]);
    }
    level_alloc_fields(L0);
    P->vol_fluid = 0.0;
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                L0->active[id] = (P->type[id] == T_FLUID);
                if (L0->active[id]) P->vol_fluid += lvol(L0, i, j, k);
            }
    L0->vol_active = P->vol_fluid;
    double hmin = INFINITY;
    for (int d = 0; d < 3; ++d) if (L0->n[d] >= 2) hmin = fmin(hmin, min_width(L0, d));
    int nlev = 1;
    while (nlev < LEVEL_CAP) {
        level_t *F = &P->lev[nlev - 1];
        level_t *C = &P->lev[nlev];
        const int64_t nf = (int64_t)F->n[0] * F->n[1] * F->n[2];
        for (int d = 0; d < 3; ++d) C->cs[d] = ialloc(F->n[d] + 1);
        double wmax = MERGE_WIDTH * ldexp(hmin, nlev - 1);
        int any = 0;
        for (int rise = 0; rise < 64; ++rise, wmax *= 1.25) {
            int64_t nc = 1;
            int full = 1;
            any = 0;
            for (int d = 0; d < 3; ++d) {
                C->n[d] = merge_axis(F, d, wmax, C->cs[d]);
                nc *= C->n[d];
                any |= C->n[d] < F->n[d];
                if (F->n[d] >= 4 && C->n[d] != (F->n[d] + 1) / 2) full = 0;
            }
            if (2 * nc <= nf || full) break;
        }
        for (int d = 0; d < 3; ++d) C->halved[d] = C->n[d] < F->n[d];
        if (!any) {
            for (int d = 0; d < 3; ++d) { free(C->cs[d]); C->cs[d] = NULL; }
            break;
        }
        for (int d = 0; d < 3; ++d) {
            F->par[d] = ialloc(F->n[d]);
            for (int I = 0; I < C->n[d]; ++I)
                for (int i = C->cs[d][I]; i < C->cs[d][I + 1]; ++i) F->par[d][i] = I;
            C->f[d] = dalloc(C->n[d] + 1);
            for (int q = 0; q <= C->n[d]; ++q) C->f[d][q] = F->f[d][C->cs[d][q]];
            C->c[d] = dalloc(C->n[d]); C->w[d] = dalloc(C->n[d]);
            axis_metrics(C->n[d], C->f[d], C->c[d], C->w[d]);
        }
        level_alloc_fields(C);
        /* active: any active child */
        C->vol_active = 0.0;
        for (int K = 0; K < C->n[2]; ++K)
            for (int J = 0; J < C->n[1]; ++J)
                for (int I = 0; I < C->n[0]; ++I) {
                    int i0, i1, j0, j1, k0, k1, act = 0;
                    child_range(C->cs[0], I, &i0, &i1);
                    child_range(C->cs[1], J, &j0, &j1);
                    child_range(C->cs[2], K, &k0, &k1);
                    for (int k = k0; k <= k1; ++k)
                        for (int j = j0; j <= j1; ++j)
                            for (int i = i0; i <= i1; ++i) act |= F->active[LIDX(F, i, j, k)];
                    C->active[LIDX(C, I, J, K)] = (uint8_t)act;
                    if (act) C->vol_active += lvol(C, I, J, K);
                }
        /* staircase transmissibility of each coarse low face: open child-face area over the
           coarse centre distance; a child face is open iff both of its cells are active */
        for (int d = 0; d < 3; ++d) {
            int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
            for (int K = 0; K < C->n[2]; ++K)
                for (int J = 0; J < C->n[1]; ++J)
                    for (int I = 0; I < C->n[0]; ++I) {
                        int Ic[3] = {I, J, K};
                        int64_t cid = LIDX(C, I, J, K);
                        if (Ic[d] == 0) { C->T[d][cid] = 0.0; continue; }
                        int fface = C->cs[d][Ic[d]];
                        int a0, a1, b0, b1;
                        child_range(C->cs[e1], Ic[e1], &a0, &a1);
                        child_range(C->cs[e2], Ic[e2], &b0, &b1);
                        double area = 0.0;
                        for (int b = b0; b <= b1; ++b)
                            for (int a = a0; a <= a1; ++a) {
                                int lo[3], hi[3];
                                lo[d] = fface - 1; hi[d] = fface;
                                lo[e1] = hi[e1] = a;
                                lo[e2] = hi[e2] = b;
                                if (F->active[LIDX(F, lo[0], lo[1], lo[2])] && F->active[LIDX(F, hi[0], hi[1], hi[2])])
                                    area += F->w[e1][a] * F->w[e2][b];
                            }
                        double dist = C->c[d][Ic[d]] - C->c[d][Ic[d] - 1];
                        C->T[d][cid] = area / dist;
                    }
        }
        /* prolongation tables for level nlev-1 from level nlev, per axis: value at fine
           index i = (1-t) e[lo] + t e[hi] in physical coordinates, lo the parent and hi the
           parent's neighbour on the side of the fine centre (clamped at the walls); a cell
           kept whole takes its parent alone */
        for (int d = 0; d < 3; ++d) {
            F->plo[d] = ialloc(F->n[d]); F->phi[d] = ialloc(F->n[d]); F->pt[d] = dalloc(F->n[d]);
            for (int i = 0; i < F->n[d]; ++i) {
                int I = F->par[d][i];
                if (C->cs[d][I + 1] - C->cs[d][I] == 1) { F->plo[d][i] = I; F->phi[d][i] = I; F->pt[d][i] = 0.0; continue; }
                double x = F->c[d][i], X = C->c[d][I];
                int Jn = (x < X) ? I - 1 : I + 1;
                if (Jn < 0 || Jn >= C->n[d]) { F->plo[d][i] = I; F->phi[d][i] = I; F->pt[d][i] = 0.0; continue; }
                F->plo[d][i] = I; F->phi[d][i] = Jn;
                F->pt[d][i] = (x - X) / (C->c[d][Jn] - X);
            }
        }
        nlev++;
    }
    P->nlev = nlev;
    return ORC_OK;
}

int orc_num_levels(orc_problem *P) {
    if (!P->nlev) build_hierarchy(P);
    return P->nlev;
}
void orc_level_info(orc_problem *P, int l, int *dims, int *halved, double *vol_active) {
    if (!P->nlev) build_hierarchy(P);
    level_t *L = &P->lev[l];
    for (int d = 0; d < 3; ++d) { dims[d] = L->n[d]; halved[d] = L->halved[d]; }
    *vol_active = L->vol_active;
}
/* children starts of level l >= 1 along axis d (n_l[d] + 1 entries) */
void orc_level_map(orc_problem *P, int l, int d, int *cs) {
    if (!P->nlev) build_hierarchy(P);
    const level_t *L = &P->lev[l];
    if (l < 1 || l >= P->nlev) return;
    memcpy(cs, L->cs[d], sizeof(int) * (size_t)(L->n[d] + 1));
}

void orc_level_arrays(orc_problem *P, int l, uint8_t *active, double *Tx, double *Ty, double *Tz) {
    if (!P->nlev) build_hierarchy(P);
    level_t *L = &P->lev[l];
    int64_t nc = (int64_t)L->n[0] * L->n[1] * L->n[2];
    if (active) memcpy(active, L->active, (size_t)nc);
    if (l > 0) {
        if (Tx) memcpy(Tx, L->T[0], sizeof(double) * nc);
        if (Ty) memcpy(Ty, L->T[1], sizeof(double) * nc);
        if (Tz) memcpy(Tz, L->T[2], sizeof(double) * nc);
    }
}

/* coarse-level stencil (integrated form) */
static inline void stencilC(const level_t *L, const double *e, int I, int J, int K, double *num, double *diag) {
    int64_t id = LIDX(L, I, J, K);
    const int64_t sx = 1, sy = L->n[0], sz = (int64_t)L->n[0] * L->n[1];
    double txm = L->T[0][id], txp = (I < L->n[0] - 1) ? L->T[0][id + sx] : 0.0;
    double tym = L->T[1][id], typ = (J < L->n[1] - 1) ? L->T[1][id + sy] : 0.0;
    double tzm = L->T[2][id], tzp = (K < L->n[2] - 1) ? L->T[2][id + sz] : 0.0;
    double s = 0.0;
    s = s + (I > 0 ? txm * e[id - sx] : 0.0);
    s = s + (I < L->n[0] - 1 ? txp * e[id + sx] : 0.0);
    s = s + (J > 0 ? tym * e[id - sy] : 0.0);
    s = s + (J < L->n[1] - 1 ? typ * e[id + sy] : 0.0);
    s = s + (K > 0 ? tzm * e[id - sz] : 0.0);
    s = s + (K < L->n[2] - 1 ? tzp * e[id + sz] : 0.0);
    double d = txm + txp;
    d = d + tym;
    d = d + typ;
    d = d + tzm;
    d = d + tzp;
    *num = s;
    *diag = d;
}

/* RB Gauss-Seidel on a coarse level: sum_F T_F (e_NB - e_C) = R_C - V_C mu */
static void sweepC(level_t *L) {
    for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for
        for (int K = 0; K < L->n[2]; ++K)
            for (int J = 0; J < L->n[1]; ++J)
                for (int I = 0; I < L->n[0]; ++I) {
                    if (((I + J + K) & 1) != colour) continue;
                    int64_t id = LIDX(L, I, J, K);
                    if (!L->active[id]) continue;
                    double num, diag;
                    stencilC(L, L->e, I, J, K, &num, &diag);
                    if (diag > 0.0) L->e[id] = (num - (L->R[id] - lvol(L, I, J, K) * L->mu)) / diag;
                }
    }
}

static void residualC(level_t *L) {
#pragma omp parallel for
    for (int K = 0; K < L->n[2]; ++K)
        for (int J = 0; J < L->n[1]; ++J)
            for (int I = 0; I < L->n[0]; ++I) {
                int64_t id = LIDX(L, I, J, K);
                if (!L->active[id]) { L->r[id] = 0.0; continue; }
                double num, diag;
                stencilC(L, L->e, I, J, K, &num, &diag);
                L->r[id] = (L->R[id] - lvol(L, I, J, K) * L->mu) - (num - diag * L->e[id]);
            }
}

/* R_{l+1}[C] = sum of the (volume-integrated) residuals of the active children; then the
   compatibility shift mu_{l+1} = sum R / sum V over active coarse cells */
static void restrict_to(level_t *F, level_t *C, const double *rint) {
    for (int K = 0; K < C->n[2]; ++K)
        for (int J = 0; J < C->n[1]; ++J)
            for (int I = 0; I < C->n[0]; ++I) {
                int i0, i1, j0, j1, k0, k1;
                child_range(C->cs[0], I, &i0, &i1);
                child_range(C->cs[1], J, &j0, &j1);
                child_range(C->cs[2], K, &k0, &k1);
                double s = 0.0;
                for (int k = k0; k <= k1; ++k)
                    for (int j = j0; j <= j1; ++j)
                        for (int i = i0; i <= i1; ++i) {
                            int64_t fid = LIDX(F, i, j, k);
                            if (F->active[fid]) s += rint[fid];
                        }
                C->R[LIDX(C, I, J, K)] = s;
            }
    double sr = 0.0;
    int64_t nc = (int64_t)C->n[0] * C->n[1] * C->n[2];
    for (int64_t q = 0; q < nc; ++q) if (C->active[q]) sr += C->R[q];
    C->mu = C->vol_active > 0.0 ? sr / C->vol_active : 0.0;
}

/* e_F += P e_C on active fine cells: trilinear from the nearest coarse centres, or the
   parent's value when any contributing coarse cell is inactive */
static void prolong_add(level_t *F, const level_t *C, double *target) {
#pragma omp parallel for
    for (int k = 0; k < F->n[2]; ++k)
        for (int j = 0; j < F->n[1]; ++j)
            for (int i = 0; i < F->n[0]; ++i) {
                int64_t fid = LIDX(F, i, j, k);
                if (!F->active[fid]) continue;
                int ix[2] = {F->plo[0][i], F->phi[0][i]}, iy[2] = {F->plo[1][j], F->phi[1][j]}, iz[2] = {F->plo[2][k], F->phi[2][k]};
                double wx[2] = {1.0 - F->pt[0][i], F->pt[0][i]}, wy[2] = {1.0 - F->pt[1][j], F->pt[1][j]}, wz[2] = {1.0 - F->pt[2][k], F->pt[2][k]};
                int nx_ = (ix[0] == ix[1]) ? 1 : 2, ny_ = (iy[0] == iy[1]) ? 1 : 2, nz_ = (iz[0] == iz[1]) ? 1 : 2;
                int all = 1;
                double s = 0.0;
                for (int c = 0; c < nz_; ++c)
                    for (int b = 0; b < ny_; ++b)
                        for (int a = 0; a < nx_; ++a) {
                            int64_t cid = LIDX(C, ix[a], iy[b], iz[c]);
                            if (!C->active[cid]) all = 0;
                            s += (wx[a] * wy[b]) * wz[c] * C->e[cid];
                        }
                if (!all) {
                    int pi = F->par[0][i], pj = F->par[1][j], pk = F->par[2][k];
                    s = C->e[LIDX(C, pi, pj, pk)];
                }
                target[fid] += s;
            }
}

static void remove_mean(level_t *L) {
    double s = 0.0;
    for (int K = 0; K < L->n[2]; ++K)
        for (int J = 0; J < L->n[1]; ++J)
            for (int I = 0; I < L->n[0]; ++I) {
                int64_t id = LIDX(L, I, J, K);
                if (L->active[id]) s += lvol(L, I, J, K) * L->e[id];
            }
    double m = L->vol_active > 0.0 ? s / L->vol_active : 0.0;
    int64_t nc = (int64_t)L->n[0] * L->n[1] * L->n[2];
    for (int64_t q = 0; q < nc; ++q) if (L->active[q]) L->e[q] -= m;
}

/* level-0 residual r = (f - lambda) - S p on fluid cells, stored volume-integrated in
   `rint` for restriction */
static void residual0_integrated(const orc_problem *P, const double *p, const double *f, double lambda, double *rint) {
    const level_t *L0 = &P->lev[0];
#pragma omp parallel for
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] != T_FLUID) { rint[id] = 0.0; continue; }
                double num, diag;
                stencil0(P, p, i, j, k, &num, &diag);
                double r = (f[id] - lambda) - (num - diag * p[id]);
                rint[id] = lvol(L0, i, j, k) * r;
            }
}

/* One V(nu1,nu2) cycle on level 0 for S p = f - lambda with ghost right-hand sides gh. */
static void vcycle_h(orc_problem *P, double *p, const double *f, double lambda, const double *gh, const orc_opts *o) {
    level_t *L0 = &P->lev[0];
    for (int s = 0; s < o->nu1; ++s) { sweep0(P, p, f, lambda, 0); ghost_refresh_h(P, p, gh); }
    if (P->nlev > 1) {
        residual0_integrated(P, p, f, lambda, L0->r);
        restrict_to(L0, &P->lev[1], L0->r);
        for (int l = 1; l < P->nlev; ++l) {
            level_t *L = &P->lev[l];
            int64_t nc = (int64_t)L->n[0] * L->n[1] * L->n[2];
            memset(L->e, 0, sizeof(double) * nc);
            if (l == P->nlev - 1) {
                for (int s = 0; s < o->coarsest_sweeps; ++s) sweepC(L);
                remove_mean(L);
            } else {
                for (int s = 0; s < o->nu1; ++s) sweepC(L);
                residualC(L);
                restrict_to(L, &P->lev[l + 1], L->r);
            }
        }
        for (int l = P->nlev - 2; l >= 1; --l) {
            prolong_add(&P->lev[l], &P->lev[l + 1], P->lev[l].e);
            for (int s = 0; s < o->nu2; ++s) sweepC(&P->lev[l]);
        }
        prolong_add(L0, &P->lev[1], p);
        ghost_refresh_h(P, p, gh);
    }
    for (int s = 0; s < o->nu2; ++s) { sweep0(P, p, f, lambda, 0); ghost_refresh_h(P, p, gh); }
}

static void vcycle(orc_problem *P, double *p, const double *f, double lambda, const orc_opts *o) {
    vcycle_h(P, p, f, lambda, P->gh, o);
}

/* r = f - S p on fluid rows; lambda = sum V r / sum V; returns || r - lambda ||_2 */
static double residual_norm(const orc_problem *P, const double *p, const double *f, double *lambda_out, double *rbuf) {
    const level_t *L0 = &P->lev[0];
#pragma omp parallel for
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] != T_FLUID) { rbuf[id] = 0.0; continue; }
                double num, diag;
                stencil0(P, p, i, j, k, &num, &diag);
                rbuf[id] = f[id] - (num - diag * p[id]);
            }
    double svr = 0.0;
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] == T_FLUID) svr += lvol(L0, i, j, k) * rbuf[id];
            }
    double lambda = svr / P->vol_fluid;
    double s2 = 0.0;
    for (int64_t id = 0; id < P->ncell; ++id)
        if (P->type[id] == T_FLUID) { double r = rbuf[id] - lambda; s2 += r * r; }
    *lambda_out = lambda;
    return sqrt(s2);
}

/* ------------------------------------------------------------------------------------ */
/* Krylov acceleration: BiCGStab (van der Vorst 1992; the paper's pressure solver family, */
/* Section 2.1) right-preconditioned by one V-cycle.                                     */
/*   unknowns : p on fluid and ghost cells (dead cells stay 0)                            */
/*   operator : fluid rows (S p)_c; ghost rows s_g (p_g - sum_{m != g} beta_m p_m), with  */
/*              s_g the diagonal of the flux stencil at the ghost cell, so both kinds of  */
/*              rows carry the same scale                                                 */
/*   rhs      : f on fluid rows, s_g h_g on ghost rows                                    */
/* The fluid part of every residual and operator image is projected to zero volume-       */
/* weighted mean: that removed mean is the lambda of the V-cycle iteration, so both        */
/* methods converge to the same discrete solution.                                         */
/* ------------------------------------------------------------------------------------ */

static double ghost_scale(const orc_problem *P, int64_t id) {
    int i = (int)(id % P->nx), j = (int)((id / P->nx) % P->ny), k = (int)(id / ((int64_t)P->nx * P->ny));
    double d = P->axm[i] + P->axp[i];
    d = d + P->aym[j];
    d = d + P->ayp[j];
    d = d + P->azm[k];
    d = d + P->azp[k];
    return d;
}

static void apply_full(const orc_problem *P, const double *y, double *out) {
    orc_apply_S(P, y, out);
#pragma omp parallel for
    for (int64_t g = 0; g < P->nghost; ++g) {
        int64_t id = P->gcell[g];
        double target;
        if (P->gflags[g] & GF_DEGENERATE) target = fluid_neighbour_mean(P, y, id);
        else {
            const int32_t *st = P->gst + 8 * g;
            const double *beta = P->gbeta + 8 * g;
            double s = 0.0;
            for (int m = 0; m < 8; ++m) if (st[m] >= 0) s = s + beta[m] * y[st[m]];
            target = s;
        }
        out[id] = ghost_scale(P, id) * (y[id] - target);
    }
}

/* remove the volume-weighted mean of the fluid part; returns that mean */
static double project_fluid_mean(const orc_problem *P, double *v) {
    const level_t *L0 = &P->lev[0];
    double s = 0.0;
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] == T_FLUID) s += lvol(L0, i, j, k) * v[id];
            }
    double m = s / P->vol_fluid;
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] == T_FLUID) v[id] -= m;
    return m;
}

static double dot_active(const orc_problem *P, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] != T_DEAD) s += a[id] * b[id];
    return s;
}

static double norm_fluid(const orc_problem *P, const double *a) {
    double s = 0.0;
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] == T_FLUID) s += a[id] * a[id];
    return sqrt(s);
}

/* m relaxed Jacobi sweeps of the fluid rows of A e = r (Section 2.1: the paper preconditions
   BiCGStab with scheduled relaxed Jacobi), sweep k with factor omega[k]:
     e_c <- (1 - w) e_c + w (sum_f a_f e_nb - r_c) / sum_f a_f,
   each followed by one pass of the ghost rows (right-hand sides gh) */
static void srj_sweeps(orc_problem *P, double *e, const double *r, const double *gh, int m, const double *omega) {
    const int64_t n = P->ncell;
    double *tmp = dalloc(n);
    for (int q = 0; q < m; ++q) {
        const double w = omega[q];
#pragma omp parallel for
        for (int64_t id = 0; id < n; ++id) {
            if (P->type[id] != T_FLUID) { tmp[id] = e[id]; continue; }
            int i = (int)(id % P->nx), j = (int)((id / P->nx) % P->ny), k = (int)(id / ((int64_t)P->nx * P->ny));
            double num, diag;
            stencil0(P, e, i, j, k, &num, &diag);
            tmp[id] = (1.0 - w) * e[id] + w * ((num - r[id]) / diag);
        }
        memcpy(e, tmp, sizeof(double) * (size_t)n);
        ghost_refresh_h(P, e, gh);
    }
    free(tmp);
}

/* e = M r from e = 0 (lambda 0, ghost right-hand sides r_g/s_g): one V-cycle (method 1) or
   the scheduled relaxed Jacobi sweeps (method 2) */
static void precondition(orc_problem *P, const double *r, double *e, double *gh, const orc_opts *o) {
    for (int64_t g = 0; g < P->nghost; ++g) {
        int64_t id = P->gcell[g];
        gh[g] = r[id] / ghost_scale(P, id);
    }
    memset(e, 0, sizeof(double) * (size_t)P->ncell);
    ghost_refresh_h(P, e, gh);
    if (o->method == 2) srj_sweeps(P, e, r, gh, o->srj_m, o->srj_omega);
    else vcycle_h(P, e, r, 0.0, gh, o);
}

/* b - A x, projected */
static void true_residual(orc_problem *P, const double *f, const double *x, double *r) {
    apply_full(P, x, r);
    for (int64_t id = 0; id < P->ncell; ++id) {
        if (P->type[id] == T_FLUID) r[id] = f[id] - r[id];
        else if (P->type[id] == T_DEAD) r[id] = 0.0;
    }
    for (int64_t g = 0; g < P->nghost; ++g) {
        int64_t id = P->gcell[g];
        r[id] = ghost_scale(P, id) * P->gh[g] - r[id];
    }
    project_fluid_mean(P, r);
}

/* Near-breakdown of BiCGStab: an inner product whose modulus is at most breakdown_tol times
   the product of its factors' norms (the shadow residual against the residual, or against
   the image A y), or omega = 0, ends the step without the quotient (alpha = 0, beta = 0) and
   restarts the shadow residual from the residual. */

/* returns the iteration count; *rel_out = ||r_fluid|| / ref of the true residual */
static int bicgstab(orc_problem *P, const double *f, double *x, const orc_opts *o, double ref, double *hist,
                    int hist_len, double *rel_out, int *status, int *restarts) {
    const double eps = o->breakdown_tol;
    const int64_t n = P->ncell;
    double *r = dalloc(n), *rh = dalloc(n), *pd = dalloc(n), *v = dalloc(n), *sv = dalloc(n), *t = dalloc(n);
    double *y = dalloc(n), *z = dalloc(n), *gh = dalloc(P->nghost);
    true_residual(P, f, x, r);
    memcpy(rh, r, sizeof(double) * n);
    double rho = dot_active(P, rh, r), rh2 = rho;
    double alpha = 0.0, omega = 0.0, beta = 0.0;
    const int nit = o->fixed_cycles > 0 ? o->fixed_cycles : o->max_cycles;
    double rel = norm_fluid(P, r) / ref;
    int it;
    *status = ORC_OK;
    for (it = 1; it <= nit; ++it) {
        int brk = 0;
        for (int64_t id = 0; id < n; ++id) pd[id] = r[id] + beta * (pd[id] - omega * v[id]);
        precondition(P, pd, y, gh, o);
        apply_full(P, y, v);
        project_fluid_mean(P, v);
        double rv = dot_active(P, rh, v), vv = dot_active(P, v, v);
        if (fabs(rv) > eps * sqrt(rh2 * vv)) alpha = rho / rv;
        else { alpha = 0.0; brk = 1; }
        for (int64_t id = 0; id < n; ++id) sv[id] = r[id] - alpha * v[id];
        precondition(P, sv, z, gh, o);
        apply_full(P, z, t);
        project_fluid_mean(P, t);
        double tt = dot_active(P, t, t);
        omega = tt > 0.0 ? dot_active(P, t, sv) / tt : 0.0;
        for (int64_t id = 0; id < n; ++id) {
            x[id] += alpha * y[id] + omega * z[id];
            r[id] = sv[id] - omega * t[id];
        }
        double rho_new = dot_active(P, rh, r), rr = dot_active(P, r, r);
        if (omega == 0.0 || !(fabs(rho_new) > eps * sqrt(rh2 * rr))) brk = 1;
        beta = brk ? 0.0 : (rho_new / rho) * (alpha / omega);
        rho = rho_new;
        rel = norm_fluid(P, r) / ref;
        if (hist && it - 1 < hist_len) hist[it - 1] = rel;
        if (!isfinite(rel) || !isfinite(beta)) { *status = ORC_E_NUMERIC; break; }
        int restart = 0;
        if (o->fixed_cycles > 0) {
            if (brk) { restart = 1; ++*restarts; }
        } else if (rel <= o->rel_tol) {
            true_residual(P, f, x, r);  /* confirm with the true residual */
            rel = norm_fluid(P, r) / ref;
            if (rel <= o->rel_tol) break;
            restart = 1;
        } else if (brk) {
            restart = 1;
            ++*restarts;
        }
        if (restart) { /* restart the shadow residual from the residual */
            memcpy(rh, r, sizeof(double) * n);
            rho = dot_active(P, rh, r);
            rh2 = rho;
            beta = 0.0;
        }
    }
    if (it > nit) it = nit;
    if (*status == ORC_OK && o->fixed_cycles <= 0 && rel > o->rel_tol) *status = ORC_NOT_CONVERGED;
    free(r); free(rh); free(pd); free(v); free(sv); free(t); free(y); free(z); free(gh);
    *rel_out = rel;
    return it;
}

/* Solve S p = f - lambda (fluid rows) with the ghost equations, V-mean of p over the fluid
   cells = 0.  p: in (initial guess if requested) / out.  hist (optional) receives the
   relative residual after each cycle. */
int orc_solve(orc_problem *P, const double *f, double *p, const orc_opts *o, orc_stats *st, double *hist, int hist_len) {
    if (!P->classified) return ORC_E_STATE;
    if (P->nghost > 0 && !P->stencils) return ORC_E_STATE;
    if (!P->nlev) build_hierarchy(P);
    if (P->vol_fluid <= 0.0) return ORC_E_GEOMETRY;
    for (int64_t id = 0; id < P->ncell; ++id) {
        if (P->type[id] == T_FLUID && !isfinite(f[id])) return ORC_E_NUMERIC;
    }
    if (!o->use_initial_guess) memset(p, 0, sizeof(double) * (size_t)P->ncell);
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] == T_DEAD) p[id] = 0.0;
    ghost_refresh(P, p);
    double *rbuf = dalloc(P->ncell);
    /* reference norm: || f - V-mean(f) || over fluid rows */
    double sf = 0.0;
    const level_t *L0 = &P->lev[0];
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] == T_FLUID) sf += lvol(L0, i, j, k) * f[id];
            }
    double fm = sf / P->vol_fluid, fn = 0.0;
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] == T_FLUID) fn += (f[id] - fm) * (f[id] - fm);
    fn = sqrt(fn);
    double lambda;
    double r0 = residual_norm(P, p, f, &lambda, rbuf);
    double ref = fn > 0.0 ? fn : r0;
    int status = ORC_OK, cyc = 0, restarts = 0;
    double rel = ref > 0.0 ? r0 / ref : 0.0;
    st->first_norm = r0;
    if ((o->method == 1 || o->method == 2) && !(o->breakdown_tol >= 0.0 && o->breakdown_tol < 1.0)) {
        free(rbuf);
        return ORC_E_ARG;
    }
    if (o->method == 2 && (o->srj_m < 1 || !o->srj_omega)) { free(rbuf); return ORC_E_ARG; }
    if (ref > 0.0 && (o->method == 1 || o->method == 2)) {
        cyc = bicgstab(P, f, p, o, ref, hist, hist_len, &rel, &status, &restarts);
        residual_norm(P, p, f, &lambda, rbuf);
    } else if (ref > 0.0) {
        int ncyc = o->fixed_cycles > 0 ? o->fixed_cycles : o->max_cycles;
        for (cyc = 1; cyc <= ncyc; ++cyc) {
            vcycle(P, p, f, lambda, o);
            double rn = residual_norm(P, p, f, &lambda, rbuf);
            rel = rn / ref;
            if (hist && cyc - 1 < hist_len) hist[cyc - 1] = rel;
            if (!isfinite(rn)) { status = ORC_E_NUMERIC; break; }
            if (rn > 1e3 * fmax(r0, ref)) { status = ORC_E_NUMERIC; break; }
            if (o->fixed_cycles <= 0 && rel <= o->rel_tol) break;
        }
        if (cyc > ncyc) cyc = ncyc;
        if (status == ORC_OK && o->fixed_cycles <= 0 && rel > o->rel_tol) status = ORC_NOT_CONVERGED;
    }
    /* gauge: zero V-weighted mean over the fluid cells (ghosts shift with it) */
    double sp = 0.0;
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] == T_FLUID) sp += lvol(L0, i, j, k) * p[id];
            }
    double pm = sp / P->vol_fluid;
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] != T_DEAD) p[id] -= pm;
    st->cycles = cyc;
    st->status = status;
    st->rel_residual = rel;
    st->lambda = lambda;
    st->ref_norm = ref;
    st->ghost_residual_max = ghost_residual_max(P, p);
    st->restarts = restarts;
    free(rbuf);
    return status;
}

/* ------------------------------------------------------------------------------------ */
/* projection (Section 2.1, fractional step)                                            */
/* ------------------------------------------------------------------------------------ */

/* f = (D u*) / dt on fluid cells, 0 elsewhere.  u[nz][ny][nx+1], v[nz][ny+1][nx], w[nz+1][ny][nx] */
void orc_rhs(const orc_problem *P, const double *u, const double *v, const double *w, double dt, double *f) {
    const int nx = P->nx, ny = P->ny, nz = P->nz;
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t id = IDX(P, i, j, k);
                if (P->type[id] != T_FLUID) { f[id] = 0.0; continue; }
                int64_t iu = ((int64_t)k * ny + j) * (nx + 1) + i;
                int64_t iv = ((int64_t)k * (ny + 1) + j) * nx + i;
                int64_t iw = ((int64_t)k * ny + j) * nx + i;
                double div = (u[iu + 1] - u[iu]) / P->wx[i];
                div = div + (v[iv + nx] - v[iv]) / P->wy[j];
                div = div + (w[iw + (int64_t)nx * ny] - w[iw]) / P->wz[k];
                f[id] = div / dt;
            }
}

/* max |D u| over the fluid cells */
double orc_div_max(const orc_problem *P, const double *u, const double *v, const double *w) {
    double *f = dalloc(P->ncell);
    orc_rhs(P, u, v, w, 1.0, f);
    double m = 0.0;
    for (int64_t id = 0; id < P->ncell; ++id) if (P->type[id] == T_FLUID) m = fmax(m, fabs(f[id]));
    free(f);
    return m;
}

/* u_f -= dt (p_nb - p_c)/d_f on interior faces with at least one fluid cell */
void orc_correct(const orc_problem *P, double *u, double *v, double *w, const double *p, double dt) {
    const int nx = P->nx, ny = P->ny, nz = P->nz;
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 1; i < nx; ++i) {
                int64_t a = IDX(P, i - 1, j, k), b = IDX(P, i, j, k);
                if (P->type[a] != T_FLUID && P->type[b] != T_FLUID) continue;
                u[((int64_t)k * ny + j) * (nx + 1) + i] -= dt * (p[b] - p[a]) / P->dcx[i];
            }
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 1; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t a = IDX(P, i, j - 1, k), b = IDX(P, i, j, k);
                if (P->type[a] != T_FLUID && P->type[b] != T_FLUID) continue;
                v[((int64_t)k * (ny + 1) + j) * nx + i] -= dt * (p[b] - p[a]) / P->dcy[j];
            }
#pragma omp parallel for
    for (int k = 1; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t a = IDX(P, i, j, k - 1), b = IDX(P, i, j, k);
                if (P->type[a] != T_FLUID && P->type[b] != T_FLUID) continue;
                w[((int64_t)k * ny + j) * nx + i] -= dt * (p[b] - p[a]) / P->dcz[k];
            }
}

/* full projection: f = (D u*) / dt, solve, correct u in place, p out */
int orc_project(orc_problem *P, double *u, double *v, double *w, double dt, double *p, const orc_opts *o,
                orc_stats *st, double *div_max) {
    double *f = dalloc(P->ncell);
    orc_rhs(P, u, v, w, dt, f);
    int s = orc_solve(P, f, p, o, st, NULL, 0);
    free(f);
    if (s < 0) return s;
    orc_correct(P, u, v, w, p, dt);
    if (div_max) *div_max = orc_div_max(P, u, v, w);
    return s;
}

/* ------------------------------------------------------------------------------------ */
/* host memory bandwidth for the CPU baseline's context: STREAM triad a = b + s c over n  */
/* doubles with the OpenMP threads in use; returns the best of `reps` runs in GB/s        */
/* (24 bytes moved per element).                                                        */
/* ------------------------------------------------------------------------------------ */
#include <omp.h>

double orc_stream_triad(int64_t n, int reps) {
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    if (!a || !b || !c) { free(a); free(b); free(c); return -1.0; }
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) { a[i] = 0.0; b[i] = 1.0; c[i] = 2.0; }
    double best = 0.0;
    for (int r = 0; r < reps; ++r) {
        double t0 = omp_get_wtime();
#pragma omp parallel for
        for (int64_t i = 0; i < n; ++i) a[i] = b[i] + 3.0 * c[i];
        double t = omp_get_wtime() - t0;
        double gbs = 24.0 * (double)n / t / 1e9;
        if (gbs > best) best = gbs;
    }
    volatile double sink = a[n / 2];
    (void)sink;
    free(a); free(b); free(c);
    return best;
}

int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { omp_set_num_threads(n); }
