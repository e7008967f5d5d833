// Advection-diffusion half-step of the fractional-step method (Section 2.1): conservative
// central-difference convection (Adams-Bashforth), Crank-Nicolson viscous term solved by
// scheduled relaxed Jacobi, with the no-slip (Dirichlet) ghost rows of Section 2.2.
//
// Cell-centred velocity components live in three arrays of the level-0 layout [nz][ny][nx].
// Every kernel here is a single pass over the grid; neighbour values come through the
// caches (the six neighbours of a cell are re-read by its neighbours' threads).
#include "device_util.hpp"
#include "ibm_impl.hpp"

namespace ibm {

namespace {

constexpr int MOM_NT = 256;      // threads per block of the cell passes
constexpr int DREF_NT = 256;     // ghost refresh: eight lanes per ghost

struct CV3 {
    const double *c[3];
};
struct V3 {
    double *c[3];
};

struct MomView {
    int nx, ny, nz;
    const double *xc, *yc, *zc;  // centres
    const double *xf, *yf, *zf;  // faces
    const double *wx, *wy, *wz;  // widths
    const double *axm, *axp, *aym, *ayp, *azm, *azp;  // flux coefficients per unit volume
    const uint8_t *type;
};

MomView mom_view(ibm_grid *g) {
    MomView M;
    M.nx = g->nx;
    M.ny = g->ny;
    M.nz = g->nz;
    M.xc = g->c0[0];
    M.yc = g->c0[1];
    M.zc = g->c0[2];
    M.xf = g->faces[0];
    M.yf = g->faces[1];
    M.zf = g->faces[2];
    M.wx = g->w0[0];
    M.wy = g->w0[1];
    M.wz = g->w0[2];
    M.axm = g->am0[0];
    M.axp = g->ap0[0];
    M.aym = g->am0[1];
    M.ayp = g->ap0[1];
    M.azm = g->am0[2];
    M.azp = g->ap0[2];
    M.type = g->type;
    return M;
}

// dst = src with dead cells cleared (three components)
__global__ void k_mom_prep(int64_t N, const uint8_t *__restrict__ type, CV3 src, V3 dst) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const bool dead = type[id] == T_DEAD;
#pragma unroll
    for (int q = 0; q < 3; ++q) dst.c[q][id] = dead ? 0.0 : src.c[q][id];
}

// Dirichlet ghost rows, one pass: u_g = (2 - betaD_g) u_BI - sum_{m != g} betaD_m u_m with
// fluid members read from dst (already updated) and ghost members from src (the values
// before the pass).  Lane m of a group of eight takes member m; three shuffle steps sum the
// group.  A degenerate ghost takes 2 u_BI minus the mean of its fluid 26-neighbours.
__global__ void __launch_bounds__(DREF_NT)
    k_dirichlet_refresh(GhostView G, const double *__restrict__ betaD, const double *__restrict__ betaDg,
                        const double *__restrict__ ubi, CV3 src, V3 dst, int nx, int ny, int nz,
                        const uint8_t *__restrict__ type) {
    const int64_t g = ((int64_t)blockIdx.x * DREF_NT + threadIdx.x) >> 3;
    const int m = threadIdx.x & 7;
    const bool live = g < G.ng;
    const int64_t gc = live ? g : 0;
    const int32_t q = G.st[8 * gc + m];
    const double b = betaD[8 * gc + m];
    const unsigned gm = G.gmask[gc];
    double t[3] = {0.0, 0.0, 0.0};
    if (live && q >= 0) {
        const bool from_src = ((gm >> m) & 1u) != 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c] = b * (from_src ? src.c[c][q] : dst.c[c][q]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        t[c] += __shfl_xor(t[c], 1, 64);
        t[c] += __shfl_xor(t[c], 2, 64);
        t[c] += __shfl_xor(t[c], 4, 64);
    }
    if (!live || m != 0) return;
    const int64_t cell = G.cell[gc];
    const double ub[3] = {ubi[3 * gc], ubi[3 * gc + 1], ubi[3 * gc + 2]};
    if (G.flags[gc] & GF_DEGENERATE) {
        int i, j, k;
        unflatten(cell, nx, ny, i, j, k);
        double sm[3] = {0.0, 0.0, 0.0};
        int n = 0;
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di, jj = j + dj, kk = k + dk;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                    const int64_t qq = ((int64_t)kk * ny + jj) * nx + ii;
                    if (type[qq] == T_FLUID) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) sm[c] += dst.c[c][qq];
                        ++n;
                    }
                }
#pragma unroll
        for (int c = 0; c < 3; ++c) dst.c[c][cell] = 2.0 * ub[c] - (n ? sm[c] / n : 0.0);
    } else {
        const double w = 2.0 - betaDg[gc];
#pragma unroll
        for (int c = 0; c < 3; ++c) dst.c[c][cell] = w * ub[c] - t[c];
    }
}

// Right-hand side of the Crank-Nicolson system on fluid rows and the convective term:
//   H = -(1/V) sum_faces (+/-) A_f Un_f (u_i)_f      (face values: linear interpolation)
//   b = u + dt (3/2 H - 1/2 H_old) + a L u,   a = nu dt / 2   (first step: H_old = H)
// H overwrites H_old in place (each thread reads and writes only its own cell).  Non-fluid
// cells get H = b = 0.  partials[block] = sum of b^2 over the block's fluid cells.
__global__ void __launch_bounds__(MOM_NT)
    k_mom_rhs(MomView M, CV3 U, V3 H, V3 B, double dt, double a, int first, double *partials) {
    __shared__ double sh[MOM_NT / 64];
    const int nx = M.nx, ny = M.ny, nz = M.nz;
    const int64_t N = (int64_t)nx * ny * nz, sy = nx, sz = (int64_t)nx * ny;
    double acc = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * MOM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * MOM_NT) {
        if (M.type[id] != T_FLUID) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                H.c[q][id] = 0.0;
                B.c[q][id] = 0.0;
            }
            continue;
        }
        int i, j, k;
        unflatten(id, nx, ny, i, j, k);
        const bool hx0 = i > 0, hx1 = i < nx - 1, hy0 = j > 0, hy1 = j < ny - 1, hz0 = k > 0, hz1 = k < nz - 1;
        // interpolation weights (low cell, high cell) of the six faces
        double xpl = 0, xph = 0, xml = 0, xmh = 0, ypl = 0, yph = 0, yml = 0, ymh = 0, zpl = 0, zph = 0, zml = 0,
               zmh = 0;
        if (hx1) {
            const double h = M.xc[i + 1] - M.xc[i];
            xpl = (M.xc[i + 1] - M.xf[i + 1]) / h;
            xph = (M.xf[i + 1] - M.xc[i]) / h;
        }
        if (hx0) {
            const double h = M.xc[i] - M.xc[i - 1];
            xml = (M.xc[i] - M.xf[i]) / h;
            xmh = (M.xf[i] - M.xc[i - 1]) / h;
        }
        if (hy1) {
            const double h = M.yc[j + 1] - M.yc[j];
            ypl = (M.yc[j + 1] - M.yf[j + 1]) / h;
            yph = (M.yf[j + 1] - M.yc[j]) / h;
        }
        if (hy0) {
            const double h = M.yc[j] - M.yc[j - 1];
            yml = (M.yc[j] - M.yf[j]) / h;
            ymh = (M.yf[j] - M.yc[j - 1]) / h;
        }
        if (hz1) {
            const double h = M.zc[k + 1] - M.zc[k];
            zpl = (M.zc[k + 1] - M.zf[k + 1]) / h;
            zph = (M.zf[k + 1] - M.zc[k]) / h;
        }
        if (hz0) {
            const double h = M.zc[k] - M.zc[k - 1];
            zml = (M.zc[k] - M.zf[k]) / h;
            zmh = (M.zf[k] - M.zc[k - 1]) / h;
        }
        const double ax = M.wz[k] * M.wy[j], ay = M.wz[k] * M.wx[i], az = M.wy[j] * M.wx[i];
        const double vol = (M.wz[k] * M.wy[j]) * M.wx[i];
        // normal velocities at the faces
        const double *u = U.c[0], *v = U.c[1], *w = U.c[2];
        const double uxp = hx1 ? xpl * u[id] + xph * u[id + 1] : 0.0;
        const double uxm = hx0 ? xml * u[id - 1] + xmh * u[id] : 0.0;
        const double vyp = hy1 ? ypl * v[id] + yph * v[id + sy] : 0.0;
        const double vym = hy0 ? yml * v[id - sy] + ymh * v[id] : 0.0;
        const double wzp = hz1 ? zpl * w[id] + zph * w[id + sz] : 0.0;
        const double wzm = hz0 ? zml * w[id - sz] + zmh * w[id] : 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double *f = U.c[q];
            const double fc = f[id];
            const double fxp = hx1 ? f[id + 1] : 0.0, fxm = hx0 ? f[id - 1] : 0.0;
            const double fyp = hy1 ? f[id + sy] : 0.0, fym = hy0 ? f[id - sy] : 0.0;
            const double fzp = hz1 ? f[id + sz] : 0.0, fzm = hz0 ? f[id - sz] : 0.0;
            double h = 0.0;
            if (hx1) h -= (uxp * (xpl * fc + xph * fxp)) * ax;
            if (hx0) h += (uxm * (xml * fxm + xmh * fc)) * ax;
            if (hy1) h -= (vyp * (ypl * fc + yph * fyp)) * ay;
            if (hy0) h += (vym * (yml * fym + ymh * fc)) * ay;
            if (hz1) h -= (wzp * (zpl * fc + zph * fzp)) * az;
            if (hz0) h += (wzm * (zml * fzm + zmh * fc)) * az;
            h /= vol;
            double lap = 0.0;
            if (hx1) lap += M.axp[i] * (fxp - fc);
            if (hx0) lap -= M.axm[i] * (fc - fxm);
            if (hy1) lap += M.ayp[j] * (fyp - fc);
            if (hy0) lap -= M.aym[j] * (fc - fym);
            if (hz1) lap += M.azp[k] * (fzp - fc);
            if (hz0) lap -= M.azm[k] * (fc - fzm);
            const double hp = first ? h : H.c[q][id];
            const double b = fc + dt * (1.5 * h - 0.5 * hp) + a * lap;
            H.c[q][id] = h;
            B.c[q][id] = b;
            acc += b * b;
        }
    }
    const double t = block_sum<MOM_NT>(acc, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// One relaxed Jacobi sweep of the fluid rows of (I - a L) u = b:
//   y = (1 - omega) x + omega (b + a sum_f a_f x_nb) / (1 + a sum_f a_f)
// other cells are copied (ghost rows follow in their own pass).  partials[block] = sum of
// the squared fluid-row residuals b - (I - a L) x at the input iterate.
__global__ void __launch_bounds__(MOM_NT)
    k_srj_sweep(MomView M, CV3 X, V3 Y, CV3 B, double a, double omega, double *partials) {
    __shared__ double sh[MOM_NT / 64];
    const int nx = M.nx, ny = M.ny, nz = M.nz;
    const int64_t N = (int64_t)nx * ny * nz, sy = nx, sz = (int64_t)nx * ny;
    double acc = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * MOM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * MOM_NT) {
        if (M.type[id] != T_FLUID) {
#pragma unroll
            for (int q = 0; q < 3; ++q) Y.c[q][id] = X.c[q][id];
            continue;
        }
        int i, j, k;
        unflatten(id, nx, ny, i, j, k);
        const bool hx0 = i > 0, hx1 = i < nx - 1, hy0 = j > 0, hy1 = j < ny - 1, hz0 = k > 0, hz1 = k < nz - 1;
        const double cxp = hx1 ? M.axp[i] : 0.0, cxm = hx0 ? M.axm[i] : 0.0;
        const double cyp = hy1 ? M.ayp[j] : 0.0, cym = hy0 ? M.aym[j] : 0.0;
        const double czp = hz1 ? M.azp[k] : 0.0, czm = hz0 ? M.azm[k] : 0.0;
        const double d = ((czm + czp) + (cym + cyp)) + (cxm + cxp);
        const double den = 1.0 + a * d;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double *x = X.c[q];
            double s = 0.0;
            if (hx1) s += cxp * x[id + 1];
            if (hx0) s += cxm * x[id - 1];
            if (hy1) s += cyp * x[id + sy];
            if (hy0) s += cym * x[id - sy];
            if (hz1) s += czp * x[id + sz];
            if (hz0) s += czm * x[id - sz];
            const double xc = x[id];
            const double num = B.c[q][id] + a * s;
            const double r = num - den * xc;
            Y.c[q][id] = (1.0 - omega) * xc + omega * (num / den);
            acc += r * r;
        }
    }
    const double t = block_sum<MOM_NT>(acc, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void k_mom_sum(const double *partials, int n, double *out) {
    __shared__ double sh[4];
    double a = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) a += partials[q];
    a = block_sum<256>(a, sh, threadIdx.x);
    if (threadIdx.x == 0) *out = a;
}

CV3 cv3(const double *a, const double *b, const double *c) {
    CV3 v;
    v.c[0] = a;
    v.c[1] = b;
    v.c[2] = c;
    return v;
}
V3 v3(double *a, double *b, double *c) {
    V3 v;
    v.c[0] = a;
    v.c[1] = b;
    v.c[2] = c;
    return v;
}

GhostView ghosts(ibm_grid *g) {
    GhostView G;
    G.ng = g->ng;
    G.cell = g->g_cell;
    G.st = g->g_st;
    G.gmask = g->g_mask;
    G.beta = g->g_betaD;
    G.h = nullptr;
    G.flags = g->g_flags;
    return G;
}

hipError_t refresh(ibm_grid *g, CV3 src, V3 dst, hipStream_t s) {
    if (g->ng == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dirichlet_refresh, dim3((unsigned)((8 * g->ng + DREF_NT - 1) / DREF_NT)), dim3(DREF_NT), 0,
                       s, ghosts(g), g->g_betaD, g->g_betaDg, g->g_ubi, src, dst, g->nx, g->ny, g->nz, g->type);
    return hipGetLastError();
}

}  // namespace

// ---- host driver ------------------------------------------------------------------------
// uvw: three device arrays (u, v, w) of N doubles, in: u^n, out: u*.  hc: three arrays, in
// H^{n-1} (ignored on the first step), out H^n.  work: six N-arrays of workspace.
// omega: the schedule (m factors), one cycle = m sweeps.  Reads one pinned scalar per cycle.
hipError_t momentum_enqueue_prep(ibm_grid *g, double *const uvw[3], double *const hc[3], double *const work[6],
                                 double dt, double a, int first, hipStream_t s) {
    const int64_t N = g->N;
    const CV3 U = cv3(uvw[0], uvw[1], uvw[2]);
    const V3 W = v3(work[3], work[4], work[5]);
    hipLaunchKernelGGL(k_mom_prep, dim3((unsigned)((N + MOM_NT - 1) / MOM_NT)), dim3(MOM_NT), 0, s, N, g->type, U, W);
    hipError_t e = refresh(g, U, W, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mom_rhs, dim3(RED_BLOCKS), dim3(MOM_NT), 0, s, mom_view(g), cv3(work[3], work[4], work[5]),
                       v3(hc[0], hc[1], hc[2]), v3(work[0], work[1], work[2]), dt, a, first, g->partials);
    hipLaunchKernelGGL(k_mom_sum, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, &g->sc->mom_b2);
    return hipGetLastError();
}

// one sweep from X into Y followed by the ghost rows; the residual sum of the input
// iterate lands in sc->mom_r2 when `sum` is set
hipError_t momentum_enqueue_sweep(ibm_grid *g, double *const X[3], double *const Y[3], double *const work[6],
                                  double a, double omega, bool sum, hipStream_t s) {
    const CV3 x = cv3(X[0], X[1], X[2]);
    const V3 y = v3(Y[0], Y[1], Y[2]);
    hipLaunchKernelGGL(k_srj_sweep, dim3(RED_BLOCKS), dim3(MOM_NT), 0, s, mom_view(g), x, y,
                       cv3(work[0], work[1], work[2]), a, omega, g->partials);
    if (sum) hipLaunchKernelGGL(k_mom_sum, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, &g->sc->mom_r2);
    return refresh(g, x, y, s);
}

}  // namespace ibm
