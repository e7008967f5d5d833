// Advection-diffusion half-step of the fractional-step method (Section 2.1): conservative
// central-difference convection (Adams-Bashforth), Crank-Nicolson viscous term solved by
// scheduled relaxed Jacobi, with the no-slip (Dirichlet) ghost rows of Section 2.2.
//
// Cell-centred velocity components live in three arrays of the level-0 layout [nz][ny][nx].
// The two cell passes (right-hand side, relaxed Jacobi sweep) are z-marches over 64 x 4
// column tiles: a thread owns a column, keeps the centre values of the planes below and
// above in registers, and issues every load of the next plane before computing the current
// one; x and y neighbours come from the lanes' common cache lines.
#include "device_util.hpp"
#include "ibm_impl.hpp"
#include "zmarch.hpp"

namespace ibm {

namespace {

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

// Dirichlet ghost rows, one pass: u_g = (2 - betaD_g) u_BI - sum_{m != g} betaD_m u_m with
// fluid members read from dst (already updated) and ghost members from src (the values
// before the pass).  Lane m of a group of eight takes member m; three shuffle steps sum the
// group.  A degenerate ghost takes 2 u_BI minus the mean of its fluid 26-neighbours.
__global__ void __launch_bounds__(DREF_NT)
    k_dirichlet_refresh(GhostView G, const double *__restrict__ betaDg, const double *__restrict__ ubi, CV3 src,
                        V3 dst, int nx, int ny, int nz, const uint8_t *__restrict__ type, double *scr) {
    const int64_t g = ((int64_t)blockIdx.x * DREF_NT + threadIdx.x) >> 3;
    const int m = threadIdx.x & 7;
    const bool live = g < G.ng;
    const int64_t gc = live ? g : 0;
    const int32_t q = G.st[8 * gc + m];
    const double b = G.beta[8 * gc + m];  // the Dirichlet weights (ghosts() below)
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
        for (int c = 0; c < 3; ++c) t[c] = 2.0 * ub[c] - (n ? sm[c] / n : 0.0);
    } else {
        const double w = 2.0 - betaDg[gc];
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c] = w * ub[c] - t[c];
    }
    if (scr) {  // values held back, scattered by k_ghost_scatter (an in-place pass)
#pragma unroll
        for (int c = 0; c < 3; ++c) scr[3 * gc + c] = t[c];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) dst.c[c][cell] = t[c];
    }
}

__global__ void k_ghost_scatter(int64_t ng, const int32_t *__restrict__ gcell, const double *__restrict__ scr, V3 dst) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int64_t cell = gcell[g];
#pragma unroll
    for (int c = 0; c < 3; ++c) dst.c[c][cell] = scr[3 * g + c];
}

// one plane of a column for the right-hand side pass: the four lateral neighbours and the
// centre of the plane above, per component, the previous convective term and the type
struct RhsPlane {
    double xm[3], xp[3], ym[3], yp[3], up[3], hold[3];
    double azm, azp, zpl, zph, zml, zmh, wz;
    uint8_t ty;
};

// Right-hand side of the Crank-Nicolson system on fluid rows and the convective term:
//   H = -(1/V) sum_faces (+/-) A_f Un_f (u_i)_f      (face values: linear interpolation)
//   b = u + dt (3/2 H - 1/2 H_old) + a L u,   a = nu dt / 2   (first step: H_old = H)
// H overwrites H_old in place (each thread reads and writes only its own cells).  Non-fluid
// cells get H = b = 0.  partials[block] = sum of b^2 over the block's fluid cells.
__global__ void __launch_bounds__(ZM_NT)
    k_mom_rhs(MomView M, CV3 U, V3 H, V3 B, double dt, double a, int first, ZTiles t, double *partials) {
    __shared__ double sh[ZM_NT / 64];
    const ZPos z = zpos(t, M.nz);
    if (!z.live) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int nx = M.nx, ny = M.ny, nz = M.nz;
    const bool in = z.i < nx && z.j < ny;
    const int i = min(z.i, nx - 1), j = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, row = (int64_t)j * nx + i;
    const bool hx0 = i > 0, hx1 = i < nx - 1, hy0 = j > 0, hy1 = j < ny - 1;
    const int64_t dxm = hx0 ? -1 : 0, dxp = hx1 ? 1 : 0, dym = hy0 ? -(int64_t)nx : 0, dyp = hy1 ? (int64_t)nx : 0;
    // interpolation weights (low cell, high cell) of the four lateral faces
    double xpl = 0, xph = 0, xml = 0, xmh = 0, ypl = 0, yph = 0, yml = 0, ymh = 0;
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
    const double wx = M.wx[i], wy = M.wy[j];
    const double cxm = M.axm[i], cxp = M.axp[i], cym = M.aym[j], cyp = M.ayp[j];
    auto ld = [&](int k) -> RhsPlane {
        RhsPlane d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + row;
        const int64_t up = (kk < nz - 1) ? base + plane : base;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            d.xm[q] = U.c[q][base + dxm];
            d.xp[q] = U.c[q][base + dxp];
            d.ym[q] = U.c[q][base + dym];
            d.yp[q] = U.c[q][base + dyp];
            d.up[q] = U.c[q][up];
            d.hold[q] = H.c[q][base];
        }
        d.ty = M.type[base];
        d.azm = M.azm[kk];
        d.azp = M.azp[kk];
        d.wz = M.wz[kk];
        d.zpl = d.zph = d.zml = d.zmh = 0.0;
        if (kk < nz - 1) {
            const double h = M.zc[kk + 1] - M.zc[kk];
            d.zpl = (M.zc[kk + 1] - M.zf[kk + 1]) / h;
            d.zph = (M.zf[kk + 1] - M.zc[kk]) / h;
        }
        if (kk > 0) {
            const double h = M.zc[kk] - M.zc[kk - 1];
            d.zml = (M.zc[kk] - M.zf[kk]) / h;
            d.zmh = (M.zf[kk] - M.zc[kk - 1]) / h;
        }
        return d;
    };
    double cm[3], cc[3];  // centres of the planes k - 1 and k
    {
        const int64_t b0 = (int64_t)z.k0 * plane + row;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            cc[q] = U.c[q][b0];
            cm[q] = z.k0 > 0 ? U.c[q][b0 - plane] : 0.0;
        }
    }
    double acc = 0.0;
    auto compute = [&](const RhsPlane &D, int k) {
        const int64_t id = (int64_t)k * plane + row;
        if (in && k < z.k1) {
            if (D.ty != T_FLUID) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    H.c[q][id] = 0.0;
                    B.c[q][id] = 0.0;
                }
            } else {
                const bool hz0 = k > 0, hz1 = k < nz - 1;
                const double ax = D.wz * wy, ay = D.wz * wx, az = wy * wx;
                const double vol = (D.wz * wy) * wx;
                const double uxp = hx1 ? xpl * cc[0] + xph * D.xp[0] : 0.0;
                const double uxm = hx0 ? xml * D.xm[0] + xmh * cc[0] : 0.0;
                const double vyp = hy1 ? ypl * cc[1] + yph * D.yp[1] : 0.0;
                const double vym = hy0 ? yml * D.ym[1] + ymh * cc[1] : 0.0;
                const double wzp = hz1 ? D.zpl * cc[2] + D.zph * D.up[2] : 0.0;
                const double wzm = hz0 ? D.zml * cm[2] + D.zmh * cc[2] : 0.0;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double fc = cc[q];
                    const double fxp = D.xp[q], fxm = D.xm[q], fyp = D.yp[q], fym = D.ym[q];
                    const double fzp = D.up[q], fzm = cm[q];
                    double h = 0.0;
                    if (hx1) h -= (uxp * (xpl * fc + xph * fxp)) * ax;
                    if (hx0) h += (uxm * (xml * fxm + xmh * fc)) * ax;
                    if (hy1) h -= (vyp * (ypl * fc + yph * fyp)) * ay;
                    if (hy0) h += (vym * (yml * fym + ymh * fc)) * ay;
                    if (hz1) h -= (wzp * (D.zpl * fc + D.zph * fzp)) * az;
                    if (hz0) h += (wzm * (D.zml * fzm + D.zmh * fc)) * az;
                    h /= vol;
                    double lap = 0.0;
                    if (hx1) lap += cxp * (fxp - fc);
                    if (hx0) lap -= cxm * (fc - fxm);
                    if (hy1) lap += cyp * (fyp - fc);
                    if (hy0) lap -= cym * (fc - fym);
                    if (hz1) lap += D.azp * (fzp - fc);
                    if (hz0) lap -= D.azm * (fc - fzm);
                    const double hp = first ? h : D.hold[q];
                    const double b = fc + dt * (1.5 * h - 0.5 * hp) + a * lap;
                    __builtin_nontemporal_store(h, H.c[q] + id);  // streaming, as in the sweep
                    __builtin_nontemporal_store(b, B.c[q] + id);
                    acc += b * b;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            cm[q] = cc[q];
            cc[q] = D.up[q];
        }
    };
    RhsPlane qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        compute(qa, k);
        qa = ld(k + 2);
        compute(qb, k + 1);
    }
    const double tot = block_sum<ZM_NT>(acc, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

struct SrjPlane {
    double xm[3], xp[3], ym[3], yp[3], up[3], b[3];
    double azm, azp;
    uint8_t ty;
};

// One relaxed Jacobi sweep of the fluid rows of (I - a L) u = b:
//   y = (1 - omega) x + omega (b + a sum_f a_f x_nb) / (1 + a sum_f a_f)
// ghost cells are copied (their rows follow in their own pass), dead cells cleared.
// partials[block] = sum of the squared fluid-row residuals b - (I - a L) x at the input.
__global__ void __launch_bounds__(ZM_NT)
    k_srj_sweep(MomView M, CV3 X, V3 Y, CV3 B, double a, double omega, ZTiles t, double *partials) {
    __shared__ double sh[ZM_NT / 64];
    const ZPos z = zpos(t, M.nz);
    if (!z.live) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int nx = M.nx, ny = M.ny, nz = M.nz;
    const bool in = z.i < nx && z.j < ny;
    const int i = min(z.i, nx - 1), j = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, row = (int64_t)j * nx + i;
    const bool hx0 = i > 0, hx1 = i < nx - 1, hy0 = j > 0, hy1 = j < ny - 1;
    const int64_t dxm = hx0 ? -1 : 0, dxp = hx1 ? 1 : 0, dym = hy0 ? -(int64_t)nx : 0, dyp = hy1 ? (int64_t)nx : 0;
    const double cxp = hx1 ? M.axp[i] : 0.0, cxm = hx0 ? M.axm[i] : 0.0;
    const double cyp = hy1 ? M.ayp[j] : 0.0, cym = hy0 ? M.aym[j] : 0.0;
    auto ld = [&](int k) -> SrjPlane {
        SrjPlane d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + row;
        const int64_t up = (kk < nz - 1) ? base + plane : base;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            d.xm[q] = X.c[q][base + dxm];
            d.xp[q] = X.c[q][base + dxp];
            d.ym[q] = X.c[q][base + dym];
            d.yp[q] = X.c[q][base + dyp];
            d.up[q] = X.c[q][up];
            d.b[q] = B.c[q][base];
        }
        d.ty = M.type[base];
        d.azm = M.azm[kk];
        d.azp = M.azp[kk];
        return d;
    };
    double cm[3], cc[3];
    {
        const int64_t b0 = (int64_t)z.k0 * plane + row;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            cc[q] = X.c[q][b0];
            cm[q] = z.k0 > 0 ? X.c[q][b0 - plane] : 0.0;
        }
    }
    double acc = 0.0;
    auto compute = [&](const SrjPlane &D, int k) {
        const int64_t id = (int64_t)k * plane + row;
        if (in && k < z.k1) {
            if (D.ty != T_FLUID) {
                const bool dead = D.ty == T_DEAD;
#pragma unroll
                for (int q = 0; q < 3; ++q) Y.c[q][id] = dead ? 0.0 : cc[q];
            } else {
                const bool hz0 = k > 0, hz1 = k < nz - 1;
                const double czp = hz1 ? D.azp : 0.0, czm = hz0 ? D.azm : 0.0;
                const double d = ((czm + czp) + (cym + cyp)) + (cxm + cxp);
                const double den = 1.0 + a * d;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    double s = 0.0;
                    if (hx1) s += cxp * D.xp[q];
                    if (hx0) s += cxm * D.xm[q];
                    if (hy1) s += cyp * D.yp[q];
                    if (hy0) s += cym * D.ym[q];
                    if (hz1) s += czp * D.up[q];
                    if (hz0) s += czm * cm[q];
                    const double xc = cc[q];
                    const double num = D.b[q] + a * s;
                    const double r = num - den * xc;
                    // full-field result, not re-read by this pass: non-temporal (measured faster)
                    __builtin_nontemporal_store((1.0 - omega) * xc + omega * (num / den), Y.c[q] + id);
                    acc += r * r;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            cm[q] = cc[q];
            cc[q] = D.up[q];
        }
    };
    SrjPlane qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        compute(qa, k);
        qa = ld(k + 2);
        compute(qb, k + 1);
    }
    const double tot = block_sum<ZM_NT>(acc, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
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

// the ghost list with the Dirichlet weights in place of the Neumann ones
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

hipError_t refresh(ibm_grid *g, CV3 src, V3 dst, hipStream_t s, double *scr = nullptr) {
    if (g->ng == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dirichlet_refresh, dim3((unsigned)((8 * g->ng + DREF_NT - 1) / DREF_NT)), dim3(DREF_NT), 0,
                       s, ghosts(g), g->g_betaDg, g->g_ubi, src, dst, g->nx, g->ny, g->nz, g->type, scr);
    if (scr)
        hipLaunchKernelGGL(k_ghost_scatter, dim3((unsigned)((g->ng + 255) / 256)), dim3(256), 0, s, g->ng, g->g_cell,
                           scr, dst);
    return hipGetLastError();
}

// Fresh-cell values (one pass over the fresh list, members read from the field as it is):
//   u_c = (u_BI + sum_{m != c} beta_m u_m) / (2 - beta_c);
// a degenerate fresh cell takes the mean of its fluid, non-fresh 26-neighbours (u_BI if it
// has none).  Results go to scr (three per fresh cell) and are scattered afterwards.
__global__ void k_fresh_fill(int64_t nf, const int32_t *__restrict__ fcell, const int32_t *__restrict__ fst,
                             const double *__restrict__ fbeta, const double *__restrict__ fbetac,
                             const int32_t *__restrict__ fflags, const double *__restrict__ ubi, CV3 U,
                             const uint8_t *__restrict__ type, const uint8_t *__restrict__ prev, int nx, int ny,
                             int nz, double *scr) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nf) return;
    double v[3];
    if (fflags[q] & GF_DEGENERATE) {
        int i, j, k;
        unflatten(fcell[q], nx, ny, i, j, k);
        double sm[3] = {0.0, 0.0, 0.0};
        int n = 0;
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di, jj = j + dj, kk = k + dk;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                    const int64_t x = ((int64_t)kk * ny + jj) * nx + ii;
                    if (type[x] == T_FLUID && prev[x] == T_FLUID) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) sm[c] += U.c[c][x];
                        ++n;
                    }
                }
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = n ? sm[c] / n : ubi[3 * q + c];
    } else {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < 8; ++m) {
            const int32_t x = fst[8 * q + m];
            if (x < 0) continue;
            const double b = fbeta[8 * q + m];
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += b * U.c[c][x];
        }
        const double den = 2.0 - fbetac[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = (ubi[3 * q + c] + acc[c]) / den;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) scr[3 * q + c] = v[c];
}

}  // namespace

hipError_t fresh_enqueue_fill(ibm_grid *g, double *const uvw[3], hipStream_t s) {
    if (g->nfresh <= 0) return hipSuccess;
    const int64_t nf = g->nfresh;
    hipLaunchKernelGGL(k_fresh_fill, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, nf, g->f_cell, g->f_st,
                       g->f_beta, g->f_betac, g->f_flags, g->f_ubi, cv3(uvw[0], uvw[1], uvw[2]), g->type, g->type_prev,
                       g->nx, g->ny, g->nz, g->f_scr);
    hipLaunchKernelGGL(k_ghost_scatter, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, nf, g->f_cell, g->f_scr,
                       v3(uvw[0], uvw[1], uvw[2]));
    return hipGetLastError();
}

// ---- host driver ------------------------------------------------------------------------
// uvw: three device arrays (u, v, w) of N doubles, in: u^n (its ghost rows are applied in
// place, from a snapshot held in a per-ghost scratch), out: u*.  hc: three arrays, in
// H^{n-1} (ignored on the first step), out H^n.  work: the right-hand side b (0..2) and the
// second iterate buffer (3..5).
hipError_t momentum_enqueue_prep(ibm_grid *g, double *const uvw[3], double *const hc[3], double *const work[6],
                                 double dt, double a, int first, hipStream_t s) {
    const CV3 U = cv3(uvw[0], uvw[1], uvw[2]);
    hipError_t e = refresh(g, U, v3(uvw[0], uvw[1], uvw[2]), s, g->g_uscr);
    if (e != hipSuccess) return e;
    const ZTiles t = ztiles(g->nx, g->ny, g->nz);
    hipLaunchKernelGGL(k_mom_rhs, dim3(t.grid), dim3(ZM_NT), 0, s, mom_view(g), U, v3(hc[0], hc[1], hc[2]),
                       v3(work[0], work[1], work[2]), dt, a, first, t, g->partials);
    hipLaunchKernelGGL(k_mom_sum, dim3(1), dim3(256), 0, s, g->partials, t.grid, &g->sc->mom_b2);
    return hipGetLastError();
}

// one sweep from X into Y followed by the ghost rows; the residual sum of the input
// iterate lands in sc->mom_r2 when `sum` is set
hipError_t momentum_enqueue_sweep(ibm_grid *g, double *const X[3], double *const Y[3], double *const work[6],
                                  double a, double omega, bool sum, hipStream_t s) {
    const CV3 x = cv3(X[0], X[1], X[2]);
    const V3 y = v3(Y[0], Y[1], Y[2]);
    const ZTiles t = ztiles(g->nx, g->ny, g->nz);
    hipLaunchKernelGGL(k_srj_sweep, dim3(t.grid), dim3(ZM_NT), 0, s, mom_view(g), x, y, cv3(work[0], work[1], work[2]),
                       a, omega, t, g->partials);
    if (sum) hipLaunchKernelGGL(k_mom_sum, dim3(1), dim3(256), 0, s, g->partials, t.grid, &g->sc->mom_r2);
    return refresh(g, x, y, s);
}

}  // namespace ibm
