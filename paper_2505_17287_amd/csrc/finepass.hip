// Fine-level (level 0) stencil passes of the multigrid cycle and of the Krylov operator,
// written as z-marches (paper Section 2.1: the pressure equation on a non-uniform Cartesian
// grid, solved with multigrid):
//   - residual + restriction to level 1 with block partials of the restricted sum,
//   - trilinear prolongation of the level-1 correction (injection where a contributor is
//     inactive),
//   - the operator S y on fluid rows with block partials of sum V (S y).
//
// A workgroup owns a tile of 64 x 4 columns and a chunk of z-planes; each thread owns one
// column and marches upward.  Per-column metrics and prolongation tables are loaded once;
// per-plane ones are uniform across the workgroup (scalar loads); the centre values of the
// planes below and above stay in registers.  Every load of a plane is independent of the
// others, so a plane costs one memory round trip, and there is no data-dependent branch
// before the loads.  Chunks start at even planes, so a halved z pair never straddles two
// workgroups.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.hpp"
#include "ibm_impl.hpp"
#include "zmarch.hpp"

namespace ibm {

namespace {

// sum of a_f y_nb over the six faces and the diagonal, in the order of the two-pass
// definition (wall terms contribute nothing)
template <typename T>
__device__ __forceinline__ void zm_stencil(T axm, T axp, T aym, T ayp, T azm, T azp, bool hx0, bool hx1, bool hy0,
                                           bool hy1, bool hz0, bool hz1, T xm, T xp, T ym, T yp, T zm, T zp, T &num,
                                           T &diag) {
    T s = 0;
    s = s + (hx0 ? axm * xm : T(0));
    s = s + (hx1 ? axp * xp : T(0));
    s = s + (hy0 ? aym * ym : T(0));
    s = s + (hy1 ? ayp * yp : T(0));
    s = s + (hz0 ? azm * zm : T(0));
    s = s + (hz1 ? azp * zp : T(0));
    T d = axm + axp;
    d = d + aym;
    d = d + ayp;
    d = d + azm;
    d = d + azp;
    num = s;
    diag = d;
}

// a full-field result nobody re-reads in this pass: non-temporal in FP64 (in FP32 the plain
// store measured faster)
template <typename T>
__device__ __forceinline__ void store_stream(T *p, T v) {
    if constexpr (sizeof(T) == 8) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int NT>
__device__ __forceinline__ void zm_block_sum_store(double v, double *partials) {
    __shared__ double sh[NT / 64];
    const double s = block_sum<NT>(v, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// NS sums per workgroup, stored at partials[NS * block + q]
template <int NT, int NS>
__device__ __forceinline__ void zm_block_sums_store(const double (&v)[NS], double *partials) {
    __shared__ double sh[NT / 64];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const double s = block_sum<NT>(v[q], sh, threadIdx.x);
        if (threadIdx.x == 0) partials[NS * blockIdx.x + q] = s;
    }
}

// Sums of the Krylov operator passes.  DOTS 0: w = S y, sum V w.  DOTS 1 and 2: w = S y - mu
// (the image with its volume-weighted fluid mean, known beforehand, removed), sum o w and
// sum w w (o is the vector the image is dotted with: the shadow residual or s; w w gives
// omega, and the near-breakdown test of alpha).  DOTS 3: the residual w = o - S y (o the
// right-hand side), sum V w.
template <int DOTS>
struct ApplySums {
    static constexpr int NS = (DOTS == 1 || DOTS == 2) ? 2 : 1;
};

// ---- residual + restriction --------------------------------------------------------------
// R_1(C) = sum over fluid children c of V_c r_c with r = (f - lambda) - S p; e_1 = 0;
// partials[block] = sum of the R_1 written by the block.  The loads of plane k+1 are issued
// before plane k is computed (two plane slots, alternating by name).
template <typename T>
struct RPlane {
    T pp, xm, xp, ym, yp, fv;  // p(k+1) at the column, in-plane neighbours of plane k, f(k)
    T azm, azp, wz;            // z metrics of plane k (prefetched with the plane)
    uint8_t ty;
};

template <typename T>
__global__ void __launch_bounds__(ZM_NT)
    k_restrict0_zm(Fine<T> F, const T *__restrict__ p, const T *__restrict__ f, const T *__restrict__ lamp,
                   Coarse<T> C, int hx, int hy, int hz, ZTiles t, double *partials) {
    __shared__ T srow[ZM_TY][ZM_TX];
    const ZPos z = zpos(t, F.nz);
    if (!z.live) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i < nx && z.j < ny;
    const int ic = min(z.i, nx - 1), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    const bool hx0 = ic > 0, hx1 = ic < nx - 1, hy0 = jc > 0, hy1 = jc < ny - 1;
    const int64_t dxm = hx0 ? -1 : 0, dxp = hx1 ? 1 : 0, dym = hy0 ? -(int64_t)nx : 0, dyp = hy1 ? (int64_t)nx : 0;
    const T axm = F.axm[ic], axp = F.axp[ic], aym = F.aym[jc], ayp = F.ayp[jc];
    const T vxy = F.wx[ic] * F.wy[jc];
    const T lam = *lamp;
    const bool writer = in && (!hx || (z.lane & 1) == 0) && (!hy || (z.wave & 1) == 0);
    const int I = hx ? ic >> 1 : ic, J = hy ? jc >> 1 : jc;
    auto ld = [=](int k) -> RPlane<T> {
        RPlane<T> d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + rowoff;
        d.pp = p[base + (kk < nz - 1 ? plane : 0)];
        d.xm = p[base + dxm];
        d.xp = p[base + dxp];
        d.ym = p[base + dym];
        d.yp = p[base + dyp];
        d.fv = f[base];
        d.ty = F.type[base];
        d.azm = F.azm[kk];
        d.azp = F.azp[kk];
        d.wz = F.wz[kk];
        return d;
    };
    T pm = (z.k0 > 0) ? p[(int64_t)(z.k0 - 1) * plane + rowoff] : T(0);
    T pc = p[(int64_t)z.k0 * plane + rowoff];
    T acc = 0;
    double psum = 0.0;
    // one plane: k >= k1 (the odd tail of the last chunk) computes from clamped data and
    // writes nothing; the barriers stay uniform across the workgroup
#define IBM_RESTRICT_PLANE(D, kk)                                                                                 \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        T num, diag;                                                                                               \
        zm_stencil<T>(axm, axp, aym, ayp, (D).azm, (D).azp, hx0, hx1, hy0, hy1, k_ > 0, k_ < nz - 1, (D).xm,        \
                      (D).xp, (D).ym, (D).yp, pm, (D).pp, num, diag);                                              \
        const T r = ((D).fv - lam) - (num - diag * pc);                                                           \
        T v = (in && k_ < z.k1 && (D).ty == T_FLUID) ? (vxy * (D).wz) * r : T(0);                                 \
        if (hx) v = v + __shfl_xor(v, 1, 64);                                                                      \
        if (hy) {                                                                                                  \
            srow[z.wave][z.lane] = v;                                                                              \
            __syncthreads();                                                                                       \
            v = v + srow[z.wave ^ 1][z.lane];                                                                      \
            __syncthreads();                                                                                       \
        }                                                                                                          \
        acc = (hz && (k_ & 1)) ? acc + v : v;                                                                      \
        if ((!hz || (k_ & 1)) && writer && k_ < z.k1) {                                                            \
            const int K_ = hz ? k_ >> 1 : k_;                                                                      \
            const int64_t cid = ((int64_t)K_ * C.n[1] + J) * C.n[0] + I;                                           \
            C.R[cid] = acc;                                                                                        \
            C.e[cid] = T(0);                                                                                       \
            psum += (double)acc;                                                                                   \
        }                                                                                                          \
        pm = pc;                                                                                                   \
        pc = (D).pp;                                                                                               \
    }
    RPlane<T> qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        IBM_RESTRICT_PLANE(qa, k);
        qa = ld(k + 2);
        IBM_RESTRICT_PLANE(qb, k + 1);
    }
#undef IBM_RESTRICT_PLANE
    zm_block_sum_store<ZM_NT>(psum, partials);
}

// Residual and restriction for any child map (cells merged on some axes only where they are
// narrow).  A tile is RM_CX coarse columns x RM_W coarse rows x a chunk of coarse planes;
// each wave owns one coarse row J (one or two fine rows), and lane l the fine column
// cs_x[I0] + l (the children of RM_CX coarse columns span at most 64 columns).  The lane
// marches up the fine planes with both fine rows in registers (the planes below and above
// in registers, in-plane neighbours through the caches, the plane k+1 loads issued before
// plane k is computed), forms the residual (f - lambda) - S p of each fine cell with the
// arithmetic of k_restrict0_zm, and adds its volume-weighted value on fluid cells to a
// running sum over the rows and fine planes of the current coarse plane.  When the coarse
// plane is complete, lane I - I0 gathers the sums of the one or two lanes holding the
// children of coarse column I (the same sum as the oracle's, in another order).  No data
// crosses waves inside the march.  Workgroups take tiles in a grid-stride loop, in the
// XCD-aware order (a contiguous range of tiles per XCD and round).
constexpr int RM_TILES_PER_CU = 16, RM_KMIN = 1;  // tiles per CU, least coarse planes per tile

template <typename T>
struct RMPlane {
    T pp0, pp1;  // p at plane k+1 above the lane's column, first and second row
    T ylo, yhi;  // p at plane k in the rows below the first and above the last
    T f0, f1;
    T em0, ep0, em1, ep1;  // p at plane k just outside the tile's columns, both rows (uniform)
    T azm, azp, wz;        // z metrics of plane k (uniform)
    uint8_t t0, t1;
};

// One wave's coarse row J of the tile (I0..I1-1, K0..K1-1); TWO: the row has two fine rows.
// Returns the sum of the R_1 values the wave stored (valid in every lane that stored one).
template <typename T, bool TWO>
__device__ __forceinline__ double restrict_map_row(const Fine<T> &F, const T *__restrict__ p,
                                                   const T *__restrict__ f, T lam, const Coarse<T> &C,
                                                   const ChildMap &M, int I0, int I1, int J, int K0, int K1,
                                                   int lane) {
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const int64_t plane = (int64_t)nx * ny;
    const int fx0 = M.cs[0][I0], fx1 = M.cs[0][I1];
    const int i = fx0 + lane;
    const bool inx = i < fx1;
    const int ic = min(i, nx - 1);
    const int ja = M.cs[1][J], jb = TWO ? ja + 1 : ja;
    const int64_t o0 = (int64_t)ja * nx + ic, o1 = (int64_t)jb * nx + ic;
    const int64_t olo = (int64_t)max(ja - 1, 0) * nx + ic, ohi = (int64_t)min(jb + 1, ny - 1) * nx + ic;
    const bool hx0 = ic > 0, hx1 = ic < nx - 1;
    // the x neighbours come from the adjacent lanes (every lane holds its column, or the
    // last column where it lies past the grid, whose value then meets a wall); lanes 0 and
    // 63 take the columns just outside the tile from the edge loads.  The shuffles run in
    // every lane before the edge lanes pick their loaded value: a shuffle evaluated only in
    // some lanes would read the others' registers while they are switched off.
    const int64_t eom = (int64_t)ja * nx + max(fx0 - 1, 0), eop = (int64_t)ja * nx + min(fx0 + 64, nx - 1);
    const T axm = F.axm[ic], axp = F.axp[ic];
    const T aym0 = F.aym[ja], ayp0 = F.ayp[ja], aym1 = F.aym[jb], ayp1 = F.ayp[jb];
    const bool hy00 = ja > 0, hy10 = ja < ny - 1, hy01 = jb > 0, hy11 = jb < ny - 1;
    const T vxy0 = F.wx[ic] * F.wy[ja], vxy1 = F.wx[ic] * F.wy[jb];
    // the owner lane of coarse column I0 + lane: where its children sit among the lanes
    const bool own = lane < I1 - I0;
    const int Io = min(I0 + lane, I1);  // every lane reads inside the map
    const int ca = own ? M.cs[0][Io] - fx0 : 0;
    const bool pair = own && M.cs[0][min(Io + 1, I1)] - M.cs[0][Io] == 2;
    const int cb = min(ca + 1, 63);
    const int k0 = M.cs[2][K0], k1 = M.cs[2][K1];
    auto ld = [=](int k) -> RMPlane<T> {
        RMPlane<T> d;
        const int kk = min(k, nz - 1);
        const int64_t b = (int64_t)kk * plane;
        const int64_t up = (kk < nz - 1) ? plane : 0;
        d.pp0 = p[b + o0 + up];
        d.em0 = p[b + eom];
        d.ep0 = p[b + eop];
        d.ylo = p[b + olo];
        d.yhi = p[b + ohi];
        d.f0 = f[b + o0];
        d.t0 = F.type[b + o0];
        if constexpr (TWO) {
            d.pp1 = p[b + o1 + up];
            d.em1 = p[b + eom + nx];
            d.ep1 = p[b + eop + nx];
            d.f1 = f[b + o1];
            d.t1 = F.type[b + o1];
        } else {
            d.pp1 = d.em1 = d.ep1 = d.f1 = T(0);
            d.t1 = 0;
        }
        d.azm = F.azm[kk];
        d.azp = F.azp[kk];
        d.wz = F.wz[kk];
        return d;
    };
    T pm0 = (k0 > 0) ? p[(int64_t)(k0 - 1) * plane + o0] : T(0);
    T pc0 = p[(int64_t)k0 * plane + o0];
    T pm1 = T(0), pc1 = T(0);
    if constexpr (TWO) {
        pm1 = (k0 > 0) ? p[(int64_t)(k0 - 1) * plane + o1] : T(0);
        pc1 = p[(int64_t)k0 * plane + o1];
    }
    T acc = 0;
    double psum = 0.0;
    int K = K0, kend = M.cs[2][K0 + 1];  // the coarse plane and its end
    // one fine plane; the loop is unrolled by two so the two plane slots change roles by name
#define IBM_RMAP_PLANE(D, kk)                                                                                     \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        T num, diag;                                                                                               \
        const T su0_ = __shfl_up(pc0, 1, 64), sd0_ = __shfl_down(pc0, 1, 64); /* in every lane */               \
        const T xm0_ = (lane == 0) ? (D).em0 : su0_;                                                               \
        const T xp0_ = (lane == 63) ? (D).ep0 : sd0_;                                                              \
        zm_stencil<T>(axm, axp, aym0, ayp0, (D).azm, (D).azp, hx0, hx1, hy00, hy10, k_ > 0, k_ < nz - 1, xm0_,     \
                      xp0_, (D).ylo, TWO ? pc1 : (D).yhi, pm0, (D).pp0, num, diag);                                 \
        const T r0 = ((D).f0 - lam) - (num - diag * pc0);                                                         \
        acc += (inx && (D).t0 == T_FLUID) ? (vxy0 * (D).wz) * r0 : T(0);                                           \
        if constexpr (TWO) {                                                                                       \
            const T su1_ = __shfl_up(pc1, 1, 64), sd1_ = __shfl_down(pc1, 1, 64);                                 \
            const T xm1_ = (lane == 0) ? (D).em1 : su1_;                                                           \
            const T xp1_ = (lane == 63) ? (D).ep1 : sd1_;                                                          \
            zm_stencil<T>(axm, axp, aym1, ayp1, (D).azm, (D).azp, hx0, hx1, hy01, hy11, k_ > 0, k_ < nz - 1,       \
                          xm1_, xp1_, pc0, (D).yhi, pm1, (D).pp1, num, diag);                                        \
            const T r1 = ((D).f1 - lam) - (num - diag * pc1);                                                     \
            acc += (inx && (D).t1 == T_FLUID) ? (vxy1 * (D).wz) * r1 : T(0);                                       \
        }                                                                                                          \
        if (k_ + 1 == kend) { /* the coarse plane K is complete */                                                \
            T s = __shfl(acc, ca, 64);                                                                             \
            const T s2 = __shfl(acc, cb, 64);                                                                      \
            if (pair) s = s + s2;                                                                                  \
            if (own) {                                                                                             \
                const int64_t cid = ((int64_t)K * C.n[1] + J) * C.n[0] + I0 + lane;                                \
                C.R[cid] = s;                                                                                      \
                C.e[cid] = T(0);                                                                                   \
                psum += (double)s;                                                                                 \
            }                                                                                                      \
            acc = T(0);                                                                                            \
            ++K;                                                                                                   \
            kend = M.cs[2][min(K + 1, K1)];                                                                        \
        }                                                                                                          \
        pm0 = pc0;                                                                                                 \
        pc0 = (D).pp0;                                                                                             \
        pm1 = pc1;                                                                                                 \
        pc1 = (D).pp1;                                                                                             \
    }
    RMPlane<T> qa = ld(k0), qb;
    for (int k = k0; k < k1; k += 2) {
        qb = ld(k + 1);
        IBM_RMAP_PLANE(qa, k);
        if (k + 1 >= k1) break;
        qa = ld(k + 2);
        IBM_RMAP_PLANE(qb, k + 1);
    }
#undef IBM_RMAP_PLANE
    return psum;
}

template <typename T>
__global__ void __launch_bounds__(RM_NT)
    k_restrict0_map(Fine<T> F, const T *__restrict__ p, const T *__restrict__ f, const T *__restrict__ lamp,
                    Coarse<T> C, ChildMap M, RowTiles t, double *partials) {
    const int lane = (int)threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const T lam = *lamp;
    double psum = 0.0;
    const int per = gridDim.x >> 3;  // the grid is a multiple of 8
    for (int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3); tile < t.ntiles; tile += gridDim.x) {
        int q = tile;
        const int txi = q % t.ntx;
        q /= t.ntx;
        const int tyi = q % t.nty;
        const int chunk = q / t.nty;
        const int J = tyi * RM_W + wave;
        if (J >= C.n[1]) continue;
        const int I0 = txi * RM_CX, I1 = min(I0 + RM_CX, C.n[0]);
        const int K0 = chunk * t.kc, K1 = min(C.n[2], K0 + t.kc);
        if (M.cs[1][J + 1] - M.cs[1][J] == 2)
            psum += restrict_map_row<T, true>(F, p, f, lam, C, M, I0, I1, J, K0, K1, lane);
        else
            psum += restrict_map_row<T, false>(F, p, f, lam, C, M, I0, I1, J, K0, K1, lane);
    }
    __shared__ double sh[RM_NT / 64];
    const double tot = block_sum<RM_NT>(psum, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// ---- prolongation ------------------------------------------------------------------------
// pnext = pcur + P e_1 on fluid cells (ghost cells are refreshed afterwards).  The loads of
// plane k+1 (its z table entry, fine values and the coarse contributors) are issued before
// plane k is computed.  A cell with an inactive contributor takes its parent's value; the
// parent is the first contributor on every axis (lo of the table), and the per-cell flag is
// fixed by the geometry (computed with the hierarchy), so no activity is read here.
template <typename T>
struct PPlane {
    T pv, e[8];
    uint8_t ty, inj;
    double tz;
    bool twoz;
};

template <typename T>
__global__ void __launch_bounds__(ZM_NT)
    k_prolong0_zm(Fine<T> F, const T *__restrict__ pcur, T *__restrict__ pnext, Coarse<T> C, ProlongTab P,
                  ZTiles t) {
    const ZPos z = zpos(t, F.nz);
    if (!z.live) return;
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i < nx && z.j < ny;
    const int ic = min(z.i, nx - 1), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    const int ix[2] = {P.lo[0][ic], P.hi[0][ic]}, iy[2] = {P.lo[1][jc], P.hi[1][jc]};
    const double tx = P.t[0][ic], ty = P.t[1][jc];
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty};
    const bool twox = ix[0] != ix[1], twoy = iy[0] != iy[1];
    const int64_t cny = C.n[1], cnx = C.n[0];
    auto ld = [=](int k) -> PPlane<T> {
        PPlane<T> d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + rowoff;
        const int iz[2] = {P.lo[2][kk], P.hi[2][kk]};
        d.tz = P.t[2][kk];
        d.twoz = iz[0] != iz[1];
        d.ty = F.type[base];
        d.inj = F.inject[base];
        d.pv = pcur[base];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    d.e[4 * c + 2 * b + a] = C.e[((int64_t)iz[c] * cny + iy[b]) * cnx + ix[a]];
        return d;
    };
#define IBM_PROLONG_PLANE(D, kk)                                                                                  \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        const double wz[2] = {1.0 - (D).tz, (D).tz};                                                               \
        double s = 0.0;                                                                                            \
        _Pragma("unroll") for (int c = 0; c < 2; ++c) _Pragma("unroll") for (int b = 0; b < 2; ++b)                \
            _Pragma("unroll") for (int a = 0; a < 2; ++a) {                                                        \
            const bool ok = (a == 0 || twox) && (b == 0 || twoy) && (c == 0 || (D).twoz);                          \
            const double term = (wx[a] * wy[b]) * wz[c] * (double)(D).e[4 * c + 2 * b + a];                       \
            if (ok) s += term;                                                                                     \
        }                                                                                                          \
        if ((D).inj) s = (double)(D).e[0];                                                                         \
        if (in && k_ < z.k1 && (D).ty == T_FLUID) {                                                                \
            store_stream<T>(pnext + (int64_t)k_ * plane + rowoff, (T)((double)(D).pv + s));                     \
        }                                                                                                          \
    }
    PPlane<T> qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        IBM_PROLONG_PLANE(qa, k);
        qa = ld(k + 2);
        IBM_PROLONG_PLANE(qb, k + 1);
    }
#undef IBM_PROLONG_PLANE
}

// Prolongation for any child map, with the coarse values staged in LDS: a workgroup's 64 x 4
// fine columns draw on at most PL_CW x PL_CH coarse columns, so each coarse plane the chunk
// needs is read once into a ring of four LDS planes (the next one while the current fine
// plane is computed) instead of eight gathers per fine cell.  Same arithmetic, order of
// summation and injection rule as k_prolong0_zm.
constexpr int PL_CW = 68, PL_CH = 6, PL_RING = 4, PL_PER = (PL_CW * PL_CH + ZM_NT - 1) / ZM_NT;

template <typename T>
struct PFine {
    T pv;
    uint8_t ty, inj;
};

template <typename T>
__global__ void __launch_bounds__(ZM_NT)
    k_prolong0_lds(Fine<T> F, const T *__restrict__ pcur, T *__restrict__ pnext, Coarse<T> C, ProlongTab P,
                   ZTiles t) {
    __shared__ T ec[PL_RING][PL_CH][PL_CW];
    const ZPos z = zpos(t, F.nz);
    if (!z.live) return;
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i < nx && z.j < ny;
    const int ic = min(z.i, nx - 1), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    // the tile's coarse window (tables are monotone: lo non-decreasing, hi = lo or lo +- 1)
    const int ia = min(z.i - z.lane, nx - 1), ib = min(z.i - z.lane + ZM_TX - 1, nx - 1);
    const int ja = min(z.j - z.wave, ny - 1), jb = min(z.j - z.wave + ZM_TY - 1, ny - 1);
    const int cx0 = min(P.lo[0][ia], P.hi[0][ia]), cx1 = max(P.lo[0][ib], P.hi[0][ib]);
    const int cy0 = min(P.lo[1][ja], P.hi[1][ja]), cy1 = max(P.lo[1][jb], P.hi[1][jb]);
    const int cw = cx1 - cx0 + 1, ch = cy1 - cy0 + 1;
    const int ix[2] = {P.lo[0][ic] - cx0, P.hi[0][ic] - cx0}, iy[2] = {P.lo[1][jc] - cy0, P.hi[1][jc] - cy0};
    const double tx = P.t[0][ic], ty = P.t[1][jc];
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty};
    const bool twox = ix[0] != ix[1], twoy = iy[0] != iy[1];
    const int64_t cny = C.n[1], cnx = C.n[0];
    // coarse values this thread stages for one coarse plane
    auto cload = [=](int K, T (&v)[PL_PER]) {
#pragma unroll
        for (int q = 0; q < PL_PER; ++q) {
            const int e = (int)threadIdx.x + q * ZM_NT;
            const int r = e / PL_CW, c = e % PL_CW;
            const bool ok = r < ch && c < cw;
            v[q] = ok ? C.e[((int64_t)K * cny + cy0 + r) * cnx + cx0 + c] : T(0);
        }
    };
    auto cstore = [&](int K, const T (&v)[PL_PER]) {
#pragma unroll
        for (int q = 0; q < PL_PER; ++q) {
            const int e = (int)threadIdx.x + q * ZM_NT;
            if (e < PL_CW * PL_CH) ec[K & (PL_RING - 1)][e / PL_CW][e % PL_CW] = v[q];
        }
    };
    auto fload = [=](int k) -> PFine<T> {
        PFine<T> d;
        const int64_t base = (int64_t)min(k, nz - 1) * plane + rowoff;
        d.pv = pcur[base];
        d.ty = F.type[base];
        d.inj = F.inject[base];
        return d;
    };
    // coarse planes needed by fine plane k: [lo, hi] of its z table
    auto need_hi = [=](int k) { return max(P.lo[2][k], P.hi[2][k]); };
    const int k0 = z.k0, k1 = z.k1;
    int have;  // highest coarse plane staged
    {
        const int a = min(P.lo[2][k0], P.hi[2][k0]), b = need_hi(k0);
        T v[PL_PER];
        for (int K = a; K <= b; ++K) {
            cload(K, v);
            cstore(K, v);
        }
        have = b;
        __syncthreads();
    }
    PFine<T> qa = fload(k0);
    for (int k = k0; k < k1; ++k) {
        const PFine<T> qb = fload(k + 1);
        // the next fine plane needs at most one more coarse plane: load it now, stage it after
        const int nb = (k + 1 < nz) ? need_hi(k + 1) : have;
        const bool more = nb > have;
        T v[PL_PER];
        if (more) cload(nb, v);
        const int iz[2] = {P.lo[2][k], P.hi[2][k]};
        const double tz = P.t[2][k];
        const double wz[2] = {1.0 - tz, tz};
        const bool twoz = iz[0] != iz[1];
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const bool ok = (a == 0 || twox) && (b == 0 || twoy) && (c == 0 || twoz);
                    const double term = (wx[a] * wy[b]) * wz[c] * (double)ec[iz[c] & (PL_RING - 1)][iy[b]][ix[a]];
                    if (ok) s += term;
                }
        if (qa.inj) s = (double)ec[iz[0] & (PL_RING - 1)][iy[0]][ix[0]];
        if (in && qa.ty == T_FLUID) store_stream<T>(pnext + (int64_t)k * plane + rowoff, (T)((double)qa.pv + s));
        if (more) {
            __syncthreads();  // every thread is done with the slot the new plane goes to
            cstore(nb, v);
            have = nb;
        }
        __syncthreads();
        qa = qb;
    }
}

// Prolongation when z is halved (the usual case).  Fine planes 2K and 2K+1 have the coarse
// plane K as their first contributor and K-1 or K+1 as their second, so a column needs one
// new coarse plane per pair of fine planes: a window of three coarse planes (four
// contributor values each) stays in registers, and the next coarse plane and the next two
// fine planes are loaded before the current pair is computed.  Same arithmetic, order of
// summation and injection rule as k_prolong0_zm.
template <typename T>
struct CPlane4 {
    T v[4];  // [b][a]: y contributor b, x contributor a
};
template <typename T>
struct FPlaneZ {
    T pv;
    uint8_t ty, inj;
    int dz;     // second z contributor minus the first: -1, 0 or +1
    double tz;  // its weight
};

template <typename T>
__global__ void __launch_bounds__(ZM_NT)
    k_prolong0_zh(Fine<T> F, const T *__restrict__ pcur, T *__restrict__ pnext, Coarse<T> C, ProlongTab P,
                  ZTiles t) {
    const ZPos z = zpos(t, F.nz);
    if (!z.live) return;
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i < nx && z.j < ny;
    const int ic = min(z.i, nx - 1), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    const int ix[2] = {P.lo[0][ic], P.hi[0][ic]}, iy[2] = {P.lo[1][jc], P.hi[1][jc]};
    const double tx = P.t[0][ic], ty = P.t[1][jc];
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty};
    const bool twox = ix[0] != ix[1], twoy = iy[0] != iy[1];
    const int64_t cny = C.n[1], cnx = C.n[0];
    const int cnz = C.n[2];
    auto ldc = [&](int K) -> CPlane4<T> {
        CPlane4<T> c;
        const int64_t Kc = min(max(K, 0), cnz - 1);
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) c.v[2 * b + a] = C.e[(Kc * cny + iy[b]) * cnx + ix[a]];
        return c;
    };
    auto ldf = [&](int k) -> FPlaneZ<T> {
        FPlaneZ<T> d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + rowoff;
        d.pv = pcur[base];
        d.ty = F.type[base];
        d.inj = F.inject[base];
        d.dz = P.hi[2][kk] - P.lo[2][kk];
        d.tz = P.t[2][kk];
        return d;
    };
    auto fine = [&](const FPlaneZ<T> &D, int k, const CPlane4<T> &lo, const CPlane4<T> &hi) {
        const double wz[2] = {1.0 - D.tz, D.tz};
        const bool twoz = D.dz != 0;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const bool ok = (a == 0 || twox) && (b == 0 || twoy) && (c == 0 || twoz);
                    const double e = (double)(c == 0 ? lo.v[2 * b + a] : hi.v[2 * b + a]);
                    const double term = (wx[a] * wy[b]) * wz[c] * e;
                    if (ok) s += term;
                }
        if (D.inj) s = (double)lo.v[0];
        if (in && k < z.k1 && D.ty == T_FLUID)
            store_stream<T>(pnext + (int64_t)k * plane + rowoff, (T)((double)D.pv + s));
    };
    // four coarse-plane slots and two fine-pair slots rotate by name (unrolled by four
    // pairs), so no register copy of a value still in flight stalls the queue
    const int K0 = z.k0 >> 1;
    CPlane4<T> q0 = ldc(K0 - 1), q1 = ldc(K0), q2 = ldc(K0 + 1), q3;
    FPlaneZ<T> fa = ldf(z.k0), fb = ldf(z.k0 + 1), ga, gb;
#define IBM_PROLONG_PAIR(CM, C0, CP, CN, FA, FB, NA, NB, kk)                                                      \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        CN = ldc((k_ >> 1) + 2);                                                                                   \
        NA = ldf(k_ + 2);                                                                                          \
        NB = ldf(k_ + 3);                                                                                          \
        fine(FA, k_, C0, FA.dz < 0 ? CM : (FA.dz > 0 ? CP : C0));                                                  \
        fine(FB, k_ + 1, C0, FB.dz < 0 ? CM : (FB.dz > 0 ? CP : C0));                                              \
    }
    for (int k = z.k0; k < z.k1; k += 8) {
        IBM_PROLONG_PAIR(q0, q1, q2, q3, fa, fb, ga, gb, k);
        IBM_PROLONG_PAIR(q1, q2, q3, q0, ga, gb, fa, fb, k + 2);
        IBM_PROLONG_PAIR(q2, q3, q0, q1, fa, fb, ga, gb, k + 4);
        IBM_PROLONG_PAIR(q3, q0, q1, q2, ga, gb, fa, fb, k + 6);
    }
#undef IBM_PROLONG_PAIR
}

// ---- Krylov operator ---------------------------------------------------------------------
// The FP64 level-0 results of the prolongation and operator passes are written with
// non-temporal stores (store_stream): the writing pass does not read them again, and keeping
// these full fields from displacing cached data measured faster over a whole projection.
// w = S y on fluid rows, 0 elsewhere, with the sums of ApplySums<DOTS> over the block (the
// fluid rows' contributions; w is 0 elsewhere).  The loads of plane k+1 are issued before
// plane k is computed.  Off the fluid rows o is not read into a sum at all (selected out, not
// multiplied by the zero image): the shadow residual is never written on dead cells, so its
// values there are whatever the workspace held, possibly NaN or Inf.
template <int DOTS>
__global__ void __launch_bounds__(ZM_NT)
    k_apply_fluid_zm(Fine<double> F, const double *__restrict__ y, double *__restrict__ w,
                     const double *__restrict__ o, const double *__restrict__ mup, ZTiles t, double *partials) {
    constexpr int NS = ApplySums<DOTS>::NS;
    const double mu = (DOTS == 1 || DOTS == 2) ? *mup : 0.0;
    const ZPos z = zpos(t, F.nz);
    if (!z.live) {
        if (threadIdx.x == 0)
            for (int q = 0; q < NS; ++q) partials[NS * blockIdx.x + q] = 0.0;
        return;
    }
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i < nx && z.j < ny;
    const int ic = min(z.i, nx - 1), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    const bool hx0 = ic > 0, hx1 = ic < nx - 1, hy0 = jc > 0, hy1 = jc < ny - 1;
    const int64_t dxm = hx0 ? -1 : 0, dxp = hx1 ? 1 : 0, dym = hy0 ? -(int64_t)nx : 0, dyp = hy1 ? (int64_t)nx : 0;
    const double axm = F.axm[ic], axp = F.axp[ic], aym = F.aym[jc], ayp = F.ayp[jc];
    const double vxy = F.wx[ic] * F.wy[jc];
    auto ld = [=](int k) -> RPlane<double> {
        RPlane<double> d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + rowoff;
        d.pp = y[base + (kk < nz - 1 ? plane : 0)];
        d.xm = y[base + dxm];
        d.xp = y[base + dxp];
        d.ym = y[base + dym];
        d.yp = y[base + dyp];
        d.ty = F.type[base];
        d.azm = F.azm[kk];
        d.azp = F.azp[kk];
        d.wz = F.wz[kk];
        d.fv = DOTS ? o[base] : 0.0;
        return d;
    };
    double ym1 = (z.k0 > 0) ? y[(int64_t)(z.k0 - 1) * plane + rowoff] : 0.0;
    double yc = y[(int64_t)z.k0 * plane + rowoff];
    double acc[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[q] = 0.0;
#define IBM_APPLY_PLANE(D, kk)                                                                                    \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        double num, diag;                                                                                          \
        zm_stencil<double>(axm, axp, aym, ayp, (D).azm, (D).azp, hx0, hx1, hy0, hy1, k_ > 0, k_ < nz - 1, (D).xm,  \
                           (D).xp, (D).ym, (D).yp, ym1, (D).pp, num, diag);                                        \
        const bool fl = in && (D).ty == T_FLUID;                                                                   \
        const double a = fl ? (DOTS == 3 ? (D).fv - (num - diag * yc)                                              \
                                         : (DOTS ? (num - diag * yc) - mu : num - diag * yc))                      \
                            : 0.0;                                                                                 \
        if (in && k_ < z.k1) {                                                                                     \
            __builtin_nontemporal_store(a, w + (int64_t)k_ * plane + rowoff);                                      \
            if (DOTS == 0 || DOTS == 3) acc[0] += (vxy * (D).wz) * a;                                              \
            if (DOTS == 1 || DOTS == 2) acc[0] += fl ? (D).fv * a : 0.0;                                           \
            if (DOTS == 1 || DOTS == 2) acc[1 % NS] += a * a;                                                      \
        }                                                                                                          \
        ym1 = yc;                                                                                                  \
        yc = (D).pp;                                                                                               \
    }
    RPlane<double> qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        IBM_APPLY_PLANE(qa, k);
        qa = ld(k + 2);
        IBM_APPLY_PLANE(qb, k + 1);
    }
#undef IBM_APPLY_PLANE
    zm_block_sums_store<ZM_NT, NS>(acc, partials);
}

// ---- relaxed Jacobi sweep (the scheduled-Jacobi preconditioner) -------------------------
// out = (1 - omega) y + omega (sum_f a_f y_nb - f) / sum_f a_f on fluid cells, y elsewhere
// (ghost cells are refreshed afterwards).  Same z-march as the operator above.
__global__ void __launch_bounds__(ZM_NT)
    k_jacobi0_zm(Fine<double> F, const double *__restrict__ y, const double *__restrict__ f, double *__restrict__ out,
                 double omega, ZTiles t) {
    const ZPos z = zpos(t, F.nz);
    if (!z.live) return;
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i < nx && z.j < ny;
    const int ic = min(z.i, nx - 1), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    const bool hx0 = ic > 0, hx1 = ic < nx - 1, hy0 = jc > 0, hy1 = jc < ny - 1;
    const int64_t dxm = hx0 ? -1 : 0, dxp = hx1 ? 1 : 0, dym = hy0 ? -(int64_t)nx : 0, dyp = hy1 ? (int64_t)nx : 0;
    const double axm = F.axm[ic], axp = F.axp[ic], aym = F.aym[jc], ayp = F.ayp[jc];
    auto ld = [=](int k) -> RPlane<double> {
        RPlane<double> d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + rowoff;
        d.pp = y[base + (kk < nz - 1 ? plane : 0)];
        d.xm = y[base + dxm];
        d.xp = y[base + dxp];
        d.ym = y[base + dym];
        d.yp = y[base + dyp];
        d.fv = f[base];
        d.ty = F.type[base];
        d.azm = F.azm[kk];
        d.azp = F.azp[kk];
        return d;
    };
    double ym1 = (z.k0 > 0) ? y[(int64_t)(z.k0 - 1) * plane + rowoff] : 0.0;
    double yc = y[(int64_t)z.k0 * plane + rowoff];
#define IBM_JACOBI_PLANE(D, kk)                                                                                   \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        double num, diag;                                                                                          \
        zm_stencil<double>(axm, axp, aym, ayp, (D).azm, (D).azp, hx0, hx1, hy0, hy1, k_ > 0, k_ < nz - 1, (D).xm,  \
                           (D).xp, (D).ym, (D).yp, ym1, (D).pp, num, diag);                                        \
        const double v = ((D).ty == T_FLUID) ? (1.0 - omega) * yc + omega * ((num - (D).fv) / diag) : yc;         \
        if (in && k_ < z.k1) store_stream<double>(out + (int64_t)k_ * plane + rowoff, v);                          \
        ym1 = yc;                                                                                                  \
        yc = (D).pp;                                                                                               \
    }
    RPlane<double> qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        IBM_JACOBI_PLANE(qa, k);
        qa = ld(k + 2);
        IBM_JACOBI_PLANE(qb, k + 1);
    }
#undef IBM_JACOBI_PLANE
}

// ---- paired-column variants (nx even) ----------------------------------------------------
// A thread owns two adjacent columns (16-byte loads); a 256-thread workgroup covers 64 x 8
// columns and a wave holds two rows (lanes l and l + 32).  For the restriction a thread's
// pair is exactly one coarse cell's x children and a wave's row pair its y children, so the
// in-plane part of the sum needs no LDS and no barrier.
constexpr int ZP_TX = 64, ZP_TY = 8, ZP_NT = 256;

ZTiles ztiles2(int nx, int ny, int nz) {
    ZTiles t;
    t.ntx = (nx + ZP_TX - 1) / ZP_TX;
    t.nty = (ny + ZP_TY - 1) / ZP_TY;
    const int64_t per_slab = (int64_t)t.ntx * t.nty;
    int nchunk = (int)std::max<int64_t>(1, (int64_t)8 * device_cu_count() / per_slab);
    nchunk = std::min(nchunk, std::max(1, nz / 2));
    int kc = (nz + nchunk - 1) / nchunk;
    kc += kc & 1;
    nchunk = (nz + kc - 1) / kc;
    t.kc = kc;
    t.ntiles = (int)(per_slab * nchunk);
    t.grid = ((t.ntiles + 7) / 8) * 8;
    return t;
}

struct ZPos2 {
    bool live;
    int i0, j, k0, k1, half;  // first column of the pair, row, chunk, lane half (row within the wave)
};

__device__ __forceinline__ ZPos2 zpos2(const ZTiles &t, int nz) {
    ZPos2 z;
    const int per = gridDim.x >> 3;
    const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    z.live = logical < t.ntiles;
    int tile = logical;
    const int txi = tile % t.ntx;
    tile /= t.ntx;
    const int tyi = tile % t.nty;
    const int chunk = tile / t.nty;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    z.half = lane >> 5;
    z.i0 = txi * ZP_TX + 2 * (lane & 31);
    z.j = tyi * ZP_TY + 2 * wave + z.half;
    z.k0 = chunk * t.kc;
    z.k1 = min(nz, z.k0 + t.kc);
    return z;
}

template <typename T>
struct Vec2T;
template <>
struct Vec2T<double> {
    using type = double2;
};
template <>
struct Vec2T<float> {
    using type = float2;
};

template <typename T>
struct RPlane2 {
    typename Vec2T<T>::type pp, ym, yp, fv;  // pairs: p(k+1), p(j-1), p(j+1), f(k)
    T xm, xp;                                // p(i0-1), p(i0+2) of plane k
    T azm, azp, wz;
    uint16_t tt;                             // the two cell types
};

template <typename T>
__global__ void __launch_bounds__(ZP_NT)
    k_restrict0_zm2(Fine<T> F, const T *__restrict__ p, const T *__restrict__ f, const T *__restrict__ lamp,
                    Coarse<T> C, int hx, int hy, int hz, ZTiles t, double *partials) {
    using V = typename Vec2T<T>::type;
    const ZPos2 z = zpos2(t, F.nz);
    if (!z.live) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i0 < nx && z.j < ny;  // nx even: the pair is wholly inside or outside
    const int ic = min(z.i0, nx - 2), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    const bool hx0 = ic > 0, hx1 = ic + 2 < nx, hy0 = jc > 0, hy1 = jc < ny - 1;
    const int64_t dxm = hx0 ? -1 : 0, dxp = hx1 ? 2 : 1, dym = hy0 ? -(int64_t)nx : 0, dyp = hy1 ? (int64_t)nx : 0;
    const T axm0 = F.axm[ic], axp0 = F.axp[ic], axm1 = F.axm[ic + 1], axp1 = F.axp[ic + 1];
    const T aym = F.aym[jc], ayp = F.ayp[jc];
    const T vxy0 = F.wx[ic] * F.wy[jc], vxy1 = F.wx[ic + 1] * F.wy[jc];
    const T lam = *lamp;
    const bool writer = in && (!hy || z.half == 0);
    const int I = hx ? ic >> 1 : ic, J = hy ? jc >> 1 : jc;
    auto ld = [=](int k) -> RPlane2<T> {
        RPlane2<T> d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + rowoff;
        d.pp = *reinterpret_cast<const V *>(p + base + (kk < nz - 1 ? plane : 0));
        d.ym = *reinterpret_cast<const V *>(p + base + dym);
        d.yp = *reinterpret_cast<const V *>(p + base + dyp);
        d.fv = *reinterpret_cast<const V *>(f + base);
        d.xm = p[base + dxm];
        d.xp = p[base + dxp];
        d.tt = *reinterpret_cast<const uint16_t *>(F.type + base);
        d.azm = F.azm[kk];
        d.azp = F.azp[kk];
        d.wz = F.wz[kk];
        return d;
    };
    V pm = (z.k0 > 0) ? *reinterpret_cast<const V *>(p + (int64_t)(z.k0 - 1) * plane + rowoff) : V{T(0), T(0)};
    V pc = *reinterpret_cast<const V *>(p + (int64_t)z.k0 * plane + rowoff);
    T acc0 = 0, acc1 = 0;
    double psum = 0.0;
#define IBM_RESTRICT_PLANE2(D, kk)                                                                                \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        const bool z0_ = k_ > 0, z1_ = k_ < nz - 1;                                                                \
        T n0, d0, n1, d1;                                                                                          \
        zm_stencil<T>(axm0, axp0, aym, ayp, (D).azm, (D).azp, hx0, true, hy0, hy1, z0_, z1_, (D).xm, pc.y,        \
                      (D).ym.x, (D).yp.x, pm.x, (D).pp.x, n0, d0);                                                 \
        zm_stencil<T>(axm1, axp1, aym, ayp, (D).azm, (D).azp, true, hx1, hy0, hy1, z0_, z1_, pc.x, (D).xp,        \
                      (D).ym.y, (D).yp.y, pm.y, (D).pp.y, n1, d1);                                                 \
        const T r0 = ((D).fv.x - lam) - (n0 - d0 * pc.x);                                                          \
        const T r1 = ((D).fv.y - lam) - (n1 - d1 * pc.y);                                                          \
        const bool ok_ = in && k_ < z.k1;                                                                          \
        T v0 = (ok_ && ((D).tt & 0xff) == T_FLUID) ? (vxy0 * (D).wz) * r0 : T(0);                                  \
        T v1 = (ok_ && ((D).tt >> 8) == T_FLUID) ? (vxy1 * (D).wz) * r1 : T(0);                                    \
        if (hx) {                                                                                                  \
            v0 = v0 + v1;                                                                                          \
            v1 = T(0);                                                                                             \
        }                                                                                                          \
        if (hy) {                                                                                                  \
            v0 = v0 + __shfl_xor(v0, 32, 64);                                                                      \
            v1 = v1 + __shfl_xor(v1, 32, 64);                                                                      \
        }                                                                                                          \
        acc0 = (hz && (k_ & 1)) ? acc0 + v0 : v0;                                                                  \
        acc1 = (hz && (k_ & 1)) ? acc1 + v1 : v1;                                                                  \
        if ((!hz || (k_ & 1)) && writer && k_ < z.k1) {                                                            \
            const int K_ = hz ? k_ >> 1 : k_;                                                                      \
            const int64_t cid = ((int64_t)K_ * C.n[1] + J) * C.n[0] + I;                                           \
            C.R[cid] = acc0;                                                                                       \
            C.e[cid] = T(0);                                                                                       \
            psum += (double)acc0;                                                                                  \
            if (!hx) {                                                                                             \
                C.R[cid + 1] = acc1;                                                                               \
                C.e[cid + 1] = T(0);                                                                               \
                psum += (double)acc1;                                                                              \
            }                                                                                                      \
        }                                                                                                          \
        pm = pc;                                                                                                   \
        pc = (D).pp;                                                                                               \
    }
    RPlane2<T> qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        IBM_RESTRICT_PLANE2(qa, k);
        qa = ld(k + 2);
        IBM_RESTRICT_PLANE2(qb, k + 1);
    }
#undef IBM_RESTRICT_PLANE2
    zm_block_sum_store<ZP_NT>(psum, partials);
}

template <int DOTS>
__global__ void __launch_bounds__(ZP_NT)
    k_apply_fluid_zm2(Fine<double> F, const double *__restrict__ y, double *__restrict__ w,
                      const double *__restrict__ o, const double *__restrict__ mup, ZTiles t, double *partials) {
    using V = double2;
    typedef double NV __attribute__((ext_vector_type(2)));  // native pair for the streaming store
    constexpr int NS = ApplySums<DOTS>::NS;
    const double mu = (DOTS == 1 || DOTS == 2) ? *mup : 0.0;
    const ZPos2 z = zpos2(t, F.nz);
    if (!z.live) {
        if (threadIdx.x == 0)
            for (int q = 0; q < NS; ++q) partials[NS * blockIdx.x + q] = 0.0;
        return;
    }
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool in = z.i0 < nx && z.j < ny;
    const int ic = min(z.i0, nx - 2), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    const bool hx0 = ic > 0, hx1 = ic + 2 < nx, hy0 = jc > 0, hy1 = jc < ny - 1;
    const int64_t dxm = hx0 ? -1 : 0, dxp = hx1 ? 2 : 1, dym = hy0 ? -(int64_t)nx : 0, dyp = hy1 ? (int64_t)nx : 0;
    const double axm0 = F.axm[ic], axp0 = F.axp[ic], axm1 = F.axm[ic + 1], axp1 = F.axp[ic + 1];
    const double aym = F.aym[jc], ayp = F.ayp[jc];
    const double vxy0 = F.wx[ic] * F.wy[jc], vxy1 = F.wx[ic + 1] * F.wy[jc];
    auto ld = [=](int k) -> RPlane2<double> {
        RPlane2<double> d;
        const int kk = min(k, nz - 1);
        const int64_t base = (int64_t)kk * plane + rowoff;
        d.pp = *reinterpret_cast<const V *>(y + base + (kk < nz - 1 ? plane : 0));
        d.ym = *reinterpret_cast<const V *>(y + base + dym);
        d.yp = *reinterpret_cast<const V *>(y + base + dyp);
        d.xm = y[base + dxm];
        d.xp = y[base + dxp];
        d.tt = *reinterpret_cast<const uint16_t *>(F.type + base);
        d.azm = F.azm[kk];
        d.azp = F.azp[kk];
        d.wz = F.wz[kk];
        d.fv = DOTS ? *reinterpret_cast<const V *>(o + base) : V{0.0, 0.0};
        return d;
    };
    V ym1 = (z.k0 > 0) ? *reinterpret_cast<const V *>(y + (int64_t)(z.k0 - 1) * plane + rowoff) : V{0.0, 0.0};
    V yc = *reinterpret_cast<const V *>(y + (int64_t)z.k0 * plane + rowoff);
    double acc[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[q] = 0.0;
#define IBM_APPLY_PLANE2(D, kk)                                                                                   \
    {                                                                                                              \
        const int k_ = (kk);                                                                                       \
        const bool z0_ = k_ > 0, z1_ = k_ < nz - 1;                                                                \
        double n0, d0, n1, d1;                                                                                     \
        zm_stencil<double>(axm0, axp0, aym, ayp, (D).azm, (D).azp, hx0, true, hy0, hy1, z0_, z1_, (D).xm, yc.y,   \
                           (D).ym.x, (D).yp.x, ym1.x, (D).pp.x, n0, d0);                                           \
        zm_stencil<double>(axm1, axp1, aym, ayp, (D).azm, (D).azp, true, hx1, hy0, hy1, z0_, z1_, yc.x, (D).xp,   \
                           (D).ym.y, (D).yp.y, ym1.y, (D).pp.y, n1, d1);                                           \
        const bool f0_ = in && ((D).tt & 0xff) == T_FLUID, f1_ = in && ((D).tt >> 8) == T_FLUID;                  \
        const double a0 = f0_                                                                                      \
                              ? (DOTS == 3 ? (D).fv.x - (n0 - d0 * yc.x)                                           \
                                           : (DOTS ? (n0 - d0 * yc.x) - mu : n0 - d0 * yc.x))                      \
                              : 0.0;                                                                               \
        const double a1 = f1_                                                                                      \
                              ? (DOTS == 3 ? (D).fv.y - (n1 - d1 * yc.y)                                           \
                                           : (DOTS ? (n1 - d1 * yc.y) - mu : n1 - d1 * yc.y))                      \
                              : 0.0;                                                                               \
        if (in && k_ < z.k1) {                                                                                     \
            const NV o_ = {a0, a1};                                                                                \
            __builtin_nontemporal_store(o_, reinterpret_cast<NV *>(w + (int64_t)k_ * plane + rowoff));             \
            if (DOTS == 0 || DOTS == 3) {                                                                          \
                acc[0] += (vxy0 * (D).wz) * a0;                                                                    \
                acc[0] += (vxy1 * (D).wz) * a1;                                                                    \
            }                                                                                                      \
            if (DOTS == 1 || DOTS == 2) {                                                                          \
                acc[0] += f0_ ? (D).fv.x * a0 : 0.0;                                                               \
                acc[0] += f1_ ? (D).fv.y * a1 : 0.0;                                                               \
            }                                                                                                      \
            if (DOTS == 1 || DOTS == 2) {                                                                          \
                acc[1 % NS] += a0 * a0;                                                                            \
                acc[1 % NS] += a1 * a1;                                                                            \
            }                                                                                                      \
        }                                                                                                          \
        ym1 = yc;                                                                                                  \
        yc = (D).pp;                                                                                               \
    }
    RPlane2<double> qa = ld(z.k0), qb;
    for (int k = z.k0; k < z.k1; k += 2) {
        qb = ld(k + 1);
        IBM_APPLY_PLANE2(qa, k);
        qa = ld(k + 2);
        IBM_APPLY_PLANE2(qb, k + 1);
    }
#undef IBM_APPLY_PLANE2
    zm_block_sums_store<ZP_NT, NS>(acc, partials);
}

}  // namespace

template <typename T>
hipError_t launch_restrict0(const Fine<T> &F, const T *p, const T *f, const T *lam, const Coarse<T> &C,
                            const ChildMap &M, double *partials, int *nparts, hipStream_t s) {
    if (!((M.halved[0] || M.same[0]) && (M.halved[1] || M.same[1]) && (M.halved[2] || M.same[2]))) {
        // some axis merges only part of its cells: the generic pass
        RowTiles t;
        int grid;
        const hipError_t e = row_tiles(C.n, RM_TILES_PER_CU, RM_KMIN, zmarch_partials_max(F.nx, F.ny, F.nz), &t, &grid);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_restrict0_map<T>, dim3(grid), dim3(RM_NT), 0, s, F, p, f, lam, C, M, t, partials);
        *nparts = grid;
        return hipGetLastError();
    }
    const int halved[3] = {M.halved[0], M.halved[1], M.halved[2]};
    if ((F.nx & 1) == 0 && F.nx >= 2) {
        const ZTiles t = ztiles2(F.nx, F.ny, F.nz);
        hipLaunchKernelGGL(k_restrict0_zm2<T>, dim3(t.grid), dim3(ZP_NT), 0, s, F, p, f, lam, C, halved[0],
                           halved[1], halved[2], t, partials);
        *nparts = t.grid;
        return hipGetLastError();
    }
    const ZTiles t = ztiles(F.nx, F.ny, F.nz);
    hipLaunchKernelGGL(k_restrict0_zm<T>, dim3(t.grid), dim3(ZM_NT), 0, s, F, p, f, lam, C, halved[0], halved[1],
                       halved[2], t, partials);
    *nparts = t.grid;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong0(const Fine<T> &F, const T *pcur, T *pnext, const Coarse<T> &C, const ProlongTab &P,
                           hipStream_t s) {
    const ZTiles t = ztiles(F.nx, F.ny, F.nz);  // chunks start at even planes and have even length
    if (P.halved[2] && (F.nz & 1) == 0)
        hipLaunchKernelGGL(k_prolong0_zh<T>, dim3(t.grid), dim3(ZM_NT), 0, s, F, pcur, pnext, C, P, t);
    else
        hipLaunchKernelGGL(k_prolong0_lds<T>, dim3(t.grid), dim3(ZM_NT), 0, s, F, pcur, pnext, C, P, t);
    return hipGetLastError();
}

template <int DOTS>
static hipError_t apply_fluid_dots(const Fine<double> &F, const double *y, double *w, const double *o,
                                   const double *mu, double *partials, int *nparts, hipStream_t s) {
    if ((F.nx & 1) == 0 && F.nx >= 2) {
        const ZTiles t = ztiles2(F.nx, F.ny, F.nz);
        hipLaunchKernelGGL(k_apply_fluid_zm2<DOTS>, dim3(t.grid), dim3(ZP_NT), 0, s, F, y, w, o, mu, t, partials);
        *nparts = t.grid;
        return hipGetLastError();
    }
    const ZTiles t = ztiles(F.nx, F.ny, F.nz);
    hipLaunchKernelGGL(k_apply_fluid_zm<DOTS>, dim3(t.grid), dim3(ZM_NT), 0, s, F, y, w, o, mu, t, partials);
    *nparts = t.grid;
    return hipGetLastError();
}

hipError_t launch_apply_fluid(const Fine<double> &F, const double *y, double *w, const double *o, const double *mu,
                              int dots, double *partials, int *nparts, hipStream_t s) {
    if (dots == 1) return apply_fluid_dots<1>(F, y, w, o, mu, partials, nparts, s);
    if (dots == 2) return apply_fluid_dots<2>(F, y, w, o, mu, partials, nparts, s);
    if (dots == 3) return apply_fluid_dots<3>(F, y, w, o, mu, partials, nparts, s);
    return apply_fluid_dots<0>(F, y, w, o, mu, partials, nparts, s);
}

hipError_t launch_jacobi0(const Fine<double> &F, const double *y, const double *f, double *out, double omega,
                          hipStream_t s) {
    const ZTiles t = ztiles(F.nx, F.ny, F.nz);
    hipLaunchKernelGGL(k_jacobi0_zm, dim3(t.grid), dim3(ZM_NT), 0, s, F, y, f, out, omega, t);
    return hipGetLastError();
}

hipError_t row_tiles(const int cn[3], int per_cu, int kmin, int64_t cap, RowTiles *t, int *grid) {
    t->ntx = (cn[0] + RM_CX - 1) / RM_CX;
    t->nty = (cn[1] + RM_W - 1) / RM_W;
    const int64_t per_slab = (int64_t)t->ntx * t->nty;
    const int64_t want = (int64_t)per_cu * device_cu_count();
    int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(want / per_slab, cn[2] / std::max(1, kmin)));
    t->kc = (cn[2] + nchunk - 1) / nchunk;
    nchunk = (cn[2] + t->kc - 1) / t->kc;
    const int64_t ntiles = per_slab * nchunk;
    if (ntiles > INT32_MAX) return hipErrorInvalidValue;
    t->ntiles = (int)ntiles;
    cap = std::max<int64_t>(8, cap / 8 * 8);
    *grid = (int)std::min<int64_t>((ntiles + 7) / 8 * 8, cap);
    return hipSuccess;
}

// upper bound of the workgroup count of any z-march launch, whatever the CU count
int64_t zmarch_partials_max(int nx, int ny, int nz) {
    const int64_t per_slab = (int64_t)((nx + ZM_TX - 1) / ZM_TX) * ((ny + ZM_TY - 1) / ZM_TY);
    return per_slab * std::max(1, nz / 2 + 1) + 8;
}

template hipError_t launch_restrict0<double>(const Fine<double> &, const double *, const double *, const double *,
                                             const Coarse<double> &, const ChildMap &, double *, int *, hipStream_t);
template hipError_t launch_restrict0<float>(const Fine<float> &, const float *, const float *, const float *,
                                            const Coarse<float> &, const ChildMap &, double *, int *, hipStream_t);
template hipError_t launch_prolong0<double>(const Fine<double> &, const double *, double *, const Coarse<double> &,
                                            const ProlongTab &, hipStream_t);
template hipError_t launch_prolong0<float>(const Fine<float> &, const float *, float *, const Coarse<float> &,
                                           const ProlongTab &, hipStream_t);

}  // namespace ibm
