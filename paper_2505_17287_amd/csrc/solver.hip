// Pressure Poisson solve (paper Section 2.1: pressure equation of the fractional step,
// solved iteratively; multigrid and red-black Gauss-Seidel are among the solvers the paper
// evaluated) and the projection passes: divergence right-hand side, velocity correction,
// gauge.  Ghost equations (Section 2.2, Eq. 2) are refreshed after every fine-level sweep.
//
// Fine level (level 0) work is out of place between two pressure buffers; every pass reads
// one buffer and writes the other, so no pass ever reads a value another thread of the same
// pass writes.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cmath>
#include <utility>

#include "device_util.hpp"
#include "ibm_impl.hpp"
#include "zmarch.hpp"

namespace ibm {


// =======================================================================================
// ghost refresh: p_g = sum_{m != g} beta_m p_m + h_g from one snapshot (Jacobi over ghosts)
// fluid members are read from dst (already updated), ghost members from src_ghost (the
// values before this pass); degenerate ghosts take the mean of their fluid 26-neighbours.
// Weights are FP64; the right-hand sides gh may be absent (homogeneous error equation).
// =======================================================================================

// Eight lanes per ghost: lane m of a group takes stencil member m (the index and weight
// loads of a wave are contiguous and the eight gathers are in flight together), and the
// group sums its terms with three shuffle steps.  Degenerate ghosts (mean of the fluid
// 26-neighbours) are handled by the group's first lane.
constexpr int REFRESH_NT = 256;
// T: precision of the cycle (each new value is rounded to it); TS, TD: types of the two
// buffers (TD wider than T only after the widening last sweep of the mixed cycle).
template <typename T, typename TS = T, typename TD = T>
__global__ void __launch_bounds__(REFRESH_NT)
    k_ghost_refresh(GhostView G, const TS *__restrict__ src_ghost, TD *dst, int nx, int ny, int nz,
                    const uint8_t *__restrict__ type, const double *__restrict__ gh) {
    const int64_t g = ((int64_t)blockIdx.x * REFRESH_NT + threadIdx.x) >> 3;
    const int m = threadIdx.x & 7;
    const bool live = g < G.ng;
    const int64_t gc = live ? g : 0;
    const int32_t q = G.st[8 * gc + m];
    const double beta = G.beta[8 * gc + m];
    const unsigned gm = G.gmask[gc];
    const int32_t flags = G.flags[gc];
    // issued with the stencil loads, so the store needs no further round trip
    const int64_t cell = G.cell[gc];
    const double hg = gh ? gh[gc] : 0.0;
    double term = 0.0;
    if (live && q >= 0) term = beta * (double)(((gm >> m) & 1u) ? src_ghost[q] : dst[q]);
    term += __shfl_xor(term, 1, 64);
    term += __shfl_xor(term, 2, 64);
    term += __shfl_xor(term, 4, 64);
    if (!live || m != 0) return;
    double v;
    if (flags & GF_DEGENERATE) {
        int i, j, k;
        unflatten(cell, nx, ny, i, j, k);
        double sm = 0.0;
        int n = 0;
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    int ii = i + di, jj = j + dj, kk = k + dk;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                    int64_t qq = ((int64_t)kk * ny + jj) * nx + ii;
                    if (type[qq] == T_FLUID) {
                        sm += (double)dst[qq];
                        ++n;
                    }
                }
        v = n ? sm / n : 0.0;
    } else {
        v = gh ? term + hg : term;
    }
    dst[cell] = (TD)(T)v;
}

static GhostView ghost_view(ibm_grid *g) {
    GhostView G;
    G.ng = g->ng;
    G.cell = g->g_cell;
    G.st = g->g_st;
    G.gmask = g->g_mask;
    G.beta = g->g_beta;
    G.h = g->g_h;
    G.flags = g->g_flags;
    return G;
}

template <typename T>
static hipError_t launch_refresh(ibm_grid *g, const T *src_ghost, T *dst, const double *gh, hipStream_t s) {
    if (g->ng == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_refresh<T>, dim3((unsigned)((8 * g->ng + REFRESH_NT - 1) / REFRESH_NT)),
                       dim3(REFRESH_NT), 0, s, ghost_view(g),
                       src_ghost, dst, g->nx, g->ny, g->nz, g->type, gh);
    return hipGetLastError();
}

// the refresh after the widening last sweep of the mixed cycle: FP32 arithmetic as in
// launch_refresh<float>, members read from the FP32 input and the FP64 result
static hipError_t launch_refresh_widen(ibm_grid *g, const float *src_ghost, double *dst, const double *gh,
                                       hipStream_t s) {
    if (g->ng == 0) return hipSuccess;
    hipLaunchKernelGGL((k_ghost_refresh<float, float, double>), dim3((unsigned)((8 * g->ng + REFRESH_NT - 1) / REFRESH_NT)),
                       dim3(REFRESH_NT), 0, s, ghost_view(g), src_ghost, dst, g->nx, g->ny, g->nz, g->type, gh);
    return hipGetLastError();
}

// =======================================================================================
// fine-level operator view helpers
// =======================================================================================

static Fine<double> fine64(ibm_grid *g) {
    Fine<double> F;
    F.nx = g->nx;
    F.ny = g->ny;
    F.nz = g->nz;
    F.axm = g->am0[0];
    F.axp = g->ap0[0];
    F.aym = g->am0[1];
    F.ayp = g->ap0[1];
    F.azm = g->am0[2];
    F.azp = g->ap0[2];
    F.wx = g->w0[0];
    F.wy = g->w0[1];
    F.wz = g->w0[2];
    F.type = g->type;
    F.inject = g->inject0;
    return F;
}
static Fine<float> fine32(ibm_grid *g) {
    Fine<float> F;
    F.nx = g->nx;
    F.ny = g->ny;
    F.nz = g->nz;
    F.axm = g->am0f[0];
    F.axp = g->ap0f[0];
    F.aym = g->am0f[1];
    F.ayp = g->ap0f[1];
    F.azm = g->am0f[2];
    F.azp = g->ap0f[2];
    F.wx = g->w0f[0];
    F.wy = g->w0f[1];
    F.wz = g->w0f[2];
    F.type = g->type;
    F.inject = g->inject0;
    return F;
}
template <typename T>
static Coarse<T> coarse_view(ibm_grid *g, int l);
template <>
Coarse<double> coarse_view<double>(ibm_grid *g, int l) {
    LevelHost &L = g->lev[l];
    Coarse<double> C;
    for (int d = 0; d < 3; ++d) {
        C.n[d] = L.n[d];
        C.w[d] = L.w64[d];
        C.Tl[d] = L.T64[d];
    }
    C.active = L.active;
    C.e = L.e64;
    C.R = L.R64;
    C.mu = &g->sc->mu[l];
    return C;
}
template <>
Coarse<float> coarse_view<float>(ibm_grid *g, int l) {
    LevelHost &L = g->lev[l];
    Coarse<float> C;
    for (int d = 0; d < 3; ++d) {
        C.n[d] = L.n[d];
        C.w[d] = L.w32[d];
        C.Tl[d] = L.T32[d];
    }
    C.active = L.active;
    C.e = L.e32;
    C.R = L.R32;
    C.mu = &g->sc->mu[l];
    return C;
}
static ProlongTab prolong_tab(ibm_grid *g, int l) {  // table of level l from level l+1
    ProlongTab P;
    for (int d = 0; d < 3; ++d) {
        P.lo[d] = g->lev[l].plo[d];
        P.hi[d] = g->lev[l].phi[d];
        P.t[d] = g->lev[l].pt[d];
        P.halved[d] = g->lev[l + 1].halved[d];
    }
    return P;
}

template <typename T>
static T *&level_e(LevelHost &L);
template <>
double *&level_e<double>(LevelHost &L) { return L.e64; }
template <>
float *&level_e<float>(LevelHost &L) { return L.e32; }
template <typename T>
static T *&level_e2(LevelHost &L);
template <>
double *&level_e2<double>(LevelHost &L) { return L.e64b; }
template <>
float *&level_e2<float>(LevelHost &L) { return L.e32b; }

template <typename T>
__device__ __forceinline__ void fine_stencil(const Fine<T> &F, const T *__restrict__ p, int i, int j, int k, int64_t id,
                                             T &num, T &diag) {
    const int64_t sy = F.nx, sz = (int64_t)F.nx * F.ny;
    const T axm = F.axm[i], axp = F.axp[i], aym = F.aym[j], ayp = F.ayp[j], azm = F.azm[k], azp = F.azp[k];
    T s = 0;
    s = s + (i > 0 ? axm * p[id - 1] : T(0));
    s = s + (i < F.nx - 1 ? axp * p[id + 1] : T(0));
    s = s + (j > 0 ? aym * p[id - sy] : T(0));
    s = s + (j < F.ny - 1 ? ayp * p[id + sy] : T(0));
    s = s + (k > 0 ? azm * p[id - sz] : T(0));
    s = s + (k < F.nz - 1 ? azp * p[id + sz] : T(0));
    T d = axm + axp;
    d = d + aym;
    d = d + ayp;
    d = d + azm;
    d = d + azp;
    num = s;
    diag = d;
}

template <typename T>
__device__ __forceinline__ void coarse_stencil(const Coarse<T> &L, const T *__restrict__ e, int I, int J, int K,
                                               int64_t id, T &num, T &diag) {
    const int64_t sy = L.n[0], sz = (int64_t)L.n[0] * L.n[1];
    const T txm = L.Tl[0][id], txp = (I < L.n[0] - 1) ? L.Tl[0][id + 1] : T(0);
    const T tym = L.Tl[1][id], typ = (J < L.n[1] - 1) ? L.Tl[1][id + sy] : T(0);
    const T tzm = L.Tl[2][id], tzp = (K < L.n[2] - 1) ? L.Tl[2][id + sz] : T(0);
    T s = 0;
    s = s + (I > 0 ? txm * e[id - 1] : T(0));
    s = s + (I < L.n[0] - 1 ? txp * e[id + 1] : T(0));
    s = s + (J > 0 ? tym * e[id - sy] : T(0));
    s = s + (J < L.n[1] - 1 ? typ * e[id + sy] : T(0));
    s = s + (K > 0 ? tzm * e[id - sz] : T(0));
    s = s + (K < L.n[2] - 1 ? tzp * e[id + sz] : T(0));
    T d = txm + txp;
    d = d + tym;
    d = d + typ;
    d = d + tzm;
    d = d + tzp;
    num = s;
    diag = d;
}

// =======================================================================================
// residual + restriction, fused with block partial sums of the coarse right-hand side
// =======================================================================================

// level l -> l+1 (l >= 1): R_{l+1}(C) = sum over active children of r, r = (R - V mu) - S e;
// the children (one or two per axis) are summed x fastest, then y, then z
template <typename T>
__global__ void k_resrestrictC(Coarse<T> L, Coarse<T> C, ChildMap M, double *partials) {
    __shared__ double sh[4];
    const int64_t NC = (int64_t)C.n[0] * C.n[1] * C.n[2];
    const int64_t cid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double Rsum = 0.0;
    if (cid < NC) {
        const T mu = (T)(*L.mu);
        int I, J, K;
        unflatten(cid, C.n[0], C.n[1], I, J, K);
        const int i0 = M.cs[0][I], i1 = M.cs[0][I + 1], j0 = M.cs[1][J], j1 = M.cs[1][J + 1];
        const int k0 = M.cs[2][K], k1 = M.cs[2][K + 1];
        T R = 0;
        for (int k = k0; k < k1; ++k)
            for (int j = j0; j < j1; ++j)
                for (int i = i0; i < i1; ++i) {
                    const int64_t id = ((int64_t)k * L.n[1] + j) * L.n[0] + i;
                    T num, diag;
                    coarse_stencil(L, L.e, i, j, k, id, num, diag);
                    const T vol = (L.w[0][i] * L.w[1][j]) * L.w[2][k];
                    const T rc = (L.R[id] - vol * mu) - (num - diag * L.e[id]);
                    if (L.active[id]) R += rc;
                }
        C.R[cid] = R;
        C.e[cid] = T(0);
        Rsum = (double)R;
    }
    double s = block_sum<256>(Rsum, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// The same for any child map, row-wise (the tiling of the level-0 restriction k_restrict0_map):
// a wave owns one coarse row J (one or two finer rows) of a tile of RM_CX coarse columns, a
// lane one finer column, and the lane marches up the finer planes with both rows in
// registers; the x neighbours and the high x face come from the adjacent lanes (lanes 0 and
// 63 from edge loads), the high y face of the first row is the second row's low face, the
// high z face the next plane's low face, loaded with that plane.  Per cell the operations
// are those of coarse_stencil; each lane sums its active cells over the rows and planes of
// the current coarse plane, and when that plane is complete lane I - I0 adds the sums of the
// one or two lanes holding the children of coarse column I (the same sum as
// k_resrestrictC's, in another order).
// the row-wise pass from levels of at least this many cells (below, a thread per coarse cell)
constexpr int64_t RC_MAP_MIN_CELLS = 1 << 17;
constexpr int RC_TILES_PER_CU = 8, RC_KMIN = 4;

template <typename T>
struct RCPlane {
    T en0, en1, tzn0, tzn1;  // e and the low z face of plane k+1
    T r0, r1, tx0, tx1, ty0, ty1;
    T ylo, yhi, tyh;         // e below the first and above the last row, the low y face above the last
    T eL0, eR0, eL1, eR1, txR0, txR1;  // e just outside the tile's columns, the low x face right of it
    T w2;
    uint8_t a0, a1;
};

template <typename T, bool TWO>
__device__ __forceinline__ double resrestrict_row(const Coarse<T> &L, const Coarse<T> &C, const ChildMap &M, T mu,
                                                  int I0, int I1, int J, int K0, int K1, int lane) {
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int64_t plane = (int64_t)nx * ny;
    const int fx0 = M.cs[0][I0], fx1 = M.cs[0][I1];
    const int i = fx0 + lane;
    const bool inx = i < fx1;
    const int ic = min(i, nx - 1);
    const int ja = M.cs[1][J], jb = TWO ? ja + 1 : ja;
    const int64_t o0 = (int64_t)ja * nx + ic, o1 = (int64_t)jb * nx + ic;
    const int64_t olo = (int64_t)max(ja - 1, 0) * nx + ic, ohi = (int64_t)min(jb + 1, ny - 1) * nx + ic;
    const bool hx0 = ic > 0, hx1 = ic < nx - 1;
    const bool hy00 = ja > 0, hy10 = ja < ny - 1, hy01 = jb > 0, hy11 = jb < ny - 1;
    const int64_t eom = (int64_t)ja * nx + max(fx0 - 1, 0), eop = (int64_t)ja * nx + min(fx0 + 64, nx - 1);
    const T w0 = L.w[0][ic];
    const T vxy0 = w0 * L.w[1][ja], vxy1 = w0 * L.w[1][jb];
    const bool own = lane < I1 - I0;
    const int Io = min(I0 + lane, I1);
    const int ca = own ? M.cs[0][Io] - fx0 : 0;
    const bool pair = own && M.cs[0][min(Io + 1, I1)] - M.cs[0][Io] == 2;
    const int cb = min(ca + 1, 63);
    const int k0 = M.cs[2][K0], k1 = M.cs[2][K1];
    const T *__restrict__ pe = L.e;
    const T *__restrict__ pr = L.R;
    const T *__restrict__ px = L.Tl[0];
    const T *__restrict__ py = L.Tl[1];
    const T *__restrict__ pz = L.Tl[2];
    auto ld = [=](int k) -> RCPlane<T> {
        RCPlane<T> d;
        const int kk = min(k, nz - 1);
        const int64_t b = (int64_t)kk * plane, bn = (int64_t)min(kk + 1, nz - 1) * plane;
        d.en0 = pe[bn + o0];
        d.tzn0 = pz[bn + o0];
        d.r0 = pr[b + o0];
        d.tx0 = px[b + o0];
        d.ty0 = py[b + o0];
        d.a0 = L.active[b + o0];
        d.ylo = pe[b + olo];
        d.yhi = pe[b + ohi];
        d.tyh = py[b + ohi];
        d.eL0 = pe[b + eom];
        d.eR0 = pe[b + eop];
        d.txR0 = px[b + eop];
        if constexpr (TWO) {
            d.en1 = pe[bn + o1];
            d.tzn1 = pz[bn + o1];
            d.r1 = pr[b + o1];
            d.tx1 = px[b + o1];
            d.ty1 = py[b + o1];
            d.a1 = L.active[b + o1];
            d.eL1 = pe[b + eom + nx];
            d.eR1 = pe[b + eop + nx];
            d.txR1 = px[b + eop + nx];
        } else {
            d.en1 = d.tzn1 = d.r1 = d.tx1 = d.ty1 = d.eL1 = d.eR1 = d.txR1 = T(0);
            d.a1 = 0;
        }
        d.w2 = L.w[2][kk];
        return d;
    };
    T em0 = (k0 > 0) ? pe[(int64_t)(k0 - 1) * plane + o0] : T(0);
    T ec0 = pe[(int64_t)k0 * plane + o0], tzc0 = pz[(int64_t)k0 * plane + o0];
    T em1 = T(0), ec1 = T(0), tzc1 = T(0);
    if constexpr (TWO) {
        em1 = (k0 > 0) ? pe[(int64_t)(k0 - 1) * plane + o1] : T(0);
        ec1 = pe[(int64_t)k0 * plane + o1];
        tzc1 = pz[(int64_t)k0 * plane + o1];
    }
    T acc = 0;
    double psum = 0.0;
    int K = K0, kend = M.cs[2][K0 + 1];
    // one cell of plane k: coarse_stencil's operations, then the residual
#define IBM_RC_CELL(TXM, TXP, TYM, TYP, TZM, TZP, XM, XP, YM, YP, ZM, ZP, EC, HY0, HY1, RV, VXY, W2, ACT)      \
    {                                                                                                          \
        const T txp_ = hx1 ? (TXP) : T(0), typ_ = (HY1) ? (TYP) : T(0), tzp_ = hz1_ ? (TZP) : T(0);            \
        T s_ = 0;                                                                                              \
        s_ = s_ + (hx0 ? (TXM) * (XM) : T(0));                                                                 \
        s_ = s_ + (hx1 ? txp_ * (XP) : T(0));                                                                  \
        s_ = s_ + ((HY0) ? (TYM) * (YM) : T(0));                                                               \
        s_ = s_ + ((HY1) ? typ_ * (YP) : T(0));                                                                \
        s_ = s_ + (hz0_ ? (TZM) * (ZM) : T(0));                                                                \
        s_ = s_ + (hz1_ ? tzp_ * (ZP) : T(0));                                                                 \
        T d_ = (TXM) + txp_;                                                                                   \
        d_ = d_ + (TYM);                                                                                       \
        d_ = d_ + typ_;                                                                                        \
        d_ = d_ + (TZM);                                                                                       \
        d_ = d_ + tzp_;                                                                                        \
        const T vol_ = (VXY) * (W2);                                                                           \
        const T rc_ = ((RV) - vol_ * mu) - (s_ - d_ * (EC));                                                   \
        acc += (inx && (ACT)) ? rc_ : T(0);                                                                    \
    }
#define IBM_RC_PLANE(D, kk)                                                                                    \
    {                                                                                                          \
        const int k_ = (kk);                                                                                   \
        const bool hz0_ = k_ > 0, hz1_ = k_ < nz - 1;                                                          \
        /* shuffles in every lane; the edge lanes then pick their loaded values */                             \
        const T su0_ = __shfl_up(ec0, 1, 64), sd0_ = __shfl_down(ec0, 1, 64), st0_ = __shfl_down((D).tx0, 1, 64); \
        IBM_RC_CELL((D).tx0, lane == 63 ? (D).txR0 : st0_, (D).ty0, TWO ? (D).ty1 : (D).tyh, tzc0, (D).tzn0,     \
                    lane == 0 ? (D).eL0 : su0_, lane == 63 ? (D).eR0 : sd0_, (D).ylo, TWO ? ec1 : (D).yhi, em0,  \
                    (D).en0, ec0, hy00, hy10, (D).r0, vxy0, (D).w2, (D).a0 != 0);                              \
        if constexpr (TWO) {                                                                                   \
            const T su1_ = __shfl_up(ec1, 1, 64), sd1_ = __shfl_down(ec1, 1, 64),                              \
                    st1_ = __shfl_down((D).tx1, 1, 64);                                                        \
            IBM_RC_CELL((D).tx1, lane == 63 ? (D).txR1 : st1_, (D).ty1, (D).tyh, tzc1, (D).tzn1,               \
                        lane == 0 ? (D).eL1 : su1_, lane == 63 ? (D).eR1 : sd1_, ec0, (D).yhi, em1, (D).en1, ec1, \
                        hy01, hy11, (D).r1, vxy1, (D).w2, (D).a1 != 0);                                        \
        }                                                                                                      \
        if (k_ + 1 == kend) { /* the coarse plane K is complete */                                            \
            T s = __shfl(acc, ca, 64);                                                                         \
            const T s2 = __shfl(acc, cb, 64);                                                                  \
            if (pair) s = s + s2;                                                                              \
            if (own) {                                                                                         \
                const int64_t cid = ((int64_t)K * C.n[1] + J) * C.n[0] + I0 + lane;                            \
                C.R[cid] = s;                                                                                  \
                C.e[cid] = T(0);                                                                               \
                psum += (double)s;                                                                             \
            }                                                                                                  \
            acc = T(0);                                                                                        \
            ++K;                                                                                               \
            kend = M.cs[2][min(K + 1, K1)];                                                                    \
        }                                                                                                      \
        em0 = ec0;                                                                                             \
        ec0 = (D).en0;                                                                                         \
        tzc0 = (D).tzn0;                                                                                       \
        em1 = ec1;                                                                                             \
        ec1 = (D).en1;                                                                                         \
        tzc1 = (D).tzn1;                                                                                       \
    }
    RCPlane<T> qa = ld(k0), qb;
    for (int k = k0; k < k1; k += 2) {
        qb = ld(k + 1);
        IBM_RC_PLANE(qa, k);
        if (k + 1 >= k1) break;
        qa = ld(k + 2);
        IBM_RC_PLANE(qb, k + 1);
    }
#undef IBM_RC_PLANE
#undef IBM_RC_CELL
    return psum;
}

template <typename T>
__global__ void __launch_bounds__(RM_NT)
    k_resrestrictC_map(Coarse<T> L, Coarse<T> C, ChildMap M, RowTiles t, double *partials) {
    const int lane = (int)threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const T mu = (T)(*L.mu);
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
            psum += resrestrict_row<T, true>(L, C, M, mu, I0, I1, J, K0, K1, lane);
        else
            psum += resrestrict_row<T, false>(L, C, M, mu, I0, I1, J, K0, K1, lane);
    }
    __shared__ double sh[RM_NT / 64];
    const double tot = block_sum<RM_NT>(psum, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// The same for a level pair with every axis halved: a thread per coarse cell loads its
// 2 x 2 x 2 children as x pairs (one vector access per row and array), the neighbour layers
// around the block and the high-face transmissibilities once, all before any arithmetic,
// instead of rebuilding each child's stencil from scalar loads.  Per child the operations
// are those of coarse_stencil, and the children are summed in the same order (x fastest,
// then y, then z), so the result is bitwise that of k_resrestrictC.
template <typename T>
__global__ void __launch_bounds__(256) k_resrestrictC8(Coarse<T> L, Coarse<T> C, double *partials) {
    using V = typename Pair2<T>::type;
    __shared__ double sh[4];
    const int64_t NC = (int64_t)C.n[0] * C.n[1] * C.n[2];
    const int64_t cid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double Rsum = 0.0;
    if (cid < NC) {
        int I, J, K;
        unflatten(cid, C.n[0], C.n[1], I, J, K);
        const int n0 = L.n[0], n1 = L.n[1], n2 = L.n[2];
        const int64_t sy = n0, sz = (int64_t)n0 * n1;
        const int i0 = 2 * I, j0 = 2 * J, k0 = 2 * K;
        const int im = max(i0 - 1, 0), ip = min(i0 + 2, n0 - 1);
        const int jm = max(j0 - 1, 0), jp = min(j0 + 2, n1 - 1);
        const int km = max(k0 - 1, 0), kp = min(k0 + 2, n2 - 1);
        auto at = [&](int j, int k) -> int64_t { return (int64_t)k * sz + (int64_t)j * sy; };
        V E[2][2], RR[2][2], X[2][2], Y[2][2], Z[2][2];
        T Exm[2][2], Exp[2][2], Xh[2][2];
        uint16_t A[2][2];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int64_t r = at(j0 + b, k0 + c);
                E[b][c] = *reinterpret_cast<const V *>(L.e + r + i0);
                RR[b][c] = *reinterpret_cast<const V *>(L.R + r + i0);
                X[b][c] = *reinterpret_cast<const V *>(L.Tl[0] + r + i0);
                Y[b][c] = *reinterpret_cast<const V *>(L.Tl[1] + r + i0);
                Z[b][c] = *reinterpret_cast<const V *>(L.Tl[2] + r + i0);
                A[b][c] = *reinterpret_cast<const uint16_t *>(L.active + r + i0);
                Exm[b][c] = L.e[r + im];
                Exp[b][c] = L.e[r + ip];
                Xh[b][c] = L.Tl[0][r + ip];
            }
        V EYm[2], EYp[2], YH[2], EZm[2], EZp[2], ZH[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            EYm[q] = *reinterpret_cast<const V *>(L.e + at(jm, k0 + q) + i0);
            EYp[q] = *reinterpret_cast<const V *>(L.e + at(jp, k0 + q) + i0);
            YH[q] = *reinterpret_cast<const V *>(L.Tl[1] + at(jp, k0 + q) + i0);
            EZm[q] = *reinterpret_cast<const V *>(L.e + at(j0 + q, km) + i0);
            EZp[q] = *reinterpret_cast<const V *>(L.e + at(j0 + q, kp) + i0);
            ZH[q] = *reinterpret_cast<const V *>(L.Tl[2] + at(j0 + q, kp) + i0);
        }
        const T mu = (T)(*L.mu);
        T R = 0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int i = i0 + a, j = j0 + b, k = k0 + c;
                    const T ev = a ? E[b][c].y : E[b][c].x;
                    const T txm = a ? X[b][c].y : X[b][c].x;
                    const T txp = a ? ((i < n0 - 1) ? Xh[b][c] : T(0)) : X[b][c].y;
                    const T tym = a ? Y[b][c].y : Y[b][c].x;
                    const T typ = b ? ((j < n1 - 1) ? (a ? YH[c].y : YH[c].x) : T(0)) : (a ? Y[1][c].y : Y[1][c].x);
                    const T tzm = a ? Z[b][c].y : Z[b][c].x;
                    const T tzp = c ? ((k < n2 - 1) ? (a ? ZH[b].y : ZH[b].x) : T(0)) : (a ? Z[b][1].y : Z[b][1].x);
                    const T exm = a ? E[b][c].x : Exm[b][c];
                    const T exp = a ? Exp[b][c] : E[b][c].y;
                    const T eym = b ? (a ? E[0][c].y : E[0][c].x) : (a ? EYm[c].y : EYm[c].x);
                    const T eyp = b ? (a ? EYp[c].y : EYp[c].x) : (a ? E[1][c].y : E[1][c].x);
                    const T ezm = c ? (a ? E[b][0].y : E[b][0].x) : (a ? EZm[b].y : EZm[b].x);
                    const T ezp = c ? (a ? EZp[b].y : EZp[b].x) : (a ? E[b][1].y : E[b][1].x);
                    T sm = 0;
                    sm = sm + (i > 0 ? txm * exm : T(0));
                    sm = sm + (i < n0 - 1 ? txp * exp : T(0));
                    sm = sm + (j > 0 ? tym * eym : T(0));
                    sm = sm + (j < n1 - 1 ? typ * eyp : T(0));
                    sm = sm + (k > 0 ? tzm * ezm : T(0));
                    sm = sm + (k < n2 - 1 ? tzp * ezp : T(0));
                    T d = txm + txp;
                    d = d + tym;
                    d = d + typ;
                    d = d + tzm;
                    d = d + tzp;
                    const T vol = (L.w[0][i] * L.w[1][j]) * L.w[2][k];
                    const T rv = a ? RR[b][c].y : RR[b][c].x;
                    const T rc = (rv - vol * mu) - (sm - d * ev);
                    const bool act = ((A[b][c] >> (8 * a)) & 0xff) != 0;
                    if (act) R += rc;
                }
        C.R[cid] = R;
        C.e[cid] = T(0);
        Rsum = (double)R;
    }
    double s = block_sum<256>(Rsum, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// mu = sum(partials) / vol  (fixed order)
__global__ void k_finalize_mu(const double *partials, int n, const double *vol, double *mu) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) s += partials[q];
    s = block_sum<256>(s, sh, threadIdx.x);
    if (threadIdx.x == 0) *mu = (*vol > 0.0) ? s / *vol : 0.0;
}

// =======================================================================================
// coarse levels: red-black GS on  sum_F T_F (e_NB - e_C) = R_C - V_C mu
// =======================================================================================

// one colour of a red-black sweep of a coarse level: a thread per cell of that colour (in
// each x pair of a row exactly one cell has the colour), every load issued before the
// activity test
template <typename T>
__global__ void k_sweepC(Coarse<T> L, int colour) {
    const int hx = (L.n[0] + 1) >> 1;
    const int64_t npair = (int64_t)hx * L.n[1] * L.n[2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npair) return;
    int P, J, K;
    unflatten(t, hx, L.n[1], P, J, K);
    const int I = 2 * P + ((J + K + colour) & 1);
    if (I >= L.n[0]) return;
    const int64_t id = ((int64_t)K * L.n[1] + J) * L.n[0] + I;
    const uint8_t act = L.active[id];
    T num, diag;
    coarse_stencil(L, L.e, I, J, K, id, num, diag);
    const T vol = (L.w[0][I] * L.w[1][J]) * L.w[2][K];
    const T r = L.R[id];
    if (act && diag > T(0)) L.e[id] = (num - (r - vol * (T)(*L.mu))) / diag;
}


// coarsest level in one workgroup: e = 0 (set by the restriction), n sweeps, then removal
// of the volume-weighted mean over the active cells
// nsweeps red-black sweeps of a level of at most SMALL_LEVEL cells in one workgroup of 1024
// threads: each thread keeps the coefficients of up to SMALL_CPT cells in registers and the
// iterate lives in LDS, so a colour costs one LDS pass and one barrier instead of a launch.
// remove_mean != 0 (coarsest level): afterwards subtract the volume-weighted mean over the
// active cells.  The arithmetic of every cell is that of k_sweepC.
constexpr int SMALL_CPT = 4, SMALL_LEVEL = 1024 * SMALL_CPT;
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_smallC(Coarse<T> L, int nsweeps, const double *vol, int remove_mean) {
    __shared__ double sh[NT / 64];
    __shared__ T es[NT * SMALL_CPT];
    __shared__ double mean_s;
    const int NC = L.n[0] * L.n[1] * L.n[2];
    const int sy = L.n[0], sz = L.n[0] * L.n[1];
    const T mu = (T)(*L.mu);
    // per cell: bit 0 live, 1 active, 2 colour, 3..8 neighbour present at -x,+x,-y,+y,-z,+z
    unsigned fl[SMALL_CPT];
    T txm[SMALL_CPT], txp[SMALL_CPT], tym[SMALL_CPT], typ[SMALL_CPT], tzm[SMALL_CPT], tzp[SMALL_CPT];
    T rhs[SMALL_CPT], dg[SMALL_CPT];
#pragma unroll
    for (int c = 0; c < SMALL_CPT; ++c) {
        const int id = (int)threadIdx.x + NT * c;
        const bool live = id < NC;
        const int idc = live ? id : 0;
        const int I = idc % L.n[0], J = (idc / L.n[0]) % L.n[1], K = idc / sz;
        const bool hx0 = I > 0, hx1 = I < L.n[0] - 1, hy0 = J > 0, hy1 = J < L.n[1] - 1, hz0 = K > 0,
                   hz1 = K < L.n[2] - 1;
        fl[c] = (live ? 1u : 0u) | ((live && L.active[idc] != 0) ? 2u : 0u) | ((unsigned)((I + J + K) & 1) << 2) |
                (hx0 ? 8u : 0u) | (hx1 ? 16u : 0u) | (hy0 ? 32u : 0u) | (hy1 ? 64u : 0u) | (hz0 ? 128u : 0u) |
                (hz1 ? 256u : 0u);
        txm[c] = L.Tl[0][idc];
        txp[c] = hx1 ? L.Tl[0][idc + 1] : T(0);
        tym[c] = L.Tl[1][idc];
        typ[c] = hy1 ? L.Tl[1][idc + sy] : T(0);
        tzm[c] = L.Tl[2][idc];
        tzp[c] = hz1 ? L.Tl[2][idc + sz] : T(0);
        const T v = (L.w[0][I] * L.w[1][J]) * L.w[2][K];
        rhs[c] = L.R[idc] - v * mu;
        T d = txm[c] + txp[c];
        d = d + tym[c];
        d = d + typ[c];
        d = d + tzm[c];
        d = d + tzp[c];
        dg[c] = d;
        if (live) es[id] = L.e[id];
    }
    __syncthreads();
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (unsigned col = 0; col < 2; ++col) {
#pragma unroll
            for (int c = 0; c < SMALL_CPT; ++c) {
                const int id = (int)threadIdx.x + NT * c;
                const unsigned f = fl[c];
                if ((f & 2u) && ((f >> 2) & 1u) == col && dg[c] > T(0)) {
                    T num = 0;
                    num = num + ((f & 8u) ? txm[c] * es[id - 1] : T(0));
                    num = num + ((f & 16u) ? txp[c] * es[id + 1] : T(0));
                    num = num + ((f & 32u) ? tym[c] * es[id - sy] : T(0));
                    num = num + ((f & 64u) ? typ[c] * es[id + sy] : T(0));
                    num = num + ((f & 128u) ? tzm[c] * es[id - sz] : T(0));
                    num = num + ((f & 256u) ? tzp[c] * es[id + sz] : T(0));
                    es[id] = (num - rhs[c]) / dg[c];
                }
            }
            __syncthreads();
        }
    }
    double mean = 0.0;
    if (remove_mean) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < SMALL_CPT; ++c) {
            const int id = (int)threadIdx.x + NT * c;
            if (fl[c] & 2u) {
                const int I = id % L.n[0], J = (id / L.n[0]) % L.n[1], K = id / sz;
                acc += (double)((L.w[0][I] * L.w[1][J]) * L.w[2][K]) * (double)es[id];
            }
        }
        const double tot = block_sum<NT>(acc, sh, threadIdx.x);
        if (threadIdx.x == 0) mean_s = (*vol > 0.0) ? tot / *vol : 0.0;
        __syncthreads();
        mean = mean_s;
    }
#pragma unroll
    for (int c = 0; c < SMALL_CPT; ++c) {
        const int id = (int)threadIdx.x + NT * c;
        if (fl[c] & 1u) L.e[id] = (remove_mean && (fl[c] & 2u)) ? es[id] - (T)mean : es[id];
    }
}

// ---------------------------------------------------------------------------------------
// The tail of the V-cycle in one workgroup: every level from the first one with at most
// SMALL_LEVEL cells down to the coarsest.  Pre-smoothing, residual and restriction, the
// coarsest sweeps with mean removal, prolongation and post-smoothing of these levels run
// with the iterates in LDS, separated by workgroup barriers; right-hand sides and
// coefficients stay in global memory (they are small and cache-resident).  Per cell the
// arithmetic is that of k_sweepC / k_resrestrictC / k_prolongC / k_coarsest.
// ---------------------------------------------------------------------------------------
constexpr int TAIL_MAX = 8, TAIL_NT = 1024, TAIL_E = 2 * SMALL_LEVEL;

template <typename T>
struct TailArgs {
    int nl;                   // tail levels; index 0 is the first, nl - 1 the coarsest
    Coarse<T> L[TAIL_MAX];    // level views (e and R in global memory)
    ProlongTab P[TAIL_MAX];   // P[q]: table of tail level q from level q + 1
    const int *cs[TAIL_MAX][3];  // cs[q]: children starts of tail level q + 1 in level q
    int off[TAIL_MAX];        // offset of each level's iterate in LDS
    const double *vol[TAIL_MAX];
    double *mu[TAIL_MAX];
    const double *partials;   // restriction partials of tail level 0
    int nparts, nu1, nu2, ncoarse;
};

template <typename T>
__device__ __forceinline__ void tail_ijk(const Coarse<T> &L, int id, int &I, int &J, int &K) {
    I = id % L.n[0];
    J = (id / L.n[0]) % L.n[1];
    K = id / (L.n[0] * L.n[1]);
}

// prolongation into a tail level from the next coarser one (both held in LDS)
template <typename T>
struct TailUp {
    const T *ec;           // coarser iterate
    const uint8_t *cact;   // coarser active flags
    int cn0, cn1;          // coarser x and y sizes
    const ProlongTab *P;   // table of this level from the coarser one
};

// One tail level in one workgroup: optional prolongation from the coarser level (up leg),
// ns red-black sweeps on the LDS iterate es, optional removal of the volume-weighted active
// mean (coarsest level), optional residual into rs (down leg).  A thread owns cells
// tid + TAIL_NT c and keeps their coefficients in registers through all three phases; the
// sweep multiplies by the reciprocal of the diagonal.  act: the level's active flags (LDS).
template <typename T>
__device__ void tail_smooth(const Coarse<T> &L, T *es, const uint8_t *act, int ns, T mu, const double *vol,
                            int remove_mean, const TailUp<T> *up, T *rs, double *sh, double *mean_s) {
    const int NC = L.n[0] * L.n[1] * L.n[2];
    const int sy = L.n[0], sz = L.n[0] * L.n[1];
    unsigned fl[SMALL_CPT];
    T txm[SMALL_CPT], txp[SMALL_CPT], tym[SMALL_CPT], typ[SMALL_CPT], tzm[SMALL_CPT], tzp[SMALL_CPT];
    T rhs[SMALL_CPT], inv[SMALL_CPT];
#pragma unroll
    for (int c = 0; c < SMALL_CPT; ++c) {
        const int id = (int)threadIdx.x + TAIL_NT * c;
        const bool live = id < NC;
        const int idc = live ? id : 0;
        int I, J, K;
        tail_ijk(L, idc, I, J, K);
        const bool hx1 = I < L.n[0] - 1, hy1 = J < L.n[1] - 1, hz1 = K < L.n[2] - 1;
        fl[c] = (live ? 1u : 0u) | ((live && act[idc] != 0) ? 2u : 0u) | ((unsigned)((I + J + K) & 1) << 2) |
                (I > 0 ? 8u : 0u) | (hx1 ? 16u : 0u) | (J > 0 ? 32u : 0u) | (hy1 ? 64u : 0u) | (K > 0 ? 128u : 0u) |
                (hz1 ? 256u : 0u);
        txm[c] = L.Tl[0][idc];
        txp[c] = hx1 ? L.Tl[0][idc + 1] : T(0);
        tym[c] = L.Tl[1][idc];
        typ[c] = hy1 ? L.Tl[1][idc + sy] : T(0);
        tzm[c] = L.Tl[2][idc];
        tzp[c] = hz1 ? L.Tl[2][idc + sz] : T(0);
        const T v = (L.w[0][I] * L.w[1][J]) * L.w[2][K];
        rhs[c] = L.R[idc] - v * mu;
        T d = txm[c] + txp[c];
        d = d + tym[c];
        d = d + typ[c];
        d = d + tzm[c];
        d = d + tzp[c];
        inv[c] = d > T(0) ? T(1) / d : T(0);
        if (up && (fl[c] & 2u)) {
            // trilinear from the 2 x 2 x 2 nearest coarser centres, or the parent's value when
            // one of them is inactive (the parent is the first contributor on every axis)
            const ProlongTab &P = *up->P;
            const int ix[2] = {P.lo[0][I], P.hi[0][I]}, iy[2] = {P.lo[1][J], P.hi[1][J]},
                      iz[2] = {P.lo[2][K], P.hi[2][K]};
            const double tx = P.t[0][I], ty = P.t[1][J], tz = P.t[2][K];
            const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
            const int nx_ = (ix[0] == ix[1]) ? 1 : 2, ny_ = (iy[0] == iy[1]) ? 1 : 2, nz_ = (iz[0] == iz[1]) ? 1 : 2;
            bool all = true;
            double sv = 0.0;
            for (int cz = 0; cz < nz_; ++cz)
                for (int b = 0; b < ny_; ++b)
                    for (int a = 0; a < nx_; ++a) {
                        const int cid = (iz[cz] * up->cn1 + iy[b]) * up->cn0 + ix[a];
                        if (!up->cact[cid]) all = false;
                        sv += (wx[a] * wy[b]) * wz[cz] * (double)up->ec[cid];
                    }
            if (!all) sv = (double)up->ec[(iz[0] * up->cn1 + iy[0]) * up->cn0 + ix[0]];
            es[id] = (T)((double)es[id] + sv);  // the thread's own cell: no other thread reads it yet
        }
    }
    if (up) __syncthreads();
    // a level that the first wave holds alone (cells of a thread are tid + TAIL_NT c, so with
    // NC <= 64 only lanes of wave 0 own cells) is swept by that wave in registers, one cell
    // per lane: the neighbours' values arrive by lane permutation (their lanes are the cell
    // offsets -1, +1, -sy, +sy, -sz, +sz, clamped into the wave; a missing neighbour is masked
    // by its flag), so a colour costs one permute round trip and no LDS store or barrier
    const bool one_wave = NC <= 64;
    if (one_wave) {
        if (threadIdx.x < 64) {
            const int id = (int)threadIdx.x;
            const unsigned f = fl[0];
            const bool upd = (f & 2u) && inv[0] > T(0);
            const unsigned mycol = (f >> 2) & 1u;
            const int lxm = max(id - 1, 0), lxp = min(id + 1, 63), lym = max(id - sy, 0), lyp = min(id + sy, 63),
                      lzm = max(id - sz, 0), lzp = min(id + sz, 63);
            T x = (f & 1u) ? es[id] : T(0);
            for (int sw = 0; sw < ns; ++sw) {
                for (unsigned col = 0; col < 2; ++col) {
                    const T xm = __shfl(x, lxm, 64), xp = __shfl(x, lxp, 64), ym = __shfl(x, lym, 64),
                            yp = __shfl(x, lyp, 64), zm = __shfl(x, lzm, 64), zp = __shfl(x, lzp, 64);
                    if (upd && mycol == col) {
                        T num = 0;
                        num = num + ((f & 8u) ? txm[0] * xm : T(0));
                        num = num + ((f & 16u) ? txp[0] * xp : T(0));
                        num = num + ((f & 32u) ? tym[0] * ym : T(0));
                        num = num + ((f & 64u) ? typ[0] * yp : T(0));
                        num = num + ((f & 128u) ? tzm[0] * zm : T(0));
                        num = num + ((f & 256u) ? tzp[0] * zp : T(0));
                        x = (num - rhs[0]) * inv[0];
                    }
                }
            }
            if (f & 1u) es[id] = x;
        }
        __syncthreads();
    } else {
        for (int sw = 0; sw < ns; ++sw) {
            for (unsigned col = 0; col < 2; ++col) {
#pragma unroll
                for (int c = 0; c < SMALL_CPT; ++c) {
                    const int id = (int)threadIdx.x + TAIL_NT * c;
                    const unsigned f = fl[c];
                    if ((f & 2u) && ((f >> 2) & 1u) == col && inv[c] > T(0)) {
                        T num = 0;
                        num = num + ((f & 8u) ? txm[c] * es[id - 1] : T(0));
                        num = num + ((f & 16u) ? txp[c] * es[id + 1] : T(0));
                        num = num + ((f & 32u) ? tym[c] * es[id - sy] : T(0));
                        num = num + ((f & 64u) ? typ[c] * es[id + sy] : T(0));
                        num = num + ((f & 128u) ? tzm[c] * es[id - sz] : T(0));
                        num = num + ((f & 256u) ? tzp[c] * es[id + sz] : T(0));
                        es[id] = (num - rhs[c]) * inv[c];
                    }
                }
                __syncthreads();
            }
        }
    }
    if (remove_mean) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < SMALL_CPT; ++c) {
            const int id = (int)threadIdx.x + TAIL_NT * c;
            if (fl[c] & 2u) {
                int I, J, K;
                tail_ijk(L, id, I, J, K);
                acc += (double)((L.w[0][I] * L.w[1][J]) * L.w[2][K]) * (double)es[id];
            }
        }
        const double tot = block_sum<TAIL_NT>(acc, sh, threadIdx.x);
        if (threadIdx.x == 0) *mean_s = (*vol > 0.0) ? tot / *vol : 0.0;
        __syncthreads();
        const T m = (T)*mean_s;
#pragma unroll
        for (int c = 0; c < SMALL_CPT; ++c) {
            const int id = (int)threadIdx.x + TAIL_NT * c;
            if (fl[c] & 2u) es[id] -= m;
        }
        __syncthreads();
    }
    if (rs) {
        // residual (R - V mu) - (A e) of the active cells, 0 elsewhere
#pragma unroll
        for (int c = 0; c < SMALL_CPT; ++c) {
            const int id = (int)threadIdx.x + TAIL_NT * c;
            const unsigned f = fl[c];
            if (!(f & 1u)) continue;
            T r = T(0);
            if (f & 2u) {
                T sm = 0;
                sm = sm + ((f & 8u) ? txm[c] * es[id - 1] : T(0));
                sm = sm + ((f & 16u) ? txp[c] * es[id + 1] : T(0));
                sm = sm + ((f & 32u) ? tym[c] * es[id - sy] : T(0));
                sm = sm + ((f & 64u) ? typ[c] * es[id + sy] : T(0));
                sm = sm + ((f & 128u) ? tzm[c] * es[id - sz] : T(0));
                sm = sm + ((f & 256u) ? tzp[c] * es[id + sz] : T(0));
                T d = txm[c] + txp[c];
                d = d + tym[c];
                d = d + typ[c];
                d = d + tzm[c];
                d = d + tzp[c];
                r = rhs[c] - (sm - d * es[id]);
            }
            rs[id] = r;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(TAIL_NT) k_tailC(TailArgs<T> A) {
    __shared__ T es[TAIL_E];           // iterates of all tail levels
    __shared__ T rs[SMALL_LEVEL];      // residual of the level being restricted
    __shared__ uint8_t acts[TAIL_E];   // active flags of all tail levels
    __shared__ double sh[TAIL_NT / 64];
    __shared__ double mean_s, mu_s[TAIL_MAX];
    const int tid = threadIdx.x;
    {   // mu of the first tail level from the restriction partials; activity of every level
        double a = 0.0;
        for (int q = tid; q < A.nparts; q += TAIL_NT) a += A.partials[q];
        for (int q = 0; q < A.nl; ++q) {
            const int n = A.L[q].n[0] * A.L[q].n[1] * A.L[q].n[2];
            for (int id = tid; id < n; id += TAIL_NT) acts[A.off[q] + id] = A.L[q].active[id];
        }
        const double tot = block_sum<TAIL_NT>(a, sh, tid);
        if (tid == 0) {
            const double m = (*A.vol[0] > 0.0) ? tot / *A.vol[0] : 0.0;
            mu_s[0] = m;
            *A.mu[0] = m;
        }
        const int n0 = A.L[0].n[0] * A.L[0].n[1] * A.L[0].n[2];
        for (int id = tid; id < n0; id += TAIL_NT) es[A.off[0] + id] = T(0);
        __syncthreads();
    }
    // down: smooth and form the residual, restrict it (inactive cells hold a zero residual)
    for (int q = 0; q + 1 < A.nl; ++q) {
        const Coarse<T> &L = A.L[q];
        tail_smooth<T>(L, es + A.off[q], acts + A.off[q], A.nu1, (T)mu_s[q], A.vol[q], 0, nullptr, rs, sh, &mean_s);
        const Coarse<T> &C = A.L[q + 1];
        const int *const *cs = A.cs[q];
        const int NCC = C.n[0] * C.n[1] * C.n[2];
        double psum = 0.0;
        for (int cid = tid; cid < NCC; cid += TAIL_NT) {
            int I, J, K;
            tail_ijk(C, cid, I, J, K);
            T R = 0;
            for (int k = cs[2][K]; k < cs[2][K + 1]; ++k)
                for (int j = cs[1][J]; j < cs[1][J + 1]; ++j)
                    for (int i = cs[0][I]; i < cs[0][I + 1]; ++i) R += rs[(k * L.n[1] + j) * L.n[0] + i];
            C.R[cid] = R;
            es[A.off[q + 1] + cid] = T(0);
            psum += (double)R;
        }
        const double tot = block_sum<TAIL_NT>(psum, sh, tid);
        if (tid == 0) {
            const double m = (*A.vol[q + 1] > 0.0) ? tot / *A.vol[q + 1] : 0.0;
            mu_s[q + 1] = m;
            *A.mu[q + 1] = m;
        }
        __syncthreads();
    }
    // coarsest
    {
        const int q = A.nl - 1;
        tail_smooth<T>(A.L[q], es + A.off[q], acts + A.off[q], A.ncoarse, (T)mu_s[q], A.vol[q], 1, nullptr, nullptr,
                       sh, &mean_s);
    }
    // up: prolong and smooth
    for (int q = A.nl - 2; q >= 0; --q) {
        TailUp<T> up;
        up.ec = es + A.off[q + 1];
        up.cact = acts + A.off[q + 1];
        up.cn0 = A.L[q + 1].n[0];
        up.cn1 = A.L[q + 1].n[1];
        up.P = &A.P[q];
        tail_smooth<T>(A.L[q], es + A.off[q], acts + A.off[q], A.nu2, (T)mu_s[q], A.vol[q], 0, &up, nullptr, sh,
                       &mean_s);
    }
    // the first tail level's correction goes back to global memory for the prolongation above
    {
        const Coarse<T> &L = A.L[0];
        const int NC = L.n[0] * L.n[1] * L.n[2];
        for (int id = tid; id < NC; id += TAIL_NT) L.e[id] = es[A.off[0] + id];
    }
}

// the smallest workgroup that holds the level (one wave for the tiny levels, where barriers
// are nearly free)
template <typename T>
static void launch_smallC(const Coarse<T> &L, int64_t ncell, int nsweeps, const double *vol, int remove_mean,
                          hipStream_t s) {
    if (ncell <= 64 * SMALL_CPT)
        hipLaunchKernelGGL((k_smallC<T, 64>), dim3(1), dim3(64), 0, s, L, nsweeps, vol, remove_mean);
    else if (ncell <= 256 * SMALL_CPT)
        hipLaunchKernelGGL((k_smallC<T, 256>), dim3(1), dim3(256), 0, s, L, nsweeps, vol, remove_mean);
    else
        hipLaunchKernelGGL((k_smallC<T, 1024>), dim3(1), dim3(1024), 0, s, L, nsweeps, vol, remove_mean);
}

template <typename T>
__global__ void __launch_bounds__(1024) k_coarsest(Coarse<T> L, int nsweeps, const double *vol) {
    __shared__ double sh[16];
    const int64_t NC = (int64_t)L.n[0] * L.n[1] * L.n[2];
    const T mu = (T)(*L.mu);
    for (int s = 0; s < nsweeps; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t id = threadIdx.x; id < NC; id += 1024) {
                int I, J, K;
                unflatten(id, L.n[0], L.n[1], I, J, K);
                if (((I + J + K) & 1) != colour || !L.active[id]) continue;
                T num, diag;
                coarse_stencil(L, L.e, I, J, K, id, num, diag);
                if (diag > T(0)) {
                    const T v = (L.w[0][I] * L.w[1][J]) * L.w[2][K];
                    L.e[id] = (num - (L.R[id] - v * mu)) / diag;
                }
            }
            __syncthreads();
        }
    }
    double acc = 0.0;
    for (int64_t id = threadIdx.x; id < NC; id += 1024) {
        if (!L.active[id]) continue;
        int I, J, K;
        unflatten(id, L.n[0], L.n[1], I, J, K);
        acc += (double)((L.w[0][I] * L.w[1][J]) * L.w[2][K]) * (double)L.e[id];
    }
    __shared__ double mean;
    double tot = block_sum<1024>(acc, sh, threadIdx.x);
    if (threadIdx.x == 0) mean = (*vol > 0.0) ? tot / *vol : 0.0;
    __syncthreads();
    const T m = (T)mean;
    for (int64_t id = threadIdx.x; id < NC; id += 1024)
        if (L.active[id]) L.e[id] -= m;
}

// prolongation with correction on a coarse level l from l+1: e_l += P e_{l+1} on active
// cells (trilinear in physical coordinates, or the parent's value when a contributing
// coarse cell is inactive)
template <typename T>
__device__ __forceinline__ double prolong_value(const Coarse<T> &C, const ProlongTab &P, int i, int j, int k) {
    const int ix[2] = {P.lo[0][i], P.hi[0][i]}, iy[2] = {P.lo[1][j], P.hi[1][j]}, iz[2] = {P.lo[2][k], P.hi[2][k]};
    const double tx = P.t[0][i], ty = P.t[1][j], tz = P.t[2][k];
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
    const bool two[3] = {ix[0] != ix[1], iy[0] != iy[1], iz[0] != iz[1]};
    bool all = true;
    double s = 0.0;
    // fixed 2x2x2 loop (a second contributor that coincides with the first is skipped),
    // unrolled so that all coarse loads are issued together
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const bool ok = (a == 0 || two[0]) && (b == 0 || two[1]) && (c == 0 || two[2]);
                const int64_t cid = ((int64_t)iz[c] * C.n[1] + iy[b]) * C.n[0] + ix[a];
                const bool act = C.active[cid] != 0;
                const double term = (wx[a] * wy[b]) * wz[c] * (double)C.e[cid];
                if (ok) {
                    if (!act) all = false;
                    s += term;
                }
            }
    if (!all) {  // the parent: the first contributor on every axis
        const int pi = P.lo[0][i], pj = P.lo[1][j], pk = P.lo[2][k];
        s = (double)C.e[((int64_t)pk * C.n[1] + pj) * C.n[0] + pi];
    }
    return s;
}

template <typename T>
__global__ void k_prolongC(Coarse<T> L, Coarse<T> C, ProlongTab P) {
    const int64_t N = (int64_t)L.n[0] * L.n[1] * L.n[2];
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N || !L.active[id]) return;
    int i, j, k;
    unflatten(id, L.n[0], L.n[1], i, j, k);
    L.e[id] = (T)((double)L.e[id] + prolong_value(C, P, i, j, k));
}

// The same for any child map, on large levels, with the coarser values staged in LDS: the
// tiling and the ring of coarser planes of the level-0 prolongation k_prolong0_lds (a
// workgroup's 64 x 4 columns draw on at most PLC_CW x PLC_CH coarser columns; each coarser
// plane it needs is read once, values and activity, the next one while the current plane is
// computed).  Per cell the terms, their order and the fallback to the parent are those of
// prolong_value, so the result is bitwise that of k_prolongC.
constexpr int PLC_CW = 68, PLC_CH = 6, PLC_RING = 4, PLC_PER = (PLC_CW * PLC_CH + ZM_NT - 1) / ZM_NT;
constexpr int64_t PROLONG_LDS_MIN_CELLS = 1 << 18;

template <typename T>
__global__ void __launch_bounds__(ZM_NT) k_prolongC_lds(Coarse<T> L, Coarse<T> C, ProlongTab P, ZTiles t) {
    __shared__ T ec[PLC_RING][PLC_CH][PLC_CW];
    __shared__ uint8_t ca[PLC_RING][PLC_CH][PLC_CW];
    const ZPos z = zpos(t, L.n[2]);
    if (!z.live) return;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const bool in = z.i < nx && z.j < ny;
    const int ic = min(z.i, nx - 1), jc = min(z.j, ny - 1);
    const int64_t plane = (int64_t)nx * ny, rowoff = (int64_t)jc * nx + ic;
    // the tile's coarser window (tables are monotone: lo non-decreasing, hi = lo or lo +- 1)
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
    // coarser values and activity this thread stages for one coarser plane
    auto cload = [=](int K, T (&v)[PLC_PER], uint8_t (&a)[PLC_PER]) {
#pragma unroll
        for (int q = 0; q < PLC_PER; ++q) {
            const int e = (int)threadIdx.x + q * ZM_NT;
            const int r = e / PLC_CW, c = e % PLC_CW;
            const bool ok = r < ch && c < cw;
            const int64_t id = ((int64_t)K * cny + cy0 + min(r, ch - 1)) * cnx + cx0 + min(c, cw - 1);
            v[q] = ok ? C.e[id] : T(0);
            a[q] = ok ? C.active[id] : (uint8_t)0;
        }
    };
    auto cstore = [&](int K, const T (&v)[PLC_PER], const uint8_t (&a)[PLC_PER]) {
#pragma unroll
        for (int q = 0; q < PLC_PER; ++q) {
            const int e = (int)threadIdx.x + q * ZM_NT;
            if (e < PLC_CW * PLC_CH) {
                ec[K & (PLC_RING - 1)][e / PLC_CW][e % PLC_CW] = v[q];
                ca[K & (PLC_RING - 1)][e / PLC_CW][e % PLC_CW] = a[q];
            }
        }
    };
    auto need_hi = [=](int k) { return max(P.lo[2][k], P.hi[2][k]); };
    const int k0 = z.k0, k1 = z.k1;
    int have;  // highest coarser plane staged
    {
        const int a = min(P.lo[2][k0], P.hi[2][k0]), b = need_hi(k0);
        T v[PLC_PER];
        uint8_t av[PLC_PER];
        for (int K = a; K <= b; ++K) {
            cload(K, v, av);
            cstore(K, v, av);
        }
        have = b;
        __syncthreads();
    }
    T ecur = L.e[(int64_t)k0 * plane + rowoff];
    uint8_t acur = L.active[(int64_t)k0 * plane + rowoff];
    for (int k = k0; k < k1; ++k) {
        const int64_t nbase = (int64_t)min(k + 1, nz - 1) * plane + rowoff;
        const T enext = L.e[nbase];
        const uint8_t anext = L.active[nbase];
        // the next plane needs at most one more coarser plane: load it now, stage it after
        const int nb = (k + 1 < nz) ? need_hi(k + 1) : have;
        const bool more = nb > have;
        T v[PLC_PER];
        uint8_t av[PLC_PER];
        if (more) cload(nb, v, av);
        const int iz[2] = {P.lo[2][k], P.hi[2][k]};
        const double tz = P.t[2][k];
        const double wz[2] = {1.0 - tz, tz};
        const bool twoz = iz[0] != iz[1];
        bool all = true;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const bool ok = (a == 0 || twox) && (b == 0 || twoy) && (c == 0 || twoz);
                    const int r = iz[c] & (PLC_RING - 1);
                    const double term = (wx[a] * wy[b]) * wz[c] * (double)ec[r][iy[b]][ix[a]];
                    if (ok) {
                        if (!ca[r][iy[b]][ix[a]]) all = false;
                        s += term;
                    }
                }
        if (!all) s = (double)ec[iz[0] & (PLC_RING - 1)][iy[0]][ix[0]];
        if (in && acur) L.e[(int64_t)k * plane + rowoff] = (T)((double)ecur + s);
        if (more) {
            __syncthreads();  // every thread is done with the slot the new plane goes to
            cstore(nb, v, av);
            have = nb;
        }
        __syncthreads();
        ecur = enext;
        acur = anext;
    }
}

// The same for a level pair with every axis halved: a thread per coarse cell updates its
// 2 x 2 x 2 children, loaded and stored as x pairs.  On a halved axis the first contributor
// of a child is its parent and the second (if any) the parent's neighbour on the child's
// side (the table's hi), so the 3 x 3 x 3 coarse neighbourhood, loaded once, holds every
// contributor.  Per child the terms, their order and the fallback to the parent are those
// of prolong_value, so the result is bitwise that of k_prolongC.
// Smaller levels keep k_prolongC: there the longer load chain of a thread outweighs the
// coalescing (64^3 from 32^3: 6.8 us against 6.4; 128^3 from 64^3: 13 us against 22).
constexpr int64_t PROLONG8_MIN_CELLS = 1 << 19;
template <typename T>
__global__ void __launch_bounds__(256) k_prolongC8(Coarse<T> L, Coarse<T> C, ProlongTab P) {
    using V = typename Pair2<T>::type;
    const int64_t NC = (int64_t)C.n[0] * C.n[1] * C.n[2];
    const int64_t cid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cid >= NC) return;
    int I, J, K;
    unflatten(cid, C.n[0], C.n[1], I, J, K);
    const int m0 = C.n[0], m1 = C.n[1], m2 = C.n[2];
    const int64_t csy = m0, csz = (int64_t)m0 * m1;
    // coarse neighbourhood, indices clamped (a clamped entry is never a contributor)
    double ce[3][3][3];
    uint32_t ca = 0;  // bit (dz*9 + dy*3 + dx): active
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int x = min(max(I + dx - 1, 0), m0 - 1), y = min(max(J + dy - 1, 0), m1 - 1),
                          z = min(max(K + dz - 1, 0), m2 - 1);
                const int64_t q = (int64_t)z * csz + (int64_t)y * csy + x;
                ce[dz][dy][dx] = (double)C.e[q];
                ca |= (C.active[q] != 0 ? 1u : 0u) << (dz * 9 + dy * 3 + dx);
            }
    // per child side (0: low, 1: high) and axis: has a second contributor, and its weight
    const int i0 = 2 * I, j0 = 2 * J, k0 = 2 * K;
    bool two[3][2];
    double tw[3][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        two[0][h] = P.lo[0][i0 + h] != P.hi[0][i0 + h];
        two[1][h] = P.lo[1][j0 + h] != P.hi[1][j0 + h];
        two[2][h] = P.lo[2][k0 + h] != P.hi[2][k0 + h];
        tw[0][h] = P.t[0][i0 + h];
        tw[1][h] = P.t[1][j0 + h];
        tw[2][h] = P.t[2][k0 + h];
    }
    const int n0 = L.n[0];
    const int64_t sy = n0, sz = (int64_t)n0 * L.n[1];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t row = (int64_t)(k0 + c) * sz + (int64_t)(j0 + b) * sy + i0;
            V ev = *reinterpret_cast<const V *>(L.e + row);
            const uint16_t fa = *reinterpret_cast<const uint16_t *>(L.active + row);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double wx[2] = {1.0 - tw[0][a], tw[0][a]}, wy[2] = {1.0 - tw[1][b], tw[1][b]},
                             wz[2] = {1.0 - tw[2][c], tw[2][c]};
                // neighbourhood index of contributor (lo, hi) on each axis: 1 is the parent
                const int hx = a ? 2 : 0, hy = b ? 2 : 0, hz = c ? 2 : 0;
                bool all = true;
                double sv = 0.0;
#pragma unroll
                for (int cz = 0; cz < 2; ++cz)
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                        for (int cx = 0; cx < 2; ++cx) {
                            const bool ok = (cx == 0 || two[0][a]) && (cy == 0 || two[1][b]) && (cz == 0 || two[2][c]);
                            const int ox = cx ? hx : 1, oy = cy ? hy : 1, oz = cz ? hz : 1;
                            const bool act = (ca >> (oz * 9 + oy * 3 + ox)) & 1u;
                            const double term = (wx[cx] * wy[cy]) * wz[cz] * ce[oz][oy][ox];
                            if (ok) {
                                if (!act) all = false;
                                sv += term;
                            }
                        }
                if (!all) sv = ce[1][1][1];
                const bool fine_act = ((fa >> (8 * a)) & 0xff) != 0;
                T &dst = a ? ev.y : ev.x;
                if (fine_act) dst = (T)((double)dst + sv);
            }
            *reinterpret_cast<V *>(L.e + row) = ev;
        }
}

// =======================================================================================
// residual norm on level 0 with the lambda update
//   r = f - S p (fluid rows);  a = r - lambda_k;  partials of sum V a, sum a^2, sum a
//   lambda_{k+1} = lambda_k + delta, delta = sum V a / sum V
//   ||r - lambda_{k+1}||^2 = sum a^2 - 2 delta sum a + delta^2 n_fluid
// WRITE_R32: also store the FP32 right-hand side a for the mixed-precision inner cycle
// =======================================================================================

constexpr int NORM_NT = 256;

template <bool WRITE_R32>
__global__ void __launch_bounds__(NORM_NT) k_norm0(Fine<double> F, const double *__restrict__ p,
                                                   const double *__restrict__ f, const double *__restrict__ lamp,
                                                   float *r32, double *partials) {
    __shared__ double sh[NORM_NT / 64];
    const int64_t N = (int64_t)F.nx * F.ny * F.nz;
    const double lam = *lamp;
    double sv = 0.0, s2 = 0.0, s1 = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * NORM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * NORM_NT) {
        if (F.type[id] != T_FLUID) {
            if (WRITE_R32) r32[id] = 0.0f;
            continue;
        }
        int i, j, k;
        unflatten(id, F.nx, F.ny, i, j, k);
        double num, diag;
        fine_stencil(F, p, i, j, k, id, num, diag);
        const double r = f[id] - (num - diag * p[id]);
        const double a = r - lam;
        sv += ((F.wx[i] * F.wy[j]) * F.wz[k]) * a;
        s2 += a * a;
        s1 += a;
        if (WRITE_R32) r32[id] = (float)a;
    }
    double t;
    t = block_sum<NORM_NT>(sv, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[3 * blockIdx.x] = t;
    t = block_sum<NORM_NT>(s2, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[3 * blockIdx.x + 1] = t;
    t = block_sum<NORM_NT>(s1, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[3 * blockIdx.x + 2] = t;
}

__global__ void k_norm_finalize(const double *partials, int nb, Scalars *sc, double nfluid, int set_ref) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) {
        a += partials[3 * q];
        b += partials[3 * q + 1];
        c += partials[3 * q + 2];
    }
    a = block_sum<256>(a, sh, threadIdx.x);
    b = block_sum<256>(b, sh, threadIdx.x);
    c = block_sum<256>(c, sh, threadIdx.x);
    if (threadIdx.x == 0) {
        const double delta = a / sc->vol[0];
        double q2 = b - 2.0 * delta * c + delta * delta * nfluid;
        if (q2 < 0.0) q2 = 0.0;
        const double nrm = sqrt(q2);
        sc->lambda = sc->lambda + delta;
        sc->delta = delta;
        sc->delta32 = (float)delta;
        sc->norm = nrm;
        if (set_ref) sc->ref = nrm;
        sc->rel = (sc->ref > 0.0) ? nrm / sc->ref : 0.0;
        if (!isfinite(nrm) || !isfinite(sc->lambda)) sc->bad = 1;
    }
}

// reference norm ||f - Vmean(f)|| over fluid cells (two passes: mean, then deviations)
__global__ void __launch_bounds__(NORM_NT) k_fsum(Fine<double> F, const double *__restrict__ f, const double *meanp,
                                                  double *partials, int pass) {
    __shared__ double sh[NORM_NT / 64];
    const int64_t N = (int64_t)F.nx * F.ny * F.nz;
    const double mean = pass ? *meanp : 0.0;
    double s = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * NORM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * NORM_NT) {
        if (F.type[id] != T_FLUID) continue;
        if (pass == 0) {
            int i, j, k;
            unflatten(id, F.nx, F.ny, i, j, k);
            s += ((F.wx[i] * F.wy[j]) * F.wz[k]) * f[id];
        } else {
            const double d = f[id] - mean;
            s += d * d;
        }
    }
    double t = block_sum<NORM_NT>(s, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void k_fsum_finalize(const double *partials, int nb, Scalars *sc, int pass) {
    __shared__ double sh[4];
    double a = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) a += partials[q];
    a = block_sum<256>(a, sh, threadIdx.x);
    if (threadIdx.x == 0) {
        if (pass == 0) sc->vmean = a / sc->vol[0];
        else sc->ref = sqrt(a);
    }
}

// volume-weighted mean of p over fluid cells, then pdst = pcur - mean (fluid, ghost), 0 (dead)
__global__ void __launch_bounds__(NORM_NT) k_psum(Fine<double> F, const double *__restrict__ p, double *partials) {
    __shared__ double sh[NORM_NT / 64];
    const int64_t N = (int64_t)F.nx * F.ny * F.nz;
    double s = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * NORM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * NORM_NT) {
        if (F.type[id] != T_FLUID) continue;
        int i, j, k;
        unflatten(id, F.nx, F.ny, i, j, k);
        s += ((F.wx[i] * F.wy[j]) * F.wz[k]) * p[id];
    }
    double t = block_sum<NORM_NT>(s, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void k_shift(const uint8_t *__restrict__ type, int64_t N, const double *__restrict__ pcur, double *pdst,
                        const Scalars *sc) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const double m = sc->vmean;
    pdst[id] = (type[id] == T_DEAD) ? 0.0 : pcur[id] - m;
}

// =======================================================================================
// launchers
// =======================================================================================

hipError_t sweep0_f64(ibm_grid *g, const double *pin, double *pout, const double *f, const double *lambda,
                      hipStream_t s) {
    return launch_sweep<double>(fine64(g), pin, pout, f, lambda, s);
}

hipError_t refresh_f64(ibm_grid *g, const double *src_ghost, double *dst, hipStream_t s) {
    return launch_refresh<double>(g, src_ghost, dst, g->g_h, s);
}

template <typename T>
__global__ void k_apply0(Fine<T> F, const T *__restrict__ p, T *out) {
    const int64_t N = (int64_t)F.nx * F.ny * F.nz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    if (F.type[id] != T_FLUID) {
        out[id] = T(0);
        return;
    }
    int i, j, k;
    unflatten(id, F.nx, F.ny, i, j, k);
    T num, diag;
    fine_stencil(F, p, i, j, k, id, num, diag);
    out[id] = num - diag * p[id];
}

hipError_t apply0_f64(ibm_grid *g, const double *p, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_apply0<double>, dim3((unsigned)((g->N + 255) / 256)), dim3(256), 0, s, fine64(g), p, out);
    return hipGetLastError();
}

static int nblk(int64_t n, int nt = 256) { return (int)((n + nt - 1) / nt); }

template <typename T>
struct FineOf;
template <>
struct FineOf<double> {
    static Fine<double> get(ibm_grid *g) { return fine64(g); }
};
template <>
struct FineOf<float> {
    static Fine<float> get(ibm_grid *g) { return fine32(g); }
};

// one V(nu1, nu2) cycle in precision T on level 0.
// bufs[0..1]: the two level-0 buffers, *cur: index of the current iterate.
// rhs: level-0 right-hand side; lam: device scalar shift of the right-hand side;
// gh: right-hand sides of the ghost equations (nullptr: homogeneous error equation).
// level-0 sweep, timed by start and end events when profiling is on
template <typename T>
static hipError_t timed_sweep(ibm_grid *g, const Fine<T> &F, const T *pin, T *pout, const T *rhs, const T *lam,
                              hipStream_t s) {
    Prof &P = g->prof;
    const bool rec = P.on && (P.seq++ % P.stride) == 0 && P.used + 2 <= (int)P.ev.size();
    hipError_t e;
    // the runtime records the two events at the kernel's own start and end
    if ((e = launch_sweep<T>(F, pin, pout, rhs, lam, s, rec ? P.ev[P.used] : nullptr,
                             rec ? P.ev[P.used + 1] : nullptr)) != hipSuccess)
        return e;
    if (rec) {
        P.kind[P.used / 2] = (sizeof(T) == 8) ? 0 : 1;
        P.used += 2;
    }
    return hipSuccess;
}

// nsweeps red-black sweeps of coarse level l (more cells than the tail takes): the fused
// out-of-place pass when the level has a second error buffer (the buffers are swapped after
// each sweep, so every later view of the level sees the current one), else two one-colour
// passes in place
template <typename T>
static hipError_t smooth_level(ibm_grid *g, int l, int nsweeps, hipStream_t s) {
    LevelHost &H = g->lev[l];
    if (level_e2<T>(H) != nullptr) {
        for (int q = 0; q < nsweeps; ++q) {
            const hipError_t e = launch_sweepC_fused<T>(coarse_view<T>(g, l), level_e2<T>(H), s);
            if (e != hipSuccess) return e;
            std::swap(level_e<T>(H), level_e2<T>(H));
        }
        return hipSuccess;
    }
    const Coarse<T> L = coarse_view<T>(g, l);
    const int nbh = nblk((int64_t)((H.n[0] + 1) / 2) * H.n[1] * H.n[2]);
    for (int q = 0; q < nsweeps; ++q) {
        hipLaunchKernelGGL(k_sweepC<T>, dim3(nbh), dim3(256), 0, s, L, 0);
        hipLaunchKernelGGL(k_sweepC<T>, dim3(nbh), dim3(256), 0, s, L, 1);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t vcycle_impl(ibm_grid *g, T **bufs, int *cur, const T *rhs, const T *lam, const double *gh,
                              const ibm_solve_opts *o, hipStream_t s, const T *start = nullptr,
                              double *wide = nullptr) {
    // start (requires nu1 > 0): the iterate the first pre-smoothing sweep reads instead of
    // bufs[*cur]; it is only read, and the sweeps continue in bufs
    // wide (FP32 cycle with nu2 > 0): the last post-smoothing sweep and its ghost refresh
    // write the result widened to FP64 there instead of into bufs (that sweep is not timed:
    // it moves 17 bytes per cell, not 13)
    const Fine<T> F = FineOf<T>::get(g);
    hipError_t e;
    for (int q = 0; q < o->nu1; ++q) {
        T *pin = (q == 0 && start) ? const_cast<T *>(start) : bufs[*cur], *pout = bufs[1 - *cur];
        if ((e = timed_sweep<T>(g, F, pin, pout, rhs, lam, s)) != hipSuccess) return e;
        if ((e = launch_refresh<T>(g, pin, pout, gh, s)) != hipSuccess) return e;
        *cur = 1 - *cur;
    }
    if (g->nlev > 1) {
        const int Lc = g->nlev - 1;
        // the tail: every level from the first one with at most SMALL_LEVEL cells down to the
        // coarsest, run by one workgroup, when those levels fit its LDS together (TAIL_E cells)
        // and number at most TAIL_MAX; else the tail starts further down
        int lt = Lc + 1;
        for (int l = 1; l <= Lc; ++l) {
            if (g->lev[l].ncell() > SMALL_LEVEL || Lc - l + 1 > TAIL_MAX) continue;
            int64_t tot = 0;
            for (int q = l; q <= Lc; ++q) tot += g->lev[q].ncell();
            if (tot <= TAIL_E) {
                lt = l;
                break;
            }
        }
        const bool tail = lt <= Lc;
        const int Lb = tail ? lt : Lc;  // levels 1 .. Lb-1 run level by level
        int nparts = 0;                 // restriction partials into level Lb
        {
            Coarse<T> C1 = coarse_view<T>(g, 1);
            if ((e = launch_restrict0<T>(F, bufs[*cur], rhs, lam, C1, child_map(g->lev[1]), g->partials, &nparts,
                                         s)) != hipSuccess)
                return e;
            if (!(tail && lt == 1))
                hipLaunchKernelGGL(k_finalize_mu, dim3(1), dim3(256), 0, s, g->partials, nparts, &g->sc->vol[1],
                                   &g->sc->mu[1]);
        }
        for (int l = 1; l < Lb; ++l) {
            if (g->lev[l].ncell() <= SMALL_LEVEL) {
                if (o->nu1 > 0) launch_smallC<T>(coarse_view<T>(g, l), g->lev[l].ncell(), o->nu1, &g->sc->vol[l], 0, s);
            } else if ((e = smooth_level<T>(g, l, o->nu1, s)) != hipSuccess) {
                return e;
            }
            Coarse<T> L = coarse_view<T>(g, l);  // after the sweeps: the current error buffer
            Coarse<T> C = coarse_view<T>(g, l + 1);
            const ChildMap M = child_map(g->lev[l + 1]);
            int nbc = nblk(g->lev[l + 1].ncell());
            if (M.halved[0] && M.halved[1] && M.halved[2]) {
                hipLaunchKernelGGL(k_resrestrictC8<T>, dim3(nbc), dim3(256), 0, s, L, C, g->partials);
            } else if (g->lev[l].ncell() >= RC_MAP_MIN_CELLS) {
                RowTiles t;
                if ((e = row_tiles(C.n, RC_TILES_PER_CU, RC_KMIN, zmarch_partials_max(g->nx, g->ny, g->nz), &t,
                                   &nbc)) != hipSuccess)
                    return e;
                hipLaunchKernelGGL(k_resrestrictC_map<T>, dim3(nbc), dim3(RM_NT), 0, s, L, C, M, t, g->partials);
            } else {
                hipLaunchKernelGGL(k_resrestrictC<T>, dim3(nbc), dim3(256), 0, s, L, C, M, g->partials);
            }
            nparts = nbc;
            if (!(tail && l + 1 == lt))
                hipLaunchKernelGGL(k_finalize_mu, dim3(1), dim3(256), 0, s, g->partials, nbc, &g->sc->vol[l + 1],
                                   &g->sc->mu[l + 1]);
        }
        if (tail) {
            TailArgs<T> A;
            A.nl = Lc - lt + 1;
            int off = 0;
            for (int q = 0; q < A.nl; ++q) {
                const int l = lt + q;
                A.L[q] = coarse_view<T>(g, l);
                if (q + 1 < A.nl) {
                    A.P[q] = prolong_tab(g, l);
                    for (int d = 0; d < 3; ++d) A.cs[q][d] = g->lev[l + 1].cs_d[d];
                }
                A.off[q] = off;
                off += (int)g->lev[l].ncell();
                A.vol[q] = &g->sc->vol[l];
                A.mu[q] = &g->sc->mu[l];
            }
            A.partials = g->partials;
            A.nparts = nparts;
            A.nu1 = o->nu1;
            A.nu2 = o->nu2;
            A.ncoarse = o->coarsest_sweeps;
            hipLaunchKernelGGL(k_tailC<T>, dim3(1), dim3(TAIL_NT), 0, s, A);
        } else if (g->lev[Lc].ncell() <= SMALL_LEVEL) {
            launch_smallC<T>(coarse_view<T>(g, Lc), g->lev[Lc].ncell(), o->coarsest_sweeps, &g->sc->vol[Lc], 1, s);
        } else {
            hipLaunchKernelGGL(k_coarsest<T>, dim3(1), dim3(1024), 0, s, coarse_view<T>(g, Lc), o->coarsest_sweeps,
                               &g->sc->vol[Lc]);
        }
        for (int l = Lb - 1; l >= 1; --l) {
            Coarse<T> L = coarse_view<T>(g, l);
            int nb = nblk(g->lev[l].ncell());
            const ProlongTab PT = prolong_tab(g, l);
            if (PT.halved[0] && PT.halved[1] && PT.halved[2] && g->lev[l].prolong_sides &&
                g->lev[l].ncell() >= PROLONG8_MIN_CELLS)
                hipLaunchKernelGGL(k_prolongC8<T>, dim3(nblk(g->lev[l + 1].ncell())), dim3(256), 0, s, L,
                                   coarse_view<T>(g, l + 1), PT);
            else if (g->lev[l].ncell() >= PROLONG_LDS_MIN_CELLS) {
                const ZTiles t = ztiles(L.n[0], L.n[1], L.n[2]);
                hipLaunchKernelGGL(k_prolongC_lds<T>, dim3(t.grid), dim3(ZM_NT), 0, s, L, coarse_view<T>(g, l + 1), PT,
                                   t);
            } else
                hipLaunchKernelGGL(k_prolongC<T>, dim3(nb), dim3(256), 0, s, L, coarse_view<T>(g, l + 1), PT);
            if (g->lev[l].ncell() <= SMALL_LEVEL) {
                if (o->nu2 > 0) launch_smallC<T>(L, g->lev[l].ncell(), o->nu2, &g->sc->vol[l], 0, s);
            } else if ((e = smooth_level<T>(g, l, o->nu2, s)) != hipSuccess) {
                return e;
            }
        }
        {
            T *pin = bufs[*cur], *pout = bufs[1 - *cur];
            if ((e = launch_prolong0<T>(F, pin, pout, coarse_view<T>(g, 1), prolong_tab(g, 0), s)) != hipSuccess)
                return e;
            if ((e = launch_refresh<T>(g, pin, pout, gh, s)) != hipSuccess) return e;
            *cur = 1 - *cur;
        }
    }
    for (int q = 0; q < o->nu2; ++q) {
        T *pin = bufs[*cur], *pout = bufs[1 - *cur];
        if constexpr (std::is_same<T, float>::value) {
            if (wide && q + 1 == o->nu2) {
                if ((e = launch_sweep_widen(F, pin, wide, rhs, lam, s)) != hipSuccess) return e;
                return launch_refresh_widen(g, pin, wide, gh, s);
            }
        }
        if ((e = timed_sweep<T>(g, F, pin, pout, rhs, lam, s)) != hipSuccess) return e;
        if ((e = launch_refresh<T>(g, pin, pout, gh, s)) != hipSuccess) return e;
        *cur = 1 - *cur;
    }
    return hipGetLastError();
}

hipError_t vcycle_f64(ibm_grid *g, double **bufs, int *cur, const double *f, hipStream_t s, const ibm_solve_opts *o) {
    return vcycle_impl<double>(g, bufs, cur, f, &g->sc->lambda, g->g_h, o, s);
}

// e32 := 0 (dead cells too), so the inner cycle starts from a zero correction
__global__ void k_zero32(float *a, float *b, int64_t N) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    a[id] = 0.0f;
    b[id] = 0.0f;
}

// p_next = p_cur + e on fluid cells (FP64 update of the refinement step)
__global__ void k_add_correction(const uint8_t *__restrict__ type, int64_t N, const double *__restrict__ pcur,
                                 const float *__restrict__ e, double *pnext) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N || type[id] != T_FLUID) return;
    pnext[id] = pcur[id] + (double)e[id];
}

// one mixed-precision refinement step: the FP32 right-hand side r32 = r - lambda_k was
// written by the preceding FP64 norm pass and delta32 = lambda_{k+1} - lambda_k; solve
// S e = r32 - delta with one FP32 V-cycle from e = 0, then p += e and an FP64 ghost refresh
hipError_t vcycle_mixed(ibm_grid *g, double **bufs, int *cur, const double *f, hipStream_t s,
                        const ibm_solve_opts *o) {
    (void)f;
    hipError_t e;
    hipLaunchKernelGGL(k_zero32, dim3(nblk(g->N)), dim3(256), 0, s, g->e32a, g->e32b, g->N);
    float *eb[2] = {g->e32a, g->e32b};
    int ecur = 0;
    if ((e = vcycle_impl<float>(g, eb, &ecur, g->r32, &g->sc->delta32, nullptr, o, s)) != hipSuccess) return e;
    double *pin = bufs[*cur], *pout = bufs[1 - *cur];
    hipLaunchKernelGGL(k_add_correction, dim3(nblk(g->N)), dim3(256), 0, s, g->type, g->N, pin, eb[ecur], pout);
    if ((e = launch_refresh<double>(g, pin, pout, g->g_h, s)) != hipSuccess) return e;
    *cur = 1 - *cur;
    return hipGetLastError();
}

hipError_t norm_pass(ibm_grid *g, const double *p, const double *f, hipStream_t s, bool write_r32, bool first) {
    if (write_r32)
        hipLaunchKernelGGL(k_norm0<true>, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, fine64(g), p, f, &g->sc->lambda, g->r32,
                           g->partials);
    else
        hipLaunchKernelGGL(k_norm0<false>, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, fine64(g), p, f, &g->sc->lambda,
                           (float *)nullptr, g->partials);
    hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, g->sc, (double)g->nfluid,
                       0);
    (void)first;
    return hipGetLastError();
}

hipError_t ref_norm_pass(ibm_grid *g, const double *f, hipStream_t s) {
    hipLaunchKernelGGL(k_fsum, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, fine64(g), f, &g->sc->vmean, g->partials, 0);
    hipLaunchKernelGGL(k_fsum_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, g->sc, 0);
    hipLaunchKernelGGL(k_fsum, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, fine64(g), f, &g->sc->vmean, g->partials, 1);
    hipLaunchKernelGGL(k_fsum_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, g->sc, 1);
    return hipGetLastError();
}

hipError_t gauge_pass(ibm_grid *g, const double *pcur, double *pdst, hipStream_t s) {
    hipLaunchKernelGGL(k_psum, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, fine64(g), pcur, g->partials);
    hipLaunchKernelGGL(k_fsum_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, g->sc, 0);
    hipLaunchKernelGGL(k_shift, dim3(nblk(g->N)), dim3(256), 0, s, g->type, g->N, pcur, pdst, g->sc);
    return hipGetLastError();
}

// start of a solve: both buffers hold the initial iterate on fluid and ghost cells (zero
// unless a guess is given) and 0 on dead cells; then the ghosts of p2 are refreshed
__global__ void k_init(const uint8_t *__restrict__ type, int64_t N, double *p, double *p2, int use_guess) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    double v = (type[id] == T_DEAD || !use_guess) ? 0.0 : p[id];
    p[id] = v;
    p2[id] = v;
}

hipError_t init_solution(ibm_grid *g, double *p, double *p2, int use_guess, hipStream_t s) {
    hipLaunchKernelGGL(k_init, dim3(nblk(g->N)), dim3(256), 0, s, g->type, g->N, p, p2, use_guess);
    return launch_refresh<double>(g, p, p2, g->g_h, s);
}

// =======================================================================================
// projection: divergence right-hand side and velocity correction (MAC faces)
// =======================================================================================

__global__ void k_rhs(Fine<double> F, const double *__restrict__ u, const double *__restrict__ v,
                      const double *__restrict__ w, double dt, double *f) {
    const int64_t N = (int64_t)F.nx * F.ny * F.nz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    if (F.type[id] != T_FLUID) {
        f[id] = 0.0;
        return;
    }
    const int nx = F.nx, ny = F.ny;
    int i, j, k;
    unflatten(id, nx, ny, i, j, k);
    const int64_t iu = ((int64_t)k * ny + j) * (nx + 1) + i;
    const int64_t iv = ((int64_t)k * (ny + 1) + j) * nx + i;
    const int64_t iw = ((int64_t)k * ny + j) * nx + i;
    double div = (u[iu + 1] - u[iu]) / F.wx[i];
    div = div + (v[iv + nx] - v[iv]) / F.wy[j];
    div = div + (w[iw + (int64_t)nx * ny] - w[iw]) / F.wz[k];
    f[id] = div / dt;
}

hipError_t rhs_pass(ibm_grid *g, const double *u, const double *v, const double *w, double dt, double *f,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, dim3(nblk(g->N)), dim3(256), 0, s, fine64(g), u, v, w, dt, f);
    return hipGetLastError();
}

// u_f -= dt (p_nb - p_c)/d_f on interior faces with at least one fluid cell.  A thread owns
// cell (i, j, k) and corrects its three low faces (the cell reads p and its type once for
// all three); the low faces of the first cells and the high faces of the last cells along
// an axis are box walls and stay as they are.
__global__ void k_correct(const uint8_t *__restrict__ type, int nx, int ny, int nz, const double *__restrict__ dcx,
                          const double *__restrict__ dcy, const double *__restrict__ dcz, const double *__restrict__ p,
                          double dt, double *u, double *v, double *w) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N) return;
    int i, j, k;
    unflatten(b, nx, ny, i, j, k);
    const bool fb = type[b] == T_FLUID;
    const double pb = p[b];
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    if (i > 0 && (fb || type[b - 1] == T_FLUID)) {
        const int64_t f = ((int64_t)k * ny + j) * (nx + 1) + i;
        u[f] -= dt * (pb - p[b - 1]) / dcx[i];
    }
    if (j > 0 && (fb || type[b - sy] == T_FLUID)) {
        const int64_t f = ((int64_t)k * (ny + 1) + j) * nx + i;
        v[f] -= dt * (pb - p[b - sy]) / dcy[j];
    }
    if (k > 0 && (fb || type[b - sz] == T_FLUID)) {
        const int64_t f = ((int64_t)k * ny + j) * nx + i;
        w[f] -= dt * (pb - p[b - sz]) / dcz[k];
    }
}

hipError_t correct_pass(ibm_grid *g, double *u, double *v, double *w, const double *p, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_correct, dim3(nblk(g->N)), dim3(256), 0, s, g->type, g->nx, g->ny, g->nz, g->dc0[0], g->dc0[1],
                       g->dc0[2], p, dt, u, v, w);
    return hipGetLastError();
}

// Fractional-step composition (cell-centred momentum, face-normal projection).
// Face velocities from cell-centred components: on every interior face along d the linear
// interpolation between the two centres, (w_b u_a + w_a u_b) / (w_a + w_b) with w the cell
// widths along d; box-wall faces 0 (no flux through the box, as in the convective term).
__global__ void k_cell_to_faces(int nx, int ny, int nz, int d, const double *__restrict__ wd,
                                const double *__restrict__ uc, double *uf) {
    const int fx = nx + (d == 0), fy = ny + (d == 1), fz = nz + (d == 2);
    const int64_t NF = (int64_t)fx * fy * fz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= NF) return;
    int i, j, k;
    unflatten(id, fx, fy, i, j, k);
    const int q = (d == 0) ? i : (d == 1) ? j : k;
    const int n = (d == 0) ? nx : (d == 1) ? ny : nz;
    if (q == 0 || q == n) {
        uf[id] = 0.0;
        return;
    }
    const int64_t b = ((int64_t)k * ny + j) * nx + i;
    const int64_t a = b - ((d == 0) ? 1 : (d == 1) ? (int64_t)nx : (int64_t)nx * ny);
    const double wa = wd[q - 1], wb = wd[q];
    uf[id] = (wb * uc[a] + wa * uc[b]) / (wa + wb);
}

// Cell-centred correction: on fluid cells u_c -= (delta_{c-1/2} + delta_{c+1/2}) / 2, where
// delta_f = dt (p_b - p_a) / d_f is the correction the projection applies to face f (the
// same arithmetic as k_correct) and 0 on box walls.
__global__ void k_correct_cells(const uint8_t *__restrict__ type, int nx, int ny, int nz, int d,
                                const double *__restrict__ dc, const double *__restrict__ p, double dt, double *uc) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N || type[id] != T_FLUID) return;
    int i, j, k;
    unflatten(id, nx, ny, i, j, k);
    const int q = (d == 0) ? i : (d == 1) ? j : k;
    const int n = (d == 0) ? nx : (d == 1) ? ny : nz;
    const int64_t st = (d == 0) ? 1 : (d == 1) ? (int64_t)nx : (int64_t)nx * ny;
    const double dm = (q > 0) ? dt * (p[id] - p[id - st]) / dc[q] : 0.0;
    const double dp = (q < n - 1) ? dt * (p[id + st] - p[id]) / dc[q + 1] : 0.0;
    uc[id] -= 0.5 * (dm + dp);
}

hipError_t cell_to_faces_pass(ibm_grid *g, const double *u, const double *v, const double *w, double *uf,
                              double *vf, double *wf, hipStream_t s) {
    const double *c[3] = {u, v, w};
    double *f[3] = {uf, vf, wf};
    for (int d = 0; d < 3; ++d) {
        const int64_t NF = (int64_t)(g->nx + (d == 0)) * (g->ny + (d == 1)) * (g->nz + (d == 2));
        hipLaunchKernelGGL(k_cell_to_faces, dim3(nblk(NF)), dim3(256), 0, s, g->nx, g->ny, g->nz, d, g->w0[d], c[d],
                           f[d]);
    }
    return hipGetLastError();
}

hipError_t correct_cells_pass(ibm_grid *g, double *u, double *v, double *w, const double *p, double dt,
                              hipStream_t s) {
    double *c[3] = {u, v, w};
    for (int d = 0; d < 3; ++d)
        hipLaunchKernelGGL(k_correct_cells, dim3(nblk(g->N)), dim3(256), 0, s, g->type, g->nx, g->ny, g->nz, d,
                           g->dc0[d], p, dt, c[d]);
    return hipGetLastError();
}

__global__ void __launch_bounds__(NORM_NT) k_divmax(Fine<double> F, const double *__restrict__ u,
                                                    const double *__restrict__ v, const double *__restrict__ w,
                                                    double *partials) {
    __shared__ double sh[NORM_NT / 64];
    const int64_t N = (int64_t)F.nx * F.ny * F.nz;
    const int nx = F.nx, ny = F.ny;
    double m = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * NORM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * NORM_NT) {
        if (F.type[id] != T_FLUID) continue;
        int i, j, k;
        unflatten(id, nx, ny, i, j, k);
        const int64_t iu = ((int64_t)k * ny + j) * (nx + 1) + i;
        const int64_t iv = ((int64_t)k * (ny + 1) + j) * nx + i;
        const int64_t iw = ((int64_t)k * ny + j) * nx + i;
        double div = (u[iu + 1] - u[iu]) / F.wx[i];
        div = div + (v[iv + nx] - v[iv]) / F.wy[j];
        div = div + (w[iw + (int64_t)nx * ny] - w[iw]) / F.wz[k];
        m = fmax(m, fabs(div));
    }
    double t = block_max<NORM_NT>(m, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_max_finalize(const double *partials, int nb, double *out) {
    __shared__ double sh[4];
    double m = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) m = fmax(m, partials[q]);
    m = block_max<256>(m, sh, threadIdx.x);
    if (threadIdx.x == 0) *out = m;
}

// max over ghosts of |p_g - sum_m beta_m p_m - h_g| (degenerate ghosts: |p_g - mean of the
// fluid 26-neighbours|), one partial maximum per block
__global__ void __launch_bounds__(256) k_ghost_res(GhostView G, const double *__restrict__ p, int nx, int ny, int nz,
                                                   const uint8_t *__restrict__ type, double *partials) {
    __shared__ double sh[4];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0;
    if (g < G.ng) {
        const int64_t cell = G.cell[g];
        double target;
        if (G.flags[g] & GF_DEGENERATE) {
            int i, j, k;
            unflatten(cell, nx, ny, i, j, k);
            double sm = 0.0;
            int n = 0;
            for (int dk = -1; dk <= 1; ++dk)
                for (int dj = -1; dj <= 1; ++dj)
                    for (int di = -1; di <= 1; ++di) {
                        const int ii = i + di, jj = j + dj, kk = k + dk;
                        if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                        const int64_t q = ((int64_t)kk * ny + jj) * nx + ii;
                        if (type[q] == T_FLUID) {
                            sm += p[q];
                            ++n;
                        }
                    }
            target = n ? sm / n : 0.0;
        } else {
            double sm = 0.0;
            for (int m = 0; m < 8; ++m) {
                const int32_t q = G.st[8 * g + m];
                if (q >= 0) sm = sm + G.beta[8 * g + m] * p[q];
            }
            target = sm + G.h[g];
        }
        r = fabs(p[cell] - target);
    }
    r = block_max<256>(r, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

hipError_t ghost_residual_pass(ibm_grid *g, const double *p, hipStream_t s) {
    if (g->ng == 0) {
        hipLaunchKernelGGL(k_max_finalize, dim3(1), dim3(256), 0, s, g->partials, 0, &g->sc->ghost_res);
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)((g->ng + 255) / 256);
    hipLaunchKernelGGL(k_ghost_res, dim3(nb), dim3(256), 0, s, ghost_view(g), p, g->nx, g->ny, g->nz, g->type,
                       g->partials);
    hipLaunchKernelGGL(k_max_finalize, dim3(1), dim3(256), 0, s, g->partials, (int)nb, &g->sc->ghost_res);
    return hipGetLastError();
}

hipError_t divmax_pass(ibm_grid *g, const double *u, const double *v, const double *w, hipStream_t s) {
    hipLaunchKernelGGL(k_divmax, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, fine64(g), u, v, w, g->partials);
    hipLaunchKernelGGL(k_max_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, &g->sc->div_max);
    return hipGetLastError();
}

// =======================================================================================
// BiCGStab (paper Section 2.1: the pressure solver family it uses), right-preconditioned by
// one V-cycle, on the fluid + ghost unknowns:
//   A y : fluid rows (S y)_c ; ghost rows s_g (y_g - sum_{m != g} beta_m y_m)
//   b   : fluid rows f       ; ghost rows s_g h_g
// s_g = diagonal of the flux stencil at the ghost cell (both row kinds on one scale).  The
// fluid part of every residual and operator image is projected to zero volume-weighted
// mean (the uniform source shift lambda of the Neumann problem).  All scalars stay on the
// device; the host reads back one status block per iteration.
// =======================================================================================

enum KOp { K_MU = 0, K_ALPHA = 1, K_OMEGA = 2, K_RHO = 3, K_INIT = 4, K_RESTART = 5 };

// ghost scale: the stencil diagonal, summed in the smoother's order
__global__ void k_ghost_scale(int64_t ng, const int32_t *__restrict__ gcell, int nx, int ny, const double *axm,
                              const double *axp, const double *aym, const double *ayp, const double *azm,
                              const double *azp, double *scale) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int64_t id = gcell[g];
    int i, j, k;
    unflatten(id, nx, ny, i, j, k);
    double d = axm[i] + axp[i];
    d = d + aym[j];
    d = d + ayp[j];
    d = d + azm[k];
    d = d + azp[k];
    scale[g] = d;
}

// ghost rows of A y (mode 0) or of b - A y (mode 1: out = s_g h_g - A y).  With gpart, the
// block sums of o_g out_g and out_g^2 over the ghost rows go to gpart[2 block + (0, 1)].
__global__ void k_apply_ghost(GhostView G, const double *__restrict__ y, double *out, const double *__restrict__ scale,
                              int nx, int ny, int nz, const uint8_t *__restrict__ type, int mode,
                              const double *__restrict__ o, double *gpart) {
    __shared__ double sh[4];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double d0 = 0.0, d1 = 0.0;
    if (g < G.ng) {
        const int64_t cell = G.cell[g];
        double target;
        if (G.flags[g] & GF_DEGENERATE) {
            int i, j, k;
            unflatten(cell, nx, ny, i, j, k);
            double s = 0.0;
            int n = 0;
            for (int dk = -1; dk <= 1; ++dk)
                for (int dj = -1; dj <= 1; ++dj)
                    for (int di = -1; di <= 1; ++di) {
                        const int ii = i + di, jj = j + dj, kk = k + dk;
                        if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                        const int64_t q = ((int64_t)kk * ny + jj) * nx + ii;
                        if (type[q] == T_FLUID) {
                            s += y[q];
                            ++n;
                        }
                    }
            target = n ? s / n : 0.0;
        } else {
            const int32_t *st = G.st + 8 * g;
            const double *beta = G.beta + 8 * g;
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (st[m] >= 0) s = s + beta[m] * y[st[m]];
            target = s;
        }
        const double a = scale[g] * (y[cell] - target);
        const double v = mode ? scale[g] * G.h[g] - a : a;
        out[cell] = v;
        if (gpart) {
            d0 = o[cell] * v;
            d1 = v * v;
        }
    }
    if (gpart) {  // uniform: every thread of the block takes part in the sums
        const double s0 = block_sum<256>(d0, sh, threadIdx.x);
        const double s1 = block_sum<256>(d1, sh, threadIdx.x);
        if (threadIdx.x == 0) {
            gpart[2 * blockIdx.x] = s0;
            gpart[2 * blockIdx.x + 1] = s1;
        }
    }
}

// The volume-weighted fluid sum of an operator image, before the image is formed.  Summed
// over the fluid rows, V_c (S y)_c = sum_f T_f (y_nb - y_c) cancels on every face between two
// fluid cells (T_f = V a_f is the same from both sides) and no flux crosses the box walls, so
// only the faces between a fluid cell and a ghost cell remain: per block, the sum over ghosts
// g and their fluid face neighbours c of V_c a_(c->g) (y_g - y_c).
__global__ void k_ghost_flux(GhostView G, Fine<double> F, const double *__restrict__ y, double *partials) {
    __shared__ double sh[4];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (g < G.ng) {
        const int64_t cell = G.cell[g];
        int i, j, k;
        unflatten(cell, F.nx, F.ny, i, j, k);
        const int64_t sy = F.nx, sz = (int64_t)F.nx * F.ny;
        const double yg = y[cell];
        if (i > 0 && F.type[cell - 1] == T_FLUID)
            acc += ((F.wx[i - 1] * F.wy[j]) * F.wz[k]) * F.axp[i - 1] * (yg - y[cell - 1]);
        if (i < F.nx - 1 && F.type[cell + 1] == T_FLUID)
            acc += ((F.wx[i + 1] * F.wy[j]) * F.wz[k]) * F.axm[i + 1] * (yg - y[cell + 1]);
        if (j > 0 && F.type[cell - sy] == T_FLUID)
            acc += ((F.wx[i] * F.wy[j - 1]) * F.wz[k]) * F.ayp[j - 1] * (yg - y[cell - sy]);
        if (j < F.ny - 1 && F.type[cell + sy] == T_FLUID)
            acc += ((F.wx[i] * F.wy[j + 1]) * F.wz[k]) * F.aym[j + 1] * (yg - y[cell + sy]);
        if (k > 0 && F.type[cell - sz] == T_FLUID)
            acc += ((F.wx[i] * F.wy[j]) * F.wz[k - 1]) * F.azp[k - 1] * (yg - y[cell - sz]);
        if (k < F.nz - 1 && F.type[cell + sz] == T_FLUID)
            acc += ((F.wx[i] * F.wy[j]) * F.wz[k + 1]) * F.azm[k + 1] * (yg - y[cell + sz]);
    }
    const double t = block_sum<256>(acc, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// start of the Krylov recurrences on the residual v: projection of its fluid part
// (v -= mu_v; mode 2) or none (restart, mode 3), then rh = v and the sums v.v (all) and v.v
// (fluid).  (The operator images of a step are projected where they are formed.)
__global__ void __launch_bounds__(NORM_NT) k_project(const uint8_t *__restrict__ type, int64_t N, double *v, double *rh,
                                                     const Scalars *sc, int mode, double *partials) {
    __shared__ double sh[NORM_NT / 64];
    const double mu = sc->mu_v;
    double a = 0.0, b = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * NORM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * NORM_NT) {
        const uint8_t t = type[id];
        if (t == T_DEAD) continue;
        double x = v[id];
        if (t == T_FLUID && mode != 3) {
            x -= mu;
            v[id] = x;
        }
        rh[id] = x;
        a += x * x;
        if (t == T_FLUID) b += x * x;
    }
    double s = block_sum<NORM_NT>(a, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[2 * blockIdx.x] = s;
    s = block_sum<NORM_NT>(b, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[2 * blockIdx.x + 1] = s;
}

// Near-breakdown of BiCGStab: an inner product whose modulus is at most brk_tol (the option
// breakdown_tol) times the product of its factors' norms (the shadow residual against the
// residual for rho, or against A y for alpha), or omega = 0.  The step then does not form the
// quotient (alpha = 0; beta = 0) and sets sc->brk; the host restarts the shadow residual from
// the residual.

// stride 3 (K_RHO): sums of rh.r, r.r on fluid rows and r.r on every active row
__global__ void k_krylov_finalize(const double *partials, int nb, int stride, Scalars *sc, int op, double brk_tol) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) {
        a += partials[stride * q];
        if (stride > 1) b += partials[stride * q + 1];
        if (stride > 2) c += partials[stride * q + 2];
    }
    a = block_sum<256>(a, sh, threadIdx.x);
    b = block_sum<256>(b, sh, threadIdx.x);
    c = block_sum<256>(c, sh, threadIdx.x);
    if (threadIdx.x != 0) return;
    switch (op) {
        case K_MU: sc->mu_v = a / sc->vol[0]; break;
        case K_ALPHA:
        case K_OMEGA: break;  // formed by k_krylov_finalize_dots
        case K_RHO:
        case K_INIT:
        case K_RESTART: {
            const double rho_new = a;
            if (op == K_RHO) {
                const bool brk = sc->brk || sc->omega == 0.0 || !(fabs(rho_new) > brk_tol * sqrt(sc->rh2 * c));
                sc->brk = brk ? 1 : 0;
                sc->beta = brk ? 0.0 : (rho_new / sc->rho) * (sc->alpha / sc->omega);
            } else {
                // the shadow residual is (re)started as the residual: rho = rh.rh
                sc->beta = 0.0;
                sc->rh2 = rho_new;
                sc->brk = 0;
            }
            sc->rho_old = sc->rho;
            sc->rho = rho_new;
            sc->norm = sqrt(b);
            sc->rel = (sc->ref > 0.0) ? sc->norm / sc->ref : 0.0;
            if (!isfinite(sc->norm) || !isfinite(sc->beta)) sc->bad = 1;
            if (op == K_INIT) sc->lambda = sc->mu_v;  // the removed mean of b - A x
            break;
        }
    }
}

// alpha = rho / rh.v or omega = t.s / t.t from the operator pass's sums (stride ns over nb
// workgroups: o w, then w w) and the ghost rows' (stride 2 over ngb blocks)
__global__ void k_krylov_finalize_dots(const double *part, int nb, int ns, const double *gpart, int ngb, Scalars *sc,
                                       int op, double brk_tol) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) {
        a += part[ns * q];
        if (ns > 1) b += part[ns * q + 1];
    }
    for (int q = threadIdx.x; q < ngb; q += 256) {
        a += gpart[2 * q];
        b += gpart[2 * q + 1];
    }
    a = block_sum<256>(a, sh, threadIdx.x);
    b = block_sum<256>(b, sh, threadIdx.x);
    if (threadIdx.x != 0) return;
    if (op == K_ALPHA) {
        // a = rh.v, b = v.v
        if (fabs(a) > brk_tol * sqrt(sc->rh2 * b)) {
            sc->alpha = sc->rho / a;
        } else {
            sc->alpha = 0.0;
            sc->brk = 1;
        }
    } else {
        sc->omega = (b > 0.0) ? a / b : 0.0;
    }
}

// pd = r + beta (pd - omega v) on fluid + ghost cells
// r32 (mixed precision, else null): the FP32 right-hand side of the preconditioner, the
// fluid part of the result rounded to FP32 and zero elsewhere
// first: the first step of a solve, p = r (beta is 0 and p, v hold nothing yet: not read)
__global__ void k_p_update(const uint8_t *__restrict__ type, int64_t N, const double *__restrict__ r,
                           const double *__restrict__ v, double *pd, const Scalars *sc, float *r32, int first) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const uint8_t ty = type[id];
    if (ty == T_DEAD) {
        pd[id] = 0.0;
        if (r32) r32[id] = 0.0f;
        return;
    }
    double pv = r[id];
    if (!first) pv = pv + sc->beta * (pd[id] - sc->omega * v[id]);
    __builtin_nontemporal_store(pv, pd + id);
    if (r32) r32[id] = (ty == T_FLUID) ? (float)pv : 0.0f;
}

// The BiCGStab vector updates write their full-field results with non-temporal stores (see
// the operator pass).
// s = r - alpha v
__global__ void k_s_update(const uint8_t *__restrict__ type, int64_t N, const double *__restrict__ r,
                           const double *__restrict__ v, double *s, const Scalars *sc, float *r32) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    const uint8_t ty = type[id];
    const double sv = (ty == T_DEAD) ? 0.0 : r[id] - sc->alpha * v[id];
    __builtin_nontemporal_store(sv, s + id);
    if (r32) r32[id] = (ty == T_FLUID) ? (float)sv : 0.0f;
}

// x += alpha y + omega z ; r = s - omega t ; partials of rh.r (all), r.r (fluid) and r.r (all)
__global__ void __launch_bounds__(NORM_NT) k_xr_update(const uint8_t *__restrict__ type, int64_t N, double *x,
                                                       const double *__restrict__ y, const double *__restrict__ z,
                                                       const double *__restrict__ s, const double *__restrict__ t,
                                                       double *r, const double *__restrict__ rh, const Scalars *sc,
                                                       double *partials) {
    __shared__ double sh[NORM_NT / 64];
    const double alpha = sc->alpha, omega = sc->omega;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * NORM_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * NORM_NT) {
        const uint8_t ty = type[id];
        if (ty == T_DEAD) continue;
        __builtin_nontemporal_store(x[id] + alpha * y[id] + omega * z[id], x + id);
        const double rv = s[id] - omega * t[id];
        __builtin_nontemporal_store(rv, r + id);
        a += rh[id] * rv;
        c += rv * rv;
        if (ty == T_FLUID) b += rv * rv;
    }
    double q = block_sum<NORM_NT>(a, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[3 * blockIdx.x] = q;
    q = block_sum<NORM_NT>(b, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[3 * blockIdx.x + 1] = q;
    q = block_sum<NORM_NT>(c, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[3 * blockIdx.x + 2] = q;
}

// preconditioner start: ghost right-hand sides gh = r_g / s_g and e_g = gh (the first ghost
// refresh of a zero field), every other cell 0.  k_precond_zero clears both buffers when no
// pre-smoothing sweep comes first; otherwise the start iterate (zero except at the ghost
// cells) is only read by the first sweep, which writes every cell of its output.
template <typename T>
__global__ void k_precond_zero(int64_t N, T *ea, T *eb) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    ea[id] = T(0);
    if (eb) eb[id] = T(0);
}
template <typename T>
__global__ void k_precond_ghosts(int64_t ng, const int32_t *__restrict__ gcell, const int32_t *__restrict__ flags,
                                 const double *__restrict__ scale, const double *__restrict__ r, double *gh, T *ea) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int64_t cell = gcell[g];
    const double h = r[cell] / scale[g];
    gh[g] = h;
    // a degenerate ghost takes the mean of its (zero) fluid neighbours
    ea[cell] = (flags[g] & GF_DEGENERATE) ? T(0) : (T)h;
}
__global__ void k_widen(const uint8_t *__restrict__ type, int64_t N, const float *__restrict__ e, double *y) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    y[id] = (type[id] == T_DEAD) ? 0.0 : (double)e[id];
}

// y = M r: one V-cycle from zero on the error equation with right-hand side r (fluid) and
// ghost right-hand sides r_g / s_g.  FP64: the result lands in one of (ya, yb), returned.
// Mixed: the cycle runs in FP32 on the workspace's FP32 buffers and is widened into ya.
// IBM_BICGSTAB_SRJ: instead of the V-cycle, the scheduled relaxed Jacobi sweeps of the
// grid's schedule, each followed by the ghost refresh (FP64).
static hipError_t precondition(ibm_grid *g, const double *r, double *ya, double *yb, double **out,
                               const ibm_solve_opts *o, hipStream_t s) {
    hipError_t e;
    const unsigned nbN = (unsigned)nblk(g->N), nbG = (unsigned)nblk(g->ng > 0 ? g->ng : 1);
    // With pre-smoothing the cycle starts from the start iterate (zero except at the ghost
    // cells, written here), which the first sweep only reads: no field is cleared per call.
    if (o->precision == IBM_MIXED) {
        const bool st = o->nu1 > 0;
        // g->r32 already holds the FP32 fluid part of r: the update kernel that formed r
        // (k_p_update, k_s_update) wrote it beside r
        float *e0 = st ? g->pz32 : g->e32a;
        if (!st) hipLaunchKernelGGL(k_precond_zero<float>, dim3(nbN), dim3(256), 0, s, g->N, g->e32a, g->e32b);
        if (g->ng > 0)
            hipLaunchKernelGGL(k_precond_ghosts<float>, dim3(nbG), dim3(256), 0, s, g->ng, g->g_cell, g->g_flags,
                               g->g_scale, r, g->g_rhs, e0);
        float *eb[2] = {g->e32a, g->e32b};
        int ecur = 0;
        // with post-smoothing, the last sweep writes the FP64 result itself
        double *wide = o->nu2 > 0 ? ya : nullptr;
        if ((e = vcycle_impl<float>(g, eb, &ecur, g->r32, &g->sc->zero32, g->g_rhs, o, s, st ? e0 : nullptr,
                                    wide)) != hipSuccess)
            return e;
        if (!wide) hipLaunchKernelGGL(k_widen, dim3(nbN), dim3(256), 0, s, g->type, g->N, eb[ecur], ya);
        *out = ya;
    } else if (o->method == IBM_BICGSTAB_SRJ) {
        // scheduled relaxed Jacobi: every sweep writes all cells of the other buffer; the first
        // one reads the start iterate
        if (g->ng > 0)
            hipLaunchKernelGGL(k_precond_ghosts<double>, dim3(nbG), dim3(256), 0, s, g->ng, g->g_cell, g->g_flags,
                               g->g_scale, r, g->g_rhs, g->pz);
        double *bufs[2] = {ya, yb};
        int cur = 0;
        bool first = true;
        const Fine<double> F = fine64(g);
        for (double w : g->srj_omega) {
            const double *pin = first ? g->pz : bufs[cur];
            if ((e = launch_jacobi0(F, pin, r, bufs[1 - cur], w, s)) != hipSuccess) return e;
            if ((e = launch_refresh<double>(g, pin, bufs[1 - cur], g->g_rhs, s)) != hipSuccess) return e;
            cur = 1 - cur;
            first = false;
        }
        if (first) {  // no sweep: the start iterate itself
            hipLaunchKernelGGL(k_precond_zero<double>, dim3(nbN), dim3(256), 0, s, g->N, ya, (double *)nullptr);
            if (g->ng > 0)
                hipLaunchKernelGGL(k_precond_ghosts<double>, dim3(nbG), dim3(256), 0, s, g->ng, g->g_cell,
                                   g->g_flags, g->g_scale, r, g->g_rhs, ya);
        }
        *out = bufs[cur];
    } else {
        const bool st = o->nu1 > 0;
        double *e0 = st ? g->pz : ya;
        if (!st) hipLaunchKernelGGL(k_precond_zero<double>, dim3(nbN), dim3(256), 0, s, g->N, ya, yb);
        if (g->ng > 0)
            hipLaunchKernelGGL(k_precond_ghosts<double>, dim3(nbG), dim3(256), 0, s, g->ng, g->g_cell, g->g_flags,
                               g->g_scale, r, g->g_rhs, e0);
        double *bufs[2] = {ya, yb};
        int cur = 0;
        if ((e = vcycle_impl<double>(g, bufs, &cur, r, &g->sc->zero, g->g_rhs, o, s, st ? e0 : nullptr)) !=
            hipSuccess)
            return e;
        *out = bufs[cur];
    }
    return hipGetLastError();
}

// w = P A y (the fluid part with its volume-weighted mean removed) and the inner products of
// `mode` (0: rh.w for alpha; 1: t.s and t.t for omega), then alpha or omega.  The mean comes
// first, from the fluid-ghost faces alone (k_ghost_flux), so the operator pass writes the
// projected image and forms its inner products in the same sweep.
static hipError_t apply_projected(ibm_grid *g, const double *y, double *w, const double *other, int mode, int op,
                                  double brk_tol, hipStream_t s) {
    const int ngb = g->ng > 0 ? nblk(g->ng) : 0;
    double *gpart = g->partials + 2 * zmarch_partials_max(g->nx, g->ny, g->nz);
    if (g->ng > 0)
        hipLaunchKernelGGL(k_ghost_flux, dim3(ngb), dim3(256), 0, s, ghost_view(g), fine64(g), y, g->partials);
    hipLaunchKernelGGL(k_krylov_finalize, dim3(1), dim3(256), 0, s, g->partials, ngb, 1, g->sc, (int)K_MU, 0.0);
    int nparts = 0;
    hipError_t e = launch_apply_fluid(fine64(g), y, w, other, &g->sc->mu_v, mode + 1, g->partials, &nparts, s);
    if (e != hipSuccess) return e;
    if (g->ng > 0)
        hipLaunchKernelGGL(k_apply_ghost, dim3(ngb), dim3(256), 0, s, ghost_view(g), y, w, g->g_scale, g->nx, g->ny,
                           g->nz, g->type, 0, other, gpart);
    hipLaunchKernelGGL(k_krylov_finalize_dots, dim3(1), dim3(256), 0, s, g->partials, nparts, 2, gpart, ngb, g->sc,
                       op, brk_tol);
    return hipGetLastError();
}

hipError_t krylov_setup(ibm_grid *g, hipStream_t s) {
    if (g->ng == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_scale, dim3(nblk(g->ng)), dim3(256), 0, s, g->ng, g->g_cell, g->nx, g->ny, g->am0[0],
                       g->ap0[0], g->am0[1], g->ap0[1], g->am0[2], g->ap0[2], g->g_scale);
    return hipGetLastError();
}

// r = P (b - A x), rh = r, rho = rh.r, norm of the fluid part; lambda = removed mean
hipError_t krylov_residual(ibm_grid *g, const double *f, const double *x, hipStream_t s) {
    double *r = g->kv[0], *rh = g->kv[1];
    // fluid rows: the z-marching operator pass in its residual form, with sum V r per workgroup
    int nparts = 0;
    hipError_t e = launch_apply_fluid(fine64(g), x, r, f, nullptr, 3, g->partials, &nparts, s);
    if (e != hipSuccess) return e;
    if (g->ng > 0)
        hipLaunchKernelGGL(k_apply_ghost, dim3(nblk(g->ng)), dim3(256), 0, s, ghost_view(g), x, r, g->g_scale, g->nx,
                           g->ny, g->nz, g->type, 1, (const double *)nullptr, (double *)nullptr);
    hipLaunchKernelGGL(k_krylov_finalize, dim3(1), dim3(256), 0, s, g->partials, nparts, 1, g->sc, (int)K_MU, 0.0);
    hipLaunchKernelGGL(k_project, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, g->type, g->N, r, rh, g->sc, 2, g->partials);
    hipLaunchKernelGGL(k_krylov_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, 2, g->sc, (int)K_INIT,
                       0.0);
    return hipGetLastError();
}

// one BiCGStab step on x (kv: r, rh, pd, v, s, t, ya, yb, za, zb)
hipError_t krylov_step(ibm_grid *g, double *x, const ibm_solve_opts *o, bool first, hipStream_t s) {
    double *r = g->kv[0], *rh = g->kv[1], *pd = g->kv[2], *v = g->kv[3], *sv = g->kv[4], *t = g->kv[5];
    double *ya = g->kv[6], *yb = g->kv[7], *za = g->kv[8], *zb = g->kv[9];
    const unsigned nbN = (unsigned)nblk(g->N);
    hipError_t e;
    float *r32 = o->precision == IBM_MIXED ? g->r32 : nullptr;  // FP32 right-hand side of the mixed cycle
    hipLaunchKernelGGL(k_p_update, dim3(nbN), dim3(256), 0, s, g->type, g->N, r, v, pd, g->sc, r32, first ? 1 : 0);
    double *y = nullptr, *z = nullptr;
    if ((e = precondition(g, pd, ya, yb, &y, o, s)) != hipSuccess) return e;
    if ((e = apply_projected(g, y, v, rh, 0, K_ALPHA, o->breakdown_tol, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_s_update, dim3(nbN), dim3(256), 0, s, g->type, g->N, r, v, sv, g->sc, r32);
    if ((e = precondition(g, sv, za, zb, &z, o, s)) != hipSuccess) return e;
    if ((e = apply_projected(g, z, t, sv, 1, K_OMEGA, o->breakdown_tol, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_xr_update, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, g->type, g->N, x, y, z, sv, t, r, rh, g->sc,
                       g->partials);
    hipLaunchKernelGGL(k_krylov_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, 3, g->sc, (int)K_RHO,
                       o->breakdown_tol);
    return hipGetLastError();
}

// restart the shadow residual after a breakdown: rh = r, rho = r.r, beta = 0
hipError_t krylov_restart(ibm_grid *g, hipStream_t s) {
    hipLaunchKernelGGL(k_project, dim3(RED_BLOCKS), dim3(NORM_NT), 0, s, g->type, g->N, g->kv[0], g->kv[1], g->sc, 3,
                       g->partials);
    hipLaunchKernelGGL(k_krylov_finalize, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, 2, g->sc,
                       (int)K_RESTART, 0.0);
    return hipGetLastError();
}

}  // namespace ibm
