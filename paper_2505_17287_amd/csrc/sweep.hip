// Fused red-black Gauss-Seidel sweep of the fine level (paper Section 2.1: red-black
// Gauss-Seidel smoothing of the pressure equation on a non-uniform Cartesian grid).
// Kept in a file of its own: it is the kernel the bandwidth figures are quoted for.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.hpp"
#include "ibm_impl.hpp"

namespace ibm {

// =======================================================================================
// fused red-black Gauss-Seidel sweep on level 0
//
// One sweep updates every red fluid cell ((i+j+k) even) from the old values, then every
// black fluid cell from the new red values:
//     p_c = (sum_f a_f p_nb - (f_c - lambda)) / sum_f a_f
// Both colours are done in one out-of-place pass.  A workgroup owns a tile of columns and a
// chunk of z-planes and marches upward; at step k it forms the red values of plane k+1
// (from old planes k, k+1, k+2) and the black values of plane k (from the red values of
// planes k-1, k, k+1).  Each thread owns two adjacent columns, so at every plane it holds
// exactly one red and one black cell: no lane of a wave idles on the colour test, and the
// pair moves as one 16-byte access.  In-plane neighbours come from double-buffered LDS
// (one barrier per plane); a ring of one column around the tile recomputes red values
// redundantly, a second ring only loads old values.  Each cell's new value is computed with
// the same operations in the same order as the two-pass definition, so the result is
// bitwise identical to it.
// Algorithmic traffic per cell: read p, f, type; write p (25 B in FP64, 13 B in FP32).
// =======================================================================================

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    using type = double2;
};
template <>
struct Vec2<float> {
    using type = float2;
};

// One plane of a thread's two columns.  With paired (vector) loads the two cell types
// arrive as one 16-bit word and are tested in place (fluid is type 0: the first cell is
// fluid iff the low byte is 0, the second iff the word is below 256).  A value carried
// around the unrolled loop must be a load's own register: a byte split out of the word
// would be formed at the loop latch, which would then wait for the newest loads.
template <typename T, bool VEC>
struct SweepPlane;
template <typename T>
struct SweepPlane<T, true> {
    T o0, o1, f0, f1;
    uint16_t tt;
    __device__ __forceinline__ bool fl0() const { return (uint8_t)tt == T_FLUID; }
    __device__ __forceinline__ bool fl1() const { return tt < 256; }
    __device__ __forceinline__ bool dd0() const { return (uint8_t)tt == T_DEAD; }
    __device__ __forceinline__ bool dd1() const { return (tt >> 8) == T_DEAD; }
};
template <typename T>
struct SweepPlane<T, false> {
    T o0, o1, f0, f1;
    uint8_t t0, t1;
    __device__ __forceinline__ bool fl0() const { return t0 == T_FLUID; }
    __device__ __forceinline__ bool fl1() const { return t1 == T_FLUID; }
    __device__ __forceinline__ bool dd0() const { return t0 == T_DEAD; }
    __device__ __forceinline__ bool dd1() const { return t1 == T_DEAD; }
};

constexpr int SW_KC_MAX = 512;  // longest z chunk of one workgroup
constexpr int SW_QD = 6;        // planes held per thread: k, k+1, k+2 in use, three in flight

// Relaxation value of one cell.  dxy = ((axm + axp) + aym) + ayp is formed once per thread;
// the remaining operations and their order are those of the two-pass definition
// (s accumulates the six neighbour products left to right; d adds azm, then azp).
template <typename T>
__device__ __forceinline__ T rb_update(T am, T ap, T bm, T bp, T cm, T cp, T dxy, T xm, T xp, T ym, T yp, T zm,
                                       T zp, T fv, T lam) {
    T s = am * xm;
    s = s + ap * xp;
    s = s + bm * ym;
    s = s + bp * yp;
    s = s + cm * zm;
    s = s + cp * zp;
    T d = dxy + cm;
    d = d + cp;
    return (s - (fv - lam)) / d;
}

// Thread layout: 32 threads span the 64 columns of a tile row (two adjacent columns each);
// a wave holds two rows of the same parity (wave w: rows 4(w/2) + (w mod 2) and that + 2).
// Tiles start at even columns, so the colour of a thread's first cell at plane k depends on
// the wave and k only: the colour phase is uniform across the wave and the plane loop is
// specialised for both phases, with no per-lane colour selection.
// VEC: nx is even, so a thread's column pair is 2-element aligned and moves as one access.
// Every thread issues the same loads for every plane (addresses clamped into the grid,
// values of cells outside it replaced by zero), which keeps the in-order memory counter
// exact: the loads of a plane are issued four plane steps before they are first used.
// TO: type of the result.  A wider TO than T (FP32 sweep, FP64 result) is the last sweep of
// the mixed-precision cycle, whose result the FP64 outer iteration takes as it is: each value
// is widened exactly and dead cells are written as zero.
template <typename T, typename TO, int BXT, int BY, bool VEC>
__global__ void __launch_bounds__(BXT *BY)
    k_rbgs_fused(Fine<T> F, const T *__restrict__ pin, TO *__restrict__ pout, const T *__restrict__ f,
                 const T *__restrict__ lamp, int ntx, int nty, int kc, int ntiles) {
    static_assert(BXT == 32 && BY % 4 == 0, "two same-parity rows of 32 threads per wave");
    using V = typename Vec2<T>::type;
    using PD = SweepPlane<T, VEC>;
    typedef TO NV __attribute__((ext_vector_type(2)));  // native pair for the streaming store
    constexpr bool WIDEN = sizeof(TO) != sizeof(T);
    constexpr int NC = 2 * BXT;  // columns of a tile including the 2-column halo
    constexpr int TXC = NC - 4, TY = BY - 4;
    // LDS planes with a guard ring (one row above and below, one column on the left, two on
    // the right keeping the pitch odd): tile row r, column c live at [r + 1][c + 1], so the
    // neighbour reads of every lane (the discarded ones of the outer rings included) stay
    // inside the arrays; the guards are zeroed once and never written again
    constexpr int GR = BY + 2, GC = NC + 3;
    __shared__ T so[2][GR][GC];  // old values of the plane whose red values are formed
    __shared__ T sr[2][GR][GC];  // red-updated values of the plane whose black values are formed
    __shared__ T saz[2][SW_KC_MAX + 8];  // z coefficients of planes k0-2 .. k1+5
    // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs; give every
    // XCD a contiguous range of tiles so neighbouring tiles share one L2
    const int per = gridDim.x >> 3;
    const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (logical >= ntiles) return;
    int tile = logical;
    const int txi = tile % ntx;
    tile /= ntx;
    const int tyi = tile % nty;
    const int chunk = tile / nty;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    const int tx = lane & (BXT - 1);
    const int ty = (wave >> 1) * 4 + (wave & 1) + 2 * (lane >> 5);
    for (int q = (int)threadIdx.x; q < kc + 8; q += BXT * BY) {
        const int kk = chunk * kc - 2 + q;
        const bool kin = kk >= 0 && kk < F.nz;
        saz[0][q] = kin ? F.azm[kk] : T(0);
        saz[1][q] = kin ? F.azp[kk] : T(0);
    }
    for (int q = (int)threadIdx.x; q < 2 * GC + 3 * BY; q += BXT * BY) {
        const int u = q - 2 * GC;
        const int r = (q < GC) ? 0 : (q < 2 * GC) ? BY + 1 : 1 + u / 3;
        const int c = (q < 2 * GC) ? q % GC : (u % 3 == 0) ? 0 : NC + u % 3;
        so[0][r][c] = T(0);
        so[1][r][c] = T(0);
        sr[0][r][c] = T(0);
        sr[1][r][c] = T(0);
    }
    const int lc = 2 * tx;              // local column of this thread's first cell
    const int ia = txi * TXC - 2 + lc;  // global column of the first cell (even); second = ia + 1
    const int j = tyi * TY - 2 + ty;
    const int nx = F.nx, ny = F.ny, nz = F.nz;
    const bool rowin = j >= 0 && j < ny;
    const bool in0 = rowin && ia >= 0 && ia < nx, in1 = rowin && ia + 1 >= 0 && ia + 1 < nx;
    const int yr = min(ty, BY - 1 - ty);
    const int xr0 = min(lc, NC - 1 - lc), xr1 = min(lc + 1, NC - 2 - lc);
    const bool red0 = in0 && yr >= 1 && xr0 >= 1, red1 = in1 && yr >= 1 && xr1 >= 1;
    const bool blk0 = in0 && yr >= 2 && xr0 >= 2, blk1 = in1 && yr >= 2 && xr1 >= 2;
    const int k0 = chunk * kc, k1 = min(nz, k0 + kc);
    const int64_t plane = (int64_t)nx * ny;
    // clamped addressing: rows and columns outside the grid read a valid cell, then zero
    const int jc = min(max(j, 0), ny - 1);
    const int ic0 = min(max(ia, 0), nx - 1), ic1 = min(max(ia + 1, 0), nx - 1);
    const int icv = min(max(ia, 0), nx - 2);  // pair start for the vector path (nx even)
    const int64_t rowoff0 = (int64_t)jc * nx + (VEC ? icv : ic0);
    const int64_t rowoff1 = (int64_t)jc * nx + ic1;
    // The outermost halo rows only supply old values: their f and type loads are pointed at
    // the adjacent row (lines the tile reads anyway), which keeps every lane's load sequence
    // identical without streaming f and type of rows nobody updates.
    const int jft = min(max((ty == 0) ? j + 1 : (ty == BY - 1) ? j - 1 : j, 0), ny - 1);
    const int64_t ftoff0 = (int64_t)jft * nx + (VEC ? icv : ic0);
    const int64_t ftoff1 = (int64_t)jft * nx + ic1;
    const T axm0 = in0 ? F.axm[ic0] : T(0), axp0 = in0 ? F.axp[ic0] : T(0);
    const T axm1 = in1 ? F.axm[ic1] : T(0), axp1 = in1 ? F.axp[ic1] : T(0);
    const T aym = rowin ? F.aym[jc] : T(0), ayp = rowin ? F.ayp[jc] : T(0);
    const T dxy0 = ((axm0 + axp0) + aym) + ayp, dxy1 = ((axm1 + axp1) + aym) + ayp;
    const T lam = *lamp;
    // the first cell is red at plane q iff (j + q) is even; phase = first cell is red at k0 - 1
    const bool phase = ((wave + (tyi * TY) + k0) & 1) != 0;  // (j + k0) odd; uniform per wave
    // planes past k1 + 1 are never needed: steps beyond the chunk re-read plane k1 + 1
    // (a cache hit) instead of streaming planes that the next chunk loads anyway
    const int klast = min(k1 + 1, nz - 1);
    // Values read through clamped addresses (rows, columns or planes outside the grid) are
    // finite copies of boundary cells.  They are never updated (the live masks exclude
    // cells outside the grid) and they only meet coefficients that are exactly zero (wall
    // faces), or feed red values of planes outside the grid that in turn only meet zero
    // wall coefficients, so they are used as loaded.
    auto load = [=](int k) -> PD {
        PD d;
        const int64_t base = (int64_t)min(max(k, 0), klast) * plane;
        if constexpr (VEC) {
            const V o = *reinterpret_cast<const V *>(pin + base + rowoff0);
            const V fv = *reinterpret_cast<const V *>(f + base + ftoff0);
            d.o0 = o.x;
            d.o1 = o.y;
            d.f0 = fv.x;
            d.f1 = fv.y;
            if constexpr (VEC) d.tt = *reinterpret_cast<const uint16_t *>(F.type + base + ftoff0);
        } else {
            d.o0 = pin[base + rowoff0];
            d.o1 = pin[base + rowoff1];
            d.f0 = f[base + ftoff0];
            d.f1 = f[base + ftoff1];
            if constexpr (!VEC) {
                d.t0 = F.type[base + ftoff0];
                d.t1 = F.type[base + ftoff1];
            }
        }
        return d;
    };

    // Red-updated values of plane q from M = plane q-1, C = plane q, P = plane q+1 and OB =
    // LDS of the old values of plane q.  FR (compile-time): the first cell is the red one.
#define IBM_RED_PAIR(q, M, C, P, OB, R0, R1, FR)                                                                    \
    {                                                                                                              \
        const int l_ = (FR) ? lc : lc + 1;                                                                         \
        const bool live_ = (FR) ? (red0 && (C).fl0()) : (red1 && (C).fl1());                      \
        const T v_ = rb_update<T>((FR) ? axm0 : axm1, (FR) ? axp0 : axp1, aym, ayp, saz[0][(q) - k0 + 2],          \
                                  saz[1][(q) - k0 + 2], (FR) ? dxy0 : dxy1, OB[ty + 1][l_], OB[ty + 1][l_ + 2],    \
                                  OB[ty][l_ + 1], OB[ty + 2][l_ + 1], (FR) ? (M).o0 : (M).o1, (FR) ? (P).o0 : (P).o1, \
                                  (FR) ? (C).f0 : (C).f1, lam);                                                    \
        R0 = ((FR) && live_) ? v_ : (C).o0;                                                                        \
        R1 = (!(FR) && live_) ? v_ : (C).o1;                                                                       \
    }

    // One plane step: A = plane k, B = k+1, C = k+2 (three more planes in flight); afterwards
    // the slot A receives plane k + SW_QD.  At step k the red cell of plane k+1 and the black
    // cell of plane k lie in the same column of the pair (FR: the first one).  Steps past the
    // chunk end compute from clamped data and store nothing, so every step issues the same
    // loads.
#define IBM_STEP(A, B, C, k, FR)                                                                                   \
    {                                                                                                              \
        so[buf][ty + 1][lc + 1] = (B).o0;                                                                          \
        so[buf][ty + 1][lc + 2] = (B).o1;                                                                          \
        sr[buf][ty + 1][lc + 1] = pb0;                                                                             \
        sr[buf][ty + 1][lc + 2] = pb1;                                                                             \
        __syncthreads();                                                                                           \
        T pc0, pc1;                                                                                                \
        IBM_RED_PAIR((k) + 1, A, B, C, so[buf], pc0, pc1, FR);                                                     \
        T out0, out1;                                                                                              \
        {                                                                                                          \
            const int l_ = (FR) ? lc : lc + 1;                                                                     \
            const bool live_ = (FR) ? (blk0 && (A).fl0()) : (blk1 && (A).fl1());                  \
            const T v_ = rb_update<T>((FR) ? axm0 : axm1, (FR) ? axp0 : axp1, aym, ayp, saz[0][(k) - k0 + 2],      \
                                      saz[1][(k) - k0 + 2], (FR) ? dxy0 : dxy1, sr[buf][ty + 1][l_],               \
                                      sr[buf][ty + 1][l_ + 2], sr[buf][ty][l_ + 1], sr[buf][ty + 2][l_ + 1],       \
                                      (FR) ? pa0 : pa1, (FR) ? pc0 : pc1, (FR) ? (A).f0 : (A).f1, lam);           \
            out0 = ((FR) && live_) ? v_ : pb0;                                                                     \
            out1 = (!(FR) && live_) ? v_ : pb1;                                                                    \
        }                                                                                                          \
        const int64_t id_ = (int64_t)(k) * plane + (int64_t)j * nx + ia;                                          \
        const bool kst_ = (k) < k1;                                                                                \
        if constexpr (VEC) { /* a pair is wholly inside or outside the tile interior: blk0 == blk1 */             \
            if (kst_ && blk0) { /* FP64: non-temporal (the pass does not re-read it; measured faster) */       \
                NV o_;                                                                                             \
                if constexpr (WIDEN)                                                                               \
                    o_ = NV{(A).dd0() ? TO(0) : (TO)out0, (A).dd1() ? TO(0) : (TO)out1};                           \
                else                                                                                               \
                    o_ = NV{out0, out1};                                                                           \
                if constexpr (sizeof(TO) == 8)                                                                     \
                    __builtin_nontemporal_store(o_, reinterpret_cast<NV *>(pout + id_));                           \
                else                                                                                               \
                    *reinterpret_cast<NV *>(pout + id_) = o_;                                                      \
            }                                                                                                      \
        } else if (kst_) {                                                                                         \
            const TO w0_ = (WIDEN && (A).dd0()) ? TO(0) : (TO)out0, w1_ = (WIDEN && (A).dd1()) ? TO(0) : (TO)out1; \
            if constexpr (sizeof(TO) == 8) {                                                                       \
                if (blk0) __builtin_nontemporal_store(w0_, pout + id_);                                            \
                if (blk1) __builtin_nontemporal_store(w1_, pout + id_ + 1);                                        \
            } else {                                                                                               \
                if (blk0) pout[id_] = w0_;                                                                         \
                if (blk1) pout[id_ + 1] = w1_;                                                                     \
            }                                                                                                      \
        }                                                                                                          \
        pa0 = pb0;                                                                                                 \
        pa1 = pb1;                                                                                                 \
        pb0 = pc0;                                                                                                 \
        pb1 = pc1;                                                                                                 \
        buf ^= 1;                                                                                                  \
        A = load((k) + SW_QD);                                                                                     \
    }

    // Queue: q2 = plane k, q3 = k+1, q4 = k+2, q5, q0, q1 = k+3..k+5 in flight; unrolled by the
    // queue depth so the slots change roles by name and no in-flight load is ever copied.
    // S: the first cell is red at plane k0 - 1 (then black at k0, red at k0 + 1, ...).
#define IBM_SWEEP_BODY(S)                                                                                         \
    {                                                                                                              \
        PD q0 = load(k0 - 2), q1 = load(k0 - 1), q2 = load(k0), q3 = load(k0 + 1), q4 = load(k0 + 2),             \
           q5 = load(k0 + 3);                                                                                      \
        T pa0, pa1, pb0, pb1; /* red-updated values of planes k-1 and k */                                         \
        so[0][ty + 1][lc + 1] = q1.o0;                                                                             \
        so[0][ty + 1][lc + 2] = q1.o1;                                                                             \
        __syncthreads();                                                                                           \
        IBM_RED_PAIR(k0 - 1, q0, q1, q2, so[0], pa0, pa1, (S));                                                    \
        q0 = load(k0 + 4);                                                                                         \
        so[1][ty + 1][lc + 1] = q2.o0;                                                                             \
        so[1][ty + 1][lc + 2] = q2.o1;                                                                             \
        __syncthreads();                                                                                           \
        IBM_RED_PAIR(k0, q1, q2, q3, so[1], pb0, pb1, !(S));                                                       \
        q1 = load(k0 + 5);                                                                                         \
        int buf = 0;                                                                                               \
        for (int k = k0; k < k1; k += SW_QD) { /* leaves as soon as plane k1 - 1 is done */                     \
            IBM_STEP(q2, q3, q4, k, (S));                                                                          \
            if (k + 1 >= k1) break;                                                                                \
            IBM_STEP(q3, q4, q5, k + 1, !(S));                                                                     \
            if (k + 2 >= k1) break;                                                                                \
            IBM_STEP(q4, q5, q0, k + 2, (S));                                                                      \
            if (k + 3 >= k1) break;                                                                                \
            IBM_STEP(q5, q0, q1, k + 3, !(S));                                                                     \
            if (k + 4 >= k1) break;                                                                                \
            IBM_STEP(q0, q1, q2, k + 4, (S));                                                                      \
            if (k + 5 >= k1) break;                                                                                \
            IBM_STEP(q1, q2, q3, k + 5, !(S));                                                                     \
        }                                                                                                          \
    }

    if (phase) IBM_SWEEP_BODY(true) else IBM_SWEEP_BODY(false)
#undef IBM_SWEEP_BODY
#undef IBM_STEP
#undef IBM_RED_PAIR
}

constexpr int SW_BXT = 32;
constexpr int SW_CHUNK_COST = 4;  // plane steps a z chunk costs beyond its own planes

// Tiles of 64 x BY columns (interior 60 x (BY - 4)).  The paired path (nx even) uses 32 rows:
// one 1024-thread workgroup per CU, 12 % fewer halo rows re-read than two 16-row tiles; the
// unpaired path keeps 16 rows (its larger register set would spill at 1024 threads).
// ev0, ev1 (optional): events the runtime records when the kernel starts and ends
template <typename T, typename TO, int BY, bool VEC>
static hipError_t launch_sweep_tiles(const Fine<T> &F, const T *pin, TO *pout, const T *f, const T *lam, hipStream_t s,
                                     hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    constexpr int TXC = 2 * SW_BXT - 4, TY = BY - 4;
    const int ntx = (F.nx + TXC - 1) / TXC, nty = (F.ny + TY - 1) / TY;
    const int64_t per_slab = (int64_t)ntx * nty;
    // Z chunks: a launch is rounds of resident workgroups (1024 threads per CU); a chunk of kc
    // planes costs about kc + SW_CHUNK_COST plane steps (three planes shared with its
    // neighbours, the two red planes of the prologue, the pipeline fill).  The chunk count
    // minimises rounds x (kc + SW_CHUNK_COST): one round when the tiles fill the CUs, else
    // several rounds of shorter chunks rather than a partly idle single round.  Workgroups
    // are ordered chunk by chunk, so those running together on one XCD are neighbouring tiles
    // at the same depth and share their halo lines in its L2.
    const int64_t slots = (int64_t)(1024 / (SW_BXT * BY)) * device_cu_count();
    const int kmin = std::min(16, F.nz);
    int nchunk = 1;
    int64_t best = -1;
    for (int c = 1; c <= F.nz; ++c) {
        const int kcc = (F.nz + c - 1) / c;
        if (kcc > SW_KC_MAX) continue;
        if (kcc < kmin) break;
        const int64_t rounds = (per_slab * c + slots - 1) / slots;
        const int64_t cost = rounds * (kcc + SW_CHUNK_COST);
        if (best < 0 || cost < best) {
            best = cost;
            nchunk = c;
        }
    }
    const int kc = (F.nz + nchunk - 1) / nchunk;
    nchunk = (F.nz + kc - 1) / kc;
    const int ntiles = (int)(per_slab * nchunk);
    const int grid = ((ntiles + 7) / 8) * 8;
    if (ev0)
        hipExtLaunchKernelGGL((k_rbgs_fused<T, TO, SW_BXT, BY, VEC>), dim3(grid), dim3(SW_BXT * BY), 0, s, ev0, ev1, 0, F,
                              pin, pout, f, lam, ntx, nty, kc, ntiles);
    else
        hipLaunchKernelGGL((k_rbgs_fused<T, TO, SW_BXT, BY, VEC>), dim3(grid), dim3(SW_BXT * BY), 0, s, F, pin, pout, f,
                           lam, ntx, nty, kc, ntiles);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const Fine<T> &F, const T *pin, T *pout, const T *f, const T *lam, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1) {
    if ((F.nx & 1) == 0) return launch_sweep_tiles<T, T, 32, true>(F, pin, pout, f, lam, s, ev0, ev1);
    return launch_sweep_tiles<T, T, 16, false>(F, pin, pout, f, lam, s, ev0, ev1);
}

hipError_t launch_sweep_widen(const Fine<float> &F, const float *pin, double *pout, const float *f, const float *lam,
                              hipStream_t s) {
    if ((F.nx & 1) == 0) return launch_sweep_tiles<float, double, 32, true>(F, pin, pout, f, lam, s);
    return launch_sweep_tiles<float, double, 16, false>(F, pin, pout, f, lam, s);
}

template hipError_t launch_sweep<double>(const Fine<double> &, const double *, double *, const double *,
                                         const double *, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sweep<float>(const Fine<float> &, const float *, float *, const float *, const float *,
                                        hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace ibm
