// Fused red-black Gauss-Seidel sweep of the coarse multigrid levels that are smoothed level
// by level (Section 2.1: red-black Gauss-Seidel smoothing, applied here to the coarse
// staircase operator of each level).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.hpp"
#include "ibm_impl.hpp"

namespace ibm {

// =======================================================================================
// One sweep updates every red cell ((I+J+K) even) from the old values, then every black
// cell from the new red values:
//     e_c = (sum_f T_f e_nb - (R_c - V_c mu)) / sum_f T_f     where sum_f T_f > 0.
// Both colours are done in one out-of-place pass with the z-march of the level-0 sweep: a
// workgroup owns a tile of 64 x BY columns (interior 60 x (BY-4)) and a chunk of planes; at
// step k it forms the red values of plane k+1 and the black values of plane k.  Each thread
// owns two adjacent columns, so it holds one red and one black cell per plane.
// The coarse operator is not separable: each cell carries the transmissibilities of its
// three low faces.  The high faces are the low faces of the +x, +y and +z neighbours: +x
// from the neighbouring lane (one shuffle), +y from LDS, +z from the next plane in the
// queue.  A face is open only when the fine cells on both of its sides are active, so a
// cell with an open face is active and an inactive cell has none: the test sum_f T_f > 0
// already excludes inactive cells, and the activity mask is not read.  Wall faces hold 0.
// Per cell the operations and their order are those of the one-colour kernel (k_sweepC),
// so both give the same bits.
// Algorithmic traffic per cell: read e, R and three transmissibilities, write e
// (48 B in FP64, 24 B in FP32).
// =======================================================================================

// one plane of a thread's two columns: old values, right-hand side, low-face
// transmissibilities in x, y and z
template <typename T>
struct CPlane {
    using V = typename Pair2<T>::type;
    V e, r, x, y, z;
};

constexpr int SWC_KC_MAX = 512;  // longest z chunk of one workgroup
constexpr int SWC_NC = 64;       // columns of a tile including the 2-column halo
constexpr int SWC_KC_MIN = 8;    // shortest z chunk (each chunk re-reads four planes)
// Levels below this size keep the two one-colour passes: there the z-march is bound by the
// latency of its plane steps, not by bandwidth (at 64^3 the fused pass took 10.4 us against
// 2 x 4.8 us; at 128^3 22 us against 2 x 19.5 us).
constexpr int64_t SWC_MIN_CELLS = 3 << 17;

// Relaxation value of one cell: the six neighbour products summed from zero in the order
// -x, +x, -y, +y, -z, +z, the diagonal summed in the same order.  A missing neighbour meets
// a zero transmissibility (a wall face, or a high face masked where the level ends), so its
// product is an exact zero; the sum starts at +0 and never becomes -0, so adding that zero
// changes nothing, and the result has the bits of the one-colour kernel, which skips the
// term.
template <typename T>
__device__ __forceinline__ T rbc_update(T txm, T txp, T tym, T typ, T tzm, T tzp, T xm, T xp, T ym, T yp, T zm, T zp,
                                        T r, T vol, T mu, T &diag) {
    T s = T(0);
    s = s + txm * xm;
    s = s + txp * xp;
    s = s + tym * ym;
    s = s + typ * yp;
    s = s + tzm * zm;
    s = s + tzp * zp;
    T d = txm + txp;
    d = d + tym;
    d = d + typ;
    d = d + tzm;
    d = d + tzp;
    diag = d;
    return (s - (r - vol * mu)) / d;
}

// Thread layout as in the level-0 sweep: 32 threads span the 64 columns of a tile row; a
// wave holds two rows of the same parity, so the colour phase is uniform per wave and the
// plane loop is specialised for both phases.  VEC (even row length): a thread's column pair
// is 2-element aligned and moves as one access; with an odd row length the two columns are
// loaded and stored one by one.
// Every thread issues the same loads for every plane (addresses clamped into the level);
// values read through clamped addresses are finite copies of level cells that only meet
// zero transmissibilities (walls, or the masked high faces of the last row, column and
// plane), so they enter no result.
template <typename T, int BY, int QD, bool VEC>
__global__ void __launch_bounds__(32 * BY)
    k_rbgsC_fused(Coarse<T> L, T *__restrict__ eout, int ntx, int nty, int kc, int ntiles) {
    static_assert(BY % 4 == 0, "two same-parity rows of 32 threads per wave");
    static_assert(QD == 4 || QD == 6, "planes held per thread");
    using V = typename Pair2<T>::type;
    typedef T U2v __attribute__((ext_vector_type(2)));
    typedef U2v U __attribute__((aligned(sizeof(T))));  // a pair at element alignment (odd rows)
    using PD = CPlane<T>;
    constexpr int NC = SWC_NC, TXC = NC - 4, TY = BY - 4;
    __shared__ T so[2][BY][NC + 1];  // old values of the plane whose red values are formed
    __shared__ T sr[2][BY][NC + 1];  // red-updated values of the plane whose black values are formed
    __shared__ T sy[3][BY][NC + 1];  // low-y transmissibilities of the planes, by plane mod 3
    __shared__ T sw[SWC_KC_MAX + 8];  // z widths of planes k0-2 .. k1+5
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
    const int tx = lane & 31;
    const int ty = (wave >> 1) * 4 + (wave & 1) + 2 * (lane >> 5);
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    const int k0 = chunk * kc, k1 = min(nz, k0 + kc);
    for (int q = (int)threadIdx.x; q < kc + 8; q += 32 * BY) {
        const int kk = k0 - 2 + q;
        sw[q] = (kk >= 0 && kk < nz) ? L.w[2][kk] : T(0);
    }
    const int lc = 2 * tx;
    const int ia = txi * TXC - 2 + lc;  // global column of the first cell (even)
    const int j = tyi * TY - 2 + ty;
    const bool rowin = j >= 0 && j < ny;
    const bool in0 = rowin && ia >= 0 && ia < nx, in1 = rowin && ia + 1 >= 0 && ia + 1 < nx;
    const int yr = min(ty, BY - 1 - ty);
    const int xr0 = min(lc, NC - 1 - lc), xr1 = min(lc + 1, NC - 2 - lc);
    const bool red0 = in0 && yr >= 1 && xr0 >= 1, red1 = in1 && yr >= 1 && xr1 >= 1;
    const bool blk0 = in0 && yr >= 2 && xr0 >= 2, blk1 = in1 && yr >= 2 && xr1 >= 2;
    const bool hx1 = ia + 2 < nx;  // the second cell has a +x neighbour
    const bool hy = j + 1 < ny;    // the row has a +y neighbour
    // element offsets fit 32 bits (a coarse level holds at most 2^28 cells), which lets the
    // loads address from a scalar base plus one 32-bit register
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const int jc = min(max(j, 0), ny - 1);
    const int icv = min(max(ia, 0), nx - 2);
    // Odd row length: rows start at alternating parity, so a thread's pair is only 8-byte
    // aligned; it still moves as one access (the target allows vector accesses at element
    // alignment), starting at icv like the aligned pairs.  On the last column of a row
    // (ia = nx - 1) the pair is (nx - 2, nx - 1) and the thread's first cell is its second
    // element (shifted); its second cell lies past the grid.
    const bool shf = !VEC && ia == nx - 1;
    const uint32_t rowoff = (uint32_t)jc * nx + icv;
    // The outermost halo rows are never updated: their right-hand side and x, z
    // transmissibilities are read from the adjacent row (lines the tile reads anyway), and
    // so is the y transmissibility of the first row (the last row's is the +y face of the
    // row below it).
    const int jr = min(max((ty == 0) ? j + 1 : (ty == BY - 1) ? j - 1 : j, 0), ny - 1);
    const int jy = min(max((ty == 0) ? j + 1 : j, 0), ny - 1);
    const uint32_t roff = (uint32_t)jr * nx + icv, yoff = (uint32_t)jy * nx + icv;
    // unpaired path: the second column is missing at the high wall of an odd row, where the
    // first column's high face is the wall (its x transmissibility must read 0, not the
    // clamped copy of the first column's low face)
    const bool x1in = VEC || ia + 1 < nx;
    const T vxy0 = in0 ? L.w[0][ia] * L.w[1][jc] : T(0);
    const T vxy1 = in1 ? L.w[0][ia + 1] * L.w[1][jc] : T(0);
    const T mu = (T)(*L.mu);
    // LDS rows and columns of the neighbours, clamped into the tile (lanes whose result is
    // discarded read valid entries)
    const int rym = max(ty - 1, 0), ryp = min(ty + 1, BY - 1);
    const int cm0 = max(lc - 1, 0), cp1 = min(lc + 2, NC - 1);
    const bool phase = ((wave + (tyi * TY) + k0) & 1) != 0;
    const int klast = min(k1 + 1, nz - 1);
    const T *__restrict__ pe = L.e;
    const T *__restrict__ pr = L.R;
    const T *__restrict__ px = L.Tl[0];
    const T *__restrict__ py = L.Tl[1];
    const T *__restrict__ pz = L.Tl[2];
    auto load = [=](int k) -> PD {
        PD d;
        const uint32_t base = (uint32_t)min(max(k, 0), klast) * plane;
        if constexpr (VEC) {
            d.e = *reinterpret_cast<const V *>(pe + base + rowoff);
            d.r = *reinterpret_cast<const V *>(pr + base + roff);
            d.x = *reinterpret_cast<const V *>(px + base + roff);
            d.y = *reinterpret_cast<const V *>(py + base + yoff);
            d.z = *reinterpret_cast<const V *>(pz + base + roff);
        } else {
            const U e2 = *reinterpret_cast<const U *>(pe + base + rowoff);
            const U r2 = *reinterpret_cast<const U *>(pr + base + roff);
            const U x2 = *reinterpret_cast<const U *>(px + base + roff);
            const U y2 = *reinterpret_cast<const U *>(py + base + yoff);
            const U z2 = *reinterpret_cast<const U *>(pz + base + roff);
            d.e.x = shf ? e2.y : e2.x;
            d.e.y = e2.y;
            d.r.x = shf ? r2.y : r2.x;
            d.r.y = r2.y;
            d.x.x = shf ? x2.y : x2.x;
            d.x.y = x1in ? x2.y : T(0);
            d.y.x = shf ? y2.y : y2.x;
            d.y.y = y2.y;
            d.z.x = shf ? z2.y : z2.x;
            d.z.y = z2.y;
        }
        return d;
    };
    // LDS buffer of plane q's y transmissibilities (q >= k0 - 1)
#define IBMC_YB(q) (((q) - k0 + 3) % 3)

    // Red-updated values of plane q from M = plane q-1, C = plane q, P = plane q+1, OB = LDS
    // of the old values of plane q.  FR (compile-time): the first cell is the red one.
#define IBMC_RED(q, M, C, P, OB, R0, R1, FR)                                                                       \
    {                                                                                                              \
        const int l_ = (FR) ? lc : lc + 1;                                                                         \
        const T xn_ = __shfl_down((C).x.x, 1, 64);                                                                 \
        const T txm_ = (FR) ? (C).x.x : (C).x.y;                                                                   \
        const T txp_ = (FR) ? (C).x.y : (hx1 ? xn_ : T(0));                                                        \
        const T tym_ = (FR) ? (C).y.x : (C).y.y;                                                                   \
        const T typ_ = hy ? sy[IBMC_YB(q)][ryp][l_] : T(0);                                                        \
        const T tzm_ = (FR) ? (C).z.x : (C).z.y;                                                                   \
        const T tzp_ = ((q) + 1 < nz) ? ((FR) ? (P).z.x : (P).z.y) : T(0);                                         \
        T d_;                                                                                                      \
        const T v_ = rbc_update<T>(txm_, txp_, tym_, typ_, tzm_, tzp_, OB[ty][(FR) ? cm0 : lc], OB[ty][(FR) ? lc + 1 : cp1], \
                                   OB[rym][l_], OB[ryp][l_], (FR) ? (M).e.x : (M).e.y, (FR) ? (P).e.x : (P).e.y,    \
                                   (FR) ? (C).r.x : (C).r.y, ((FR) ? vxy0 : vxy1) * sw[(q) - k0 + 2], mu, d_);      \
        const bool live_ = ((FR) ? red0 : red1) && (q) >= 0 && (q) < nz && d_ > T(0);                             \
        R0 = ((FR) && live_) ? v_ : (C).e.x;                                                                       \
        R1 = (!(FR) && live_) ? v_ : (C).e.y;                                                                      \
    }

    // One plane step: A = plane k, B = k+1, C = k+2 (QD - 3 more planes in flight);
    // afterwards the slot A receives plane k + QD.  Steps past the chunk end compute from clamped data
    // and store nothing.
#define IBMC_STEP(A, B, C, k, FR)                                                                                  \
    {                                                                                                              \
        so[buf][ty][lc] = (B).e.x;                                                                                 \
        so[buf][ty][lc + 1] = (B).e.y;                                                                             \
        sr[buf][ty][lc] = pb0;                                                                                     \
        sr[buf][ty][lc + 1] = pb1;                                                                                 \
        sy[IBMC_YB((k) + 1)][ty][lc] = (B).y.x;                                                                    \
        sy[IBMC_YB((k) + 1)][ty][lc + 1] = (B).y.y;                                                                \
        __syncthreads();                                                                                           \
        T pc0, pc1;                                                                                                \
        IBMC_RED((k) + 1, A, B, C, so[buf], pc0, pc1, FR);                                                         \
        T out0, out1;                                                                                              \
        {                                                                                                          \
            const int l_ = (FR) ? lc : lc + 1;                                                                     \
            const T xn_ = __shfl_down((A).x.x, 1, 64);                                                             \
            const T txm_ = (FR) ? (A).x.x : (A).x.y;                                                               \
            const T txp_ = (FR) ? (A).x.y : (hx1 ? xn_ : T(0));                                                    \
            const T tym_ = (FR) ? (A).y.x : (A).y.y;                                                               \
            const T typ_ = hy ? sy[IBMC_YB(k)][ryp][l_] : T(0);                                                    \
            const T tzm_ = (FR) ? (A).z.x : (A).z.y;                                                               \
            const T tzp_ = ((k) + 1 < nz) ? ((FR) ? (B).z.x : (B).z.y) : T(0);                                     \
            T d_;                                                                                                  \
            const T v_ = rbc_update<T>(txm_, txp_, tym_, typ_, tzm_, tzp_, sr[buf][ty][(FR) ? cm0 : lc],           \
                                       sr[buf][ty][(FR) ? lc + 1 : cp1], sr[buf][rym][l_], sr[buf][ryp][l_],       \
                                       (FR) ? pa0 : pa1, (FR) ? pc0 : pc1, (FR) ? (A).r.x : (A).r.y,               \
                                       ((FR) ? vxy0 : vxy1) * sw[(k) - k0 + 2], mu, d_);                           \
            const bool live_ = ((FR) ? blk0 : blk1) && d_ > T(0);                                                  \
            out0 = ((FR) && live_) ? v_ : pb0;                                                                     \
            out1 = (!(FR) && live_) ? v_ : pb1;                                                                    \
        }                                                                                                          \
        if constexpr (VEC) {                                                                                       \
            if ((k) < k1 && blk0) { /* a pair is wholly inside or outside the tile interior */                    \
                V o_;                                                                                              \
                o_.x = out0;                                                                                       \
                o_.y = out1;                                                                                       \
                *reinterpret_cast<V *>(eout + ((uint32_t)(k) * plane + (uint32_t)j * nx + ia)) = o_;                   \
            }                                                                                                      \
        } else if ((k) < k1) { /* both cells or, at the last column of a row, the first alone */                  \
            const uint32_t o_ = (uint32_t)(k) * plane + (uint32_t)j * nx + ia;                                     \
            if (blk0 && blk1) {                                                                                    \
                U o2_;                                                                                             \
                o2_.x = out0;                                                                                      \
                o2_.y = out1;                                                                                      \
                *reinterpret_cast<U *>(eout + o_) = o2_;                                                           \
            } else if (blk0) {                                                                                     \
                eout[o_] = out0;                                                                                   \
            }                                                                                                      \
        }                                                                                                          \
        pa0 = pb0;                                                                                                 \
        pa1 = pb1;                                                                                                 \
        pb0 = pc0;                                                                                                 \
        pb1 = pc1;                                                                                                 \
        buf ^= 1;                                                                                                  \
        A = load((k) + QD);                                                                                        \
    }

    // Queue of QD planes: at step k the slots hold planes k .. k+QD-1 (the last QD-3 in
    // flight); unrolled by the queue depth so the slots change roles by name and no in-flight
    // load is ever copied.  S: the first cell is red at plane k0 - 1.
#define IBMC_BODY(S)                                                                                               \
    {                                                                                                              \
        PD q0 = load(k0 - 2), q1 = load(k0 - 1), q2 = load(k0), q3 = load(k0 + 1);                                 \
        [[maybe_unused]] PD q4, q5;                                                                                \
        if constexpr (QD == 6) {                                                                                   \
            q4 = load(k0 + 2);                                                                                     \
            q5 = load(k0 + 3);                                                                                     \
        }                                                                                                          \
        T pa0, pa1, pb0, pb1;                                                                                      \
        so[0][ty][lc] = q1.e.x;                                                                                    \
        so[0][ty][lc + 1] = q1.e.y;                                                                                \
        sy[IBMC_YB(k0 - 1)][ty][lc] = q1.y.x;                                                                      \
        sy[IBMC_YB(k0 - 1)][ty][lc + 1] = q1.y.y;                                                                  \
        sy[IBMC_YB(k0)][ty][lc] = q2.y.x;                                                                          \
        sy[IBMC_YB(k0)][ty][lc + 1] = q2.y.y;                                                                      \
        __syncthreads();                                                                                           \
        IBMC_RED(k0 - 1, q0, q1, q2, so[0], pa0, pa1, (S));                                                        \
        q0 = load(k0 + QD - 2);                                                                                    \
        so[1][ty][lc] = q2.e.x;                                                                                    \
        so[1][ty][lc + 1] = q2.e.y;                                                                                \
        __syncthreads();                                                                                           \
        IBMC_RED(k0, q1, q2, q3, so[1], pb0, pb1, !(S));                                                           \
        q1 = load(k0 + QD - 1);                                                                                    \
        int buf = 0;                                                                                               \
        if constexpr (QD == 4) {                                                                                   \
            for (int k = k0; k < k1; k += 4) {                                                                     \
                IBMC_STEP(q2, q3, q0, k, (S));                                                                     \
                IBMC_STEP(q3, q0, q1, k + 1, !(S));                                                                \
                IBMC_STEP(q0, q1, q2, k + 2, (S));                                                                 \
                IBMC_STEP(q1, q2, q3, k + 3, !(S));                                                                \
            }                                                                                                      \
        } else {                                                                                                   \
            for (int k = k0; k < k1; k += 6) {                                                                     \
                IBMC_STEP(q2, q3, q4, k, (S));                                                                     \
                IBMC_STEP(q3, q4, q5, k + 1, !(S));                                                                \
                IBMC_STEP(q4, q5, q0, k + 2, (S));                                                                 \
                IBMC_STEP(q5, q0, q1, k + 3, !(S));                                                                \
                IBMC_STEP(q0, q1, q2, k + 4, (S));                                                                 \
                IBMC_STEP(q1, q2, q3, k + 5, !(S));                                                                \
            }                                                                                                      \
        }                                                                                                          \
    }

    if (phase) IBMC_BODY(true) else IBMC_BODY(false)
#undef IBMC_BODY
#undef IBMC_STEP
#undef IBMC_RED
#undef IBMC_YB
}

// Tile rows and queue depth per precision.  FP64: 16 rows (512 threads, so the plane queue
// stays in registers; 32 rows spill it) and four planes (a deeper queue measured slower).
// FP32: 32 rows, four planes.
template <typename T>
struct SwcRows;
template <>
struct SwcRows<double> {
    static constexpr int BY = 16, QD = 4;
};
template <>
struct SwcRows<float> {
    static constexpr int BY = 32, QD = 4;
};

bool sweepC_fused_ok(const int n[3]) {
    return n[0] >= 2 && (int64_t)n[0] * n[1] * n[2] >= SWC_MIN_CELLS;
}

template <typename T>
hipError_t launch_sweepC_fused(const Coarse<T> &L, T *eout, hipStream_t s) {
    if (!sweepC_fused_ok(L.n)) return hipErrorInvalidValue;
    constexpr int BY = SwcRows<T>::BY, QD = SwcRows<T>::QD;
    constexpr int TXC = SWC_NC - 4, TY = BY - 4;
    const int ntx = (L.n[0] + TXC - 1) / TXC, nty = (L.n[1] + TY - 1) / TY;
    const int64_t per_slab = (int64_t)ntx * nty;
    // one workgroup per CU; chunks as long as that residency allows, but no shorter than
    // kcmin planes (each chunk re-reads four planes of its neighbours)
    const int kcmin = SWC_KC_MIN;
    const int slots = device_cu_count();
    int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(slots / per_slab, L.n[2]));
    int kc = (L.n[2] + nchunk - 1) / nchunk;
    kc = std::max(kc, std::min(kcmin, L.n[2]));
    kc = std::min(kc, SWC_KC_MAX);
    nchunk = (L.n[2] + kc - 1) / kc;
    const int ntiles = (int)(per_slab * nchunk);
    const int grid = ((ntiles + 7) / 8) * 8;
    if ((L.n[0] & 1) == 0)
        hipLaunchKernelGGL((k_rbgsC_fused<T, BY, QD, true>), dim3(grid), dim3(32 * BY), 0, s, L, eout, ntx, nty, kc,
                           ntiles);
    else
        hipLaunchKernelGGL((k_rbgsC_fused<T, BY, QD, false>), dim3(grid), dim3(32 * BY), 0, s, L, eout, ntx, nty, kc,
                           ntiles);
    return hipGetLastError();
}

template hipError_t launch_sweepC_fused<double>(const Coarse<double> &, double *, hipStream_t);
template hipError_t launch_sweepC_fused<float>(const Coarse<float> &, float *, hipStream_t);

}  // namespace ibm
