// Geometry kernels: grid metrics, triangle bucket grid, ray-parity classification, ghost
// identification and compaction, body intercepts, image points and interpolation weights,
// and the multigrid hierarchy (active masks, staircase transmissibilities, prolongation
// tables).  Paper Section 2.1 (non-uniform Cartesian grid) and Section 2.2 (ghost cells).
//
// Floating-point contraction is disabled for this library, so every geometric predicate is
// evaluated with the same IEEE operations in the same order as a plain sequential
// evaluation: classification and intercepts are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "ibm_impl.hpp"

namespace ibm {

// ---------------------------------------------------------------------------------------
// grid metrics (Section 2.1): centres, widths, centre distances, flux coefficients
// ---------------------------------------------------------------------------------------

__global__ void k_axis_metrics(int n, const double *__restrict__ f, double *c, double *w, double *dc, double *am,
                               double *ap, float *amf, float *apf, float *wf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ci = 0.5 * (f[i] + f[i + 1]);
    double wi = f[i + 1] - f[i];
    c[i] = ci;
    w[i] = wi;
    // centre distance across face i (between cells i-1 and i); 0 at the low wall
    double cm = (i > 0) ? 0.5 * (f[i - 1] + f[i]) : 0.0;
    double cp = (i < n - 1) ? 0.5 * (f[i + 1] + f[i + 2]) : 0.0;
    double d_lo = (i > 0) ? ci - cm : 0.0;
    double d_hi = (i < n - 1) ? cp - ci : 0.0;
    dc[i] = d_lo;
    // per-volume flux coefficients; the box walls carry no flux (homogeneous Neumann)
    double a_m = (i > 0) ? 1.0 / (wi * d_lo) : 0.0;
    double a_p = (i < n - 1) ? 1.0 / (wi * d_hi) : 0.0;
    am[i] = a_m;
    ap[i] = a_p;
    amf[i] = (float)a_m;
    apf[i] = (float)a_p;
    wf[i] = (float)wi;
}

__global__ void k_level_axis(int n, const double *__restrict__ f, double *c, double *w, float *wf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    c[i] = 0.5 * (f[i] + f[i + 1]);
    w[i] = f[i + 1] - f[i];
    wf[i] = (float)(f[i + 1] - f[i]);
}

__global__ void k_prolong_tab(int nf, int nc, const int *__restrict__ cs, const double *__restrict__ fc,
                              const double *__restrict__ cc, int *lo, int *hi, double *t);

hipError_t launch_metrics(ibm_grid *g, hipStream_t s) {
    int n[3] = {g->nx, g->ny, g->nz};
    for (int d = 0; d < 3; ++d) {
        hipLaunchKernelGGL(k_axis_metrics, dim3((n[d] + 127) / 128), dim3(128), 0, s, n[d], g->faces[d], g->c0[d],
                           g->w0[d], g->dc0[d], g->am0[d], g->ap0[d], g->am0f[d], g->ap0f[d], g->w0f[d]);
    }
    for (int l = 1; l < g->nlev; ++l) {
        LevelHost &L = g->lev[l];
        for (int d = 0; d < 3; ++d) {
            // coarse faces were uploaded behind the centres array (see layout)
            hipLaunchKernelGGL(k_level_axis, dim3((L.n[d] + 127) / 128), dim3(128), 0, s, L.n[d],
                               L.c64[d] + L.n[d], L.c64[d], L.w64[d], L.w32[d]);
        }
    }
    // prolongation tables: they depend on the grid alone, so they are built here once
    for (int l = 1; l < g->nlev; ++l) {
        LevelHost &Fh = g->lev[l - 1], &Ch = g->lev[l];
        for (int d = 0; d < 3; ++d) {
            const double *fc = (l == 1) ? g->c0[d] : Fh.c64[d];
            hipLaunchKernelGGL(k_prolong_tab, dim3((Fh.n[d] + 127) / 128), dim3(128), 0, s, Fh.n[d], Ch.n[d],
                               Ch.cs_d[d], fc, Ch.c64[d], Fh.plo[d], Fh.phi[d], Fh.pt[d]);
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// exclusive scan of int32 counts (three kernels, fixed decomposition)
// ---------------------------------------------------------------------------------------

constexpr int SCAN_NT = 256, SCAN_PER = 16, SCAN_CH = SCAN_NT * SCAN_PER;

__global__ void __launch_bounds__(SCAN_NT) k_scan_blocks(const int32_t *in, int32_t *out, int64_t n, int64_t *blk) {
    __shared__ int64_t sh[SCAN_NT];
    int tid = threadIdx.x;
    int64_t base = (int64_t)blockIdx.x * SCAN_CH + (int64_t)tid * SCAN_PER;
    int64_t loc[SCAN_PER];
    int64_t s = 0;
    for (int q = 0; q < SCAN_PER; ++q) {
        int64_t idx = base + q;
        loc[q] = s;
        s += (idx < n) ? in[idx] : 0;
    }
    sh[tid] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread sums
    for (int o = 1; o < SCAN_NT; o <<= 1) {
        int64_t v = (tid >= o) ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += v;
        __syncthreads();
    }
    int64_t excl = sh[tid] - s;
    for (int q = 0; q < SCAN_PER; ++q) {
        int64_t idx = base + q;
        if (idx < n) out[idx] = (int32_t)(excl + loc[q]);
    }
    if (tid == SCAN_NT - 1) blk[blockIdx.x] = sh[tid];
}

// single block: exclusive scan of the block totals, total -> blk[nb]
__global__ void __launch_bounds__(SCAN_NT) k_scan_top(int64_t *blk, int64_t nb) {
    __shared__ int64_t sh[SCAN_NT];
    __shared__ int64_t carry;
    int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_NT) {
        int64_t idx = b0 + tid;
        int64_t v = (idx < nb) ? blk[idx] : 0;
        sh[tid] = v;
        __syncthreads();
        for (int o = 1; o < SCAN_NT; o <<= 1) {
            int64_t t = (tid >= o) ? sh[tid - o] : 0;
            __syncthreads();
            sh[tid] += t;
            __syncthreads();
        }
        int64_t c = carry;
        if (idx < nb) blk[idx] = c + sh[tid] - v;
        __syncthreads();
        if (tid == SCAN_NT - 1) carry = c + sh[tid];
        __syncthreads();
    }
    if (tid == 0) blk[nb] = carry;
}

__global__ void k_scan_add(int32_t *out, int64_t n, const int64_t *blk) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += (int32_t)blk[idx / SCAN_CH];
}

// exclusive scan of n counts into out[0..n) and the total into *total_dev (int64)
static hipError_t scan_counts(const int32_t *in, int32_t *out, int64_t n, int64_t *blk, hipStream_t s) {
    int64_t nb = (n + SCAN_CH - 1) / SCAN_CH;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(SCAN_NT), 0, s, in, out, n, blk);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_NT), 0, s, blk, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, blk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// triangle bucket grid for the closest-point search
// ---------------------------------------------------------------------------------------

// Each triangle is listed once, in the bucket holding the low corner of its bounding box;
// a box query reaches every triangle whose bounding box meets it by extending the box's low
// side by the largest triangle extent ext.
struct BucketGrid {
    double bmin[3], bsize[3], ext[3];
    int nb[3];
};

__device__ __forceinline__ int bucket_coord(double x, double bmin, double bsize, int nb) {
    double q = floor((x - bmin) / bsize);
    int b = (q < 0.0) ? 0 : (q >= (double)nb ? nb - 1 : (int)q);
    return b;
}

__device__ __forceinline__ void tri_bbox(const double *V, const int32_t *T, int64_t t, double lo[3], double hi[3]) {
    const int32_t a = T[3 * t], b = T[3 * t + 1], c = T[3 * t + 2];
    for (int d = 0; d < 3; ++d) {
        double x = V[3 * a + d], y = V[3 * b + d], z = V[3 * c + d];
        lo[d] = fmin(x, fmin(y, z));
        hi[d] = fmax(x, fmax(y, z));
    }
}

__global__ void k_bucket_pass(const double *__restrict__ V, const int32_t *__restrict__ T, int64_t nt, BucketGrid G,
                              int32_t *cnt, const int32_t *off, int32_t *fill, int32_t *ent, int64_t cap,
                              int64_t *overflow) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double lo[3], hi[3];
    tri_bbox(V, T, t, lo, hi);
    int bc[3];
    for (int d = 0; d < 3; ++d) bc[d] = bucket_coord(lo[d], G.bmin[d], G.bsize[d], G.nb[d]);
    const int b = (bc[2] * G.nb[1] + bc[1]) * G.nb[0] + bc[0];
    if (!ent) {
        atomicAdd(&cnt[b], 1);
    } else {
        int slot = atomicAdd(&fill[b], 1);
        int64_t pos = (int64_t)off[b] + slot;
        if (pos < cap) ent[pos] = (int32_t)t;
        else atomicAdd((unsigned long long *)overflow, 1ull);
    }
}

hipError_t launch_buckets(ibm_grid *g, hipStream_t s) {
    BucketGrid G;
    for (int d = 0; d < 3; ++d) {
        G.bmin[d] = g->bmin[d];
        G.bsize[d] = g->bsize[d];
        G.ext[d] = g->bext[d];
        G.nb[d] = g->nb[d];
    }
    int64_t nbk = (int64_t)g->nb[0] * g->nb[1] * g->nb[2];
    hipError_t e = hipMemsetAsync(g->bucket_cnt, 0, sizeof(int32_t) * (nbk + 1), s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(g->col_fill, 0, sizeof(int32_t) * (nbk + 1), s);
    if (e != hipSuccess) return e;
    unsigned nblk = (unsigned)((g->nt + 255) / 256);
    e = hipMemsetAsync(g->counters + 6, 0, sizeof(int64_t), s);
    if (e != hipSuccess) return e;
    const int64_t cap = 8 * g->nt_max + 16;
    hipLaunchKernelGGL(k_bucket_pass, dim3(nblk), dim3(256), 0, s, g->verts, g->tris, g->nt, G, g->bucket_cnt,
                       nullptr, nullptr, nullptr, cap, g->counters + 6);
    e = scan_counts(g->bucket_cnt, g->bucket_off, nbk + 1, (int64_t *)g->blk_cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_pass, dim3(nblk), dim3(256), 0, s, g->verts, g->tris, g->nt, G, nullptr,
                       g->bucket_off, g->col_fill, g->bucket_ent, cap, g->counters + 6);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// classification (Section 2.2: ray tracing).  z-rays through every column centre.
// ---------------------------------------------------------------------------------------

// Edge function of the undirected edge {u,v}, evaluated from its lower vertex index so the
// two triangles sharing the edge see exactly opposite values; > 0 when (px,py) lies left
// of the directed edge u->v.
__device__ __forceinline__ double edge_fn(const double *V, int32_t u, int32_t v, double px, double py) {
    int32_t lo = u < v ? u : v, hi = u < v ? v : u;
    double ax = V[3 * lo], ay = V[3 * lo + 1], bx = V[3 * hi], by = V[3 * hi + 1];
    double e = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
    return (u == lo) ? e : -e;
}

// a point exactly on an edge of a counter-clockwise triangle belongs to it when the edge is
// a left edge (pointing down) or a top edge (horizontal, pointing left)
__device__ __forceinline__ bool owns_edge(const double *V, int32_t u, int32_t v) {
    double dx = V[3 * v] - V[3 * u], dy = V[3 * v + 1] - V[3 * u + 1];
    return (dy < 0.0) || (dy == 0.0 && dx < 0.0);
}

__device__ __forceinline__ bool ray_hits(const double *V, const int32_t *tri, double px, double py, double *z) {
    int32_t a = tri[0], b = tri[1], c = tri[2];
    double area = edge_fn(V, a, b, V[3 * c], V[3 * c + 1]);
    if (area == 0.0) return false;
    if (area < 0.0) {
        int32_t t = b;
        b = c;
        c = t;
    }
    double wab = edge_fn(V, a, b, px, py);
    double wbc = edge_fn(V, b, c, px, py);
    double wca = edge_fn(V, c, a, px, py);
    bool in = ((wab > 0.0) || (wab == 0.0 && owns_edge(V, a, b))) && ((wbc > 0.0) || (wbc == 0.0 && owns_edge(V, b, c))) &&
              ((wca > 0.0) || (wca == 0.0 && owns_edge(V, c, a)));
    if (!in) return false;
    // barycentric z: each vertex weighted by the edge function of the opposite edge, written
    // relative to vertex a so that a horizontal facet gives its height exactly
    const double za = V[3 * a + 2];
    double num = wca * (V[3 * b + 2] - za);
    num = num + wab * (V[3 * c + 2] - za);
    double den = wbc + wca;
    den = den + wab;
    *z = za + num / den;
    return true;
}

// one column of a triangle: its +z crossing, counted (cnt) or stored at the column's next
// slot (zs)
__device__ __forceinline__ void col_cross(const double *V, const int32_t *tri, const double *xc, const double *yc,
                                          int nx, int i, int j, int32_t *cnt, const int32_t *off, int32_t *fill,
                                          double *zs, int64_t cap, int64_t *overflow) {
    double z;
    if (!ray_hits(V, tri, xc[i], yc[j], &z)) return;
    const int64_t col = (int64_t)j * nx + i;
    if (!zs) {
        atomicAdd(&cnt[col], 1);
    } else {
        const int slot = atomicAdd(&fill[col], 1);
        const int64_t pos = (int64_t)off[col] + slot;
        if (pos < cap) zs[pos] = z;
        else atomicAdd((unsigned long long *)overflow, 1ull);
    }
}

// One triangle per lane.  A lane visits the columns of its triangle's xy bounding box
// itself when there are at most COL_SMALL of them (the usual case: triangles smaller than
// a cell); triangles with more columns are then taken one at a time by the whole wave,
// its lanes striding over the columns.
constexpr int COL_NT = 256, COL_SMALL = 8;
__global__ void __launch_bounds__(COL_NT) k_col_pass(const double *__restrict__ V, const int32_t *__restrict__ T,
                                                     int64_t nt, const double *__restrict__ xc,
                                                     const double *__restrict__ yc, int nx, int ny, int32_t *cnt,
                                                     const int32_t *off, int32_t *fill, double *zs, int64_t cap,
                                                     int64_t *overflow) {
    const int64_t t = (int64_t)blockIdx.x * COL_NT + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int i0 = 0, j0 = 0, ni = 0, nj = 0;
    if (t < nt) {
        const int32_t *tri = T + 3 * t;
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        for (int q = 0; q < 3; ++q) {
            const double x = V[3 * tri[q]], y = V[3 * tri[q] + 1];
            xmin = fmin(xmin, x);
            xmax = fmax(xmax, x);
            ymin = fmin(ymin, y);
            ymax = fmax(ymax, y);
        }
        i0 = lower_idx(xc, nx, xmin);
        j0 = lower_idx(yc, ny, ymin);
        const int i1 = upper_idx(xc, nx, xmax), j1 = upper_idx(yc, ny, ymax);
        if (i1 >= i0 && j1 >= j0) {
            ni = i1 - i0 + 1;
            nj = j1 - j0 + 1;
        }
    }
    const int64_t ncols = (int64_t)ni * nj;
    if (ncols <= COL_SMALL) {
        for (int q = 0; q < (int)ncols; ++q)
            col_cross(V, T + 3 * t, xc, yc, nx, i0 + q % ni, j0 + q / ni, cnt, off, fill, zs, cap, overflow);
    }
    uint64_t big = __ballot(ncols > COL_SMALL);
    while (big) {
        const int L = __ffsll((unsigned long long)big) - 1;
        big &= big - 1;
        const int tl = __shfl((int)t, L, 64), il = __shfl(i0, L, 64), jl = __shfl(j0, L, 64), nil = __shfl(ni, L, 64),
                  njl = __shfl(nj, L, 64);
        const int64_t nc = (int64_t)nil * njl;
        for (int64_t q = lane; q < nc; q += 64)
            col_cross(V, T + 3 * (int64_t)tl, xc, yc, nx, il + (int)(q % nil), jl + (int)(q / nil), cnt, off, fill, zs,
                      cap, overflow);
    }
}

// per column: sort the crossings in place (insertion sort: few per column) and count the
// columns with an odd number of them (the host reports those)
__global__ void k_col_sort(const int32_t *__restrict__ off, double *zs, int64_t ncol, int64_t *odd, int64_t cap) {
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncol) return;
    if ((int64_t)off[ncol] > cap) return;  // overflowed: the host reports it
    const int n = off[col + 1] - off[col];
    double *z = zs + off[col];
    for (int a = 1; a < n; ++a) {
        const double v = z[a];
        int q = a - 1;
        while (q >= 0 && z[q] > v) {
            z[q + 1] = z[q];
            --q;
        }
        z[q + 1] = v;
    }
    if (n & 1) atomicAdd((unsigned long long *)odd, 1ull);
}

// one thread per cell: solid (1) iff the cell centre lies strictly between the crossings of a
// sorted pair of its column (an odd last crossing is dropped), fluid (0) otherwise
__global__ void k_col_fill(const int32_t *__restrict__ off, const double *__restrict__ zs,
                           const double *__restrict__ zc, int64_t ncol, int64_t N, uint8_t *type, int64_t cap) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    if ((int64_t)off[ncol] > cap) return;
    const uint32_t u = (uint32_t)id, k = u / (uint32_t)ncol, col = u - k * (uint32_t)ncol;  // N < 2^31
    const int b = off[col], n = (off[col + 1] - b) & ~1;
    const double zk = zc[k];
    uint8_t solid = 0;
    for (int m = 0; m < n; m += 2)
        if (zk > zs[b + m] && zk < zs[b + m + 1]) {
            solid = 1;
            break;
        }
    type[id] = solid;
}

// ghost = solid with a fluid cell among its in-range 26 neighbours; dead = other solid.
// Solid cells hold 1 on entry; rewriting them to 1 or 2 keeps "solid" readable.  A
// grid-stride loop with block-level counts keeps the counter atomics to one per block.
constexpr int MARK_NT = 256, MARK_BLOCKS = 2048;
__global__ void __launch_bounds__(MARK_NT) k_mark_ghosts(uint8_t *type, int nx, int ny, int nz, int64_t *counters) {
    __shared__ long long sh[3][MARK_NT / 64];
    const int64_t N = (int64_t)nx * ny * nz;
    long long cf = 0, cg = 0, cd = 0;
    for (int64_t id = (int64_t)blockIdx.x * MARK_NT + threadIdx.x; id < N; id += (int64_t)gridDim.x * MARK_NT) {
        const uint8_t t = type[id];
        if (t == 0) {
            cf += 1;
            continue;
        }
        int i, j, k;
        unflatten(id, nx, ny, i, j, k);
        bool fl = false;
        for (int dk = -1; dk <= 1 && !fl; ++dk)
            for (int dj = -1; dj <= 1 && !fl; ++dj)
                for (int di = -1; di <= 1 && !fl; ++di) {
                    const int ii = i + di, jj = j + dj, kk = k + dk;
                    if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                    if (type[((int64_t)kk * ny + jj) * nx + ii] == 0) fl = true;
                }
        type[id] = fl ? T_GHOST : T_DEAD;
        if (fl) cg += 1;
        else cd += 1;
    }
    cf = wave_sum_ll(cf);
    cg = wave_sum_ll(cg);
    cd = wave_sum_ll(cd);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = cf;
        sh[1][w] = cg;
        sh[2][w] = cd;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        long long v = 0;
        for (int q = 0; q < MARK_NT / 64; ++q) v += sh[threadIdx.x][q];
        if (v) atomicAdd((unsigned long long *)&counters[threadIdx.x], (unsigned long long)v);
    }
}

// The same marking for rows whose length is a multiple of 16: a thread takes 16 cells of
// one row with a single 16-byte load.  Only if one of them is solid does it load the nine
// row segments of its 3 x 3 (y, z) neighbourhood, each with the byte before and after it,
// all at once; bit b+1 of an 18-bit mask marks a fluid cell at x = i0 + b, so
// m | m >> 1 | m >> 2 marks the cells with a fluid x-neighbour (or themselves fluid), and
// the OR over the nine rows marks the solid cells whose 3 x 3 x 3 box holds a fluid cell.
// Fluid bytes are rewritten unchanged and solid bytes stay nonzero, so concurrent
// neighbour reads see the same fluid / solid state.
constexpr int MARK16_NT = 256;

__device__ __forceinline__ unsigned fluid_bits16(uint4 v) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    unsigned m = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) m |= (((w[q >> 2] >> (8 * (q & 3))) & 0xffu) == 0u ? 1u : 0u) << q;
    return m;
}

__global__ void __launch_bounds__(MARK16_NT) k_mark_ghosts16(uint8_t *type, int nx, int ny, int nz, int64_t nseg,
                                                             int64_t *part) {
    __shared__ long long sh[3][MARK16_NT / 64];
    long long cf = 0, cg = 0, cd = 0;
    const int64_t sg = (int64_t)blockIdx.x * MARK16_NT + threadIdx.x;
    if (sg < nseg) {
        const int segs = nx >> 4;
        const int64_t row = sg / segs;
        const int i0 = (int)(sg - row * segs) << 4;
        const int k = (int)(row / ny), j = (int)(row - (int64_t)k * ny);
        uint8_t *p0 = type + row * nx + i0;
        const unsigned fl = fluid_bits16(*reinterpret_cast<const uint4 *>(p0));
        const unsigned solid = ~fl & 0xffffu;
        cf = 16 - __popc(solid);
        if (solid) {
            uint4 v[9];
            uint8_t lo[9], hi[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int jj = j + q % 3 - 1, kk = k + q / 3 - 1;
                const bool in = jj >= 0 && jj < ny && kk >= 0 && kk < nz;
                const uint8_t *r = type + ((int64_t)(in ? kk : k) * ny + (in ? jj : j)) * nx + i0;
                v[q] = *reinterpret_cast<const uint4 *>(r);
                lo[q] = i0 > 0 ? r[-1] : (uint8_t)1;
                hi[q] = i0 + 16 < nx ? r[16] : (uint8_t)1;
                if (!in) {  // outside the grid: no fluid
                    v[q] = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
                    lo[q] = hi[q] = 1;
                }
            }
            unsigned near = 0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const unsigned m = (lo[q] == 0 ? 1u : 0u) | (fluid_bits16(v[q]) << 1) | ((hi[q] == 0 ? 1u : 0u) << 17);
                near |= (m | (m >> 1) | (m >> 2)) & 0xffffu;
            }
            const unsigned ghost = solid & near, dead = solid & ~near;
            cg = __popc(ghost);
            cd = __popc(dead);
            uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint32_t t = ((ghost >> q) & 1u) ? (uint32_t)T_GHOST : (((dead >> q) & 1u) ? (uint32_t)T_DEAD : 0u);
                w[q >> 2] |= t << (8 * (q & 3));
            }
            *reinterpret_cast<uint4 *>(p0) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    cf = wave_sum_ll(cf);
    cg = wave_sum_ll(cg);
    cd = wave_sum_ll(cd);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][wv] = cf;
        sh[1][wv] = cg;
        sh[2][wv] = cd;
    }
    __syncthreads();
    if (threadIdx.x < 3) {  // per-block counts (same-address atomics from every block would serialise)
        long long t = 0;
        for (int q = 0; q < MARK16_NT / 64; ++q) t += sh[threadIdx.x][q];
        part[3 * (int64_t)blockIdx.x + threadIdx.x] = t;
    }
}

// fluid, ghost and dead totals of k_mark_ghosts16's per-block counts, in one workgroup
constexpr int SUM3_NT = 1024;
__global__ void __launch_bounds__(SUM3_NT) k_sum_counts3(const int64_t *__restrict__ part, int64_t nblk,
                                                         int64_t *counters) {
    __shared__ long long sh[3][SUM3_NT / 64];
    long long a[3] = {0, 0, 0};
    for (int64_t b = threadIdx.x; b < nblk; b += SUM3_NT)
        for (int q = 0; q < 3; ++q) a[q] += part[3 * b + q];
    for (int q = 0; q < 3; ++q) a[q] = wave_sum_ll(a[q]);
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 3; ++q) sh[q][threadIdx.x >> 6] = a[q];
    __syncthreads();
    if (threadIdx.x < 3) {
        long long t = 0;
        for (int w = 0; w < SUM3_NT / 64; ++w) t += sh[threadIdx.x][w];
        counters[threadIdx.x] = t;
    }
}

// compaction of the ghost cells in increasing linear order
constexpr int CMP_NT = 256, CMP_PER = 16, CMP_CH = CMP_NT * CMP_PER;

// the listed cells: ghosts (prev == nullptr), or fresh cells (not fluid in prev, fluid now)
__device__ __forceinline__ bool listed(const uint8_t *__restrict__ type, const uint8_t *__restrict__ prev, int64_t id) {
    return prev ? (prev[id] != T_FLUID && type[id] == T_FLUID) : type[id] == T_GHOST;
}

__global__ void __launch_bounds__(CMP_NT) k_ghost_count(const uint8_t *__restrict__ type, int64_t N, int32_t *blkc,
                                                        const uint8_t *__restrict__ prev) {
    __shared__ double sh[CMP_NT / 64];
    int tid = threadIdx.x;
    int64_t base = (int64_t)blockIdx.x * CMP_CH + (int64_t)tid * CMP_PER;
    int c = 0;
    for (int q = 0; q < CMP_PER; ++q) {
        int64_t id = base + q;
        if (id < N && listed(type, prev, id)) ++c;
    }
    double s = block_sum<CMP_NT>((double)c, sh, tid);
    if (tid == 0) blkc[blockIdx.x] = (int32_t)s;
}

__global__ void __launch_bounds__(CMP_NT) k_ghost_write(const uint8_t *__restrict__ type, int64_t N,
                                                        const int32_t *blkoff, int32_t *gcell, int64_t gmax,
                                                        const uint8_t *__restrict__ prev) {
    __shared__ int sh[CMP_NT];
    int tid = threadIdx.x;
    int64_t base = (int64_t)blockIdx.x * CMP_CH + (int64_t)tid * CMP_PER;
    int c = 0;
    for (int q = 0; q < CMP_PER; ++q) {
        int64_t id = base + q;
        if (id < N && listed(type, prev, id)) ++c;
    }
    sh[tid] = c;
    __syncthreads();
    for (int o = 1; o < CMP_NT; o <<= 1) {
        int v = (tid >= o) ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += v;
        __syncthreads();
    }
    int64_t pos = (int64_t)blkoff[blockIdx.x] + sh[tid] - c;
    for (int q = 0; q < CMP_PER; ++q) {
        int64_t id = base + q;
        if (id < N && listed(type, prev, id)) {
            if (pos < gmax) gcell[pos] = (int32_t)id;
            ++pos;
        }
    }
}

// zero n 32-bit words (a kernel rather than a memset, so the no-allocation entry point that
// shares this path stays capturable in a HIP graph)
__global__ void k_clear_words(uint32_t *p, int64_t n) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n) p[id] = 0u;
}

static hipError_t clear_words(void *p, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 4;
    hipLaunchKernelGGL(k_clear_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t *)p, n);
    return hipGetLastError();
}

int64_t classify_mark16_parts(int nx, int ny, int nz) {
    if (nx % 16 != 0) return 0;
    const int64_t nseg = (int64_t)nx * ny * nz / 16;
    return 3 * ((nseg + MARK16_NT - 1) / MARK16_NT);
}

int64_t classify_scan_blocks(int64_t n) { return (n + SCAN_CH - 1) / SCAN_CH + 1; }

// cell types of every cell and counters[0..4] = fluid, ghost, dead, odd columns, crossing
// overflow; every buffer is the caller's (a handle's workspace or the static scratch)
hipError_t launch_classify_cells(const ClassifyBufs &B, hipStream_t s) {
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int64_t ncol = (int64_t)nx * ny, N = ncol * nz;
    hipError_t e;
    if ((e = clear_words(B.counters, sizeof(int64_t) * 8, s)) != hipSuccess) return e;
    if ((e = clear_words(B.col_cnt, sizeof(int32_t) * (ncol + 1), s)) != hipSuccess) return e;
    if ((e = clear_words(B.col_fill, sizeof(int32_t) * (ncol + 1), s)) != hipSuccess) return e;
    if (B.nt > 0) {
        hipLaunchKernelGGL(k_col_pass, dim3((unsigned)((B.nt + COL_NT - 1) / COL_NT)), dim3(COL_NT), 0, s, B.verts,
                           B.tris, B.nt, B.xc, B.yc, nx, ny, B.col_cnt, nullptr, nullptr, nullptr, (int64_t)0, nullptr);
    }
    e = scan_counts(B.col_cnt, B.col_off, ncol + 1, B.blk, s);
    if (e != hipSuccess) return e;
    if (B.nt > 0) {
        hipLaunchKernelGGL(k_col_pass, dim3((unsigned)((B.nt + COL_NT - 1) / COL_NT)), dim3(COL_NT), 0, s, B.verts,
                           B.tris, B.nt, B.xc, B.yc, nx, ny, nullptr, B.col_off, B.col_fill, B.crossings, B.cross_cap,
                           B.counters + 4);
    }
    hipLaunchKernelGGL(k_col_sort, dim3((unsigned)((ncol + 255) / 256)), dim3(256), 0, s, B.col_off, B.crossings,
                       (int64_t)ncol, B.counters + 3, B.cross_cap);
    hipLaunchKernelGGL(k_col_fill, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, B.col_off, B.crossings, B.zc,
                       (int64_t)ncol, N, B.type, B.cross_cap);
    if (nx % 16 == 0) {
        const int64_t nseg = N / 16, nblk = (nseg + MARK16_NT - 1) / MARK16_NT;
        hipLaunchKernelGGL(k_mark_ghosts16, dim3((unsigned)nblk), dim3(MARK16_NT), 0, s, B.type, nx, ny, nz, nseg,
                           B.mark_parts);
        hipLaunchKernelGGL(k_sum_counts3, dim3(1), dim3(SUM3_NT), 0, s, (const int64_t *)B.mark_parts, nblk,
                           B.counters);
    } else {
        hipLaunchKernelGGL(k_mark_ghosts, dim3((unsigned)std::min<int64_t>((N + MARK_NT - 1) / MARK_NT, MARK_BLOCKS)),
                           dim3(MARK_NT), 0, s, B.type, nx, ny, nz, B.counters);
    }
    return hipGetLastError();
}

hipError_t launch_classify(ibm_grid *g, hipStream_t s, int64_t counts[4]) {
    const int nx = g->nx, ny = g->ny;
    const int64_t N = g->N;
    ClassifyBufs B;
    B.nx = nx;
    B.ny = ny;
    B.nz = g->nz;
    B.verts = g->verts;
    B.tris = g->tris;
    B.nt = g->nt;
    B.xc = g->c0[0];
    B.yc = g->c0[1];
    B.zc = g->c0[2];
    B.col_cnt = g->col_cnt;
    B.col_off = g->col_off;
    B.col_fill = g->col_fill;
    B.crossings = g->crossings;
    B.cross_cap = g->cross_cap;
    B.counters = g->counters;
    B.blk = (int64_t *)g->blk_cnt;
    // per-block counts of the 16-cell ghost marking go to the reduction partials
    // (3 per block <= N / 256 + 1024 entries)
    B.mark_parts = reinterpret_cast<int64_t *>(g->partials);
    B.type = g->type;
    hipError_t e = launch_classify_cells(B, s);
    if (e != hipSuccess) return e;
    int64_t nb = (N + CMP_CH - 1) / CMP_CH;
    int32_t *blkc = g->col_cnt;  // reuse: ncol+1 >= nb is guaranteed by the layout
    int32_t *blko = g->col_fill;
    hipLaunchKernelGGL(k_ghost_count, dim3((unsigned)nb), dim3(CMP_NT), 0, s, g->type, N, blkc,
                       (const uint8_t *)nullptr);
    e = scan_counts(blkc, blko, nb, (int64_t *)g->blk_cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ghost_write, dim3((unsigned)nb), dim3(CMP_NT), 0, s, g->type, N, blko, g->g_cell,
                       g->ghost_max, (const uint8_t *)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t hc[8];
    e = hipMemcpyAsync(hc, g->counters, sizeof(hc), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    counts[0] = hc[0];
    counts[1] = hc[1];
    counts[2] = hc[2];
    counts[3] = hc[3] + (hc[4] ? (int64_t)1 << 40 : 0);  // odd columns; overflow flagged high
    return hipSuccess;
}

// ---------------------------------------------------------------------------------------
// body intercept: closest point of the mesh (Ericson, Real-Time Collision Detection, 2005,
// section 5.1.5: Voronoi-region test per triangle), argmin with lowest triangle index
// ---------------------------------------------------------------------------------------

__device__ void closest_on_triangle(const double p[3], const double a[3], const double b[3], const double c[3],
                                    double q[3]) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    for (int d = 0; d < 3; ++d) {
        ab[d] = b[d] - a[d];
        ac[d] = c[d] - a[d];
        ap[d] = p[d] - a[d];
    }
    double d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
    double d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
    if (d1 <= 0.0 && d2 <= 0.0) {
        for (int d = 0; d < 3; ++d) q[d] = a[d];
        return;
    }
    for (int d = 0; d < 3; ++d) bp[d] = p[d] - b[d];
    double d3 = ab[0] * bp[0] + ab[1] * bp[1] + ab[2] * bp[2];
    double d4 = ac[0] * bp[0] + ac[1] * bp[1] + ac[2] * bp[2];
    if (d3 >= 0.0 && d4 <= d3) {
        for (int d = 0; d < 3; ++d) q[d] = b[d];
        return;
    }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int d = 0; d < 3; ++d) q[d] = a[d] + v * ab[d];
        return;
    }
    for (int d = 0; d < 3; ++d) cp[d] = p[d] - c[d];
    double d5 = ab[0] * cp[0] + ab[1] * cp[1] + ab[2] * cp[2];
    double d6 = ac[0] * cp[0] + ac[1] * cp[1] + ac[2] * cp[2];
    if (d6 >= 0.0 && d5 <= d6) {
        for (int d = 0; d < 3; ++d) q[d] = c[d];
        return;
    }
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

__device__ __forceinline__ void consider_tri(const double *V, const int32_t *T, int32_t t, const double x[3],
                                             double &best, int32_t &bt, double bq[3]) {
    const int32_t *tri = T + 3 * (int64_t)t;
    double a[3], b[3], c[3], q[3];
    for (int d = 0; d < 3; ++d) {
        a[d] = V[3 * tri[0] + d];
        b[d] = V[3 * tri[1] + d];
        c[d] = V[3 * tri[2] + d];
    }
    closest_on_triangle(x, a, b, c, q);
    double dx = q[0] - x[0], dy = q[1] - x[1], dz = q[2] - x[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < best || (d2 == best && t < bt)) {
        best = d2;
        bt = t;
        bq[0] = q[0];
        bq[1] = q[1];
        bq[2] = q[2];
    }
}

// One wave per ghost: the lanes stride over the triangles of each bucket in the search box,
// then the wave keeps the lexicographic minimum of (squared distance, triangle index).  The
// candidate set and the tie rule are those of a sequential scan, so the result is the same.
constexpr int CLOSEST_WAVES = 4;
__device__ __forceinline__ void closest_wave_min(double &best, int32_t &bt, double bq[3]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int32_t ot = __shfl_xor(bt, off, 64);
        const double o0 = __shfl_xor(bq[0], off, 64), o1 = __shfl_xor(bq[1], off, 64),
                     o2 = __shfl_xor(bq[2], off, 64);
        if (ob < best || (ob == best && ot < bt)) {
            best = ob;
            bt = ot;
            bq[0] = o0;
            bq[1] = o1;
            bq[2] = o2;
        }
    }
}

__global__ void __launch_bounds__(64 * CLOSEST_WAVES)
    k_closest(int64_t ng, const int32_t *__restrict__ gcell, int nx, int ny, int nz, const double *__restrict__ xc,
              const double *__restrict__ yc, const double *__restrict__ zc, const double *__restrict__ V,
              const int32_t *__restrict__ T, int64_t nt, const int32_t *__restrict__ boff,
              const int32_t *__restrict__ bent, BucketGrid G, double *gbi, int32_t *gtri) {
    const int64_t g = (int64_t)blockIdx.x * CLOSEST_WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= ng) return;  // whole wave
    int64_t id = gcell[g];
    int i, j, k;
    unflatten(id, nx, ny, i, j, k);
    double x[3] = {xc[i], yc[j], zc[k]};
    const bool two_d = (nz == 1);
    // the surface crosses the segment to any fluid neighbour: search within the largest
    // centre distance to the 26 neighbours
    double rx = fmax(i > 0 ? x[0] - xc[i - 1] : 0.0, i < nx - 1 ? xc[i + 1] - x[0] : 0.0);
    double ry = fmax(j > 0 ? x[1] - yc[j - 1] : 0.0, j < ny - 1 ? yc[j + 1] - x[1] : 0.0);
    double rz = fmax(k > 0 ? x[2] - zc[k - 1] : 0.0, k < nz - 1 ? zc[k + 1] - x[2] : 0.0);
    if (two_d) rz = 0.0;
    double r = sqrt(rx * rx + ry * ry + rz * rz);
    double best = INFINITY, bq[3] = {0.0, 0.0, 0.0};
    int32_t bt = 0x7fffffff;
    int b0[3], b1[3];
    for (int d = 0; d < 3; ++d) {
        b0[d] = bucket_coord(x[d] - r - G.ext[d], G.bmin[d], G.bsize[d], G.nb[d]);
        b1[d] = bucket_coord(x[d] + r, G.bmin[d], G.bsize[d], G.nb[d]);
    }
    // The box's bucket entries are laid end to end: lane L of a chunk of 64 buckets holds
    // bucket L's offset and count, a wave prefix sum gives each bucket's first position, and
    // the lane taking position q finds its bucket as the last one starting at or before q
    // (a binary search over lanes by shuffles).  All buckets' entries are fetched in one
    // round instead of one bucket after another.
    const int nbx = b1[0] - b0[0] + 1, nby = b1[1] - b0[1] + 1, nbox = nbx * nby * (b1[2] - b0[2] + 1);
    for (int c0 = 0; c0 < nbox; c0 += 64) {
        int start = 0, cnt = 0;
        if (c0 + lane < nbox) {
            const int cb = c0 + lane, bx = b0[0] + cb % nbx, by = b0[1] + (cb / nbx) % nby, bz = b0[2] + cb / (nbx * nby);
            const int b = (bz * G.nb[1] + by) * G.nb[0] + bx;
            start = boff[b];
            cnt = boff[b + 1] - start;
        }
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int total = __shfl(incl, 63, 64), excl = incl - cnt;
        for (int q0 = 0; q0 < total; q0 += 64) {
            const int q = q0 + lane;
            int L = 0;  // the last lane whose first position is <= q
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const int e = __shfl(excl, min(L + step, 63), 64);
                if (L + step <= 63 && e <= q) L += step;
            }
            const int st = __shfl(start, L, 64), ex = __shfl(excl, L, 64);
            if (q >= total) continue;
            const int32_t t = bent[st + (q - ex)];
            double lo[3], hi[3];
            tri_bbox(V, T, t, lo, hi);
            bool far = false;
            for (int d = 0; d < 3; ++d)
                if (lo[d] > x[d] + r || hi[d] < x[d] - r) far = true;
            if (far) continue;
            consider_tri(V, T, t, x, best, bt, bq);
        }
    }
    closest_wave_min(best, bt, bq);
    if (bt == 0x7fffffff || !(best <= r * r)) {
        // nothing within the radius: search every triangle
        best = INFINITY;
        bt = 0x7fffffff;
        for (int64_t t = lane; t < nt; t += 64) consider_tri(V, T, (int32_t)t, x, best, bt, bq);
        closest_wave_min(best, bt, bq);
    }
    if (lane != 0) return;
    if (two_d) bq[2] = x[2];  // prism bodies of a one-cell-thick grid: stay in the cell plane
    gbi[3 * g] = bq[0];
    gbi[3 * g + 1] = bq[1];
    gbi[3 * g + 2] = bq[2];
    gtri[g] = bt;
}

// ---------------------------------------------------------------------------------------
// image point, interpolation box and weights (Eq. 2 and Eq. 3)
//
// The weights beta solve V^T beta = b(x_IP) for the trilinear basis b of the box; when the
// ghost is itself a member its row of V is the normal derivative of the basis at the body
// intercept.  Here the solution is written in closed form through the trilinear Lagrange
// basis L_m of the box (dual-basis form, no per-ghost factorisation):
//     no Neumann row:  beta_m = L_m(IP)
//     ghost g in box:  beta_g = L_g(IP) / dL_g/dn(BI)
//                      beta_m = L_m(IP) - dL_m/dn(BI) * beta_g      (m != g)
// dL_g/dn(BI) < 0 strictly for a mirror image point, so the form is defined; a ghost whose
// row would not satisfy it (on the surface next to a wall, where the box cannot lie on the
// normal's side) is degenerate.
// ---------------------------------------------------------------------------------------

__global__ void k_weights(int64_t ng, const int32_t *__restrict__ gcell, int nx, int ny, int nz,
                          const double *__restrict__ xc, const double *__restrict__ yc, const double *__restrict__ zc,
                          const double *__restrict__ wx, const double *__restrict__ wy, const double *__restrict__ wz,
                          const uint8_t *__restrict__ type, const double *__restrict__ V, const int32_t *__restrict__ T,
                          double *gbi, const int32_t *__restrict__ gtri, double *gn, double *gip,
                          double *gdl, int32_t *gst, uint8_t *gmask, double *gbeta, double *gbetag, int32_t *gflags,
                          int64_t *ndegen, double *gbetaD, double *gbetaDg) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    int64_t id = gcell[g];
    int i, j, k;
    unflatten(id, nx, ny, i, j, k);
    const bool two_d = (nz == 1);
    double xg[3] = {xc[i], yc[j], zc[k]};
    double bi[3] = {gbi[3 * g], gbi[3 * g + 1], gbi[3 * g + 2]};
    double dv[3] = {bi[0] - xg[0], bi[1] - xg[1], bi[2] - xg[2]};
    double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    double hloc = fmin(wx[i], wy[j]);
    if (!two_d) hloc = fmin(hloc, wz[k]);
    int flags = 0;
    double n[3];
    const bool on_surface = dist <= 1e-12 * hloc;
    if (on_surface) {
        const int32_t *tri = T + 3 * (int64_t)gtri[g];
        double u[3], v[3];
        for (int d = 0; d < 3; ++d) {
            u[d] = V[3 * tri[1] + d] - V[3 * tri[0] + d];
            v[d] = V[3 * tri[2] + d] - V[3 * tri[0] + d];
        }
        double nn[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        if (two_d) nn[2] = 0.0;
        double ln = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
        for (int d = 0; d < 3; ++d) n[d] = nn[d] / ln;
        flags |= GF_NFALLBACK;
        // the centre is on the surface: it is its own intercept (and image point)
        for (int d = 0; d < 3; ++d) {
            bi[d] = xg[d];
            gbi[3 * g + d] = xg[d];
        }
        dist = 0.0;
    } else {
        for (int d = 0; d < 3; ++d) n[d] = dv[d] / dist;
    }
    double ip[3];
    for (int d = 0; d < 3; ++d) ip[d] = (bi[d] + bi[d]) - xg[d];
    double dl = dist + dist;
    for (int d = 0; d < 3; ++d) {
        gn[3 * g + d] = n[d];
        gip[3 * g + d] = ip[d];
    }
    gdl[g] = dl;
    // box around the image point; on the surface, the cells on the side the normal points to
    // (the ghost's row is then the one-sided normal difference into the fluid)
    int i0, j0, k0;
    if (on_surface) {
        i0 = min(max(n[0] >= 0.0 ? i : i - 1, 0), nx - 2);
        j0 = min(max(n[1] >= 0.0 ? j : j - 1, 0), ny - 2);
        k0 = two_d ? 0 : min(max(n[2] >= 0.0 ? k : k - 1, 0), nz - 2);
    } else {
        i0 = box_lo(xc, nx, ip[0]);
        j0 = box_lo(yc, ny, ip[1]);
        k0 = two_d ? 0 : box_lo(zc, nz, ip[2]);
    }
    double hx = xc[i0 + 1] - xc[i0], hy = yc[j0 + 1] - yc[j0];
    double hz = two_d ? 1.0 : zc[k0 + 1] - zc[k0];
    double s[3], bl[3];
    s[0] = (ip[0] - xc[i0]) / hx;
    s[1] = (ip[1] - yc[j0]) / hy;
    s[2] = two_d ? 0.0 : (ip[2] - zc[k0]) / hz;
    for (int d = 0; d < 3; ++d) {
        if (s[d] < 0.0) {
            s[d] = 0.0;
            flags |= GF_CLAMPED;
        } else if (s[d] > 1.0) {
            s[d] = 1.0;
            flags |= GF_CLAMPED;
        }
    }
    bl[0] = (bi[0] - xc[i0]) / hx;
    bl[1] = (bi[1] - yc[j0]) / hy;
    bl[2] = two_d ? 0.0 : (bi[2] - zc[k0]) / hz;
    const double hs[3] = {hx, hy, hz};
    const int nm = two_d ? 4 : 8;
    int32_t mem[8];
    int nfl = 0, ndead = 0, self = -1;
    uint8_t gm = 0;
    for (int m = 0; m < nm; ++m) {
        int a = m & 1, b = (m >> 1) & 1, c = (m >> 2) & 1;
        int64_t mid = ((int64_t)(k0 + c) * ny + (j0 + b)) * nx + (i0 + a);
        mem[m] = (int32_t)mid;
        uint8_t ty = type[mid];
        if (ty == T_FLUID) ++nfl;
        if (ty == T_DEAD) ++ndead;
        if (mid == id) self = m;
        else if (ty == T_GHOST) gm |= (uint8_t)(1u << m);
    }
    double beta[8];
    int32_t st[8];
    for (int m = 0; m < 8; ++m) {
        beta[m] = 0.0;
        st[m] = -1;
    }
    double bg = 0.0;
    // Dirichlet weights (velocity ghost rows): the interpolant's own row is its value at the
    // intercept, so with the Lagrange basis L_m of the box
    //   betaD_m = L_m(IP) - L_m(BI) L_g(IP) / L_g(BI),  betaD_g = L_g(IP) / L_g(BI);
    // for a mirrored image point BI lies between the ghost centre and IP, so L_g(BI) >= 1/8.
    double betaD[8], bDg = 0.0;
    for (int m = 0; m < 8; ++m) betaD[m] = 0.0;
    bool degenerate = (ndead > 0 || nfl == 0);
    if (!degenerate) {
        // Lagrange basis at the image point, at the intercept, and its normal derivative there
        double L[8], dLn[8], LB[8];
        for (int m = 0; m < nm; ++m) {
            int bits[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1};
            double fi[3], fb[3];
            for (int d = 0; d < 3; ++d) {
                fi[d] = bits[d] ? s[d] : 1.0 - s[d];
                fb[d] = bits[d] ? bl[d] : 1.0 - bl[d];
            }
            LB[m] = two_d ? fb[0] * fb[1] : fb[0] * fb[1] * fb[2];
            if (two_d) {
                L[m] = fi[0] * fi[1];
                dLn[m] = n[0] * ((bits[0] ? 1.0 : -1.0) / hs[0]) * fb[1] + n[1] * ((bits[1] ? 1.0 : -1.0) / hs[1]) * fb[0];
            } else {
                L[m] = fi[0] * fi[1] * fi[2];
                dLn[m] = n[0] * ((bits[0] ? 1.0 : -1.0) / hs[0]) * (fb[1] * fb[2]) +
                         n[1] * ((bits[1] ? 1.0 : -1.0) / hs[1]) * (fb[0] * fb[2]) +
                         n[2] * ((bits[2] ? 1.0 : -1.0) / hs[2]) * (fb[0] * fb[1]);
            }
        }
        if (self < 0) {
            for (int m = 0; m < nm; ++m) {
                beta[m] = L[m];
                betaD[m] = L[m];
                st[m] = mem[m];
            }
        } else if (dLn[self] < 0.0) {
            bDg = L[self] / LB[self];
            for (int m = 0; m < nm; ++m)
                if (m != self) betaD[m] = L[m] - LB[m] * bDg;
            bg = L[self] / dLn[self];
            for (int m = 0; m < nm; ++m) {
                if (m == self) {
                    beta[m] = bg;
                    st[m] = -1;
                } else {
                    beta[m] = L[m] - dLn[m] * bg;
                    st[m] = mem[m];
                }
            }
            flags |= GF_SELF;
        } else {
            degenerate = true;
        }
    }
    if (degenerate) {
        flags |= GF_DEGENERATE;
        gm = 0;
        bg = 0.0;
        bDg = 0.0;
        for (int m = 0; m < 8; ++m) {
            beta[m] = 0.0;
            betaD[m] = 0.0;
            st[m] = -1;
        }
        atomicAdd((unsigned long long *)ndegen, 1ull);
    }
    for (int m = 0; m < 8; ++m) {
        gst[8 * g + m] = st[m];
        gbeta[8 * g + m] = beta[m];
        gbetaD[8 * g + m] = betaD[m];
    }
    gmask[g] = gm;
    gbetag[g] = bg;
    gbetaDg[g] = bDg;
    gflags[g] = flags;
}

__global__ void k_ghost_h(int64_t ng, const double *betag, const double *dl, const double *data,
                          const int32_t *flags, double *h) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    // ghost equation: p_g - sum_{m != g} beta_m p_m = (beta_g - dl) * dp/dn(BI); a degenerate
    // ghost's equation (mean of its fluid neighbours) carries no Neumann term
    h[g] = (flags[g] & GF_DEGENERATE) ? 0.0 : (betag[g] - dl[g]) * data[g];
}

hipError_t launch_stencils(ibm_grid *g, hipStream_t s) {
    if (g->ng == 0) return hipSuccess;
    BucketGrid G;
    for (int d = 0; d < 3; ++d) {
        G.bmin[d] = g->bmin[d];
        G.bsize[d] = g->bsize[d];
        G.ext[d] = g->bext[d];
        G.nb[d] = g->nb[d];
    }
    unsigned nb = (unsigned)((g->ng + 127) / 128);
    hipLaunchKernelGGL(k_closest, dim3((unsigned)((g->ng + CLOSEST_WAVES - 1) / CLOSEST_WAVES)),
                       dim3(64 * CLOSEST_WAVES), 0, s, g->ng, g->g_cell, g->nx, g->ny, g->nz, g->c0[0], g->c0[1],
                       g->c0[2], g->verts, g->tris, g->nt, g->bucket_off, g->bucket_ent, G, g->g_bi, g->g_tri);
    hipLaunchKernelGGL(k_weights, dim3(nb), dim3(128), 0, s, g->ng, g->g_cell, g->nx, g->ny, g->nz, g->c0[0], g->c0[1],
                       g->c0[2], g->w0[0], g->w0[1], g->w0[2], g->type, g->verts, g->tris, g->g_bi, g->g_tri, g->g_n,
                       g->g_ip, g->g_dl, g->g_st, g->g_mask, g->g_beta, g->g_betag, g->g_flags, g->counters + 5,
                       g->g_betaD, g->g_betaDg);
    return hipGetLastError();
}

hipError_t launch_ghost_h(ibm_grid *g, hipStream_t s) {
    if (g->ng == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_h, dim3((unsigned)((g->ng + 255) / 256)), dim3(256), 0, s, g->ng, g->g_betag, g->g_dl,
                       g->g_data, g->g_flags, g->g_h);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// fresh cells of a moved body (Section 2.2): not fluid before the move, fluid after it.  The
// image point is the mirror of the intercept through the cell centre (IP = 2 x_c - BI), so
// u_c = (u_BI + u_IP) / 2 with u_IP trilinear (Eq. 2) over the 8 (2D: 4) cells around IP;
// the fresh cell's own weight, when it is one of them, is kept apart (beta_c) and moved to
// the left side at fill time.  A box with a dead cell or without a fluid cell is degenerate.
// ---------------------------------------------------------------------------------------

__global__ void k_fresh_weights(int64_t nf, const int32_t *__restrict__ fcell, int nx, int ny, int nz,
                                const double *__restrict__ xc, const double *__restrict__ yc,
                                const double *__restrict__ zc, const uint8_t *__restrict__ type,
                                const double *__restrict__ fbi, double *fip, int32_t *fst, double *fbeta,
                                double *fbetac, int32_t *fflags) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nf) return;
    const int64_t id = fcell[q];
    int i, j, k;
    unflatten(id, nx, ny, i, j, k);
    const bool two_d = (nz == 1);
    const double x[3] = {xc[i], yc[j], zc[k]};
    double ip[3];
    for (int d = 0; d < 3; ++d) {
        ip[d] = (x[d] + x[d]) - fbi[3 * q + d];
        fip[3 * q + d] = ip[d];
    }
    const int i0 = box_lo(xc, nx, ip[0]), j0 = box_lo(yc, ny, ip[1]), k0 = two_d ? 0 : box_lo(zc, nz, ip[2]);
    double sl[3];
    sl[0] = (ip[0] - xc[i0]) / (xc[i0 + 1] - xc[i0]);
    sl[1] = (ip[1] - yc[j0]) / (yc[j0 + 1] - yc[j0]);
    sl[2] = two_d ? 0.0 : (ip[2] - zc[k0]) / (zc[k0 + 1] - zc[k0]);
    int flags = 0;
    for (int d = 0; d < 3; ++d) {
        if (sl[d] < 0.0) {
            sl[d] = 0.0;
            flags |= GF_CLAMPED;
        } else if (sl[d] > 1.0) {
            sl[d] = 1.0;
            flags |= GF_CLAMPED;
        }
    }
    const int nm = two_d ? 4 : 8;
    int nfl = 0, ndead = 0;
    int32_t mem[8];
    for (int m = 0; m < nm; ++m) {
        const int a = m & 1, b = (m >> 1) & 1, c = (m >> 2) & 1;
        const int64_t mid = ((int64_t)(k0 + c) * ny + (j0 + b)) * nx + (i0 + a);
        mem[m] = (int32_t)mid;
        const uint8_t ty = type[mid];
        if (ty == T_FLUID) ++nfl;
        if (ty == T_DEAD) ++ndead;
    }
    const bool degenerate = ndead > 0 || nfl == 0;
    double bc = 0.0;
    for (int m = 0; m < 8; ++m) {
        double w = 0.0;
        int32_t st = -1;
        if (!degenerate && m < nm) {
            const int bits[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1};
            w = (bits[0] ? sl[0] : 1.0 - sl[0]) * (bits[1] ? sl[1] : 1.0 - sl[1]);
            if (!two_d) w *= bits[2] ? sl[2] : 1.0 - sl[2];
            if (mem[m] == id) {
                bc = w;
                w = 0.0;
            } else {
                st = mem[m];
            }
        }
        fst[8 * q + m] = st;
        fbeta[8 * q + m] = w;
    }
    fbetac[q] = bc;
    fflags[q] = flags | (degenerate ? GF_DEGENERATE : 0) | (bc != 0.0 ? GF_SELF : 0);
}

// the list of fresh cells (increasing linear order), their intercepts and weights;
// *nfresh receives the count (the list holds at most ghost_max of them)
hipError_t launch_fresh(ibm_grid *g, hipStream_t s, int64_t *nfresh) {
    const int64_t N = g->N;
    const int64_t nb = (N + CMP_CH - 1) / CMP_CH;
    int32_t *blkc = g->col_cnt, *blko = g->col_fill;
    hipLaunchKernelGGL(k_ghost_count, dim3((unsigned)nb), dim3(CMP_NT), 0, s, g->type, N, blkc,
                       (const uint8_t *)g->type_prev);
    hipError_t e = scan_counts(blkc, blko, nb, (int64_t *)g->blk_cnt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ghost_write, dim3((unsigned)nb), dim3(CMP_NT), 0, s, g->type, N, blko, g->f_cell,
                       g->ghost_max, (const uint8_t *)g->type_prev);
    int32_t last[2];
    if ((e = hipMemcpyAsync(&last[0], blko + nb - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&last[1], blkc + nb - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const int64_t nf = (int64_t)last[0] + last[1];
    *nfresh = nf;
    if (nf == 0 || nf > g->ghost_max) return hipSuccess;
    BucketGrid G;
    for (int d = 0; d < 3; ++d) {
        G.bmin[d] = g->bmin[d];
        G.bsize[d] = g->bsize[d];
        G.ext[d] = g->bext[d];
        G.nb[d] = g->nb[d];
    }
    hipLaunchKernelGGL(k_closest, dim3((unsigned)((nf + CLOSEST_WAVES - 1) / CLOSEST_WAVES)), dim3(64 * CLOSEST_WAVES),
                       0, s, nf, g->f_cell, g->nx, g->ny, g->nz, g->c0[0], g->c0[1], g->c0[2], g->verts, g->tris, g->nt,
                       g->bucket_off, g->bucket_ent, G, g->f_bi, g->f_tri);
    hipLaunchKernelGGL(k_fresh_weights, dim3((unsigned)((nf + 127) / 128)), dim3(128), 0, s, nf, g->f_cell, g->nx,
                       g->ny, g->nz, g->c0[0], g->c0[1], g->c0[2], g->type, g->f_bi, g->f_ip, g->f_st, g->f_beta,
                       g->f_betac, g->f_flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// multigrid hierarchy: active masks, staircase transmissibilities, prolongation tables
// ---------------------------------------------------------------------------------------

struct LevelDims {
    int n[3];
    const int *cs[3];  // children starts in the finer level (coarse side of a pair only)
};

// active(C) = any active child; fine level 0 active = fluid
__global__ void k_coarsen_active(LevelDims F, LevelDims C, const uint8_t *__restrict__ fine_active, bool fine_is_type,
                                 uint8_t *coarse_active, const double *__restrict__ cw0, const double *__restrict__ cw1,
                                 const double *__restrict__ cw2, double *partials) {
    __shared__ double sh[4];
    int64_t NC = (int64_t)C.n[0] * C.n[1] * C.n[2];
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double vol = 0.0;
    if (id < NC) {
        int I, J, K;
        unflatten(id, C.n[0], C.n[1], I, J, K);
        const int i0 = C.cs[0][I], i1 = C.cs[0][I + 1] - 1;
        const int j0 = C.cs[1][J], j1 = C.cs[1][J + 1] - 1;
        const int k0 = C.cs[2][K], k1 = C.cs[2][K + 1] - 1;
        uint8_t act = 0;
        for (int k = k0; k <= k1; ++k)
            for (int j = j0; j <= j1; ++j)
                for (int i = i0; i <= i1; ++i) {
                    uint8_t v = fine_active[((int64_t)k * F.n[1] + j) * F.n[0] + i];
                    act |= fine_is_type ? (uint8_t)(v == T_FLUID) : v;
                }
        coarse_active[id] = act;
        if (act) vol = (cw0[I] * cw1[J]) * cw2[K];
    }
    double s = block_sum<256>(vol, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// level-0 active volume
__global__ void k_fluid_volume(const uint8_t *__restrict__ type, int nx, int ny, int nz, const double *__restrict__ wx,
                               const double *__restrict__ wy, const double *__restrict__ wz, double *partials) {
    __shared__ double sh[4];
    int64_t N = (int64_t)nx * ny * nz;
    double vol = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < N; id += (int64_t)gridDim.x * blockDim.x) {
        if (type[id] == T_FLUID) {
            int i, j, k;
            unflatten(id, nx, ny, i, j, k);
            vol += (wx[i] * wy[j]) * wz[k];
        }
    }
    double s = block_sum<256>(vol, sh, threadIdx.x);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// one workgroup of 256 threads; fixed combination order, so the sum is reproducible
__global__ void __launch_bounds__(256) k_sum_partials(const double *partials, int n, double *out) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) s += partials[q];
    s = block_sum<256>(s, sh, threadIdx.x);
    if (threadIdx.x == 0) *out = s;
}

// open child-face area over the coarse centre distance, for each cell's low face along d
// Level-0 cells whose trilinear prolongation would read an inactive level-1 cell: those fluid
// cells take the parent's value instead (the parent is always the first contributor).  The
// flag is fixed by the geometry, so it is computed once with the hierarchy.
__global__ void k_inject0(int nx, int ny, int nz, const uint8_t *__restrict__ type, LevelDims C,
                          const uint8_t *__restrict__ cactive, const int *lo0, const int *hi0, const int *lo1,
                          const int *hi1, const int *lo2, const int *hi2, uint8_t *inject) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    uint8_t v = 0;
    if (type[id] == T_FLUID) {
        int i, j, k;
        unflatten(id, nx, ny, i, j, k);
        const int ix[2] = {lo0[i], hi0[i]}, iy[2] = {lo1[j], hi1[j]}, iz[2] = {lo2[k], hi2[k]};
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    if (!cactive[((int64_t)iz[c] * C.n[1] + iy[b]) * C.n[0] + ix[a]]) v = 1;
    }
    inject[id] = v;
}

struct FaceAxes {  // per axis: coarse centres and the transmissibility outputs
    const double *cc[3];
    double *T64[3];
    float *T32[3];
};

// the three axes in one launch: blockIdx.y is the axis
__global__ void k_face_T(LevelDims F, LevelDims C, const uint8_t *__restrict__ fine_active, bool fine_is_type,
                         const double *__restrict__ fw0, const double *__restrict__ fw1, const double *__restrict__ fw2,
                         FaceAxes A) {
    const int d = (int)blockIdx.y;
    const double *__restrict__ cc = A.cc[d];
    double *T64 = A.T64[d];
    float *T32 = A.T32[d];
    int64_t NC = (int64_t)C.n[0] * C.n[1] * C.n[2];
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= NC) return;
    int Ic[3];
    unflatten(id, C.n[0], C.n[1], Ic[0], Ic[1], Ic[2]);
    if (Ic[d] == 0) {
        T64[id] = 0.0;
        T32[id] = 0.0f;
        return;
    }
    const double *fw[3] = {fw0, fw1, fw2};
    int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
    const int fface = C.cs[d][Ic[d]];
    const int a0 = C.cs[e1][Ic[e1]], a1 = C.cs[e1][Ic[e1] + 1] - 1;
    const int b0 = C.cs[e2][Ic[e2]], b1 = C.cs[e2][Ic[e2] + 1] - 1;
    double area = 0.0;
    for (int b = b0; b <= b1; ++b)
        for (int a = a0; a <= a1; ++a) {
            int lo[3], hi[3];
            lo[d] = fface - 1;
            hi[d] = fface;
            lo[e1] = hi[e1] = a;
            lo[e2] = hi[e2] = b;
            uint8_t va = fine_active[((int64_t)lo[2] * F.n[1] + lo[1]) * F.n[0] + lo[0]];
            uint8_t vb = fine_active[((int64_t)hi[2] * F.n[1] + hi[1]) * F.n[0] + hi[0]];
            bool oa = fine_is_type ? (va == T_FLUID) : (va != 0);
            bool ob = fine_is_type ? (vb == T_FLUID) : (vb != 0);
            if (oa && ob) area += fw[e1][a] * fw[e2][b];
        }
    double dist = cc[Ic[d]] - cc[Ic[d] - 1];
    double t = area / dist;
    T64[id] = t;
    T32[id] = (float)t;
}

// prolongation table of a fine axis: value(i) = (1-t) e[lo] + t e[hi], physical coordinates;
// lo is the parent (the coarse cell holding i, found in the children starts cs), hi the
// parent's neighbour on the side of the fine centre, clamped at the walls; a cell kept whole
// takes its parent alone
__global__ void k_prolong_tab(int nf, int nc, const int *__restrict__ cs, const double *__restrict__ fc,
                              const double *__restrict__ cc, int *lo, int *hi, double *t) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    int a = 0, b = nc;  // cs[a] <= i < cs[b]
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (cs[m] <= i)
            a = m;
        else
            b = m;
    }
    const int I = a;
    if (cs[I + 1] - cs[I] == 1) {
        lo[i] = I;
        hi[i] = I;
        t[i] = 0.0;
        return;
    }
    double x = fc[i], X = cc[I];
    int Jn = (x < X) ? I - 1 : I + 1;
    if (Jn < 0 || Jn >= nc) {
        lo[i] = I;
        hi[i] = I;
        t[i] = 0.0;
        return;
    }
    lo[i] = I;
    hi[i] = Jn;
    t[i] = (x - X) / (cc[Jn] - X);
}

hipError_t launch_hierarchy(ibm_grid *g, hipStream_t s) {
    // level-0 fluid volume
    hipLaunchKernelGGL(k_fluid_volume, dim3(RED_BLOCKS), dim3(256), 0, s, g->type, g->nx, g->ny, g->nz, g->w0[0],
                       g->w0[1], g->w0[2], g->partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, g->partials, RED_BLOCKS, &g->sc->vol[0]);
    for (int l = 1; l < g->nlev; ++l) {
        LevelHost &Fh = g->lev[l - 1], &Ch = g->lev[l];
        LevelDims F, C;
        for (int d = 0; d < 3; ++d) {
            F.n[d] = Fh.n[d];
            F.cs[d] = nullptr;
            C.n[d] = Ch.n[d];
            C.cs[d] = Ch.cs_d[d];
        }
        const bool fine_type = (l == 1);
        const uint8_t *fa = fine_type ? g->type : Fh.active;
        int64_t NC = Ch.ncell();
        unsigned nb = (unsigned)((NC + 255) / 256);
        // the partial sums of this kernel can exceed RED_BLOCKS: sum them directly
        double *parts = (double *)g->crossings;  // geometry scratch is free after classification
        hipLaunchKernelGGL(k_coarsen_active, dim3(nb), dim3(256), 0, s, F, C, fa, fine_type, Ch.active, Ch.w64[0],
                           Ch.w64[1], Ch.w64[2], parts);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, parts, (int)nb, &g->sc->vol[l]);
        const double *fw0 = (l == 1) ? g->w0[0] : Fh.w64[0];
        const double *fw1 = (l == 1) ? g->w0[1] : Fh.w64[1];
        const double *fw2 = (l == 1) ? g->w0[2] : Fh.w64[2];
        FaceAxes A;
        for (int d = 0; d < 3; ++d) {
            A.cc[d] = Ch.c64[d];
            A.T64[d] = Ch.T64[d];
            A.T32[d] = Ch.T32[d];
        }
        hipLaunchKernelGGL(k_face_T, dim3(nb, 3), dim3(256), 0, s, F, C, fa, fine_type, fw0, fw1, fw2, A);
    }
    if (g->nlev > 1) {
        const LevelHost &F0 = g->lev[0], &C1 = g->lev[1];
        LevelDims C;
        for (int d = 0; d < 3; ++d) {
            C.n[d] = C1.n[d];
            C.cs[d] = C1.cs_d[d];
        }
        hipLaunchKernelGGL(k_inject0, dim3((unsigned)((g->N + 255) / 256)), dim3(256), 0, s, g->nx, g->ny, g->nz,
                           g->type, C, C1.active, F0.plo[0], F0.phi[0], F0.plo[1], F0.phi[1], F0.plo[2], F0.phi[2],
                           g->inject0);
    }
    return hipGetLastError();
}

}  // namespace ibm
