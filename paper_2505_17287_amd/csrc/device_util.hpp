// Device helpers: deterministic block reductions and small index utilities (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

namespace ibm {

// Compute units of the current device (queried once per device; 256 on MI355X).
inline int device_cu_count() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a block of NT threads (1D flat thread index `tid`); result valid in thread 0.
// Fixed combination order -> bitwise reproducible for a fixed launch shape.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh, int tid) {
    v = wave_sum(v);
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0) {
        for (int w = 0; w < NT / 64; ++w) r += sh[w];
    }
    __syncthreads();
    return r;
}
template <int NT>
__device__ __forceinline__ double block_max(double v, double *sh, int tid) {
    v = wave_max(v);
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0) {
        for (int w = 0; w < NT / 64; ++w) r = fmax(r, sh[w]);
    }
    __syncthreads();
    return r;
}

// two adjacent elements moved as one access (8- or 16-byte aligned pairs)
template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
    using type = double2;
};
template <>
struct Pair2<float> {
    using type = float2;
};

// (i, j, k) of the flat index id = (k ny + j) nx + i.  Grids hold fewer than 2^31 cells,
// so 32-bit unsigned arithmetic is exact (and far cheaper than 64-bit division).
__device__ __forceinline__ void unflatten(int64_t id, int nx, int ny, int &i, int &j, int &k) {
    const uint32_t u = (uint32_t)id, row = u / (uint32_t)nx;
    i = (int)(u - row * (uint32_t)nx);
    k = (int)(row / (uint32_t)ny);
    j = (int)(row - (uint32_t)k * (uint32_t)ny);
}

// largest i in [0, n-2] with c[i] <= x (0 if x < c[0]); n >= 2
__device__ __forceinline__ int box_lo(const double *c, int n, double x) {
    int lo = 0, hi = n - 2;
    if (x < c[0]) return 0;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (c[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// first index i with c[i] >= x (n if none)
__device__ __forceinline__ int lower_idx(const double *c, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (c[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
// last index i with c[i] <= x (-1 if none)
__device__ __forceinline__ int upper_idx(const double *c, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (c[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo - 1;
}

}  // namespace ibm
