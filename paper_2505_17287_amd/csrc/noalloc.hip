// Cell classification without a handle or a workspace, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  It runs the kernels of ibm_classify (geometry.hip) on caller-owned inputs and
// output, with every intermediate buffer (cell centres, per-column crossing counts, offsets
// and lists, scan totals, counters) in one fixed array of device memory per GPU, `scratch`.
//
// `scratch` is a file-scope __device__ array: each GPU the library runs on holds its own copy
// from the first use until the process ends.  In host code its name is only a stand-in for
// the symbol, so its device address is taken once per device with hipGetSymbolAddress (with
// that device current) and kept; kernels receive that address.  Every call on one GPU shares
// the array and leaves the last call's contents in it: everything that must start at zero is
// cleared by a kernel at the start of each call, and calls that overlap on one GPU (other
// threads, other streams) race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ibm_impl.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(IBM_NOALLOC_SCRATCH_MB) << 20;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// device address of this GPU's scratch array (taken once per device, with it current)
hipError_t scratch_address(int dev, unsigned char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return hipSuccess;
}

// centres of one axis from its face coordinates (the arithmetic of the handle's metrics)
__global__ void k_centres(int n, const double *__restrict__ f, double *c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0.5 * (f[i] + f[i + 1]);
}

// sub-buffer carving of the scratch array (256-byte aligned pieces)
struct Carve {
    size_t off = 0;
    template <typename T>
    size_t take(int64_t count) {
        off = (off + 255) & ~size_t(255);
        const size_t at = off;
        off += sizeof(T) * (size_t)(count > 0 ? count : 1);
        return at;
    }
};

}  // namespace

extern "C" ibm_status ibm_classify_noalloc(int nx, int ny, int nz, const double *xf, const double *yf,
                                           const double *zf, const double *verts, int64_t nv, const int32_t *tris,
                                           int64_t nt, uint8_t *type_out, int64_t counts_out[3], void *stream) {
    using namespace ibm;
    if (nx < 2 || ny < 2 || nz < 1) return report_error(IBM_E_ARG, "ibm_classify_noalloc: need nx, ny >= 2 and nz >= 1");
    if ((int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return report_error(IBM_E_ARG, "ibm_classify_noalloc: more than 2^31 cells");
    if (!xf || !yf || !zf || !verts || !tris || !type_out || !counts_out)
        return report_error(IBM_E_ARG, "ibm_classify_noalloc: NULL argument");
    if (nv < 3 || nt < 1) return report_error(IBM_E_ARG, "ibm_classify_noalloc: empty mesh");
    const int64_t ncol = (int64_t)nx * ny;
    // fixed part of the carving; whatever remains holds the crossings
    Carve C;
    const size_t o_xc = C.take<double>(nx), o_yc = C.take<double>(ny), o_zc = C.take<double>(nz);
    const size_t o_cnt = C.take<int32_t>(ncol + 1), o_off = C.take<int32_t>(ncol + 1),
                 o_fill = C.take<int32_t>(ncol + 1);
    const size_t o_blk = C.take<int64_t>(classify_scan_blocks(ncol + 1));
    const size_t o_ctr = C.take<int64_t>(8);
    const size_t o_mark = C.take<int64_t>(classify_mark16_parts(nx, ny, nz));
    const size_t o_cross = (C.off + 255) & ~size_t(255);
    const int64_t min_cross = 2 * ncol + 1024;
    if (o_cross + sizeof(double) * (size_t)min_cross > SCRATCH_BYTES)
        return report_error(IBM_E_NOMEM, "ibm_classify_noalloc: " + std::to_string(nx) + " x " + std::to_string(ny) +
                                             " columns exceed the " + std::to_string(IBM_NOALLOC_SCRATCH_MB) +
                                             " MiB scratch (at most about " +
                                             std::to_string(SCRATCH_BYTES / 36) + " columns)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report_error(IBM_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return report_error(IBM_E_DEVICE, "ibm_classify_noalloc: device index too large");
    unsigned char *base = nullptr;
    if ((e = scratch_address(dev, &base)) != hipSuccess)
        return report_error(IBM_E_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    double *xc = reinterpret_cast<double *>(base + o_xc), *yc = reinterpret_cast<double *>(base + o_yc),
           *zc = reinterpret_cast<double *>(base + o_zc);
    hipLaunchKernelGGL(k_centres, dim3((nx + 127) / 128), dim3(128), 0, s, nx, xf, xc);
    hipLaunchKernelGGL(k_centres, dim3((ny + 127) / 128), dim3(128), 0, s, ny, yf, yc);
    hipLaunchKernelGGL(k_centres, dim3((nz + 127) / 128), dim3(128), 0, s, nz, zf, zc);
    ClassifyBufs B;
    B.nx = nx;
    B.ny = ny;
    B.nz = nz;
    B.verts = verts;
    B.tris = tris;
    B.nt = nt;
    B.xc = xc;
    B.yc = yc;
    B.zc = zc;
    B.col_cnt = reinterpret_cast<int32_t *>(base + o_cnt);
    B.col_off = reinterpret_cast<int32_t *>(base + o_off);
    B.col_fill = reinterpret_cast<int32_t *>(base + o_fill);
    B.crossings = reinterpret_cast<double *>(base + o_cross);
    B.cross_cap = (int64_t)((SCRATCH_BYTES - o_cross) / sizeof(double));
    B.counters = reinterpret_cast<int64_t *>(base + o_ctr);
    B.blk = reinterpret_cast<int64_t *>(base + o_blk);
    B.mark_parts = reinterpret_cast<int64_t *>(base + o_mark);
    B.type = type_out;
    if ((e = launch_classify_cells(B, s)) != hipSuccess)
        return report_error(IBM_E_DEVICE, std::string("ibm_classify_noalloc: ") + hipGetErrorString(e));
    int64_t hc[8];
    if ((e = hipMemcpyAsync(hc, B.counters, sizeof(hc), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return report_error(IBM_E_DEVICE, std::string("ibm_classify_noalloc: ") + hipGetErrorString(e));
    if (hc[4]) return report_error(IBM_E_NOMEM, "ibm_classify_noalloc: more ray crossings than the scratch holds");
    if (hc[3])
        return report_error(IBM_E_GEOMETRY, "ibm_classify_noalloc: " + std::to_string(hc[3]) +
                                                " columns with an odd number of ray crossings (mesh not watertight)");
    counts_out[0] = hc[0];
    counts_out[1] = hc[1];
    counts_out[2] = hc[2];
    if (hc[0] == 0) return report_error(IBM_E_GEOMETRY, "ibm_classify_noalloc: no fluid cell");
    return IBM_OK;
}
