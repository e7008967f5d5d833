// Column-march tiling of level 0 shared by the z-marching passes (finepass.hip,
// momentum.hip): a workgroup owns a tile of 64 x 4 columns and a chunk of z-planes; each
// thread owns one column and marches upward.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_util.hpp"

namespace ibm {

constexpr int ZM_TX = 64, ZM_TY = 4, ZM_NT = ZM_TX * ZM_TY;

struct ZTiles {
    int ntx, nty, kc, ntiles, grid;
};

// Tile the grid so that about eight workgroups per CU are launched (all resident at once).
inline ZTiles ztiles(int nx, int ny, int nz) {
    ZTiles t;
    t.ntx = (nx + ZM_TX - 1) / ZM_TX;
    t.nty = (ny + ZM_TY - 1) / ZM_TY;
    const int64_t per_slab = (int64_t)t.ntx * t.nty;
    int nchunk = (int)std::max<int64_t>(1, (int64_t)8 * device_cu_count() / per_slab);
    nchunk = std::min(nchunk, std::max(1, nz / 2));
    int kc = (nz + nchunk - 1) / nchunk;
    kc += kc & 1;  // even chunk starts
    nchunk = (nz + kc - 1) / kc;
    t.kc = kc;
    t.ntiles = (int)(per_slab * nchunk);
    t.grid = ((t.ntiles + 7) / 8) * 8;
    return t;
}

struct ZPos {
    bool live;  // the workgroup has a tile
    int i, j, k0, k1, lane, wave;
};

// XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs, so each XCD
// receives a contiguous range of tiles and neighbouring tiles share one L2.
__device__ __forceinline__ ZPos zpos(const ZTiles &t, int nz) {
    ZPos z;
    const int per = gridDim.x >> 3;
    const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    z.live = logical < t.ntiles;
    int tile = logical;
    const int txi = tile % t.ntx;
    tile /= t.ntx;
    const int tyi = tile % t.nty;
    const int chunk = tile / t.nty;
    z.lane = (int)threadIdx.x & (ZM_TX - 1);
    z.wave = (int)threadIdx.x / ZM_TX;
    z.i = txi * ZM_TX + z.lane;
    z.j = tyi * ZM_TY + z.wave;
    z.k0 = chunk * t.kc;
    z.k1 = min(nz, z.k0 + t.kc);
    return z;
}

}  // namespace ibm
