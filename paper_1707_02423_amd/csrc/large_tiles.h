// Tile map of the tiled path (shared by the FP32 gather kernels of large.hip
// and the BF16 MFMA kernels of large_mfma.hip): every pair's state is cut
// into 128-row x 64-column tiles, numbered pair by pair (tile_off), with the
// pair of each tile in tile_pair; each tile leaves FP64 partials of the
// norms that a per-pair kernel sums in tile order.
#pragma once

#include "cfsim_internal.h"
#include "pair_device.h"

namespace cfsim {
namespace tiled {

constexpr int kTileRows = 128;                  // rows per tile
constexpr int kStepThreads = 256;               // 4 waves, 32 rows each
constexpr int kNWStep = kStepThreads / kWave;
constexpr int kRowsPerWave = kTileRows / kNWStep;

__device__ inline int tiles_of(int nC, int nR) { return ((nR + kTileRows - 1) / kTileRows) * ((nC + 63) / 64); }
static_assert(kTileRows == 128, "large_tiles() in cfsim_internal.h assumes 128-row tiles");

// Pair p's buffer b of slot_elems elements.
template <typename T>
__device__ inline T* buf_of(const LargeJob& J, int p, int b) {
    return reinterpret_cast<T*>(J.bufs) + ((long long)p * J.nslots + b) * J.slot_elems;
}

__device__ inline int pair_of_tile(const LargeJob& J, long long t) { return J.tile_pair[t]; }

// ---------------------------------------------------------------- tiles
struct Tile {
    int r0, c0;
};

// XCD-aware tile order: workgroups are dealt to the 8 XCDs round-robin, so
// the workgroups of one XCD take one contiguous range of tiles (neighbouring
// row strips of one pair share rows of the iterate through that XCD's L2).
struct TileRange {
    long long first, end, stride;
};
__device__ inline TileRange tile_range(const LargeJob& J) {
    const long long total = J.tile_off[J.n_pairs];
    const int xcd = blockIdx.x & 7, y = blockIdx.x >> 3;
    TileRange r;
    r.first = total * xcd / 8 + y;
    r.end = total * (xcd + 1) / 8;
    r.stride = gridDim.x >> 3;
    return r;
}

__device__ inline Tile tile_at(const LargeJob& J, long long t, const LargeState* s, int p) {
    Tile x;
    const int lt = (int)(t - J.tile_off[p]);
    const int nct = (s->nC + 63) / 64;
    x.r0 = (lt / nct) * kTileRows;
    x.c0 = (lt % nct) * 64;
    return x;
}

// Per-tile partials (fixed order: waves, then lanes).
__device__ inline void tile_partials(const LargeJob& J, long long t, double nu2, double d2, double* red) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    nu2 = dev::wave_sum(nu2);
    d2 = dev::wave_sum(d2);
    if (lane == 0) {
        red[wave] = nu2;
        red[kNWStep + wave] = d2;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kNWStep; ++w) {
            a += red[w];
            b += red[kNWStep + w];
        }
        J.part_nu[t] = a;
        J.part_delta[t] = b;
    }
    __syncthreads();
}

}  // namespace tiled
}  // namespace cfsim
