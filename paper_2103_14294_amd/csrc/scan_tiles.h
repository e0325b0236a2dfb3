// Building blocks of the exclusive prefix sum over 4096-element tiles
// (256 threads x 16 elements): wave and workgroup scans, the sum of one tile
// and the scan of one tile with a carry-in.  Shared by the device-wide scans
// (prims.hip) and the batched rounds, which scan many short arrays in one launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace huge {
namespace scan {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;  // 4096

__device__ __forceinline__ int64_t wave_incl_scan(int64_t x) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of one 256-thread block's values; returns the block total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *warp_sums /* LDS[4] */, int64_t &excl) {
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(x);
    if (lane == 63) warp_sums[w] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) {
        int64_t s = warp_sums[i];
        if (i < w) base += s;
        tot += s;
    }
    excl = base + inc - x;
    __syncthreads();
    return tot;
}

// Sum of tile t of in[0, n) (every thread of the workgroup calls it).
template <typename Tin>
__device__ __forceinline__ int64_t tile_sum(const Tin *__restrict__ in, int64_t n, int64_t t) {
    __shared__ int64_t ws[kScanThreads / 64];
    int64_t base = t * kScanTile;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        int64_t i = base + j * kScanThreads + threadIdx.x;
        if (i < n) s += (int64_t)in[i];
    }
    int64_t ex;
    return block_excl_scan(s, ws, ex);
}

// Scans tile t of in[0, n): out[i] = c + exclusive prefix within the tile;
// returns the tile's sum (every thread of the workgroup calls it).
template <typename Tin>
__device__ __forceinline__ int64_t tile_scan(const Tin *__restrict__ in, int64_t n, int64_t c, int64_t *__restrict__ out,
                                             int64_t t) {
    __shared__ int64_t buf[kScanTile];
    __shared__ int64_t ws[kScanThreads / 64];
    int64_t base = t * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        int64_t i = base + j * kScanThreads + threadIdx.x;
        buf[j * kScanThreads + threadIdx.x] = i < n ? (int64_t)in[i] : 0;
    }
    __syncthreads();
    int64_t loc[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        loc[j] = s;
        s += buf[threadIdx.x * kScanPer + j];
    }
    int64_t ex;
    int64_t tot = block_excl_scan(s, ws, ex);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) buf[threadIdx.x * kScanPer + j] = c + ex + loc[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        int64_t i = base + j * kScanThreads + threadIdx.x;
        if (i < n) out[i] = buf[j * kScanThreads + threadIdx.x];
    }
    return tot;
}

}  // namespace scan
}  // namespace huge
