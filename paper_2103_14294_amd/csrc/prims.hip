// Device-wide primitives used by graph loading and by the level scheduler:
//   * exclusive prefix sum (recursive reduce / scan / add, 4096-element tiles)
//   * stable least-significant-digit radix sort of (uint32 key, uint32 value)
//     pairs, 8-bit digits, with wave64 ballot-based stable ranking.
// Written for gfx950: 64-lane wavefronts, 256-thread workgroups.
#include "prims.h"
#include "scan_tiles.h"

namespace huge {

namespace {

using namespace scan;

template <typename Tin>
__global__ __launch_bounds__(kScanThreads) void k_tile_reduce(const Tin *__restrict__ in, int64_t n,
                                                              int64_t *__restrict__ partial) {
    const int64_t tot = tile_sum(in, n, blockIdx.x);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Scan one tile: out[i] = carry[tile] + exclusive prefix within the tile.
template <typename Tin>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const Tin *__restrict__ in, int64_t n,
                                                            const int64_t *__restrict__ carry,
                                                            int64_t *__restrict__ out, int64_t *__restrict__ total) {
    const int64_t c = carry ? carry[blockIdx.x] : 0;
    const int64_t tot = tile_scan(in, n, c, out, blockIdx.x);
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = c + tot;
}

// The same three steps with the element count read from device memory at run
// time (fixed grids sized for the largest count; tiles past the count and
// every kernel of a zero count do nothing), so that they can be recorded once
// in a graph.  out[n] receives the total.
__global__ __launch_bounds__(kScanThreads) void k_tile_reduce_dn(const int32_t *__restrict__ in,
                                                                 const int64_t *__restrict__ n_dev,
                                                                 int64_t *__restrict__ partial) {
    const int64_t n = *n_dev;
    if ((int64_t)blockIdx.x * kScanTile >= n) return;
    const int64_t tot = tile_sum(in, n, blockIdx.x);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_partial_scan_dn(const int64_t *__restrict__ n_dev,
                                                                  int64_t *__restrict__ partial) {
    const int64_t n = *n_dev;
    if (n <= kScanTile) return;  // a single tile needs no carries
    const int64_t nb = (n + kScanTile - 1) / kScanTile;  // <= kScanTile
    tile_scan(partial, nb, 0, partial, 0);
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan_dn(const int32_t *__restrict__ in,
                                                               const int64_t *__restrict__ n_dev,
                                                               const int64_t *__restrict__ partial,
                                                               int64_t *__restrict__ out) {
    const int64_t n = *n_dev;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    if (base >= n) return;
    const int64_t c = n > kScanTile ? partial[blockIdx.x] : 0;
    const int64_t tot = tile_scan(in, n, c, out, blockIdx.x);
    if (base + kScanTile >= n && threadIdx.x == 0) out[n] = c + tot;
}

template <typename Tin>
void scan_rec(const Tin *in, int64_t *out, int64_t n, int64_t *total, int64_t *tmp, hipStream_t st) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_tile_scan<Tin>, dim3(1), dim3(kScanThreads), 0, st, in, n, (const int64_t *)nullptr, out,
                           total);
        return;
    }
    int64_t *partial = tmp;
    int64_t *rest = tmp + nb;
    hipLaunchKernelGGL(k_tile_reduce<Tin>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, partial);
    scan_rec<int64_t>(partial, partial, nb, nullptr, rest, st);
    hipLaunchKernelGGL(k_tile_scan<Tin>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n,
                       (const int64_t *)partial, out, total);
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsPer = 32;
constexpr int kRsTile = kRsThreads * kRsPer;  // 8192 pairs per workgroup

__global__ __launch_bounds__(kRsThreads) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                           uint32_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
    for (int j = 0; j < kRsPer; ++j) {
        int64_t i = base + j * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsThreads) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                              const uint32_t *__restrict__ vin, int64_t n, int shift,
                                                              const int64_t *__restrict__ offs, int64_t nblocks,
                                                              uint32_t *__restrict__ kout,
                                                              uint32_t *__restrict__ vout) {
    __shared__ int64_t gbase[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t off[4][256];
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = __lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    gbase[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    run[t] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) cnt[q][t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int j = 0; j < kRsPer; ++j) {
        int64_t i = base + j * kRsThreads + t;
        bool act = i < n;
        uint32_t key = act ? kin[i] : 0u;
        uint32_t val = act ? vin[i] : 0u;
        uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        uint32_t rnk = (uint32_t)__popcll(peers & lt);
        if (act && rnk == 0) cnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t r = run[t];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                off[q][t] = r;
                r += cnt[q][t];
                cnt[q][t] = 0;
            }
            run[t] = r;
        }
        __syncthreads();
        if (act) {
            int64_t p = gbase[d] + off[w][d] + rnk;
            kout[p] = key;
            vout[p] = val;
        }
    }
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) {
    int64_t tot = 0;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    while (nb > 1) {
        tot += nb;
        nb = (nb + kScanTile - 1) / kScanTile;
    }
    return tot + 8;
}

void scan_excl(const uint32_t *in, int64_t *out, int64_t n, int64_t *total, int64_t *tmp, hipStream_t st) {
    if (n <= 0) {
        if (total) HUGE_HIP(hipMemsetAsync(total, 0, sizeof(int64_t), st));
        return;
    }
    scan_rec<uint32_t>(in, out, n, total, tmp, st);
}
void scan_excl(const int32_t *in, int64_t *out, int64_t n, int64_t *total, int64_t *tmp, hipStream_t st) {
    if (n <= 0) {
        if (total) HUGE_HIP(hipMemsetAsync(total, 0, sizeof(int64_t), st));
        return;
    }
    scan_rec<int32_t>(in, out, n, total, tmp, st);
}

int64_t scan_devn_max() { return (int64_t)kScanTile * kScanTile; }

void scan_excl_devn(const int32_t *in, int64_t *out, const int64_t *n_dev, int64_t nmax, int64_t *tmp,
                    hipStream_t st) {
    if (nmax <= 0) return;
    if (nmax > scan_devn_max()) HUGE_FAIL(HUGE_EINVAL, "scan_excl_devn: %lld elements exceed the limit", (long long)nmax);
    const unsigned nb = (unsigned)((nmax + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_tile_reduce_dn, dim3(nb), dim3(kScanThreads), 0, st, in, n_dev, tmp);
    hipLaunchKernelGGL(k_partial_scan_dn, dim3(1), dim3(kScanThreads), 0, st, n_dev, tmp);
    hipLaunchKernelGGL(k_tile_scan_dn, dim3(nb), dim3(kScanThreads), 0, st, in, n_dev, (const int64_t *)tmp, out);
}

int64_t radix_sort_hist_elems(int64_t n) {
    int64_t nb = (n + kRsTile - 1) / kRsTile;
    return nb * 256;
}

// Returns true when the sorted result is in (k1, v1), false when in (k0, v0).
bool radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits, uint32_t *hist,
                      int64_t *offs, int64_t *scan_tmp, hipStream_t st) {
    if (n <= 1 || bits <= 0) return false;
    int64_t nb = (n + kRsTile - 1) / kRsTile;
    bool flip = false;
    for (int shift = 0; shift < bits; shift += 8) {
        const uint32_t *ki = flip ? k1 : k0;
        const uint32_t *vi = flip ? v1 : v0;
        uint32_t *ko = flip ? k0 : k1;
        uint32_t *vo = flip ? v0 : v1;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kRsThreads), 0, st, ki, n, shift, hist, nb);
        scan_excl(hist, offs, nb * 256, nullptr, scan_tmp, st);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kRsThreads), 0, st, ki, vi, n, shift,
                           (const int64_t *)offs, nb, ko, vo);
        flip = !flip;
    }
    HUGE_HIP(hipGetLastError());
    return flip;
}

}  // namespace huge
