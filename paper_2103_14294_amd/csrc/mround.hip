// Batched rounds: many queries of a batch advance together (Section 4.2's
// batching of operator input, Algorithm 5 per query, Section 5.3's sharing of
// workers between busy and idle work), with the scheduling on the device.
//
// Each query keeps its own Algorithm 5 state (GState), queues and segment
// buffers.  One round is a fixed sequence of launches:
//   k_mround_sched    one thread per query takes that query's next action
//                     (round_sched_step: prepare a segment of level W, or
//                     extend a range of its work items), then the workgroup
//                     turns the actions into exclusive prefixes over queries:
//                     prepare workgroups, scan tiles, and extend tiles per
//                     extend launch;
//   k_mround_prepare  every query's prepared segment, whatever its level;
//   k_mscan_*         the bounds scan of every prepared segment (tile sums,
//                     carries, tiles), the total landing at off[n];
//   k_mround_extend   one launch per (level W, last level or not): its
//                     workgroups claim tiles in order across the queries
//                     extending at W, so small queries fill the chip together
//                     and a hub row of one query spreads over every CU; each
//                     query's tiles are lane merges or binary searches, as
//                     its tuned buckets at that level favour.
// The round holds no memset or copy, so it can be recorded once in a graph
// and replayed until every query is done.
#include <algorithm>

#include "internal.h"
#include "round_sched.h"
#include "scan_tiles.h"
#include "tiles.h"

namespace huge {
namespace {

using namespace tiles;

constexpr int64_t kMRoundMaxItems = 1ll << 30;  // largest extend action of one query in one round
constexpr unsigned kMGrid = 4096;               // workgroups of the grid-stride prepare and scan launches

// Exclusive scan of x over the scheduler workgroup (kMaxBatch threads); every
// thread calls it.  out[t] receives thread t's prefix for t < np, out[np] the total.
__device__ __forceinline__ void sched_scan(int64_t x, int np, int64_t *out, int64_t *lds /* [kMaxBatch/64 + 1] */) {
    const int t = threadIdx.x, lane = __lane_id(), w = t >> 6;
    int64_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int q = 0; q < kMaxBatch / 64; ++q) {
        if (q < w) base += lds[q];
        tot += lds[q];
    }
    if (t < np) out[t] = base + inc - x;
    if (t == 0) out[np] = tot;
    __syncthreads();
}

__global__ __launch_bounds__(kMaxBatch) void k_mround_sched(MPat *mp, MRound *mr, MConst mc) {
    __shared__ int64_t s_w[kMaxBatch / 64 + 1];
    __shared__ int32_t s_alive[kMaxBatch / 64];
    __shared__ int32_t s_err;
    const int p = threadIdx.x;
    const int np = mc.np;
    if (p == 0) s_err = 0;
    __syncthreads();
    int64_t prep_blocks = 0, scan_tiles = 0, ext_tiles = 0;
    int pw = 0, lid = -1, alive = 0;
    if (p < np) {
        MPat &m = mp[p];
        GState &s = *m.gs;
        round_sched_step(s, m.gc, m.ctrl->qcount, kMRoundMaxItems);
        alive = s.done ? 0 : 1;
        if (s.error) atomicOr(&s_err, 1);
        for (int W = 2; W <= m.gc.lastW; ++W) {
            if (s.n_prep[W] > 0) {
                pw = W;
                prep_blocks = (s.n_prep[W] + kT - 1) / kT;
                scan_tiles = (s.n_prep[W] + scan::kScanTile - 1) / scan::kScanTile;
            }
            if (s.ext_w1[W] > s.ext_w0[W]) {
                lid = (W - 2) * 2 + (W == m.gc.lastW ? 1 : 0);
                const int64_t ti = m.search[W] ? (int64_t)kTile : (int64_t)mc.tile_items[lid];
                ext_tiles = (s.ext_w1[W] - s.ext_w0[W] + ti - 1) / ti;
            }
        }
        mr->prep_W[p] = pw;
    }
    sched_scan(prep_blocks, np, mr->prep_pre, s_w);
    sched_scan(scan_tiles, np, mr->scan_pre, s_w);
    for (int l = 0; l < kMLaunches; ++l)
        if ((mc.lids >> l) & 1u) sched_scan(lid == l ? ext_tiles : 0, np, mr->ext_pre[l], s_w);
    if (p < kMLaunches) mr->claim[p] = 0;
    {
        const uint64_t m = __ballot(alive != 0);
        if (__lane_id() == 0) s_alive[p >> 6] = __popcll(m);
    }
    __syncthreads();
    if (p == 0) {
        int a = 0;
        for (int q = 0; q < kMaxBatch / 64; ++q) a += s_alive[q];
        mr->active = a;
        if (s_err) mr->error = 1;
    }
}

// largest p in [0, np - 1] with pre[p] <= t (t < pre[np]): the query owning item t
__device__ __forceinline__ int owner(const int64_t *pre, int np, int64_t t) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int W>
__device__ __forceinline__ void mprepare_w(const MPat &m, int64_t i) {
    const GState &gs = *m.gs;
    const int64_t n = gs.n_prep[W], row0 = gs.lv[W].seg_row0;
    if (W == m.gc.lastW)
        prepare_row<W, true>(m.q[W], row0, n, m.g, m.P, m.sb[W], m.ctrl, i);
    else
        prepare_row<W, false>(m.q[W], row0, n, m.g, m.P, m.sb[W], m.ctrl, i);
}

__global__ __launch_bounds__(kT) void k_mround_prepare(const MPat *__restrict__ mp, const MRound *__restrict__ mr,
                                                       int np) {
    const int64_t total = mr->prep_pre[np];
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int p = __builtin_amdgcn_readfirstlane(owner(mr->prep_pre, np, b));
        const MPat &m = mp[p];
        const int64_t i = (b - mr->prep_pre[p]) * kT + threadIdx.x;
        switch (mr->prep_W[p]) {
            case 2: mprepare_w<2>(m, i); break;
            case 3: mprepare_w<3>(m, i); break;
            case 4: mprepare_w<4>(m, i); break;
            case 5: mprepare_w<5>(m, i); break;
            case 6: mprepare_w<6>(m, i); break;
            case 7: mprepare_w<7>(m, i); break;
            default: break;
        }
        __syncthreads();
    }
}

// The bounds scan of every prepared segment: tile sums (segments of more than
// one tile), the scan of those sums (one workgroup per query), then the tiles
// with their carries; the last tile of a segment writes its total at off[n].
__global__ __launch_bounds__(scan::kScanThreads) void k_mscan_reduce(const MPat *__restrict__ mp,
                                                                     const MRound *__restrict__ mr, int np) {
    const int64_t total = mr->scan_pre[np];
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int p = __builtin_amdgcn_readfirstlane(owner(mr->scan_pre, np, b));
        const int64_t tiles = mr->scan_pre[p + 1] - mr->scan_pre[p];
        if (tiles > 1) {
            const MPat &m = mp[p];
            const int W = mr->prep_W[p];
            const int64_t t = b - mr->scan_pre[p];
            const int64_t s = scan::tile_sum(m.sb[W].bound, m.gs->n_prep[W], t);
            if (threadIdx.x == 0) m.scan_part[t] = s;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(scan::kScanThreads) void k_mscan_carry(const MPat *__restrict__ mp,
                                                                    const MRound *__restrict__ mr, int np) {
    for (int p = blockIdx.x; p < np; p += gridDim.x) {
        const int64_t tiles = mr->scan_pre[p + 1] - mr->scan_pre[p];
        if (tiles > 1) scan::tile_scan(mp[p].scan_part, tiles, 0, mp[p].scan_part, 0);
        __syncthreads();
    }
}

__global__ __launch_bounds__(scan::kScanThreads) void k_mscan_tiles(const MPat *__restrict__ mp,
                                                                    const MRound *__restrict__ mr, int np) {
    const int64_t total = mr->scan_pre[np];
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
        const int p = __builtin_amdgcn_readfirstlane(owner(mr->scan_pre, np, b));
        const MPat &m = mp[p];
        const int W = mr->prep_W[p];
        const int64_t tiles = mr->scan_pre[p + 1] - mr->scan_pre[p];
        const int64_t t = b - mr->scan_pre[p];
        const int64_t n = m.gs->n_prep[W];
        const int64_t c = tiles > 1 ? m.scan_part[t] : 0;
        const int64_t tot = scan::tile_scan(m.sb[W].bound, n, c, m.sb[W].off, t);
        if (t == tiles - 1 && threadIdx.x == 0) m.sb[W].off[n] = c + tot;
        __syncthreads();
    }
}

// SEARCH: the launch also serves queries whose level W runs binary-search
// tiles (a branch that is uniform over the workgroup, by the tile's query)
template <int W, int MODE, int RUN, bool BLK, bool SEARCH = false>
__global__ __launch_bounds__(kT) void k_mround_extend(const MPat *__restrict__ mp, MRound *__restrict__ mr, int np,
                                                      int lid) {
    __shared__ int64_t s_t;
    __shared__ int32_t s_p;
    const int64_t *pre = mr->ext_pre[lid];
    const int64_t total = pre[np];
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t t = (int64_t)atomicAdd(&mr->claim[lid], 1ull);
            s_t = t;
            s_p = t < total ? owner(pre, np, t) : 0;
        }
        __syncthreads();
        const int64_t t = s_t;
        const int p = __builtin_amdgcn_readfirstlane(s_p);
        __syncthreads();
        if (t >= total) return;
        const MPat &m = mp[p];
        const GState &gs = *m.gs;
        ExtArgs a;
        a.rows = m.q[W];
        a.row0 = gs.lv[W].seg_row0;
        a.rid = nullptr;
        a.off = m.sb[W].off;
        a.pinfo = m.sb[W].pinfo;
        a.hpre = m.sb[W].hpre;
        a.nrows = gs.lv[W].seg_n;
        a.w0 = gs.ext_w0[W];
        a.w1 = gs.ext_w1[W];
        a.out = MODE == MODE_EMIT ? m.q[W + 1] : nullptr;
        a.ctrl = m.ctrl;
        a.inv_rank = m.inv_rank;
        a.g = m.g;
        a.P = m.P;
        if constexpr (SEARCH) {
            if (m.search[W])
                extend_tile<W, MODE, STRAT_BSEARCH>(a, t - pre[p]);
            else
                merge_tile<W, MODE, RUN, BLK>(a, t - pre[p]);
        } else {
            merge_tile<W, MODE, RUN, BLK>(a, t - pre[p]);
        }
        __syncthreads();
    }
}

// Workgroups of f that fit on the device at once.
template <typename F>
unsigned resident(F f) {
    int dev = 0, cus = 0, per = 0;
    HUGE_HIP(hipGetDevice(&dev));
    HUGE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HUGE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kT, 0));
    return (unsigned)std::max(1, cus * std::max(1, per));
}

template <int W, int MODE, int RUN, bool BLK>
void mextend(bool search, const MPat *mp, MRound *mr, int np, int lid, hipStream_t st) {
    if (search) {
        auto f = k_mround_extend<W, MODE, RUN, BLK, true>;
        hipLaunchKernelGGL(f, dim3(resident(f)), dim3(kT), 0, st, mp, mr, np, lid);
    } else {
        auto f = k_mround_extend<W, MODE, RUN, BLK, false>;
        hipLaunchKernelGGL(f, dim3(resident(f)), dim3(kT), 0, st, mp, mr, np, lid);
    }
}

// RUN and BLK of a lane-merge strategy; emitting kernels stage at most 16 rows per lane
void merge_shape(int strategy, bool emit, int &run, bool &blk) {
    switch (strategy) {
        case STRAT_MERGE_SHORT: run = 4; blk = false; break;
        case STRAT_MERGE_LONG: run = 64; blk = false; break;
        case STRAT_BLOCK_MERGE: run = 16; blk = true; break;
        case STRAT_BLOCK_MERGE_LONG: run = 64; blk = true; break;
        case STRAT_LANE_MERGE: run = 16; blk = false; break;
        default: HUGE_FAIL(HUGE_EINVAL, "batched rounds take lane-merge strategies (2..6), not %d", strategy);
    }
    if (emit && run > 16) run = 16;
}

template <int W, int MODE>
void mextend_mode(int run, bool blk, bool search, const MPat *mp, MRound *mr, int np, int lid, hipStream_t st) {
    if (blk) {
        if (run == 16) mextend<W, MODE, 16, true>(search, mp, mr, np, lid, st);
        else if (MODE != MODE_EMIT) mextend<W, MODE, (MODE == MODE_EMIT ? 16 : 64), true>(search, mp, mr, np, lid, st);
    } else {
        if (run == 4) mextend<W, MODE, 4, false>(search, mp, mr, np, lid, st);
        else if (run == 16) mextend<W, MODE, 16, false>(search, mp, mr, np, lid, st);
        else if (MODE != MODE_EMIT) mextend<W, MODE, (MODE == MODE_EMIT ? 16 : 64), false>(search, mp, mr, np, lid, st);
    }
}

template <int W>
void mextend_w(bool last, int count_mode, int run, bool blk, bool search, const MPat *mp, MRound *mr, int np,
               int lid, hipStream_t st) {
    if (!last)
        mextend_mode<W, MODE_EMIT>(run, blk, search, mp, mr, np, lid, st);
    else if (count_mode == MODE_COUNT_NOHASH)
        mextend_mode<W, MODE_COUNT_NOHASH>(run, blk, search, mp, mr, np, lid, st);
    else
        mextend_mode<W, MODE_COUNT>(run, blk, search, mp, mr, np, lid, st);
}

}  // namespace

void launch_mround_sched(MPat *mp, MRound *mr, const MConst &mc, hipStream_t st) {
    hipLaunchKernelGGL(k_mround_sched, dim3(1), dim3(kMaxBatch), 0, st, mp, mr, mc);
    HUGE_HIP(hipGetLastError());
}

void launch_mround_prepare(const MPat *mp, const MRound *mr, int np, hipStream_t st) {
    hipLaunchKernelGGL(k_mround_prepare, dim3(kMGrid), dim3(kT), 0, st, mp, mr, np);
    HUGE_HIP(hipGetLastError());
}

void launch_mround_scan(const MPat *mp, MRound *mr, int np, int64_t max_tiles, hipStream_t st) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(max_tiles, kMGrid));
    hipLaunchKernelGGL(k_mscan_reduce, dim3(grid), dim3(scan::kScanThreads), 0, st, mp, (const MRound *)mr, np);
    hipLaunchKernelGGL(k_mscan_carry, dim3((unsigned)std::min(np, 1024)), dim3(scan::kScanThreads), 0, st, mp,
                       (const MRound *)mr, np);
    hipLaunchKernelGGL(k_mscan_tiles, dim3(grid), dim3(scan::kScanThreads), 0, st, mp, (const MRound *)mr, np);
    HUGE_HIP(hipGetLastError());
}

int mround_tile_items(int lid, int strategy) {
    int run = 16;
    bool blk = false;
    merge_shape(strategy, (lid & 1) == 0, run, blk);
    return kT * run;
}

void launch_mround_extend(int lid, int count_mode, int strategy, bool search, const MPat *mp, MRound *mr, int np,
                          hipStream_t st) {
    const int W = lid / 2 + 2;
    const bool last = (lid & 1) != 0;
    int run = 16;
    bool blk = false;
    merge_shape(strategy, !last, run, blk);
    switch (W) {
        case 2: mextend_w<2>(last, count_mode, run, blk, search, mp, mr, np, lid, st); break;
        case 3: mextend_w<3>(last, count_mode, run, blk, search, mp, mr, np, lid, st); break;
        case 4: mextend_w<4>(last, count_mode, run, blk, search, mp, mr, np, lid, st); break;
        case 5: mextend_w<5>(last, count_mode, run, blk, search, mp, mr, np, lid, st); break;
        case 6: mextend_w<6>(last, count_mode, run, blk, search, mp, mr, np, lid, st); break;
        case 7: mextend_w<7>(last, count_mode, run, blk, search, mp, mr, np, lid, st); break;
        default: HUGE_FAIL(HUGE_EINVAL, "bad extend launch %d", lid);
    }
    HUGE_HIP(hipGetLastError());
}

}  // namespace huge
