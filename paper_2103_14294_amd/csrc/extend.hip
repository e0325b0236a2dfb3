// PULL-EXTEND on gfx950 (Section 4.2 semantics, Algorithm 4's intersect
// stage): for every partial match f of the induced prefix pi_0..pi_{W-1},
// the candidates for the next query vertex pi_W are
//     C = intersection over p in Ext of N(f[p])              (Eq. 2)
// kept when v differs from every f[p] outside Ext (injectivity), and when v
// respects the symmetry-breaking constraints between pi_W and the prefix.
//
// One segment of input rows is handled in two launches:
//   k_prepare : per row, the constraints become one window [lo, hi) on v
//               (lo = 1 + max f[p] over "f[p] < v", hi = min f[p] over
//               "v < f[p]"); each list N(f[p]), p in Ext, is trimmed to the
//               window by binary search and the shortest trimmed list is the
//               probe.  Its length bounds the row's output (used for
//               bounded-memory chunking) and is the row's work.
//   k_extend  : a flat, load-balanced pass over the segment's work items
//               (one probe element each): locate the row (binary search in
//               the exclusive scan of the bounds), test the probe element
//               against the other Ext lists (binary search), apply the
//               injectivity and slice filters, then either append the
//               extended row to the next level's queue (wave ballot +
//               one atomic per workgroup) or, at the last level, fold it into
//               the counting SINK (count, set-hash sum and xor).
#include <algorithm>

#include "devfuncs.h"
#include "internal.h"
#include "prims.h"
#include "round_sched.h"
#include "tiles.h"

namespace huge {
namespace {

using namespace dev;
using namespace tiles;

template <int W, bool LAST>
__global__ __launch_bounds__(kT) void k_prepare(const int32_t *__restrict__ rows, int64_t row0, int64_t nrows,
                                                GraphDev g, DevPlan P, SegBufs s, Ctrl *ctrl) {
    prepare_row<W, LAST>(rows, row0, nrows, g, P, s, ctrl, (int64_t)blockIdx.x * kT + threadIdx.x);
}

template <int W, int MODE, int STRAT>
__global__ __launch_bounds__(kT) void k_extend(ExtArgs a) {
    extend_tile<W, MODE, STRAT>(a, blockIdx.x);
}

// k == 2: every valid level-2 row is a match.
__global__ __launch_bounds__(kT) void k_edge_sink(GraphDev g, DevPlan P, int64_t e0, int64_t e1, int mode,
                                                  int32_t *out, const int32_t *inv_rank, Ctrl *ctrl) {
    __shared__ unsigned long long s_red[3][kT / 64];
    __shared__ int32_t s_cnt[kT / 64];
    __shared__ unsigned long long s_base;
    const int64_t e = e0 + (int64_t)blockIdx.x * kT + threadIdx.x;
    bool ok = false;
    int32_t f[2] = {0, 0};
    if (e < e1) {
        load_row<2>(nullptr, g, e, f);
        ok = level2_ok(f, P, g);
    }
    const int wv = threadIdx.x >> 6;
    if (mode == MODE_COUNT) {
        unsigned long long c = ok ? 1 : 0, h = ok ? mix64(mix64(edge_key(f[0], f[1]))) : 0;
        unsigned long long cs = wave_sum_u64(c), hs = wave_sum_u64(h), hx = wave_xor_u64(h);
        if (__lane_id() == 0) {
            s_red[0][wv] = cs;
            s_red[1][wv] = hs;
            s_red[2][wv] = hx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long a = 0, s = 0, x = 0;
            for (int q = 0; q < kT / 64; ++q) {
                a += s_red[0][q];
                s += s_red[1][q];
                x ^= s_red[2][q];
            }
            if (a) {
                atomicAdd(&ctrl->acc[0], a);
                atomicAdd(&ctrl->acc[1], s);
                atomicXor(&ctrl->acc[2], x);
                atomicAdd(&ctrl->level[1], a);
            }
        }
    } else {
        uint64_t m = __ballot(ok);
        const int lane = __lane_id();
        if (lane == 0) s_cnt[wv] = __popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int q = 0; q < kT / 64; ++q) t += s_cnt[q];
            s_base = t ? atomicAdd(&ctrl->qcount[HUGE_KMAX], (unsigned long long)t) : 0;
            if (t) atomicAdd(&ctrl->level[1], (unsigned long long)t);
        }
        __syncthreads();
        if (ok) {
            int wb = 0;
            for (int q = 0; q < wv; ++q) wb += s_cnt[q];
            int64_t o = (int64_t)s_base + wb + __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            // row indexed by query vertex: vertex q sits at position pos[q]
            const int32_t a0 = P.pos[0] == 0 ? f[0] : f[1];
            const int32_t a1 = P.pos[1] == 0 ? f[0] : f[1];
            out[o * 2 + 0] = inv_rank ? inv_rank[a0] : a0;
            out[o * 2 + 1] = inv_rank ? inv_rank[a1] : a1;
        }
    }
}

__global__ __launch_bounds__(kT) void k_root_count(GraphDev g, DevPlan P, Ctrl *ctrl) {
    __shared__ unsigned long long s[kT / 64];
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    unsigned long long c =
        (v < g.n && slices_ok(P.st[0].slice, (int32_t)v, P) && label_ok(g, P.st[0].label, (int32_t)v)) ? 1 : 0;
    c = wave_sum_u64(c);
    if (__lane_id() == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < kT / 64; ++q) t += s[q];
        if (t) atomicAdd(&ctrl->level[0], t);
    }
}

// degree of each root of a strided slice (ranks s, s + S, ...)
__global__ __launch_bounds__(kT) void k_l2_degrees(const int64_t *__restrict__ rp, int64_t roots, uint32_t S,
                                                   uint32_t s, int32_t *deg) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= roots) return;
    const int64_t r = (int64_t)s + j * (int64_t)S;
    deg[j] = (int32_t)(rp[r + 1] - rp[r]);
}

// entry i of the gathered level 2: root j holding it (largest j with off[j] <= i,
// which skips roots without entries) and its offset in j's list
__global__ __launch_bounds__(kT) void k_l2_fill(const int64_t *__restrict__ rp, int64_t roots, uint32_t S, uint32_t s,
                                                const int64_t *__restrict__ off, int64_t cap, int64_t *idx) {
    const int64_t total = min(off[roots], cap);
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < total; i += (int64_t)gridDim.x * kT) {
        const int64_t j = find_row(off, 0, roots - 1, i);
        idx[i] = rp[(int64_t)s + j * (int64_t)S] + (i - off[j]);
    }
}

template <int W>
void prepare_w(bool last, const GraphDev &g, const DevPlan &P, const int32_t *rows, int64_t row0, int64_t nrows,
               const SegBufs &s, Ctrl *ctrl, hipStream_t st) {
    dim3 grid((unsigned)((nrows + kT - 1) / kT));
    if (last)
        hipLaunchKernelGGL((k_prepare<W, true>), grid, dim3(kT), 0, st, rows, row0, nrows, g, P, s, ctrl);
    else
        hipLaunchKernelGGL((k_prepare<W, false>), grid, dim3(kT), 0, st, rows, row0, nrows, g, P, s, ctrl);
}

template <int W, int MODE, int RUN, bool BLK>
__global__ __launch_bounds__(kT) void k_extend_merge(ExtArgs a) {
    merge_tile<W, MODE, RUN, BLK>(a, blockIdx.x);
}

template <int W, int MODE, int RUN, bool BLK>
void merge_launch(const ExtArgs &a, hipStream_t st) {
    const int64_t items = a.w1 - a.w0;
    dim3 grid((unsigned)((items + (int64_t)kT * RUN - 1) / ((int64_t)kT * RUN)));
    hipLaunchKernelGGL((k_extend_merge<W, MODE, RUN, BLK>), grid, dim3(kT), 0, st, a);
}

template <int W, int RUN, bool BLK = false>
void merge_mode(int mode, const ExtArgs &a, hipStream_t st) {
    if (mode == MODE_COUNT)
        merge_launch<W, MODE_COUNT, RUN, BLK>(a, st);
    else if (mode == MODE_COUNT_NOHASH)
        merge_launch<W, MODE_COUNT_NOHASH, RUN, BLK>(a, st);
    else if (mode == MODE_EMIT)
        merge_launch<W, MODE_EMIT, (RUN > 16 ? 16 : RUN), BLK>(a, st);
    else
        merge_launch<W, MODE_OUTPUT, (RUN > 16 ? 16 : RUN), BLK>(a, st);
}

template <int W, int STRAT>
void extend_ws(int mode, const ExtArgs &a, hipStream_t st) {
    const int64_t items = a.w1 - a.w0;
    dim3 grid((unsigned)((items + kTile - 1) / kTile));
    if (mode == MODE_COUNT)
        hipLaunchKernelGGL((k_extend<W, MODE_COUNT, STRAT>), grid, dim3(kT), 0, st, a);
    else if (mode == MODE_COUNT_NOHASH)
        hipLaunchKernelGGL((k_extend<W, MODE_COUNT_NOHASH, STRAT>), grid, dim3(kT), 0, st, a);
    else if (mode == MODE_EMIT)
        hipLaunchKernelGGL((k_extend<W, MODE_EMIT, STRAT>), grid, dim3(kT), 0, st, a);
    else
        hipLaunchKernelGGL((k_extend<W, MODE_OUTPUT, STRAT>), grid, dim3(kT), 0, st, a);
}

template <int W>
void extend_w(int mode, int strategy, const ExtArgs &a, hipStream_t st) {
    switch (strategy) {
        case STRAT_BSEARCH: extend_ws<W, STRAT_BSEARCH>(mode, a, st); break;
        case STRAT_WAVE_STAGED: extend_ws<W, STRAT_WAVE_STAGED>(mode, a, st); break;
        case STRAT_MERGE_SHORT: merge_mode<W, 4>(mode, a, st); break;
        case STRAT_MERGE_LONG: merge_mode<W, 64>(mode, a, st); break;
        case STRAT_BLOCK_MERGE: merge_mode<W, 16, true>(mode, a, st); break;
        case STRAT_BLOCK_MERGE_LONG: merge_mode<W, 64, true>(mode, a, st); break;
        default: merge_mode<W, 16>(mode, a, st); break;
    }
}

// ---------------------------------------------------------------------------
// device-driven rounds: one scheduler thread takes Algorithm 5's next step
// (a segment to prepare, or a range of work items to extend), and fixed-grid
// prepare / scan / extend launches of every level read it and stay idle
// unless it is theirs.  The same round can then be replayed from a graph.
// ---------------------------------------------------------------------------
constexpr int64_t kRoundMaxItems = 1ll << 30;
constexpr unsigned kRoundGrid = 4096;  // workgroups of a round's prepare and partition launches (grid-stride)

__global__ void k_round_sched(GState *gs, GConst c, Ctrl *ctrl) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    round_sched_step(*gs, c, ctrl->qcount, kRoundMaxItems);
}

template <int W, bool LAST>
__global__ __launch_bounds__(kT) void k_round_prepare(const int32_t *__restrict__ rows, const GState *gs, GraphDev g,
                                                      DevPlan P, SegBufs s, Ctrl *ctrl) {
    const int64_t n = gs->n_prep[W];
    if (n <= 0) return;
    const int64_t row0 = gs->lv[W].seg_row0;
    for (int64_t b = (int64_t)blockIdx.x * kT; b < n; b += (int64_t)gridDim.x * kT) {
        prepare_row<W, LAST>(rows, row0, n, g, P, s, ctrl, b + threadIdx.x);
        __syncthreads();
    }
}

// This round's work items of level W, restricted to bucket c (c < 0: all).
template <int W>
__device__ __forceinline__ bool round_range(const GState *gs, int c, int64_t &w0, int64_t &w1) {
    w0 = gs->ext_w0[W];
    w1 = gs->ext_w1[W];
    if (c >= 0) {
        w0 = max(w0, gs->bw[W][c]);
        w1 = min(w1, gs->bw[W][c + 1]);
    }
    return w1 > w0;
}

template <int W, int MODE, int RUN, bool BLK>
__global__ __launch_bounds__(kT) void k_round_extend(ExtArgs a, GState *gs, int c) {
    int64_t w0, w1;
    if (!round_range<W>(gs, c, w0, w1)) return;
    a.row0 = gs->lv[W].seg_row0;
    a.nrows = gs->lv[W].seg_n;
    a.w0 = w0;
    a.w1 = w1;
    const int64_t tiles = (w1 - w0 + (int64_t)kT * RUN - 1) / ((int64_t)kT * RUN);
    for (int64_t t; (t = claim_tile(&gs->tile_next[W][c + 1], tiles)) >= 0;) {
        merge_tile<W, MODE, RUN, BLK>(a, t);
        __syncthreads();
    }
}

template <int W, int MODE, int STRAT>
__global__ __launch_bounds__(kT) void k_round_extend_ws(ExtArgs a, GState *gs, int c) {
    int64_t w0, w1;
    if (!round_range<W>(gs, c, w0, w1)) return;
    a.row0 = gs->lv[W].seg_row0;
    a.nrows = gs->lv[W].seg_n;
    a.w0 = w0;
    a.w1 = w1;
    const int64_t tiles = (w1 - w0 + kTile - 1) / kTile;
    for (int64_t t; (t = claim_tile(&gs->tile_next[W][c + 1], tiles)) >= 0;) {
        extend_tile<W, MODE, STRAT>(a, t);
        __syncthreads();
    }
}

// Workgroups of kernel f that fit on the device at once: the grid of a
// round's extend launches (each claims tiles until none is left).
template <typename F>
unsigned resident_grid(F f) {
    int dev = 0, cus = 0, per = 0;
    HUGE_HIP(hipGetDevice(&dev));
    HUGE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HUGE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kT, 0));
    return (unsigned)std::max(1, cus * std::max(1, per));
}

template <typename F>
void round_launch(F f, const ExtArgs &a, GState *gs, int c, hipStream_t st) {
    hipLaunchKernelGGL(f, dim3(resident_grid(f)), dim3(kT), 0, st, a, gs, c);
}

template <int W, int RUN, bool BLK>
void round_extend_mode(int mode, const ExtArgs &a, GState *gs, int c, hipStream_t st) {
    if (mode == MODE_COUNT)
        round_launch(k_round_extend<W, MODE_COUNT, RUN, BLK>, a, gs, c, st);
    else if (mode == MODE_COUNT_NOHASH)
        round_launch(k_round_extend<W, MODE_COUNT_NOHASH, RUN, BLK>, a, gs, c, st);
    else
        round_launch(k_round_extend<W, MODE_EMIT, (RUN > 16 ? 16 : RUN), BLK>, a, gs, c, st);
}

template <int W, int STRAT>
void round_extend_ws(int mode, const ExtArgs &a, GState *gs, int c, hipStream_t st) {
    if (mode == MODE_COUNT)
        round_launch(k_round_extend_ws<W, MODE_COUNT, STRAT>, a, gs, c, st);
    else if (mode == MODE_COUNT_NOHASH)
        round_launch(k_round_extend_ws<W, MODE_COUNT_NOHASH, STRAT>, a, gs, c, st);
    else
        round_launch(k_round_extend_ws<W, MODE_EMIT, STRAT>, a, gs, c, st);
}

template <int W>
void round_extend_w(int mode, int strategy, const ExtArgs &a, GState *gs, int c, hipStream_t st) {
    switch (strategy) {
        case STRAT_BSEARCH: round_extend_ws<W, STRAT_BSEARCH>(mode, a, gs, c, st); break;
        case STRAT_WAVE_STAGED: round_extend_ws<W, STRAT_WAVE_STAGED>(mode, a, gs, c, st); break;
        case STRAT_MERGE_SHORT: round_extend_mode<W, 4, false>(mode, a, gs, c, st); break;
        case STRAT_MERGE_LONG: round_extend_mode<W, 64, false>(mode, a, gs, c, st); break;
        case STRAT_BLOCK_MERGE: round_extend_mode<W, 16, true>(mode, a, gs, c, st); break;
        case STRAT_BLOCK_MERGE_LONG: round_extend_mode<W, 64, true>(mode, a, gs, c, st); break;
        default: round_extend_mode<W, 16, false>(mode, a, gs, c, st); break;
    }
}

// ---------------------------------------------------------------------------
// probe-length buckets: a stable counting partition of a prepared segment by
// the bucket of each row's probe length, so that every bucket's work items
// are contiguous and can run with their own strategy
// ---------------------------------------------------------------------------
__device__ __forceinline__ int probe_bucket(int32_t len) {
    return len < (1 << 6) ? 0 : len < (1 << 9) ? 1 : len < (1 << 12) ? 2 : len < (1 << 15) ? 3 : 4;
}

// bcnt[c * nblk + b] = rows of bucket c in block b
__device__ __forceinline__ void bucket_count_block(const int32_t *bound, int64_t n, int32_t *bcnt, int64_t nblk,
                                                   int64_t b) {
    __shared__ int32_t s_c[kT / 64][HUGE_TUNE_BUCKETS];
    const int64_t i = b * kT + threadIdx.x;
    const int c = i < n ? probe_bucket(bound[i]) : -1;
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < HUGE_TUNE_BUCKETS; ++q) {
        const uint64_t m = __ballot(c == q);
        if (__lane_id() == 0) s_c[wv][q] = (int32_t)__popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < HUGE_TUNE_BUCKETS) {
        int32_t t = 0;
        for (int q = 0; q < kT / 64; ++q) t += s_c[q][threadIdx.x];
        bcnt[(int64_t)threadIdx.x * nblk + b] = t;
    }
}
__global__ __launch_bounds__(kT) void k_bucket_count(const int32_t *bound, int64_t n, int32_t *bcnt, int64_t nblk) {
    bucket_count_block(bound, n, bcnt, nblk, blockIdx.x);
}

// Moves row i's prepared data to its stable position in bucket order.
__device__ __forceinline__ void bucket_scatter_block(const int32_t *bound_in, const uint64_t *pinfo_in,
                                                     const uint64_t *hpre_in, int64_t n, int64_t nblk,
                                                     const int64_t *bscan, int32_t *bound, uint64_t *pinfo,
                                                     uint64_t *hpre, int32_t *rid, int64_t blk) {
    __shared__ int32_t s_c[kT / 64][HUGE_TUNE_BUCKETS];
    const int64_t i = blk * kT + threadIdx.x;
    const int32_t b = i < n ? bound_in[i] : 0;
    const int c = i < n ? probe_bucket(b) : -1;
    const int wv = threadIdx.x >> 6, lane = __lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int rank = 0;
#pragma unroll
    for (int q = 0; q < HUGE_TUNE_BUCKETS; ++q) {
        const uint64_t m = __ballot(c == q);
        if (lane == 0) s_c[wv][q] = (int32_t)__popcll(m);
        if (c == q) rank = (int)__popcll(m & lt);
    }
    __syncthreads();
    if (i < n) {
        int64_t pos = bscan[(int64_t)c * nblk + blk] + rank;
        for (int q = 0; q < wv; ++q) pos += s_c[q][c];
        bound[pos] = b;
        pinfo[pos] = pinfo_in[i];
        if (hpre_in) hpre[pos] = hpre_in[i];
        rid[pos] = (int32_t)i;
    }
}
__global__ __launch_bounds__(kT) void k_bucket_scatter(const int32_t *bound_in, const uint64_t *pinfo_in,
                                                       const uint64_t *hpre_in, int64_t n, int64_t nblk,
                                                       const int64_t *bscan, int32_t *bound, uint64_t *pinfo,
                                                       uint64_t *hpre, int32_t *rid) {
    bucket_scatter_block(bound_in, pinfo_in, hpre_in, n, nblk, bscan, bound, pinfo, hpre, rid, blockIdx.x);
}

// The partition with the row count read from device memory (graph engine):
// fixed grids, blocks past the count idle; gs->n_part[W] receives the length
// of the per-block counts so that the device-count scan can take them.
template <int W>
__global__ __launch_bounds__(kT) void k_round_bucket_count(const int32_t *bound, GState *gs, int32_t *bcnt) {
    const int64_t n = gs->n_prep[W];
    const int64_t nblk = (n + kT - 1) / kT;
    if (blockIdx.x == 0 && threadIdx.x == 0) gs->n_part[W] = HUGE_TUNE_BUCKETS * nblk;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        bucket_count_block(bound, n, bcnt, nblk, b);
        __syncthreads();
    }
}

template <int W>
__global__ __launch_bounds__(kT) void k_round_bucket_scatter(const GState *gs, SegBufs s, bool last) {
    const int64_t n = gs->n_prep[W];
    const int64_t nblk = (n + kT - 1) / kT;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        bucket_scatter_block(s.bound_in, s.pinfo_in, last ? s.hpre_in : nullptr, n, nblk, s.bscan, s.bound,
                             s.pinfo, s.hpre, s.rid, b);
        __syncthreads();
    }
}

// gs->bw[W][c] = first work item of bucket c, bw[W][B] = total
template <int W>
__global__ void k_round_bucket_bounds(GState *gs, const int64_t *bscan, const int64_t *off) {
    const int64_t n = gs->n_prep[W];
    if (n <= 0) return;
    const int64_t nblk = (n + kT - 1) / kT;
    const int t = threadIdx.x;
    if (t <= HUGE_TUNE_BUCKETS) gs->bw[W][t] = off[t < HUGE_TUNE_BUCKETS ? bscan[(int64_t)t * nblk] : n];
}

// out[c] = first work item of bucket c (c = 0..B-1), out[B] = total
__global__ void k_bucket_bounds(const int64_t *bscan, int64_t nblk, int64_t n, const int64_t *off, long long *out) {
    const int t = threadIdx.x;
    if (t <= HUGE_TUNE_BUCKETS) out[t] = off[t < HUGE_TUNE_BUCKETS ? bscan[(int64_t)t * nblk] : n];
}

}  // namespace

void launch_prepare(int width, bool last, const GraphDev &g, const DevPlan &P, const int32_t *rows, int64_t row0,
                    int64_t nrows, const SegBufs &s, Ctrl *ctrl, hipStream_t st) {
    if (nrows <= 0) return;
    switch (width) {
        case 2: prepare_w<2>(last, g, P, rows, row0, nrows, s, ctrl, st); break;
        case 3: prepare_w<3>(last, g, P, rows, row0, nrows, s, ctrl, st); break;
        case 4: prepare_w<4>(last, g, P, rows, row0, nrows, s, ctrl, st); break;
        case 5: prepare_w<5>(last, g, P, rows, row0, nrows, s, ctrl, st); break;
        case 6: prepare_w<6>(last, g, P, rows, row0, nrows, s, ctrl, st); break;
        case 7: prepare_w<7>(last, g, P, rows, row0, nrows, s, ctrl, st); break;
        default: HUGE_FAIL(HUGE_EINVAL, "bad width %d", width);
    }
    HUGE_HIP(hipGetLastError());
}

void launch_scan_bounds(const SegBufs &s, int64_t nrows, int64_t *tmp, hipStream_t st) {
    scan_excl(s.bound, s.off, nrows, s.off + nrows, tmp, st);
    HUGE_HIP(hipGetLastError());
}

void launch_extend(int width, int mode, int strategy, const GraphDev &g, const DevPlan &P, const int32_t *rows,
                   int64_t row0, const SegBufs &s, int64_t nrows, int64_t w0, int64_t w1, int32_t *out_rows,
                   Ctrl *ctrl, const int32_t *inv_rank, hipStream_t st, bool partitioned) {
    if (w1 <= w0) return;
    ExtArgs a;
    a.rows = rows;
    a.row0 = row0;
    a.rid = partitioned ? s.rid : nullptr;
    a.off = s.off;
    a.pinfo = s.pinfo;
    a.hpre = s.hpre;
    a.nrows = nrows;
    a.w0 = w0;
    a.w1 = w1;
    a.out = out_rows;
    a.ctrl = ctrl;
    a.inv_rank = inv_rank;
    a.g = g;
    a.P = P;
    switch (width) {
        case 2: extend_w<2>(mode, strategy, a, st); break;
        case 3: extend_w<3>(mode, strategy, a, st); break;
        case 4: extend_w<4>(mode, strategy, a, st); break;
        case 5: extend_w<5>(mode, strategy, a, st); break;
        case 6: extend_w<6>(mode, strategy, a, st); break;
        case 7: extend_w<7>(mode, strategy, a, st); break;
        default: HUGE_FAIL(HUGE_EINVAL, "bad width %d", width);
    }
    HUGE_HIP(hipGetLastError());
}

void launch_bucket_partition(const SegBufs &s, int64_t nrows, bool last, int64_t *scan_tmp, Ctrl *ctrl,
                             hipStream_t st) {
    if (nrows <= 0) return;
    const int64_t nblk = (nrows + kT - 1) / kT;
    hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)nblk), dim3(kT), 0, st, s.bound_in, nrows, s.bcnt, nblk);
    scan_excl(s.bcnt, s.bscan, HUGE_TUNE_BUCKETS * nblk, s.bscan + HUGE_TUNE_BUCKETS * nblk, scan_tmp, st);
    hipLaunchKernelGGL(k_bucket_scatter, dim3((unsigned)nblk), dim3(kT), 0, st, s.bound_in, s.pinfo_in,
                       last ? s.hpre_in : (const uint64_t *)nullptr, nrows, nblk, s.bscan, s.bound, s.pinfo, s.hpre,
                       s.rid);
    HUGE_HIP(hipGetLastError());
    (void)ctrl;
}

void launch_bucket_bounds(const SegBufs &s, int64_t nrows, Ctrl *ctrl, hipStream_t st) {
    const int64_t nblk = (nrows + kT - 1) / kT;
    hipLaunchKernelGGL(k_bucket_bounds, dim3(1), dim3(64), 0, st, s.bscan, nblk, nrows, s.off, ctrl->scratch);
    HUGE_HIP(hipGetLastError());
}

void launch_edge_sink(const GraphDev &g, const DevPlan &P, int64_t e0, int64_t e1, int mode, int32_t *out,
                      const int32_t *inv_rank, Ctrl *ctrl, hipStream_t st) {
    if (e1 <= e0) return;
    dim3 grid((unsigned)((e1 - e0 + kT - 1) / kT));
    hipLaunchKernelGGL(k_edge_sink, grid, dim3(kT), 0, st, g, P, e0, e1, mode, out, inv_rank, ctrl);
    HUGE_HIP(hipGetLastError());
}

void launch_gather_level2(const GraphDev &g, const DevPlan &P, int64_t roots, int32_t *deg, int64_t *off,
                          int64_t *idx, int64_t cap, int64_t *scan_tmp, hipStream_t st) {
    if (roots <= 0) {
        HUGE_HIP(hipMemsetAsync(off, 0, sizeof(int64_t), st));
        return;
    }
    hipLaunchKernelGGL(k_l2_degrees, dim3((unsigned)((roots + kT - 1) / kT)), dim3(kT), 0, st, g.rp, roots,
                       P.slice_count, P.slice_id, deg);
    scan_excl(deg, off, roots, off + roots, scan_tmp, st);
    const int64_t blocks = std::min<int64_t>((cap + kT - 1) / kT, 1 << 16);
    hipLaunchKernelGGL(k_l2_fill, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(kT), 0, st, g.rp, roots,
                       P.slice_count, P.slice_id, (const int64_t *)off, cap, idx);
    HUGE_HIP(hipGetLastError());
}

void launch_root_count(const GraphDev &g, const DevPlan &P, Ctrl *ctrl, hipStream_t st) {
    dim3 grid((unsigned)((g.n + kT - 1) / kT));
    hipLaunchKernelGGL(k_root_count, grid, dim3(kT), 0, st, g, P, ctrl);
    HUGE_HIP(hipGetLastError());
}

void launch_round_sched(GState *s, const GConst &c, Ctrl *ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_round_sched, dim3(1), dim3(64), 0, st, s, c, ctrl);
    HUGE_HIP(hipGetLastError());
}

void launch_round_prepare(int width, bool last, const GraphDev &g, const DevPlan &P, const int32_t *rows,
                          const SegBufs &s, Ctrl *ctrl, GState *gs, int64_t seg_cap, hipStream_t st) {
    const dim3 grid((unsigned)std::min<int64_t>((seg_cap + kT - 1) / kT, kRoundGrid)), blk(kT);
    switch (width * 2 + (last ? 1 : 0)) {
#define HUGE_ROUND_PREP(W)                                                                                  \
    case 2 * W: hipLaunchKernelGGL((k_round_prepare<W, false>), grid, blk, 0, st, rows, gs, g, P, s, ctrl); break; \
    case 2 * W + 1: hipLaunchKernelGGL((k_round_prepare<W, true>), grid, blk, 0, st, rows, gs, g, P, s, ctrl); break;
        HUGE_ROUND_PREP(2)
        HUGE_ROUND_PREP(3)
        HUGE_ROUND_PREP(4)
        HUGE_ROUND_PREP(5)
        HUGE_ROUND_PREP(6)
        HUGE_ROUND_PREP(7)
#undef HUGE_ROUND_PREP
        default: HUGE_FAIL(HUGE_EINVAL, "bad width %d", width);
    }
    HUGE_HIP(hipGetLastError());
}

void launch_round_scan(int width, const SegBufs &s, GState *gs, int64_t seg_cap, int64_t *tmp, hipStream_t st) {
    scan_excl_devn(s.bound, s.off, &gs->n_prep[width], seg_cap, tmp, st);
    HUGE_HIP(hipGetLastError());
}

void launch_round_partition(int width, bool last, const SegBufs &s, GState *gs, int64_t seg_cap, int64_t *tmp,
                            hipStream_t st) {
    const int64_t nblk_max = (seg_cap + kT - 1) / kT;
    const dim3 grid((unsigned)std::min<int64_t>(nblk_max, kRoundGrid)), blk(kT);
    switch (width) {
#define HUGE_ROUND_PART(W)                                                                                     \
    case W:                                                                                                    \
        hipLaunchKernelGGL(k_round_bucket_count<W>, grid, blk, 0, st, (const int32_t *)s.bound_in, gs, s.bcnt); \
        scan_excl_devn(s.bcnt, s.bscan, &gs->n_part[W], HUGE_TUNE_BUCKETS * nblk_max, tmp, st);                \
        hipLaunchKernelGGL(k_round_bucket_scatter<W>, grid, blk, 0, st, (const GState *)gs, s, last);           \
        break;
        HUGE_ROUND_PART(2)
        HUGE_ROUND_PART(3)
        HUGE_ROUND_PART(4)
        HUGE_ROUND_PART(5)
        HUGE_ROUND_PART(6)
        HUGE_ROUND_PART(7)
#undef HUGE_ROUND_PART
        default: HUGE_FAIL(HUGE_EINVAL, "bad width %d", width);
    }
    HUGE_HIP(hipGetLastError());
}

void launch_round_bucket_bounds(int width, const SegBufs &s, GState *gs, hipStream_t st) {
    switch (width) {
        case 2: hipLaunchKernelGGL(k_round_bucket_bounds<2>, dim3(1), dim3(64), 0, st, gs, (const int64_t *)s.bscan, (const int64_t *)s.off); break;
        case 3: hipLaunchKernelGGL(k_round_bucket_bounds<3>, dim3(1), dim3(64), 0, st, gs, (const int64_t *)s.bscan, (const int64_t *)s.off); break;
        case 4: hipLaunchKernelGGL(k_round_bucket_bounds<4>, dim3(1), dim3(64), 0, st, gs, (const int64_t *)s.bscan, (const int64_t *)s.off); break;
        case 5: hipLaunchKernelGGL(k_round_bucket_bounds<5>, dim3(1), dim3(64), 0, st, gs, (const int64_t *)s.bscan, (const int64_t *)s.off); break;
        case 6: hipLaunchKernelGGL(k_round_bucket_bounds<6>, dim3(1), dim3(64), 0, st, gs, (const int64_t *)s.bscan, (const int64_t *)s.off); break;
        case 7: hipLaunchKernelGGL(k_round_bucket_bounds<7>, dim3(1), dim3(64), 0, st, gs, (const int64_t *)s.bscan, (const int64_t *)s.off); break;
        default: HUGE_FAIL(HUGE_EINVAL, "bad width %d", width);
    }
    HUGE_HIP(hipGetLastError());
}

void launch_round_extend(int width, int mode, int strategy, const GraphDev &g, const DevPlan &P, const int32_t *rows,
                         const SegBufs &s, int32_t *out_rows, Ctrl *ctrl, const int32_t *inv_rank, GState *gs,
                         int bucket, hipStream_t st) {
    ExtArgs a;
    a.rows = rows;
    a.row0 = 0;
    a.rid = bucket >= 0 ? s.rid : nullptr;
    a.off = s.off;
    a.pinfo = s.pinfo;
    a.hpre = s.hpre;
    a.nrows = 0;
    a.w0 = a.w1 = 0;
    a.out = out_rows;
    a.ctrl = ctrl;
    a.inv_rank = inv_rank;
    a.g = g;
    a.P = P;
    switch (width) {
        case 2: round_extend_w<2>(mode, strategy, a, gs, bucket, st); break;
        case 3: round_extend_w<3>(mode, strategy, a, gs, bucket, st); break;
        case 4: round_extend_w<4>(mode, strategy, a, gs, bucket, st); break;
        case 5: round_extend_w<5>(mode, strategy, a, gs, bucket, st); break;
        case 6: round_extend_w<6>(mode, strategy, a, gs, bucket, st); break;
        case 7: round_extend_w<7>(mode, strategy, a, gs, bucket, st); break;
        default: HUGE_FAIL(HUGE_EINVAL, "bad width %d", width);
    }
    HUGE_HIP(hipGetLastError());
}

}  // namespace huge
