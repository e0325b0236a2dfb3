// Persistent engine: one launch of resident workgroups (WGs) runs the whole
// query, or a batch of queries.
//
// Each WG executes Algorithm 5 (DFS/BFS-adaptive scheduling, Section 5.2) on
// its own: every materialised level W (3..k-1) has a private fixed-capacity
// buffer, the WG keeps extending the current chunk of level W into level W+1
// while W+1 has room for a full tile, descends as soon as W+1 holds rows, and
// backtracks when a level is drained.  Level-2 rows (edges) are handed out in
// chunks from one global cursor per query.  The memory of intermediate
// results is bounded by (number of WGs) x (sum of level capacities), and a
// tile never emits more rows than the free space it checked for.
//
// Load balancing is the intra-machine work stealing of Section 5.3, at two
// granularities:
//   * rows: a level buffer is a deque; its owner pops chunks from the back
//     (tail) and pushes new rows at the back, and an idle WG steals half of
//     the rows from the front (head) of the shallowest non-empty level of a
//     victim.  The deque word packs head (24 bits), tail (24 bits) and the
//     query index (16 bits), so a steal CAS fails if the victim has moved to
//     another query.  A thief announces itself in the victim's per-level
//     pending counter while it copies, and the owner only rewinds an empty
//     deque to row 0 when no thief is copying.
//   * tiles: the last level does almost all the work, and one chunk of hub
//     rows can hold millions of candidates.  Its owner publishes the prepared
//     chunk on a board (global memory) and idle WGs claim 4096-candidate tiles
//     of it through one atomic word (generation | tiles | next); the owner
//     reuses the chunk's rows only after every claimed tile reports done.
//
// Termination: a global count of WGs that may hold work.  A WG enters the
// count when it starts and leaves it only when every query cursor is
// exhausted and its own levels are empty; a thief re-enters the count before
// it tries to steal.  The count is zero only when no started WG holds rows,
// and a WG that starts later finds the cursors exhausted and nothing to
// steal, so no WG waits on one that is not resident.  Every wait loop is
// bounded by a wall-clock deadline; passing it sets an error flag and the WG
// exits.
//
// Queries of 3 or 4 vertices only: the level buffers then hold rows of width
// 3, and the kernel keeps every row in registers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "devfuncs.h"
#include "internal.h"

namespace huge {
namespace {

using namespace dev;

constexpr int kT = 256;
constexpr int kR = 256;             // rows per chunk
constexpr int kPRun = 16;           // consecutive work items per lane in a tile
constexpr int kPTile = kT * kPRun;  // work items per tile (= most rows a tile emits)
constexpr int kLv = HUGE_KMAX;      // level index = row width W
constexpr int kResStride = 16;      // per query: count, hash_sum, hash_xor, pad, level[8], pad

struct Board {
    unsigned long long word;  // generation:16 | tiles:24 | next claim:24
    unsigned long long done;  // tiles finished in the current generation
    int32_t plan, W, nrows, pad;
    int64_t row0, total;
    int64_t off[kR + 1];
    uint64_t pinfo[kR];
    uint64_t hpre[kR];
};

struct PersistArgs {
    GraphDev g;
    const DevPlan *plans;
    int nplans;
    int steal;
    int32_t *bufs;               // per-WG level buffers
    int64_t wg_ints;             // int32 entries per WG region
    int64_t lvl_off[kLv];        // offset of level W inside a WG region
    int32_t cap[kLv];            // row capacity of level W
    unsigned long long *deq;     // [nwg][kLv]
    int *pending;                // [nwg][kLv]
    Board *boards;               // [nwg]
    unsigned long long *cursor;  // [nplans] next level-2 edge
    unsigned long long *res;     // [nplans][kResStride]
    int *busy;
    int *err;
    unsigned long long *stats;   // [0] row steals, [1] stolen rows, [2] sum of per-WG peak bytes, [3] helped tiles
    unsigned long long *wg_busy; // [nwg] wall-clock ticks each WG spent in tiles and prepare passes
    uint64_t limit_ticks;        // longest wait, in wall-clock ticks
};

// deque word: head | tail << 24 | plan << 48
__device__ __forceinline__ uint32_t dq_head(unsigned long long x) { return (uint32_t)(x & 0xFFFFFFull); }
__device__ __forceinline__ uint32_t dq_tail(unsigned long long x) { return (uint32_t)((x >> 24) & 0xFFFFFFull); }
__device__ __forceinline__ int dq_plan(unsigned long long x) { return (int)(x >> 48); }
__device__ __forceinline__ unsigned long long dq_make(uint32_t h, uint32_t t, int plan) {
    return (unsigned long long)h | ((unsigned long long)t << 24) | ((unsigned long long)plan << 48);
}
// board word: next | tiles << 24 | gen << 48 (same field layout)
__device__ __forceinline__ uint32_t bw_next(unsigned long long x) { return (uint32_t)(x & 0xFFFFFFull); }
__device__ __forceinline__ uint32_t bw_tiles(unsigned long long x) { return (uint32_t)((x >> 24) & 0xFFFFFFull); }
__device__ __forceinline__ uint32_t bw_gen(unsigned long long x) { return (uint32_t)(x >> 48); }

__device__ __forceinline__ unsigned long long ld_acq(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_acq_i(int *p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ bool past(uint64_t deadline) { return wall_clock64() > deadline; }

struct LvState {
    int64_t row0;   // chunk's first row (buffer row, or edge index at W = 2)
    int32_t nrows;  // rows in the chunk
    int32_t pad;
    int64_t total;  // work items of the chunk
    int64_t done;   // work items processed
};

struct Shared {
    LvState lv[kLv];
    int64_t off[kLv][kR + 1];
    uint64_t pinfo[kLv][kR];
    uint64_t hpre[kR];
    int64_t scan_ws[kT / 64];
    unsigned long long red[3][kT / 64];
    int plan;
    int k;
    int W;
    int action;
    int emitted;
    int32_t tail_base;
    int victim;
    int vlevel;
    uint32_t vhead, vcount;
    int32_t tile;
    uint32_t gen;
    unsigned long long peak_bytes;
};

// The rows, scan and probe data of one prepared chunk, in LDS (owner) or on
// a board in global memory (helpers).
struct ChunkView {
    const int32_t *rows;
    int64_t row0;
    int32_t nrows;
    const int64_t *off;
    const uint64_t *pinfo;
    const uint64_t *hpre;
};

__device__ __forceinline__ int64_t block_excl_scan64(int64_t x, Shared &sh, int64_t &total) {
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    int64_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) sh.scan_ws[w] = inc;
    __syncthreads();
    int64_t base = 0;
    total = 0;
#pragma unroll
    for (int q = 0; q < kT / 64; ++q) {
        if (q < w) base += sh.scan_ws[q];
        total += sh.scan_ws[q];
    }
    __syncthreads();
    return base + inc - x;
}

__device__ __forceinline__ int32_t *level_buf(const PersistArgs &a, int wg, int W) {
    return a.bufs + (int64_t)wg * a.wg_ints + a.lvl_off[W];
}

// Fold the lanes' count and hash into query `plan` (block-uniform call).
__device__ void flush_counts(const PersistArgs &a, Shared &sh, int plan, int k, unsigned long long &cnt,
                             unsigned long long &hs, unsigned long long &hx) {
    const int t = threadIdx.x;
    const unsigned long long c = wave_sum_u64(cnt), s = wave_sum_u64(hs), x = wave_xor_u64(hx);
    if (__lane_id() == 0) {
        sh.red[0][t >> 6] = c;
        sh.red[1][t >> 6] = s;
        sh.red[2][t >> 6] = x;
    }
    __syncthreads();
    if (t == 0 && plan >= 0) {
        unsigned long long C = 0, S = 0, X = 0;
        for (int q = 0; q < kT / 64; ++q) {
            C += sh.red[0][q];
            S += sh.red[1][q];
            X ^= sh.red[2][q];
        }
        if (C) {
            unsigned long long *r = a.res + plan * kResStride;
            atomicAdd(&r[0], C);
            atomicAdd(&r[1], S);
            atomicXor(&r[2], X);
            atomicAdd(&r[4 + k - 1], C);
        }
    }
    cnt = hs = hx = 0;
    __syncthreads();
}

// Prepare the chunk of level W held in sh.lv[W]: per row, the symmetry-
// breaking window, the shortest trimmed Ext list (probe), its length (bound)
// and the row's prefix hash; then the exclusive scan of the bounds.
template <int W>
__device__ void prepare_chunk(const PersistArgs &a, const DevPlan &P, bool last, Shared &sh) {
    const GraphDev &g = a.g;
    LvState &L = sh.lv[W];
    const int t = threadIdx.x;
    int64_t bound = 0;
    uint64_t pinfo = 0;
    bool valid = false;
    if (t < L.nrows) {
        int32_t f[W];
        load_row<W>(level_buf(a, blockIdx.x, W), g, L.row0 + t, f);
        valid = true;
        if constexpr (W == 2) valid = level2_ok(f, P, g);
        if (valid) {
            const DevStep &st = P.st[W];
            int32_t lo = 0, hi = 0x7FFFFFFF;
#pragma unroll
            for (int p = 0; p < W; ++p) {
                if ((st.lo >> p) & 1u) lo = max(lo, f[p] + 1);
                if ((st.hi >> p) & 1u) hi = min(hi, f[p]);
            }
            if (lo < hi) {
                int64_t best = -1, bb = 0;
                int bp = 0;
#pragma unroll
                for (int p = 0; p < W; ++p) {
                    if ((st.ext >> p) & 1u) {
                        const int32_t x = f[p];
                        const int64_t b = g.rp[x], e = g.rp[x + 1];
                        const int64_t s0 = lo > 0 ? lower_bound(g.col, b, e, lo) : b;
                        const int64_t s1 = hi < 0x7FFFFFFF ? lower_bound(g.col, s0, e, hi) : e;
                        if (best < 0 || s1 - s0 < best) {
                            best = s1 - s0;
                            bb = s0;
                            bp = p;
                        }
                    }
                }
                bound = best;
                pinfo = (uint64_t)bb | ((uint64_t)bp << 56);
            }
        }
        if (last) {
            uint64_t h = 0;
            for (int e = 0; e < P.ne; ++e) {
                const int b = P.eb[e];
                if (b < W) {
                    const int ea = P.ea[e];
                    int32_t fa = 0, fb = 0;
#pragma unroll
                    for (int p = 0; p < W; ++p) {
                        if (p == ea) fa = f[p];
                        if (p == b) fb = f[p];
                    }
                    h += mix64(edge_key(fa, fb));
                }
            }
            sh.hpre[t] = h;
        }
        sh.pinfo[W][t] = pinfo;
    }
    int64_t total;
    const int64_t ex = block_excl_scan64(bound, sh, total);
    if (t < L.nrows) sh.off[W][t] = ex;
    if constexpr (W == 2) {
        // level-2 rows that pass the first constraint and the slice
        int64_t vt;
        (void)block_excl_scan64(valid ? 1 : 0, sh, vt);
        if (t == 0 && vt) atomicAdd(&a.res[sh.plan * kResStride + 4 + 1], (unsigned long long)vt);
    }
    if (t == 0) {
        sh.off[W][L.nrows] = total;
        L.total = total;
        L.done = 0;
    }
    __syncthreads();
}

// One tile of a prepared chunk of level W: work items [w0, w1), each lane a
// run of kPRun consecutive items with galloping cursors (lane merge).  The
// last level folds matches into the lane's count and hash; other levels
// append rows to the WG's level W+1 at sh.tail_base + (LDS counter).
template <int W, bool LAST>
__device__ void run_tile(const PersistArgs &a, const DevPlan &P, const ChunkView &cv, Shared &sh, int64_t w0,
                         int64_t w1, unsigned long long &cnt, unsigned long long &hs, unsigned long long &hx) {
    const GraphDev &g = a.g;
    const DevStep st = P.st[W];
    int32_t *outb = LAST ? nullptr : level_buf(a, blockIdx.x, W + 1);
    const int64_t wb = w0 + (int64_t)threadIdx.x * kPRun;
    const int64_t we = min(wb + (int64_t)kPRun, w1);
    if (wb >= we) return;
    int64_t w = wb;
    int64_t r = find_row(cv.off, 0, cv.nrows - 1, w);
    while (w < we) {
        const int64_t wend = min(cv.off[r + 1], we);
        const uint64_t pi = cv.pinfo[r];
        const int pp = (int)(pi >> 56);
        const int64_t pshift = (int64_t)(pi & kPbMask) - cv.off[r];
        int32_t f[W];
        load_row<W>(cv.rows, g, cv.row0 + r, f);
        const uint64_t hp = LAST ? cv.hpre[r] : 0;
        int64_t cur[W], end[W];
        const int32_t v0 = g.col[pshift + w];
#pragma unroll
        for (int p = 0; p < W; ++p) {
            cur[p] = 0;
            end[p] = 0;
            if (((st.ext >> p) & 1u) && p != pp && f[p] < g.hub_base) {
                end[p] = g.rp[f[p] + 1];
                cur[p] = lower_bound(g.col, g.rp[f[p]], end[p], v0);
            }
        }
        for (; w < wend; ++w) {
            const int32_t v = g.col[pshift + w];
            bool ok = true;
#pragma unroll
            for (int p = 0; p < W; ++p)
                if ((st.neq >> p) & 1u) ok &= (v != f[p]);
            if (st.slice) ok &= slices_ok(st.slice, v, P);
#pragma unroll
            for (int p = 0; p < W; ++p) {
                if (ok && ((st.ext >> p) & 1u) && p != pp) {
                    if (f[p] >= g.hub_base) {
                        ok = adj_has(g, f[p], v);
                    } else {
                        cur[p] = gallop(g.col, cur[p], end[p], v);
                        ok = cur[p] < end[p] && g.col[cur[p]] == v;
                    }
                }
            }
            if (!ok) continue;
            if constexpr (LAST) {
                uint64_t h = hp;
#pragma unroll
                for (int p = 0; p < W; ++p)
                    if ((st.ext >> p) & 1u) h += mix64(edge_key(f[p], v));
                h = mix64(h);
                cnt += 1;
                hs += h;
                hx ^= h;
            } else {
                const int q = atomicAdd(&sh.emitted, 1);
                int32_t *dst = outb + (int64_t)(sh.tail_base + q) * (W + 1);
#pragma unroll
                for (int p = 0; p < W; ++p) dst[p] = f[p];
                dst[W] = v;
            }
        }
        if (w < we) r = find_row(cv.off, r + 1, cv.nrows - 1, w);
    }
}

template <int K>
__device__ void prepare_any(int W, const PersistArgs &a, const DevPlan &P, bool last, Shared &sh) {
    switch (W) {
        case 2: prepare_chunk<2>(a, P, last, sh); break;
        case 3: if constexpr (K > 3) prepare_chunk<3>(a, P, last, sh); break;
        case 4: if constexpr (K > 4) prepare_chunk<4>(a, P, last, sh); break;
        case 5: if constexpr (K > 5) prepare_chunk<5>(a, P, last, sh); break;
        case 6: if constexpr (K > 6) prepare_chunk<6>(a, P, last, sh); break;
        default: if constexpr (K > 7) prepare_chunk<7>(a, P, last, sh); break;
    }
}

template <int K>
__device__ void tile_any(int W, bool last, const PersistArgs &a, const DevPlan &P, const ChunkView &cv, Shared &sh,
                         int64_t w0, int64_t w1, unsigned long long &c, unsigned long long &s, unsigned long long &x) {
#define HUGE_TILE_CASE(WW)                                                      \
    case WW:                                                                    \
        if constexpr (K > WW) {                                                 \
            if (last) run_tile<WW, true>(a, P, cv, sh, w0, w1, c, s, x);        \
            else if constexpr (K > WW + 1) run_tile<WW, false>(a, P, cv, sh, w0, w1, c, s, x); \
        }                                                                       \
        break;
    switch (W) {
        HUGE_TILE_CASE(2)
        HUGE_TILE_CASE(3)
        HUGE_TILE_CASE(4)
        HUGE_TILE_CASE(5)
        HUGE_TILE_CASE(6)
        HUGE_TILE_CASE(7)
        default: break;
    }
#undef HUGE_TILE_CASE
}

// Owner side: publish rows appended at the tail of its level-W deque.
__device__ void dq_push(const PersistArgs &a, int W, uint32_t add) {
    unsigned long long *d = a.deq + (int64_t)blockIdx.x * kLv + W;
    __threadfence();  // rows are visible before the new tail
    for (;;) {
        const unsigned long long o = ld_acq(d);
        const unsigned long long n = dq_make(dq_head(o), dq_tail(o) + add, dq_plan(o));
        if (atomicCAS(d, o, n) == o) break;
    }
}

// Owner side: pop up to kR rows from the tail.  Returns the count (0 = empty).
__device__ int dq_pop(const PersistArgs &a, int W, int64_t &row0) {
    unsigned long long *d = a.deq + (int64_t)blockIdx.x * kLv + W;
    for (;;) {
        const unsigned long long o = ld_acq(d);
        const uint32_t h = dq_head(o), t = dq_tail(o);
        if (t <= h) return 0;
        const uint32_t c = min(t - h, (uint32_t)kR);
        if (atomicCAS(d, o, dq_make(h, t - c, dq_plan(o))) == o) {
            row0 = t - c;
            return (int)c;
        }
    }
}

// Owner side: the append position of its level-W deque for query `plan`.  A
// drained deque is re-tagged with the query and, when no thief is still
// copying out of it, rewound to row 0.
__device__ uint32_t dq_prepare_append(const PersistArgs &a, int W, int plan) {
    unsigned long long *d = a.deq + (int64_t)blockIdx.x * kLv + W;
    int *pend = a.pending + (int64_t)blockIdx.x * kLv + W;
    for (;;) {
        const unsigned long long o = ld_acq(d);
        const uint32_t h = dq_head(o), t = dq_tail(o);
        if (h != t || (t == 0 && dq_plan(o) == plan)) return t;
        const uint32_t pos = ld_acq_i(pend) == 0 ? 0u : t;
        if (atomicCAS(d, o, dq_make(pos, pos, plan)) == o) return pos;
    }
}

// Time thread 0 sees the workgroup spend in a piece of work (a tile or a
// chunk's prepare pass; each ends with a workgroup barrier), for the per-WG
// busy times that show how evenly the load is spread.
#define HUGE_BUSY(...)                                        \
    do {                                                      \
        const uint64_t busy_t0_ = wall_clock64();             \
        __VA_ARGS__;                                          \
        if (t == 0) busy_ticks += wall_clock64() - busy_t0_;  \
    } while (0)

template <int K>
__global__ __launch_bounds__(kT) void k_persist(PersistArgs a) {
    __shared__ Shared sh;
    const int t = threadIdx.x;
    uint64_t busy_ticks = 0;  // thread 0: time spent in tiles and prepare passes
    unsigned long long cnt = 0, hs = 0, hx = 0;  // per lane, for query sh.plan
    const uint64_t deadline = wall_clock64() + a.limit_ticks;
    int counted = 1;  // thread 0 only: this WG is counted in *busy
    Board &myb = a.boards[blockIdx.x];
    if (t == 0) {
        atomicAdd(a.busy, 1);
        sh.plan = -1;
        sh.k = 3;
        sh.peak_bytes = 0;
        sh.W = 2;
        sh.gen = 0;
    }
    __syncthreads();
    // level 0 of a query whose first position holds the sliced vertex: the roots in the slice
    for (int q = 0; q < a.nplans; ++q) {
        const DevPlan &Q = a.plans[q];
        if (Q.slice_count <= 1 || !Q.st[0].slice) continue;
        unsigned long long c = 0;
        for (int64_t v = (int64_t)blockIdx.x * kT + t; v < a.g.n; v += (int64_t)gridDim.x * kT)
            c += in_slice((int32_t)v, Q) ? 1ull : 0ull;
        c = wave_sum_u64(c);
        if (__lane_id() == 0 && c) atomicAdd(&a.res[q * kResStride + 4], c);
    }

    for (;;) {
        // ---- find work: a level-2 chunk of some query
        if (t == 0) {
            sh.action = 0;
            const int start = sh.plan >= 0 ? sh.plan : (int)(blockIdx.x % a.nplans);
            for (int q = 0; q < a.nplans && sh.action == 0; ++q) {
                const int p = (start + q) % a.nplans;
                if (ld_acq(&a.cursor[p]) >= (unsigned long long)a.g.nnz) continue;
                const unsigned long long e0 = atomicAdd(&a.cursor[p], (unsigned long long)kR);
                if (e0 < (unsigned long long)a.g.nnz) {
                    sh.lv[2].row0 = (int64_t)e0;
                    sh.lv[2].nrows = (int32_t)min((unsigned long long)kR, (unsigned long long)a.g.nnz - e0);
                    sh.action = (sh.plan == p) ? 1 : 2;
                    sh.victim = p;
                }
            }
        }
        __syncthreads();
        if (sh.action == 2) {
            flush_counts(a, sh, sh.plan, sh.k, cnt, hs, hx);  // results so far belong to the previous query
            if (t == 0) {
                sh.plan = sh.victim;
                sh.k = a.plans[sh.plan].k;
            }
            __syncthreads();
        }
        if (sh.action != 0) {
            if (t == 0) {
                for (int q = 2; q < kLv; ++q) sh.lv[q].total = sh.lv[q].done = 0;
                sh.W = 2;
            }
            __syncthreads();
            HUGE_BUSY(prepare_any<K>(2, a, a.plans[sh.plan], sh.k == 3, sh));
        } else {
            // ---- no fresh edges anywhere: help a big last-level chunk, steal
            // rows, or finish when nothing is left
            flush_counts(a, sh, sh.plan, sh.k, cnt, hs, hx);
            if (t == 0 && counted) {
                atomicSub(a.busy, 1);
                counted = 0;
            }
            uint32_t seed = (uint32_t)blockIdx.x * 2654435761u + 12345u;
            bool got_rows = false;
            for (;;) {
                if (t == 0) {
                    sh.action = 0;
                    const int nwg = gridDim.x;
                    // 1. a tile of another WG's published chunk
                    for (int tries = 0; tries < 16 && sh.action == 0; ++tries) {
                        seed = seed * 1664525u + 1013904223u;
                        const int v = (int)(seed % (uint32_t)nwg);
                        if (v == (int)blockIdx.x) continue;
                        Board &b = a.boards[v];
                        const unsigned long long o = ld_acq(&b.word);
                        if (bw_next(o) >= bw_tiles(o)) continue;
                        // a claim below the tile count is valid for whatever generation it
                        // landed in: that generation's owner waits for it to be done
                        const unsigned long long x = atomicAdd(&b.word, 1ull);
                        if (bw_next(x) < bw_tiles(x)) {
                            sh.action = 5;
                            sh.victim = v;
                            sh.tile = (int32_t)bw_next(x);
                        }
                    }
                    // 2. half of the rows of another WG's shallowest level
                    if (sh.action == 0 && a.steal) {
                        for (int tries = 0; tries < 8 && sh.action == 0; ++tries) {
                            seed = seed * 1664525u + 1013904223u;
                            const int v = (int)(seed % (uint32_t)nwg);
                            if (v == (int)blockIdx.x) continue;
                            for (int W = 3; W < K && sh.action == 0; ++W) {
                                unsigned long long *d = a.deq + (int64_t)v * kLv + W;
                                const unsigned long long o = ld_acq(d);
                                const uint32_t h = dq_head(o), tl = dq_tail(o);
                                if (tl < h + 2) continue;
                                const int plan = dq_plan(o);
                                if (plan >= a.nplans || W > a.plans[plan].k - 1) continue;
                                // count ourselves busy before the rows can become ours
                                atomicAdd(a.busy, 1);
                                atomicAdd(&a.pending[(int64_t)v * kLv + W], 1);
                                __threadfence();
                                const uint32_t kk = min((tl - h) / 2, (uint32_t)a.cap[W]);
                                if (atomicCAS(d, o, dq_make(h + kk, tl, plan)) == o) {
                                    sh.action = 3;
                                    sh.victim = v;
                                    sh.vlevel = W;
                                    sh.vhead = h;
                                    sh.vcount = kk;
                                    sh.plan = plan;
                                    counted = 1;
                                } else {
                                    atomicSub(&a.pending[(int64_t)v * kLv + W], 1);
                                    atomicSub(a.busy, 1);
                                }
                            }
                        }
                    }
                    if (sh.action == 0) {
                        if (ld_acq_i(a.busy) == 0) {
                            sh.action = 4;  // no rows anywhere: done
                        } else if (past(deadline)) {
                            atomicOr(a.err, 1);
                            sh.action = 4;
                        } else {
                            __builtin_amdgcn_s_sleep(4);
                        }
                    }
                }
                __syncthreads();
                const int act = sh.action;
                __syncthreads();  // every wave has read the decision before thread 0 makes the next one
                if (act == 0) continue;
                if (act == 4) break;
                if (act == 5) {
                    // process the claimed tile; its owner waits for our "done"
                    __threadfence();
                    Board &b = a.boards[sh.victim];
                    const int plan = b.plan, W = b.W, k = a.plans[plan].k;
                    ChunkView cv;
                    cv.rows = level_buf(a, sh.victim, W);
                    cv.row0 = b.row0;
                    cv.nrows = b.nrows;
                    cv.off = b.off;
                    cv.pinfo = b.pinfo;
                    cv.hpre = b.hpre;
                    const int64_t w0 = (int64_t)sh.tile * kPTile;
                    HUGE_BUSY(tile_any<K>(W, true, a, a.plans[plan], cv, sh, w0, min(w0 + (int64_t)kPTile, b.total), cnt, hs, hx));
                    flush_counts(a, sh, plan, k, cnt, hs, hx);
                    if (t == 0) {
                        __threadfence();
                        atomicAdd(&b.done, 1ull);
                        atomicAdd(&a.stats[3], 1ull);
                    }
                    __syncthreads();
                    continue;
                }
                got_rows = true;  // act == 3
                break;
            }
            if (!got_rows) break;
            // ---- take the stolen rows into our own (empty) level buffer
            const int W = sh.vlevel;
            if (t == 0) {
                sh.k = a.plans[sh.plan].k;
                int *pend = a.pending + (int64_t)blockIdx.x * kLv + W;
                while (ld_acq_i(pend) != 0 && !past(deadline)) __builtin_amdgcn_s_sleep(2);
                if (ld_acq_i(pend) != 0) atomicOr(a.err, 1);
                __hip_atomic_store(a.deq + (int64_t)blockIdx.x * kLv + W, dq_make(0, 0, sh.plan), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            __threadfence();
            {
                const int32_t *src = level_buf(a, sh.victim, W) + (int64_t)sh.vhead * W;
                int32_t *dst = level_buf(a, blockIdx.x, W);
                const int64_t n = (int64_t)sh.vcount * W;
                for (int64_t i = t; i < n; i += kT) dst[i] = src[i];
            }
            __threadfence();
            __syncthreads();
            if (t == 0) {
                atomicSub(&a.pending[(int64_t)sh.victim * kLv + W], 1);
                atomicAdd(&a.stats[0], 1ull);
                atomicAdd(&a.stats[1], (unsigned long long)sh.vcount);
                for (int q = 2; q < kLv; ++q) sh.lv[q].total = sh.lv[q].done = 0;
                sh.W = W;
                dq_push(a, W, sh.vcount);
            }
            __syncthreads();
        }

        // ---- Algorithm 5 on this WG's levels for query sh.plan
        const DevPlan &P = a.plans[sh.plan];
        const int k = sh.k;
        for (;;) {
            const int W = sh.W;
            LvState &L = sh.lv[W];
            const bool has_work = L.done < L.total;
            // every wave has read the control state before thread 0 may change it
            __syncthreads();
            if (has_work) {
                ChunkView cv;
                cv.rows = level_buf(a, blockIdx.x, W);
                cv.row0 = L.row0;
                cv.nrows = L.nrows;
                cv.off = sh.off[W];
                cv.pinfo = sh.pinfo[W];
                cv.hpre = sh.hpre;
                if (W == k - 1) {
                    // fused SINK: consume the whole chunk, then back to the precursor
                    const int64_t ntiles = (L.total + kPTile - 1) / kPTile;
                    if (ntiles <= 1) {
                        HUGE_BUSY(tile_any<K>(W, true, a, P, cv, sh, 0, L.total, cnt, hs, hx));
                    } else {
                        // publish the chunk so that idle WGs can take tiles of it
                        for (int i = t; i <= L.nrows; i += kT) myb.off[i] = sh.off[W][i];
                        for (int i = t; i < L.nrows; i += kT) {
                            myb.pinfo[i] = sh.pinfo[W][i];
                            myb.hpre[i] = sh.hpre[i];
                        }
                        if (t == 0) {
                            myb.plan = sh.plan;
                            myb.W = W;
                            myb.nrows = L.nrows;
                            myb.row0 = L.row0;
                            myb.total = L.total;
                            myb.done = 0;
                            sh.gen = (sh.gen + 1) & 0xFFFF;
                        }
                        __threadfence();
                        __syncthreads();
                        if (t == 0)
                            __hip_atomic_store(&myb.word, dq_make(0, (uint32_t)ntiles, (int)sh.gen), __ATOMIC_RELEASE,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        for (;;) {
                            if (t == 0) {
                                const unsigned long long x = atomicAdd(&myb.word, 1ull);
                                sh.tile = bw_next(x) < bw_tiles(x) ? (int32_t)bw_next(x) : -1;
                            }
                            __syncthreads();
                            const int tile = sh.tile;
                            if (tile < 0) break;
                            const int64_t w0 = (int64_t)tile * kPTile;
                            HUGE_BUSY(tile_any<K>(W, true, a, P, cv, sh, w0, min(w0 + (int64_t)kPTile, L.total), cnt, hs, hx));
                            __syncthreads();
                            if (t == 0) atomicAdd(&myb.done, 1ull);
                        }
                        if (t == 0) {
                            // the rows stay in place until every claimed tile is done
                            while (ld_acq(&myb.done) < (unsigned long long)ntiles && !past(deadline))
                                __builtin_amdgcn_s_sleep(2);
                            if (ld_acq(&myb.done) < (unsigned long long)ntiles) {
                                atomicOr(a.err, 1);
                                sh.W = -1;
                            }
                        }
                    }
                    __syncthreads();
                    if (sh.W < 0) break;
                    if (t == 0) L.done = L.total;
                    __syncthreads();
                    continue;
                }
                // extend into W+1 while it has room for a whole tile
                if (t == 0) {
                    sh.tail_base = (int32_t)dq_prepare_append(a, W + 1, sh.plan);
                    sh.action = (a.cap[W + 1] - sh.tail_base >= kPTile) ? 1 : 0;
                    sh.emitted = 0;
                }
                __syncthreads();
                if (sh.action) {
                    const int64_t w0 = L.done, w1 = min(L.done + (int64_t)kPTile, L.total);
                    HUGE_BUSY(tile_any<K>(W, false, a, P, cv, sh, w0, w1, cnt, hs, hx));
                    __threadfence();
                    __syncthreads();
                    if (t == 0) {
                        L.done = w1;
                        if (sh.emitted) {
                            dq_push(a, W + 1, (uint32_t)sh.emitted);
                            atomicAdd(&a.res[sh.plan * kResStride + 4 + W], (unsigned long long)sh.emitted);
                            unsigned long long bytes = 0;
                            for (int q = 3; q < k; ++q)
                                bytes += 4ull * q * dq_tail(ld_acq(a.deq + (int64_t)blockIdx.x * kLv + q));
                            if (bytes > sh.peak_bytes) sh.peak_bytes = bytes;
                        }
                    }
                    __syncthreads();
                }
                // Q_O full or holding rows: move to the successor
                if (t == 0) {
                    const unsigned long long o = ld_acq(a.deq + (int64_t)blockIdx.x * kLv + (W + 1));
                    if (dq_tail(o) > dq_head(o)) {
                        sh.W = W + 1;
                    } else if (!sh.action) {
                        // empty but no room: a thief is still copying out of it
                        if (past(deadline)) {
                            atomicOr(a.err, 1);
                            sh.W = -1;
                        } else {
                            __builtin_amdgcn_s_sleep(2);
                        }
                    }
                }
                __syncthreads();
                if (sh.W < 0) break;
                continue;
            }
            // chunk done: the next chunk of level W
            if (W == 2) {
                if (t == 0) {
                    sh.action = 0;
                    if (ld_acq(&a.cursor[sh.plan]) < (unsigned long long)a.g.nnz) {
                        const unsigned long long e0 = atomicAdd(&a.cursor[sh.plan], (unsigned long long)kR);
                        if (e0 < (unsigned long long)a.g.nnz) {
                            sh.lv[2].row0 = (int64_t)e0;
                            sh.lv[2].nrows = (int32_t)min((unsigned long long)kR, (unsigned long long)a.g.nnz - e0);
                            sh.action = 1;
                        }
                    }
                }
                __syncthreads();
                const int got = sh.action;
                __syncthreads();  // read before thread 0 reuses sh.action
                if (!got) break;  // this query's edges are exhausted and every deeper level is empty
                HUGE_BUSY(prepare_any<K>(2, a, P, k == 3, sh));
                continue;
            }
            if (t == 0) {
                int64_t row0 = 0;
                const int c = dq_pop(a, W, row0);
                sh.action = c;
                if (c) {
                    L.row0 = row0;
                    L.nrows = c;
                } else {
                    sh.W = W - 1;  // level drained: back to the precursor
                }
            }
            __syncthreads();
            if (sh.action) HUGE_BUSY(prepare_any<K>(W, a, P, W == k - 1, sh));
        }
        if (sh.W < 0) break;
    }
    flush_counts(a, sh, sh.plan, sh.k, cnt, hs, hx);
    if (t == 0) {
        atomicAdd(&a.stats[2], sh.peak_bytes);
        a.wg_busy[blockIdx.x] = busy_ticks;
        if (counted) atomicSub(a.busy, 1);
    }
}
#undef HUGE_BUSY

constexpr int kKMax = 4;  // largest query size the kernel is built for

}  // namespace

namespace {

// Device memory of one persistent launch, carved from one block.
struct PersistLayout {
    int nwg = 0, kmax = 3;
    int64_t rows = 0, wg_ints = 0;
    int64_t lvl_off[kLv] = {};
    int32_t cap[kLv] = {};
    uint64_t buf_bytes = 0, board_bytes = 0, ctl_bytes = 0, plan_bytes = 0, total = 0;
};

PersistLayout persist_layout(const huge_plan *const *plans, int np, const huge_exec_opts &o) {
    PersistLayout L;
    if (np < 1 || np > 4096) HUGE_FAIL(HUGE_EINVAL, "bad number of plans %d", np);
    for (int i = 0; i < np; ++i) {
        if (plans[i]->k < 3) HUGE_FAIL(HUGE_EINVAL, "the persistent engine needs queries of 3 or more vertices");
        if (plans[i]->induced || plans[i]->labelled)
            HUGE_FAIL(HUGE_EINVAL, "the persistent engine does not run induced or labelled plans");
        L.kmax = std::max(L.kmax, plans[i]->k);
    }
    if (L.kmax > kKMax) HUGE_FAIL(HUGE_EINVAL, "the persistent engine supports queries of 3 to %d vertices", kKMax);
    int dev = 0, cus = 0;
    HUGE_HIP(hipGetDevice(&dev));
    HUGE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 0;
    HUGE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_persist<kKMax>, kT, 0));
    if (per_cu < 1) HUGE_FAIL(HUGE_EDEVICE, "persistent kernel cannot be resident");
    L.nwg = cus * per_cu;
    // level capacities from the frontier budget, at least two tiles per level
    uint64_t cap = o.frontier_cap_bytes;
    if (cap == UINT64_MAX) {
        size_t fr = 0, tot = 0;
        HUGE_HIP(hipMemGetInfo(&fr, &tot));
        cap = (uint64_t)(fr * 0.5);
    }
    uint64_t row_slot_bytes = 0;
    for (int W = 3; W <= L.kmax - 1; ++W) row_slot_bytes += 4ull * W;
    int64_t rows = row_slot_bytes ? (int64_t)(cap / ((uint64_t)L.nwg * row_slot_bytes)) : 0;
    rows = std::max<int64_t>(rows, 2 * kPTile);
    L.rows = std::min<int64_t>(rows, (1 << 24) - 1);
    int64_t ints = 0;
    for (int W = 0; W < kLv; ++W) {
        L.lvl_off[W] = ints;
        if (W >= 3 && W <= L.kmax - 1) {
            L.cap[W] = (int32_t)L.rows;
            ints += L.rows * W;
        }
    }
    L.wg_ints = std::max<int64_t>(ints, 1);
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    L.buf_bytes = al(4ull * L.wg_ints * L.nwg);
    L.board_bytes = al((uint64_t)sizeof(Board) * L.nwg);
    L.ctl_bytes = al(8ull * L.nwg * kLv + 4ull * L.nwg * kLv + 8ull * np + 8ull * np * kResStride + 64 + 8ull * L.nwg);
    L.plan_bytes = al(sizeof(DevPlan) * np);
    L.total = L.buf_bytes + L.board_bytes + L.ctl_bytes + L.plan_bytes;
    return L;
}

}  // namespace

uint64_t persist_workspace_bytes(const huge_plan *const *plans, int np, const huge_exec_opts &o) {
    return persist_layout(plans, np, o).total;
}

void run_persistent(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                    huge_result *outs) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)o.stream;
    if (o.slice_mode != HUGE_SLICE_MIX || o.slice2_count > 1)
        HUGE_FAIL(HUGE_EINVAL, "the persistent engine takes mixed slices of one vertex or edge only");
    const PersistLayout L = persist_layout(plans, np, o);
    std::vector<DevPlan> dp(np);
    for (int i = 0; i < np; ++i) {
        const huge_plan *p = plans[i];
        if (!p->bushy.empty()) HUGE_FAIL(HUGE_EINVAL, "a bushy plan runs through huge_count / huge_count_bushy only");
        if (p->directed) HUGE_FAIL(HUGE_EINVAL, "the persistent engine takes undirected queries only");
        dp[i] = p->dev;
        dp[i].slice_count = o.slice_count > 1 ? o.slice_count : 1;
        dp[i].slice_id = o.slice_count > 1 ? o.slice_id : 0;
        if (dp[i].slice_count > 1 && dp[i].slice_id >= dp[i].slice_count) HUGE_FAIL(HUGE_EINVAL, "slice_id >= slice_count");
        if (o.slice_vertex < -2 || o.slice_vertex >= p->k) HUGE_FAIL(HUGE_EINVAL, "slice_vertex out of range");
        const int sv = o.slice_vertex == -1 ? p->order[0] : o.slice_vertex;  // -2: edge slice, no vertex
        for (int j = 0; j < p->k; ++j) dp[i].st[j].slice = p->order[j] == sv ? 1 : 0;
        dp[i].edge_slice = (o.slice_vertex == -2 && dp[i].slice_count > 1) ? 1 : 0;
    }
    const int nwg = L.nwg;
    PersistArgs a{};
    a.g = g->dev;
    a.nplans = np;
    a.steal = o.work_stealing ? 1 : 0;
    for (int W = 0; W < kLv; ++W) {
        a.lvl_off[W] = L.lvl_off[W];
        a.cap[W] = L.cap[W];
    }
    a.wg_ints = L.wg_ints;
    // the caller's workspace when it is large enough (huge_workspace_size), else one allocation
    struct Free {
        void *p = nullptr;
        ~Free() {
            if (p) (void)hipFree(p);
        }
    } own;
    char *mem = (char *)o.workspace;
    if (mem) {
        if (o.workspace_bytes < L.total)
            HUGE_FAIL(HUGE_ENOMEM, "workspace too small: %llu bytes given, %llu needed",
                      (unsigned long long)o.workspace_bytes, (unsigned long long)L.total);
    } else {
        HUGE_HIP(hipMalloc(&own.p, L.total));
        mem = (char *)own.p;
    }
    char *c = mem;
    a.bufs = (int32_t *)c;
    c += L.buf_bytes;
    a.boards = (Board *)c;
    char *zero_from = c;
    c += L.board_bytes;
    char *ctl = c;
    a.deq = (unsigned long long *)ctl;
    ctl += 8ull * nwg * kLv;
    a.pending = (int *)ctl;
    ctl += 4ull * nwg * kLv;
    a.cursor = (unsigned long long *)ctl;
    ctl += 8ull * np;
    a.res = (unsigned long long *)ctl;
    ctl += 8ull * np * kResStride;
    a.busy = (int *)ctl;
    a.err = (int *)(ctl + 4);
    a.stats = (unsigned long long *)(ctl + 8);
    a.wg_busy = (unsigned long long *)(ctl + 64);
    c += L.ctl_bytes;
    DevPlan *dplans = (DevPlan *)c;
    int dev = 0, wall_khz = 0;
    HUGE_HIP(hipGetDevice(&dev));
    HUGE_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
    // every wait of the kernel ends within this limit (then it reports an error), well
    // before the time limits of the callers' tests and harnesses
    double limit_s = 15.0;
    if (const char *e = getenv("HUGE_PERSIST_TIMEOUT_S")) limit_s = atof(e);
    a.limit_ticks = (uint64_t)((double)std::max(wall_khz, 1) * 1000.0 * limit_s);
    HUGE_HIP(hipMemsetAsync(zero_from, 0, L.board_bytes + L.ctl_bytes, st));
    HUGE_HIP(hipMemcpyAsync(dplans, dp.data(), sizeof(DevPlan) * np, hipMemcpyHostToDevice, st));
    a.plans = dplans;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (o.profile) {
        HUGE_HIP(hipEventCreate(&e0));
        HUGE_HIP(hipEventCreate(&e1));
        HUGE_HIP(hipEventRecord(e0, st));
    }
    hipLaunchKernelGGL(k_persist<kKMax>, dim3(nwg), dim3(kT), 0, st, a);
    HUGE_HIP(hipGetLastError());
    if (o.profile) HUGE_HIP(hipEventRecord(e1, st));
    std::vector<unsigned long long> res((size_t)np * kResStride), busy(nwg);
    int err = 0;
    unsigned long long stats[4] = {0, 0, 0, 0};
    HUGE_HIP(hipMemcpyAsync(res.data(), a.res, 8ull * np * kResStride, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(&err, a.err, 4, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(stats, a.stats, sizeof(stats), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(busy.data(), a.wg_busy, 8ull * nwg, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    float kms = 0;
    if (o.profile) {
        HUGE_HIP(hipEventElapsedTime(&kms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    if (err) HUGE_FAIL(HUGE_EDEVICE, "persistent engine: a wait exceeded its time limit");
    auto t1 = std::chrono::steady_clock::now();
    const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    // per-WG busy time: mean and standard deviation over the launch's WGs (Section 7.3's balance measure)
    double sum = 0, sq = 0;
    const double tick_ms = 1.0 / std::max(wall_khz, 1);
    for (int w = 0; w < nwg; ++w) {
        const double x = (double)busy[w] * tick_ms;
        sum += x;
        sq += x * x;
    }
    const double mean = sum / nwg, var = std::max(0.0, sq / nwg - mean * mean);
    for (int i = 0; i < np; ++i) {
        huge_result &r = outs[i];
        memset(&r, 0, sizeof(r));
        const unsigned long long *x = &res[(size_t)i * kResStride];
        r.count = x[0];
        r.hash_sum = x[1];
        r.hash_xor = x[2];
        for (int q = 1; q < HUGE_KMAX; ++q) r.level_counts[q] = x[4 + q];
        r.level_counts[0] = (dp[i].slice_count > 1 && dp[i].st[0].slice) ? x[4] : (uint64_t)g->dev.n;
        r.query_ms = ms;
        r.launches = 1;
        r.steals = stats[0] + stats[3];
        r.peak_frontier_bytes = stats[2];
        r.kernel_ms[HUGE_KC_SINK] = kms;
        r.kernel_launches[HUGE_KC_SINK] = 1;
        r.workgroups = (uint64_t)nwg;
        r.wg_busy_ms_mean = mean;
        r.wg_busy_ms_std = std::sqrt(var);
    }
}

}  // namespace huge
