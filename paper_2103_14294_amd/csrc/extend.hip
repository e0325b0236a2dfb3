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

namespace huge {
namespace {

using namespace dev;

constexpr int kT = 256;
constexpr int kIPT = 4;
constexpr int kTile = kT * kIPT;


// ---------------------------------------------------------------------------
// prepare
// ---------------------------------------------------------------------------
// Prepares segment row i (every thread of the workgroup calls it: it ends
// with a workgroup reduction).
template <int W, bool LAST>
__device__ __forceinline__ void prepare_row(const int32_t *__restrict__ rows, int64_t row0, int64_t nrows,
                                            const GraphDev &g, const DevPlan &P, const SegBufs &s, Ctrl *ctrl,
                                            int64_t i) {
    __shared__ unsigned long long s_valid[kT / 64];
    __shared__ unsigned long long s_bytes[kT / 64];
    bool valid = false;
    unsigned long long abytes = 0;  // algorithmic bytes of a merge intersection for this row
    if (i < nrows) {
        abytes = 4ull * W;
        int32_t f[W];
        load_row<W>(rows, g, row0 + i, f);
        valid = true;
        if constexpr (W == 2) valid = level2_ok(f, P);
        int32_t bound = 0;
        uint64_t pinfo = 0;
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
                        int32_t x = f[p];
                        int64_t b = g.rp[x], e = g.rp[x + 1];
                        int64_t a = lo > 0 ? lower_bound(g.col, b, e, lo) : b;
                        int64_t z = hi < 0x7FFFFFFF ? lower_bound(g.col, a, e, hi) : e;
                        abytes += 16ull + 4ull * (unsigned long long)(z - a);
                        if (best < 0 || z - a < best) {
                            best = z - a;
                            bb = a;
                            bp = p;
                        }
                    }
                }
                bound = (int32_t)best;
                pinfo = (uint64_t)bb | ((uint64_t)bp << 56);
            }
        }
        s.bound[i] = bound;
        s.pinfo[i] = pinfo;
        if constexpr (LAST) {
            uint64_t h = 0;
            for (int e = 0; e < P.ne; ++e) {
                int b = P.eb[e];
                if (b < W) {
                    int a = P.ea[e];
                    int32_t fa = 0, fb = 0;
#pragma unroll
                    for (int p = 0; p < W; ++p) {
                        if (p == a) fa = f[p];
                        if (p == b) fb = f[p];
                    }
                    h += mix64(edge_key(fa, fb));
                }
            }
            s.hpre[i] = h;
        }
    }
    {
        unsigned long long c = wave_sum_u64(valid ? 1ull : 0ull);
        unsigned long long b = wave_sum_u64(abytes);
        if (__lane_id() == 0) {
            s_valid[threadIdx.x >> 6] = c;
            s_bytes[threadIdx.x >> 6] = b;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0, tb = 0;
            for (int q = 0; q < kT / 64; ++q) {
                t += s_valid[q];
                tb += s_bytes[q];
            }
            if (W == 2 && t) atomicAdd(&ctrl->level[1], t);
            if (tb) atomicAdd(&ctrl->segbytes[W], tb);
        }
    }
}

template <int W, bool LAST>
__global__ __launch_bounds__(kT) void k_prepare(const int32_t *__restrict__ rows, int64_t row0, int64_t nrows,
                                                GraphDev g, DevPlan P, SegBufs s, Ctrl *ctrl) {
    prepare_row<W, LAST>(rows, row0, nrows, g, P, s, ctrl, (int64_t)blockIdx.x * kT + threadIdx.x);
}

// ---------------------------------------------------------------------------
// extend
// ---------------------------------------------------------------------------
struct ExtArgs {
    const int32_t *rows;
    int64_t row0;
    const int32_t *rid;  // segment row r holds input row row0 + rid[r] (NULL: row0 + r)
    const int64_t *off;
    const uint64_t *pinfo;
    const uint64_t *hpre;
    int64_t nrows;
    int64_t w0, w1;
    int32_t *out;
    Ctrl *ctrl;
    const int32_t *inv_rank;
    GraphDev g;
    DevPlan P;
};


__device__ __forceinline__ int64_t row_at(const ExtArgs &a, int64_t r) {
    return a.row0 + (a.rid ? (int64_t)a.rid[r] : r);
}

__device__ __forceinline__ bool lds_contains(const int32_t *s, int32_t n, int32_t key) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        int32_t x = s[mid];
        if (x == key) return true;
        if (x < key) lo = mid + 1; else hi = mid;
    }
    return false;
}

// Orders this wave's LDS writes before its later LDS reads (all lanes).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kStage = 512;  // staged list entries per wave

struct WaveSeg {
    int head, tail;  // first and last lane of this lane's row segment
    int ord, nseg;   // segment ordinal within the wave, number of segments
    bool big;        // segment long enough to share one window search
};

// Wave-cooperative membership test of each lane's candidate v in the list of
// vertex x (one list per row segment).  The 64 lanes hold consecutive work
// items, so a row's candidates occupy a run of lanes in increasing order.  For
// a run of >= 3 lanes, its first lane finds the first list entry >= its
// candidate and its last lane the first entry > its candidate: the run's
// candidates can only match inside that window.  The windows of all runs are
// copied into LDS with coalesced loads when they fit, and each lane then
// binary-searches LDS; otherwise each lane searches its run's window in
// global memory.  Short runs search the whole list directly.
__device__ __forceinline__ bool wave_member(const GraphDev &g, bool need_any, int32_t x, int32_t v, int lane,
                                            const WaveSeg &sg, int32_t *stage, int32_t *spref, int64_t *slb) {
    // hub lists are answered by their bitmap; only the others take part below
    const bool hub = need_any && x >= g.hub_base;
    const bool need = need_any && !hub;
    int64_t lo = 0, hi = 0;
    if (need) {
        lo = g.rp[x];
        hi = g.rp[x + 1];
    }
    const bool nb = need && sg.big;
    int64_t lbv = 0, ubv = 0;
    if (nb && lane == sg.head) lbv = lower_bound(g.col, lo, hi, v);
    if (nb && lane == sg.tail) ubv = upper_bound(g.col, lo, hi, v);
    const int64_t lb = __shfl(lbv, sg.head, 64);
    const int64_t ub = __shfl(ubv, sg.tail, 64);
    const int32_t wlen = nb ? (int32_t)(ub - lb) : 0;
    const int32_t contrib = (lane == sg.head) ? wlen : 0;
    int32_t incl = contrib;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    const int32_t total = __shfl(incl, 63, 64);
    const int32_t myoff = __shfl(incl - contrib, sg.head, 64);
    bool found = false;
    if (total > 0 && total <= kStage) {
        if (lane == sg.head) {
            spref[sg.ord] = incl - contrib;
            slb[sg.ord] = lb;
        }
        if (lane == 0) spref[sg.nseg] = total;
        wave_sync();
        for (int idx = lane; idx < total; idx += 64) {
            int s0 = 0, s1 = sg.nseg - 1;
            while (s0 < s1) {
                int m = (s0 + s1 + 1) >> 1;
                if (spref[m] <= idx) s0 = m; else s1 = m - 1;
            }
            stage[idx] = g.col[slb[s0] + (idx - spref[s0])];
        }
        wave_sync();
        if (nb) found = lds_contains(stage + myoff, wlen, v);
        wave_sync();
    } else if (nb) {
        found = contains(g.col, lb, ub, v);
    }
    if (need && !sg.big) found = contains(g.col, lo, hi, v);
    if (hub) found = adj_has(g, x, v);
    return found;
}

// One tile of kTile work items (every thread of the workgroup calls it).
template <int W, int MODE, int STRAT>
__device__ __forceinline__ void extend_tile(const ExtArgs &a, int64_t tile) {
    __shared__ int64_t s_rng[2];
    __shared__ unsigned long long s_red[3][kT / 64];
    __shared__ int32_t s_cnt[kT / 64];
    __shared__ unsigned long long s_base;
    __shared__ int32_t s_stage[STRAT == 1 ? kT / 64 : 1][STRAT == 1 ? kStage : 1];
    __shared__ int32_t s_pref[STRAT == 1 ? kT / 64 : 1][65];
    __shared__ int64_t s_lb[STRAT == 1 ? kT / 64 : 1][64];

    const int64_t tile0 = a.w0 + tile * kTile;
    const int64_t tile1 = min(tile0 + (int64_t)kTile, a.w1);
    if (threadIdx.x == 0) {
        s_rng[0] = find_row(a.off, 0, a.nrows - 1, tile0);
        s_rng[1] = find_row(a.off, s_rng[0], a.nrows - 1, tile1 - 1);
    }
    __syncthreads();
    const int64_t rlo = s_rng[0], rhi = s_rng[1];
    const DevStep st = a.P.st[W];
    const GraphDev &g = a.g;
    const int lane = __lane_id();
    const int wvi = threadIdx.x >> 6;

    unsigned long long cnt = 0, hs = 0, hx = 0;
    uint32_t okmask = 0;
    int32_t vv[kIPT];
    int32_t rr[kIPT];
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
        vv[j] = 0;
        rr[j] = 0;
        const int64_t w = tile0 + j * kT + threadIdx.x;
        const bool active = w < tile1;
        if (STRAT == 0 && !active) continue;
        int64_t r = rlo;
        int32_t v = 0;
        int pp = 0;
        int32_t f[W];
#pragma unroll
        for (int p = 0; p < W; ++p) f[p] = 0;
        if (active) {
            r = find_row(a.off, rlo, rhi, w);
            const uint64_t pi = a.pinfo[r];
            pp = (int)(pi >> 56);
            v = g.col[(int64_t)(pi & kPbMask) + (w - a.off[r])];
            load_row<W>(a.rows, g, row_at(a, r), f);
        }
        bool ok = active;
#pragma unroll
        for (int p = 0; p < W; ++p)
            if ((st.neq >> p) & 1u) ok &= (v != f[p]);
        if (st.slice && a.P.slice_count > 1) ok &= in_slice(v, a.P);
        if constexpr (STRAT == 0) {
#pragma unroll
            for (int p = 0; p < W; ++p) {
                if (ok && ((st.ext >> p) & 1u) && p != pp) ok = adj_has(g, f[p], v);
            }
        } else {
            // row segments of this wave
            const int64_t rprev = __shfl_up(r, 1, 64);
            const bool head = active && (lane == 0 || rprev != r);
            const uint64_t hmask = __ballot(head);
            const uint64_t amask = __ballot(active);
            const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
            WaveSeg sg;
            const uint64_t hle = hmask & le;
            sg.head = hle ? 63 - __clzll(hle) : 0;
            const uint64_t after = hmask & ~le;
            const int last_active = amask ? 63 - __clzll(amask) : 0;
            sg.tail = after ? __ffsll((long long)after) - 2 : last_active;
            sg.ord = __popcll(hle) - 1;
            sg.nseg = __popcll(hmask);
            sg.big = (sg.tail - sg.head) >= 2;
#pragma unroll
            for (int p = 0; p < W; ++p) {
                if ((st.ext >> p) & 1u) {
                    const bool need = active && p != pp;
                    const bool in = wave_member(g, need, f[p], v, lane, sg, s_stage[wvi], s_pref[wvi], s_lb[wvi]);
                    if (need) ok &= in;
                }
            }
        }
        if (!ok) continue;
        if constexpr (MODE == MODE_COUNT) {
            uint64_t h = a.hpre[r];
#pragma unroll
            for (int p = 0; p < W; ++p)
                if ((st.ext >> p) & 1u) h += mix64(edge_key(f[p], v));
            h = mix64(h);
            cnt += 1;
            hs += h;
            hx ^= h;
        } else if constexpr (MODE == MODE_COUNT_NOHASH) {
            cnt += 1;
        } else {
            okmask |= 1u << j;
            vv[j] = v;
            rr[j] = (int32_t)r;
        }
    }

    const int wv = wvi;
    if constexpr (MODE == MODE_COUNT || MODE == MODE_COUNT_NOHASH) {
        cnt = wave_sum_u64(cnt);
        hs = wave_sum_u64(hs);
        hx = wave_xor_u64(hx);
        if (__lane_id() == 0) {
            s_red[0][wv] = cnt;
            s_red[1][wv] = hs;
            s_red[2][wv] = hx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long c = 0, s = 0, x = 0;
            for (int q = 0; q < kT / 64; ++q) {
                c += s_red[0][q];
                s += s_red[1][q];
                x ^= s_red[2][q];
            }
            if (c) {
                atomicAdd(&a.ctrl->acc[0], c);
                atomicAdd(&a.ctrl->acc[1], s);
                atomicXor(&a.ctrl->acc[2], x);
                atomicAdd(&a.ctrl->level[W], c);
            }
        }
        return;
    } else {
        // workgroup-wide exclusive scan of per-thread output counts
        int c = __popc(okmask);
        int inc = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int y = __shfl_up(inc, d, 64);
            if (lane >= d) inc += y;
        }
        if (lane == 63) s_cnt[wv] = inc;
        __syncthreads();
        int wbase = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kT / 64; ++q) {
            if (q < wv) wbase += s_cnt[q];
            tot += s_cnt[q];
        }
        if (threadIdx.x == 0) {
            unsigned long long b = 0;
            if (tot) {
                const int qi = (MODE == MODE_EMIT) ? (W + 1) : HUGE_KMAX;
                b = atomicAdd(&a.ctrl->qcount[qi], (unsigned long long)tot);
                atomicAdd(&a.ctrl->level[W], (unsigned long long)tot);
            }
            s_base = b;
        }
        __syncthreads();
        if (!okmask) return;
        int64_t o = (int64_t)s_base + wbase + (inc - c);
#pragma unroll
        for (int j = 0; j < kIPT; ++j) {
            if (!((okmask >> j) & 1u)) continue;
            int32_t f[W];
            load_row<W>(a.rows, g, row_at(a, rr[j]), f);
            if constexpr (MODE == MODE_EMIT) {
                int32_t *dst = a.out + o * (W + 1);
#pragma unroll
                for (int p = 0; p < W; ++p) dst[p] = f[p];
                dst[W] = vv[j];
            } else {
                // final match, indexed by query vertex, original IDs
                int32_t *dst = a.out + o * (W + 1);
#pragma unroll
                for (int q = 0; q < W + 1; ++q) {
                    const int p = a.P.pos[q];
                    int32_t x = vv[j];
#pragma unroll
                    for (int t = 0; t < W; ++t)
                        if (t == p) x = f[t];
                    dst[q] = a.inv_rank[x];
                }
            }
            ++o;
        }
    }
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
        f[0] = g.src[e];
        f[1] = g.col[e];
        ok = level2_ok(f, P);
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
            out[o * 2 + 0] = inv_rank[a0];
            out[o * 2 + 1] = inv_rank[a1];
        }
    }
}

__global__ __launch_bounds__(kT) void k_root_count(int64_t n, DevPlan P, Ctrl *ctrl) {
    __shared__ unsigned long long s[kT / 64];
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    unsigned long long c = (v < n && in_slice((int32_t)v, P)) ? 1 : 0;
    c = wave_sum_u64(c);
    if (__lane_id() == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < kT / 64; ++q) t += s[q];
        if (t) atomicAdd(&ctrl->level[0], t);
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

// ---------------------------------------------------------------------------
// lane merge: every lane owns a run of RUN consecutive work items (probe
// elements, usually of one row).  For each other Ext list it finds the first
// entry >= its first candidate once, then advances that cursor by galloping
// (exponential then binary search, Bentley-Yao) as the sorted candidates
// increase, so a membership test costs O(log gap) instead of O(log degree).
// Hub lists are answered by their bitmap.
//
// With BLK, every list read goes through one aligned 16-byte block kept in
// registers per list (and one for the lane's own candidates): a cursor that
// stays inside its block, which is the common case when the lists have similar
// density, costs no load at all, and a short gallop ending in the next block
// costs one.  The kernel is limited by how many lane-divergent gathers the
// memory pipeline accepts per clock, so fewer of them is what pays.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t pick4(const int4 &q, int64_t i) {
    const int t = (int)(i & 3);
    return t == 0 ? q.x : t == 1 ? q.y : t == 2 ? q.z : q.w;
}

// First index i in [c, e) with col[i] >= key (e if none), given that every
// index before c holds a smaller value.  blk/q cache the aligned block
// col[4*blk .. 4*blk+3]; the result's value is returned in x when i < e.
__device__ __forceinline__ int64_t gallop_blk(const int32_t *__restrict__ col, int64_t c, int64_t e, int32_t key,
                                              int32_t &blk, int4 &q, int32_t &x) {
    if (c >= e) return e;
    const int32_t b = (int32_t)(c >> 2);
    if (b != blk) {
        q = reinterpret_cast<const int4 *>(col)[b];
        blk = b;
    }
    const int64_t base = (int64_t)b << 2;
    // first slot t >= c - base of the block (and before e) with a value >= key
    int64_t hit = -1;
    int32_t hv = 0;
    const int32_t qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int t = 3; t >= 0; --t) {
        const int64_t i = base + t;
        if (i >= c && i < e && qv[t] >= key) {
            hit = i;
            hv = qv[t];
        }
    }
    if (hit >= 0) {
        x = hv;
        return hit;
    }
    if (base + 4 >= e) return e;
    const int64_t r = gallop(col, base + 4, e, key);
    if (r < e) {
        blk = (int32_t)(r >> 2);
        q = reinterpret_cast<const int4 *>(col)[blk];
        x = pick4(q, r);
    }
    return r;
}

// One tile of kT * RUN work items (every thread of the workgroup calls it).
// First index in [lo, hi) with col[i] >= key (hi if none), by binary search
// over whole aligned blocks; leaves the block of the result in (blk, q).
__device__ __forceinline__ int64_t lower_bound_blk(const int32_t *__restrict__ col, int64_t lo, int64_t hi,
                                                   int32_t key, int32_t &blk, int4 &q) {
    if (lo >= hi) return hi;
    int32_t bl = (int32_t)(lo >> 2), bh = (int32_t)((hi - 1) >> 2);
    // the result's block is in [bl, bh]: the last entry of every block before
    // bh lies inside [lo, hi) and decides which side the result is on
    while (bl < bh) {
        const int32_t mid = (bl + bh) >> 1;
        if (col[((int64_t)mid << 2) + 3] < key) bl = mid + 1; else bh = mid;
    }
    if (bl != blk) {
        q = reinterpret_cast<const int4 *>(col)[bl];
        blk = bl;
    }
    const int32_t qv[4] = {q.x, q.y, q.z, q.w};
    const int64_t base = (int64_t)bl << 2;
    int64_t r = hi;
#pragma unroll
    for (int t = 3; t >= 0; --t)
        if (base + t >= lo && base + t < hi && qv[t] >= key) r = base + t;
    return r;
}

template <int W, int MODE, int RUN, bool BLK>
__device__ __forceinline__ void merge_tile(const ExtArgs &a, int64_t tile) {
    constexpr int kRun = RUN;
    constexpr int kMTile = kT * RUN;
    constexpr bool kEmit = MODE == MODE_EMIT || MODE == MODE_OUTPUT;
    // each hit is hashed in the lane that finds it, from the row in registers
    // and the row's prefix hash loaded once per row: the kernel is bound by
    // memory instructions, not VALU, so divergent hashing beats batching hits
    // and reloading their rows
    constexpr bool kHash = MODE == MODE_COUNT;
    __shared__ int64_t s_rng[2];
    __shared__ unsigned long long s_red[3][kT / 64];
    __shared__ int32_t s_cnt[kT / 64];
    __shared__ unsigned long long s_base;
    static_assert(!kEmit || RUN <= 16, "emitting kernels stage RUN rows per lane in LDS");
    __shared__ int32_t s_ov[kEmit ? kT * kRun : 1];
    __shared__ int32_t s_or[kEmit ? kT * kRun : 1];

    const int64_t tile0 = a.w0 + tile * kMTile;
    const int64_t tile1 = min(tile0 + (int64_t)kMTile, a.w1);
    if (threadIdx.x == 0) {
        s_rng[0] = find_row(a.off, 0, a.nrows - 1, tile0);
        s_rng[1] = find_row(a.off, s_rng[0], a.nrows - 1, tile1 - 1);
    }
    __syncthreads();
    const int64_t rlo = s_rng[0], rhi = s_rng[1];
    const DevStep st = a.P.st[W];
    const GraphDev &g = a.g;
    const int wv = threadIdx.x >> 6;
    const int lane = __lane_id();

    unsigned long long cnt = 0, hs = 0, hx = 0;
    int nout = 0;

    const int64_t wb = tile0 + (int64_t)threadIdx.x * kRun;
    const int64_t we = min(wb + (int64_t)kRun, tile1);
    int64_t r = rlo, rend = -1, pshift = 0;
    int pp = 0;
    int32_t f[W];
    int64_t cur[W], end[W];
    // BLK: the cached block of each list, and of the lane's candidates
    int32_t cblk[BLK ? W : 1];
    int4 cq[BLK ? W : 1];
    int32_t vblk = -1;
    int4 vq = make_int4(0, 0, 0, 0);
    uint64_t hrow = 0;  // hashing: prefix hash of the lane's current row
#pragma unroll
    for (int p = 0; p < W; ++p) {
        f[p] = 0;
        cur[p] = 0;
        end[p] = 0;
    }
#pragma unroll
    for (int p = 0; p < (BLK ? W : 1); ++p) {
        cblk[p] = -1;
        cq[p] = make_int4(0, 0, 0, 0);
    }
    auto cand = [&](int64_t i) -> int32_t {
        if constexpr (BLK) {
            const int32_t b = (int32_t)(i >> 2);
            if (b != vblk) {
                vq = reinterpret_cast<const int4 *>(g.col)[b];
                vblk = b;
            }
            return pick4(vq, i);
        } else {
            return g.col[i];
        }
    };
    for (int it = 0; it < kRun; ++it) {
        const int64_t w = wb + it;
        bool ok = false;
        int32_t v = 0;
        if (w < we) {
            if (w >= rend) {
                // enter the row that holds item w
                r = (rend < 0) ? find_row(a.off, rlo, rhi, w) : find_row(a.off, r + 1, rhi, w);
                rend = a.off[r + 1];
                const uint64_t pi = a.pinfo[r];
                pp = (int)(pi >> 56);
                pshift = (int64_t)(pi & kPbMask) - a.off[r];
                load_row<W>(a.rows, g, row_at(a, r), f);
                if constexpr (kHash) hrow = a.hpre[r];
                const int32_t v0 = cand(pshift + w);
#pragma unroll
                for (int p = 0; p < W; ++p) {
                    if (((st.ext >> p) & 1u) && p != pp) {
                        if (f[p] < g.hub_base) {
                            end[p] = g.rp[f[p] + 1];
                            if constexpr (BLK) {
                                cur[p] = lower_bound_blk(g.col, g.rp[f[p]], end[p], v0, cblk[p], cq[p]);
                            } else {
                                cur[p] = lower_bound(g.col, g.rp[f[p]], end[p], v0);
                            }
                        } else if constexpr (BLK) {
                            cblk[p] = -1;  // a new hub: its cached bitmap block is not valid
                        }
                    }
                }
            }
            v = cand(pshift + w);
            ok = true;
#pragma unroll
            for (int p = 0; p < W; ++p)
                if ((st.neq >> p) & 1u) ok &= (v != f[p]);
            if (st.slice && a.P.slice_count > 1) ok &= in_slice(v, a.P);
#pragma unroll
            for (int p = 0; p < W; ++p) {
                if (ok && ((st.ext >> p) & 1u) && p != pp) {
                    if (f[p] >= g.hub_base) {
                        if constexpr (BLK) {
                            // hub: the 16-byte bitmap block of 128 vertex IDs around v, cached
                            // under a negative key (list blocks have keys >= 0)
                            const int32_t key = -2 - (v >> 7);
                            if (cblk[p] != key) {
                                cq[p] = reinterpret_cast<const int4 *>(
                                    g.hub_bm + (int64_t)(f[p] - g.hub_base) * g.hub_words)[v >> 7];
                                cblk[p] = key;
                            }
                            ok = (((uint32_t)pick4(cq[p], (v >> 5) & 3)) >> (v & 31)) & 1u;
                        } else {
                            ok = adj_has(g, f[p], v);
                        }
                    } else if constexpr (BLK) {
                        int32_t x = 0;
                        cur[p] = gallop_blk(g.col, cur[p], end[p], v, cblk[p], cq[p], x);
                        ok = cur[p] < end[p] && x == v;
                    } else {
                        cur[p] = gallop(g.col, cur[p], end[p], v);
                        ok = cur[p] < end[p] && g.col[cur[p]] == v;
                    }
                }
            }
        }
        if constexpr (kHash) {
            if (ok) {
                uint64_t h = hrow;
#pragma unroll
                for (int p = 0; p < W; ++p)
                    if ((st.ext >> p) & 1u) h += mix64(edge_key(f[p], v));
                h = mix64(h);
                cnt += 1;
                hs += h;
                hx ^= h;
            }
        } else if constexpr (MODE == MODE_COUNT_NOHASH) {
            cnt += ok ? 1 : 0;
        } else {
            if (ok) {
                s_ov[threadIdx.x * kRun + nout] = v;
                s_or[threadIdx.x * kRun + nout] = (int32_t)r;
                ++nout;
            }
        }
    }

    if constexpr (!kEmit) {
        cnt = wave_sum_u64(cnt);
        hs = wave_sum_u64(hs);
        hx = wave_xor_u64(hx);
        if (lane == 0) {
            s_red[0][wv] = cnt;
            s_red[1][wv] = hs;
            s_red[2][wv] = hx;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long c = 0, s = 0, x = 0;
            for (int q = 0; q < kT / 64; ++q) {
                c += s_red[0][q];
                s += s_red[1][q];
                x ^= s_red[2][q];
            }
            if (c) {
                atomicAdd(&a.ctrl->acc[0], c);
                if (kHash) {
                    atomicAdd(&a.ctrl->acc[1], s);
                    atomicXor(&a.ctrl->acc[2], x);
                }
                atomicAdd(&a.ctrl->level[W], c);
            }
        }
    } else {
        int inc = nout;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int y = __shfl_up(inc, d, 64);
            if (lane >= d) inc += y;
        }
        if (lane == 63) s_cnt[wv] = inc;
        __syncthreads();
        int wbase = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kT / 64; ++q) {
            if (q < wv) wbase += s_cnt[q];
            tot += s_cnt[q];
        }
        if (threadIdx.x == 0) {
            unsigned long long b = 0;
            if (tot) {
                const int qi = (MODE == MODE_EMIT) ? (W + 1) : HUGE_KMAX;
                b = atomicAdd(&a.ctrl->qcount[qi], (unsigned long long)tot);
                atomicAdd(&a.ctrl->level[W], (unsigned long long)tot);
            }
            s_base = b;
        }
        __syncthreads();
        int64_t o = (int64_t)s_base + wbase + (inc - nout);
        for (int q = 0; q < nout; ++q, ++o) {
            const int32_t v = s_ov[threadIdx.x * kRun + q];
            int32_t ff[W];
            load_row<W>(a.rows, g, row_at(a, s_or[threadIdx.x * RUN + q]), ff);
            int32_t *dst = a.out + o * (W + 1);
            if constexpr (MODE == MODE_EMIT) {
#pragma unroll
                for (int p = 0; p < W; ++p) dst[p] = ff[p];
                dst[W] = v;
            } else {
#pragma unroll
                for (int qq = 0; qq < W + 1; ++qq) {
                    const int p = a.P.pos[qq];
                    int32_t x = v;
#pragma unroll
                    for (int t = 0; t < W; ++t)
                        if (t == p) x = ff[t];
                    dst[qq] = a.inv_rank[x];
                }
            }
        }
    }
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

// Claims the workgroup's next tile from a per-round counter, so that tiles are
// taken in order, as the hardware dispatches the workgroups of a plain launch
// (neighbouring rows share lists in L2), and a slow tile delays no other.
// Returns -1 when every tile is taken.
__device__ __forceinline__ int64_t claim_tile(unsigned long long *next, int64_t tiles) {
    __shared__ int64_t s_tile;
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(next, 1ull);
    __syncthreads();
    const int64_t t = s_tile;
    __syncthreads();
    return t < tiles ? t : -1;
}

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

void launch_root_count(const GraphDev &g, const DevPlan &P, Ctrl *ctrl, hipStream_t st) {
    dim3 grid((unsigned)((g.n + kT - 1) / kT));
    hipLaunchKernelGGL(k_root_count, grid, dim3(kT), 0, st, g.n, P, ctrl);
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
