// Per-tile device bodies of PULL-EXTEND, shared by the level engine, the
// graph engine and the batched graph engine: the prepare pass of one row
// (symmetry-breaking window, trimmed lists, probe choice), the intersection
// tiles (binary search / wave-staged LDS, and the lane merges) with their
// filters, compaction and counting SINK, and in-order tile claiming.
#pragma once
#include "devfuncs.h"
#include "internal.h"

namespace huge {
namespace tiles {

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
    // Algorithmic bytes of this row's intersection: the row, 16 bytes of list
    // bounds per Ext list, the probe window, and of every other window at
    // least one element per probe candidate unless the window is shorter (a
    // membership needs one element of it; a merge reads it whole): the fewest
    // list bytes any intersection of these windows must read.
    unsigned long long abytes = 0;
    if (i < nrows) {
        abytes = 4ull * W;
        int32_t f[W];
        load_row<W>(rows, g, row0 + i, f);
        valid = true;
        if constexpr (W == 2) valid = level2_ok(f, P, g);
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
                int64_t len[W];
#pragma unroll
                for (int p = 0; p < W; ++p) {
                    len[p] = 0;
                    if ((st.ext >> p) & 1u) {
                        int32_t x = f[p];
                        int64_t b = g.rp[x], e = g.rp[x + 1];
                        int64_t a = lo > 0 ? lower_bound(g.col, b, e, lo) : b;
                        int64_t z = hi < 0x7FFFFFFF ? lower_bound(g.col, a, e, hi) : e;
                        len[p] = z - a;
                        if (best < 0 || z - a < best) {
                            best = z - a;
                            bb = a;
                            bp = p;
                        }
                    }
                }
#pragma unroll
                for (int p = 0; p < W; ++p)
                    if ((st.ext >> p) & 1u)
                        abytes += 16ull + 4ull * (unsigned long long)(len[p] < best ? len[p] : best);
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

constexpr int kStage = 512;     // staged list entries per wave
constexpr int kRowStage = 1024; // row offsets of a binary-search tile staged in LDS

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

// The binary-search strategy's items of one lane: the kIPT work items
// w = tile0 + j * kT + threadIdx.x (every thread of the workgroup calls it: it
// stages the tile's row offsets in LDS).  Their searches run in lockstep -- the
// row of each item in the tile's offsets, then for every Ext list the
// membership of each candidate by a branch-free binary search (Khuong and
// Morin's form: halve the range on one comparison per round, test the one
// element left) -- so a round issues one load per item and the kIPT chains
// of dependent loads overlap instead of following one another.  ok[j] says
// whether item j passes every test; v[j], r[j] and f[j] are its candidate,
// segment row and row.
template <int W>
__device__ __forceinline__ void bsearch_items(const ExtArgs &a, const DevStep &st, int64_t tile0, int64_t tile1,
                                              int64_t rlo, int64_t rhi, bool (&ok)[kIPT], int32_t (&v)[kIPT],
                                              int64_t (&r)[kIPT], int32_t (&f)[kIPT][W]) {
    const GraphDev &g = a.g;
    // the tile's row offsets off[rlo .. rhi + 1], staged in LDS with coalesced
    // loads when they fit, so the row searches below run on LDS
    __shared__ int64_t s_off[kRowStage + 1];
    const int64_t nr = rhi - rlo + 1;
    const bool staged = nr <= kRowStage;
    if (staged)
        for (int64_t i = threadIdx.x; i <= nr; i += kT) s_off[i] = a.off[rlo + i];
    __syncthreads();
    const int64_t *off = staged ? s_off : a.off + rlo;  // off[i] is the offset of row rlo + i
    int64_t w[kIPT], lo[kIPT], hi[kIPT];
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
        w[j] = tile0 + j * kT + threadIdx.x;
        ok[j] = w[j] < tile1;
        lo[j] = 0;
        hi[j] = ok[j] ? nr - 1 : 0;
    }
    // rows: the last i in [0, nr) with off[i] <= w (every probe inside the tile's rows)
    for (;;) {
        bool more = false;
        int64_t x[kIPT];
#pragma unroll
        for (int j = 0; j < kIPT; ++j) x[j] = off[lo[j] < hi[j] ? (lo[j] + hi[j] + 1) >> 1 : lo[j]];
#pragma unroll
        for (int j = 0; j < kIPT; ++j) {
            if (lo[j] < hi[j]) {
                const int64_t mid = (lo[j] + hi[j] + 1) >> 1;
                if (x[j] <= w[j]) lo[j] = mid; else hi[j] = mid - 1;
                more |= lo[j] < hi[j];
            }
        }
        if (!more) break;
    }
    int pp[kIPT];
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
        r[j] = rlo + lo[j];
        const uint64_t pi = a.pinfo[r[j]];
        pp[j] = (int)(pi >> 56);
        v[j] = g.col[(int64_t)(pi & kPbMask) + (ok[j] ? w[j] - off[lo[j]] : 0)];
        load_row<W>(a.rows, g, row_at(a, r[j]), f[j]);
    }
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
        bool o = ok[j];
#pragma unroll
        for (int p = 0; p < W; ++p)
            if ((st.neq >> p) & 1u) o &= (v[j] != f[j][p]);
        if (st.slice) o &= slices_ok(st.slice, v[j], a.P);
        if (st.label >= 0) o = o && label_ok(g, st.label, v[j]);
        if (st.slice & 4) o = o && pair2_ok<W>(g, a.P, f[j], v[j]);
        if (st.dout | st.din) o = o && dirs_ok<W>(g, st, f[j], v[j]);
        ok[j] = o;
    }
#pragma unroll
    for (int p = 0; p < W; ++p) {
        if (!(((st.ext | st.vadj) >> p) & 1u)) continue;
        int64_t b[kIPT];
        int32_t n[kIPT];
        bool found[kIPT];
#pragma unroll
        for (int j = 0; j < kIPT; ++j) {
            const int32_t x = f[j][p];
            const bool need = ok[j] && p != pp[j];
            const bool hub = need && x >= g.hub_base;
            found[j] = !need;
            if (hub) {
                const uint32_t word = g.hub_bm[(int64_t)(x - g.hub_base) * g.hub_words + (v[j] >> 5)];
                found[j] = (word >> (v[j] & 31)) & 1u;
            }
            const int32_t xx = (need && !hub) ? x : 0;
            b[j] = g.rp[xx];
            n[j] = (need && !hub) ? (int32_t)(g.rp[xx + 1] - b[j]) : 0;
        }
        // found[j] for a non-hub list: the last element <= v[j] stays in [b, b + n) until n = 1
        for (;;) {
            bool more = false;
            int32_t y[kIPT];
#pragma unroll
            for (int j = 0; j < kIPT; ++j) y[j] = g.col[n[j] > 0 ? b[j] + (n[j] >> 1) : 0];
#pragma unroll
            for (int j = 0; j < kIPT; ++j) {
                const int32_t half = n[j] >> 1;
                found[j] = n[j] == 1 ? y[j] == v[j] : found[j];
                b[j] += (n[j] > 1 && y[j] <= v[j]) ? half : 0;
                n[j] = n[j] > 1 ? n[j] - half : 0;
                more |= n[j] > 0;
            }
            if (!more) break;
        }
#pragma unroll
        for (int j = 0; j < kIPT; ++j) ok[j] = ok[j] && found[j];
    }
    if (st.nadj) {  // induced mode
#pragma unroll
        for (int j = 0; j < kIPT; ++j)
#pragma unroll
            for (int p = 0; p < W; ++p)
                if (ok[j] && ((st.nadj >> p) & 1u)) ok[j] = !adj_has(g, f[j][p], v[j]);
    }
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
    // a passing item: folded into the counting SINK, or kept for the output pass
    auto accept = [&](int j, int64_t r, int32_t v, const int32_t(&f)[W]) {
        if constexpr (MODE == MODE_COUNT) {
            uint64_t h = a.hpre[r];
#pragma unroll
            for (int p = 0; p < W; ++p)
                if (((st.ext | st.vadj) >> p) & 1u) h += mix64(edge_key(f[p], v));
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
    };
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
        vv[j] = 0;
        rr[j] = 0;
    }
    if constexpr (STRAT == 0) {
        bool okb[kIPT];
        int32_t vb[kIPT];
        int64_t rb[kIPT];
        int32_t fb[kIPT][W];
        bsearch_items<W>(a, st, tile0, tile1, rlo, rhi, okb, vb, rb, fb);
#pragma unroll
        for (int j = 0; j < kIPT; ++j)
            if (okb[j]) accept(j, rb[j], vb[j], fb[j]);
    } else {
#pragma unroll
    for (int j = 0; j < kIPT; ++j) {
        const int64_t w = tile0 + j * kT + threadIdx.x;
        const bool active = w < tile1;
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
        if (st.slice) ok &= slices_ok(st.slice, v, a.P);
        if (st.label >= 0) ok = ok && label_ok(g, st.label, v);
        if (st.slice & 4) ok = ok && pair2_ok<W>(g, a.P, f, v);
        if (st.dout | st.din) ok = ok && dirs_ok<W>(g, st, f, v);
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
#pragma unroll
        for (int p = 0; p < W; ++p) {
            if (ok && ((st.nadj >> p) & 1u)) ok = !adj_has(g, f[p], v);  // induced mode
            if (ok && ((st.vadj >> p) & 1u)) ok = adj_has(g, f[p], v);   // verify-only edges
        }
        if (ok) accept(j, r, v, f);
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
                // final match, indexed by query vertex, original IDs (ranks without inv_rank)
                int32_t *dst = a.out + o * (W + 1);
#pragma unroll
                for (int q = 0; q < W + 1; ++q) {
                    const int p = a.P.pos[q];
                    int32_t x = vv[j];
#pragma unroll
                    for (int t = 0; t < W; ++t)
                        if (t == p) x = f[t];
                    dst[q] = a.inv_rank ? a.inv_rank[x] : x;
                }
            }
            ++o;
        }
    }
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
                    if ((((st.ext | st.nadj | st.vadj) >> p) & 1u) && p != pp) {
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
            if (st.slice) ok &= slices_ok(st.slice, v, a.P);
            if (st.label >= 0) ok = ok && label_ok(g, st.label, v);
            if (st.slice & 4) ok = ok && pair2_ok<W>(g, a.P, f, v);
            if (st.dout | st.din) ok = ok && dirs_ok<W>(g, st, f, v);
#pragma unroll
            for (int p = 0; p < W; ++p) {
                // Ext lists (and verify-only lists) must hold v; in induced mode
                // the lists of the other matched vertices (nadj) must not
                if (ok && (((st.ext | st.nadj | st.vadj) >> p) & 1u) && p != pp) {
                    const bool absent = (st.nadj >> p) & 1u;
                    bool in = false;
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
                            in = (((uint32_t)pick4(cq[p], (v >> 5) & 3)) >> (v & 31)) & 1u;
                        } else {
                            in = adj_has(g, f[p], v);
                        }
                    } else if constexpr (BLK) {
                        int32_t x = 0;
                        cur[p] = gallop_blk(g.col, cur[p], end[p], v, cblk[p], cq[p], x);
                        in = cur[p] < end[p] && x == v;
                    } else {
                        cur[p] = gallop(g.col, cur[p], end[p], v);
                        in = cur[p] < end[p] && g.col[cur[p]] == v;
                    }
                    ok = in != absent;
                }
            }
        }
        if constexpr (kHash) {
            if (ok) {
                uint64_t h = hrow;
#pragma unroll
                for (int p = 0; p < W; ++p)
                    if (((st.ext | st.vadj) >> p) & 1u) h += mix64(edge_key(f[p], v));
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
                    dst[qq] = a.inv_rank ? a.inv_rank[x] : x;
                }
            }
        }
    }
}


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

}  // namespace tiles
}  // namespace huge
