// Table operators of bushy plans (Sections 3.1-3.3, 4.3, 5.1): PULL-EXTEND
// steps over a materialised table, the verify-only EXTEND (a row filter on
// edges between matched vertices), and PUSH-JOIN, a hash join of two tables
// on their shared query vertices.
//
// A table holds rows of ranks, row-major, column c holding one query vertex.
// Every operator is two data-parallel passes over "work items": a prepare
// pass gives each input row its item count (candidates of the shortest
// trimmed list, 1 for a filter, the equal-key range of the other side for a
// join), an exclusive scan turns the counts into offsets, and an item pass
// maps every item back to its row by binary search in the offsets and tests
// it -- the same flattening as the level engine's, so a hub row's work
// spreads over the whole grid; each lane takes a run of consecutive items, so
// the row search and the row load are paid once per run and row.  The item pass either counts the rows that
// pass (to size the output exactly), writes them (one atomic per wave), or,
// for the plan's root, counts them with the set-hash of their edges.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "devfuncs.h"
#include "join.h"
#include "prims.h"

namespace huge {

namespace {

using namespace dev;

constexpr int kJT = 256;

__device__ __forceinline__ void load_tab_row(const int32_t *__restrict__ t, int w, int64_t r, int32_t (&f)[HUGE_KMAX]) {
#pragma unroll
    for (int c = 0; c < HUGE_KMAX; ++c) f[c] = c < w ? t[r * w + c] : -1;
}

// set-hash of one output row over the edges given as column pairs
__device__ __forceinline__ uint64_t row_hash(const int32_t (&f)[HUGE_KMAX], int ne, const int8_t *ea,
                                             const int8_t *eb) {
    uint64_t h = 0;
    for (int e = 0; e < ne; ++e) {
        int32_t a = 0, b = 0;
#pragma unroll
        for (int c = 0; c < HUGE_KMAX; ++c) {
            if (c == ea[e]) a = f[c];
            if (c == eb[e]) b = f[c];
        }
        h += mix64(edge_key(a, b));
    }
    return mix64(h);
}

// The item pass's output: append `ok` rows of width w (one atomic per wave),
// or count them (with the set-hash for the root).
struct Sink {
    int mode;  // TAB_COUNT, TAB_WRITE, TAB_ROOT
    int32_t *out;
    int64_t cap;
    int w;
    unsigned long long *acc;  // [0] rows, [1] hash_sum, [2] hash_xor, [3] overflow
    int ne;
    int8_t ea[32], eb[32];
};

__device__ __forceinline__ void sink_row(const Sink &s, bool ok, const int32_t (&f)[HUGE_KMAX]) {
    const int lane = __lane_id();
    if (s.mode == TAB_WRITE) {
        const uint64_t m = __ballot(ok);
        if (!m) return;
        unsigned long long base = 0;
        const int leader = __ffsll((long long)m) - 1;
        if (lane == leader) base = atomicAdd(&s.acc[0], (unsigned long long)__popcll(m));
        base = __shfl(base, leader, 64);
        if (ok) {
            const int64_t o = (int64_t)base + __popcll(m & ((1ull << lane) - 1));
            if (o < s.cap) {
#pragma unroll
                for (int c = 0; c < HUGE_KMAX; ++c)
                    if (c < s.w) s.out[o * s.w + c] = f[c];
            } else {
                atomicOr(&s.acc[3], 1ull);
            }
        }
        return;
    }
    unsigned long long c = ok ? 1ull : 0ull, h = 0;
    if (s.mode == TAB_ROOT && ok) h = row_hash(f, s.ne, s.ea, s.eb);
    const unsigned long long cs = wave_sum_u64(c);
    const unsigned long long hs = s.mode == TAB_ROOT ? wave_sum_u64(h) : 0ull;
    const unsigned long long hx = s.mode == TAB_ROOT ? wave_xor_u64(h) : 0ull;
    if (lane == 0 && cs) {
        atomicAdd(&s.acc[0], cs);
        if (s.mode == TAB_ROOT) {
            atomicAdd(&s.acc[1], hs);
            atomicXor(&s.acc[2], hx);
        }
    }
}

// Every lane takes kChunk consecutive work items per round: one binary search
// finds the row of the first, a forward cursor the rows of the others, and
// the row is loaded again only when it changes.
constexpr int kChunk = 8;

// the row holding item t, from a cursor at row r <= that row (rows without
// items are stepped over)
__device__ __forceinline__ int64_t advance_row(const int64_t *__restrict__ off, int64_t n, int64_t r, int64_t t) {
    while (r + 1 < n && off[r + 1] <= t) ++r;
    return r;
}

// ---------------------------------------------------------------------------
// table steps
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kJT) void k_tab_prepare(const int32_t *__restrict__ in, int64_t n, TabStep S, GraphDev g,
                                                     uint32_t *__restrict__ bound, uint64_t *__restrict__ pinfo) {
    for (int64_t i = (int64_t)blockIdx.x * kJT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kJT) {
        int32_t f[HUGE_KMAX];
        load_tab_row(in, S.w, i, f);
        bool ok = true;
        // the verify-only EXTEND: the row's edges between matched vertices
        for (int t = 0; t < S.nver && ok; ++t) {
            int32_t a = 0, b = 0;
#pragma unroll
            for (int c = 0; c < HUGE_KMAX; ++c) {
                if (c == S.va[t]) a = f[c];
                if (c == S.vb[t]) b = f[c];
            }
            ok = adj_has(g, a, b);
        }
        uint32_t cnt = ok ? 1u : 0u;
        uint64_t pi = 0;
        if (ok && S.add) {
            // Eq. 2: the shortest list among the Ext columns, trimmed to the
            // symmetry-breaking window, is the probe
            int32_t lo = 0, hi = 0x7FFFFFFF;
#pragma unroll
            for (int c = 0; c < HUGE_KMAX; ++c) {
                if ((S.lo >> c) & 1u) lo = max(lo, f[c] + 1);
                if ((S.hi >> c) & 1u) hi = min(hi, f[c]);
            }
            int64_t best = -1, bb = 0;
            int bp = 0;
            if (lo < hi) {
#pragma unroll
                for (int c = 0; c < HUGE_KMAX; ++c) {
                    if ((S.ext >> c) & 1u) {
                        const int64_t b = g.rp[f[c]], e = g.rp[f[c] + 1];
                        const int64_t a = lo > 0 ? lower_bound(g.col, b, e, lo) : b;
                        const int64_t z = hi < 0x7FFFFFFF ? lower_bound(g.col, a, e, hi) : e;
                        if (best < 0 || z - a < best) {
                            best = z - a;
                            bb = a;
                            bp = c;
                        }
                    }
                }
            }
            cnt = best > 0 ? (uint32_t)best : 0u;
            pi = (uint64_t)bb | ((uint64_t)bp << 56);
        }
        bound[i] = cnt;
        pinfo[i] = pi;
    }
}

__global__ __launch_bounds__(kJT) void k_tab_items(const int32_t *__restrict__ in, int64_t n,
                                                   const int64_t *__restrict__ off, const uint64_t *__restrict__ pinfo,
                                                   int64_t items, TabStep S, GraphDev g, Sink sk) {
    const int64_t span = (int64_t)gridDim.x * kJT * kChunk;
    const int64_t t_lane = ((int64_t)blockIdx.x * kJT + threadIdx.x) * kChunk;
    // every lane of a wave runs the same number of iterations (the sink's ballots)
    const int64_t rounds = (items + span - 1) / span;
    for (int64_t it = 0; it < rounds; ++it) {
        const int64_t t0 = it * span + t_lane;
        int64_t r = t0 < items ? find_row(off, 0, n - 1, t0) : 0, rl = -1;
        int32_t fr[HUGE_KMAX];
        uint64_t pi = 0;
        for (int j = 0; j < kChunk; ++j) {
            const int64_t t = t0 + j;
            bool ok = false;
            int32_t f[HUGE_KMAX];
#pragma unroll
            for (int c = 0; c < HUGE_KMAX; ++c) f[c] = -1;
            if (t < items) {
                r = advance_row(off, n, r, t);
                if (r != rl) {
                    load_tab_row(in, S.w, r, fr);
                    pi = S.add ? pinfo[r] : 0;
                    rl = r;
                }
#pragma unroll
                for (int c = 0; c < HUGE_KMAX; ++c) f[c] = fr[c];
                ok = true;
                if (S.add) {
                    const int pp = (int)(pi >> 56);
                    const int32_t v = g.col[(int64_t)(pi & kPbMask) + (t - off[r])];
#pragma unroll
                    for (int c = 0; c < HUGE_KMAX; ++c) {
                        if (c < S.w) {
                            ok = ok && v != f[c];  // injectivity
                            if (ok && ((S.ext >> c) & 1u) && c != pp) ok = adj_has(g, f[c], v);
                        }
                    }
                    if (ok && S.slice) ok = in_vslice(v, S.slice_count, S.slice_id, S.slice_mode);
                    if (ok && S.label >= 0) ok = label_ok(g, S.label, v);
#pragma unroll
                    for (int c = 0; c < HUGE_KMAX; ++c)
                        if (c == S.w) f[c] = v;
                }
            }
            sink_row(sk, ok, f);
        }
    }
}

// ---------------------------------------------------------------------------
// PUSH-JOIN
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t key_hash(const int32_t (&f)[HUGE_KMAX], int nkey, const int8_t *kc) {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    for (int i = 0; i < nkey; ++i) {
        int32_t x = 0;
#pragma unroll
        for (int c = 0; c < HUGE_KMAX; ++c)
            if (c == kc[i]) x = f[c];
        h = mix64(h ^ (uint64_t)(uint32_t)x);
    }
    return (uint32_t)(h >> 32);
}

__global__ __launch_bounds__(kJT) void k_join_keys(const int32_t *__restrict__ R, int64_t nr, JoinSpec J,
                                                   uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    for (int64_t i = (int64_t)blockIdx.x * kJT + threadIdx.x; i < nr; i += (int64_t)gridDim.x * kJT) {
        int32_t f[HUGE_KMAX];
        load_tab_row(R, J.wr, i, f);
        keys[i] = key_hash(f, J.nkey, J.kr);
        vals[i] = (uint32_t)i;
    }
}

// each left row: the range of right rows with its key hash in the sorted keys
__global__ __launch_bounds__(kJT) void k_join_prepare(const int32_t *__restrict__ L, int64_t nl, JoinSpec J,
                                                      const uint32_t *__restrict__ skeys, int64_t nr,
                                                      uint32_t *__restrict__ bound, int64_t *__restrict__ first,
                                                      unsigned long long *__restrict__ acc) {
    for (int64_t i = (int64_t)blockIdx.x * kJT + threadIdx.x; i < nl; i += (int64_t)gridDim.x * kJT) {
        int32_t f[HUGE_KMAX];
        load_tab_row(L, J.wl, i, f);
        const uint32_t h = key_hash(f, J.nkey, J.kl);
        int64_t lo = 0, hi = nr;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (skeys[mid] < h) lo = mid + 1; else hi = mid;
        }
        int64_t a = lo;
        hi = nr;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (skeys[mid] <= h) lo = mid + 1; else hi = mid;
        }
        const int64_t cnt = lo - a;
        if (cnt > 0xFFFFFFFFll) atomicOr(&acc[3], 2ull);
        bound[i] = (uint32_t)(cnt > 0xFFFFFFFFll ? 0xFFFFFFFFll : cnt);
        first[i] = a;
    }
}

// R's rows in key-hash order (after the sort), so that a key's rows are adjacent
__global__ __launch_bounds__(kJT) void k_gather_rows(const int32_t *__restrict__ R, int64_t nr, int w,
                                                     const uint32_t *__restrict__ svals, int32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * kJT + threadIdx.x; i < nr * w; i += (int64_t)gridDim.x * kJT) {
        const int64_t r = i / w, c = i - r * w;
        out[i] = R[(int64_t)svals[r] * w + c];
    }
}

__global__ __launch_bounds__(kJT) void k_join_items(const int32_t *__restrict__ L, int64_t nl,
                                                    const int32_t *__restrict__ Rs, const int64_t *__restrict__ off,
                                                    const int64_t *__restrict__ first, int64_t items, JoinSpec J,
                                                    Sink sk) {
    const int64_t span = (int64_t)gridDim.x * kJT * kChunk;
    const int64_t t_lane = ((int64_t)blockIdx.x * kJT + threadIdx.x) * kChunk;
    const int64_t rounds = (items + span - 1) / span;
    for (int64_t it = 0; it < rounds; ++it) {
        const int64_t t0 = it * span + t_lane;
        int64_t r = t0 < items ? find_row(off, 0, nl - 1, t0) : 0, rl = -1;
        int32_t fl[HUGE_KMAX];
        for (int jj = 0; jj < kChunk; ++jj) {
            const int64_t t = t0 + jj;
            bool ok = false;
            int32_t f[HUGE_KMAX];
#pragma unroll
            for (int c = 0; c < HUGE_KMAX; ++c) f[c] = -1;
            if (t < items) {
                r = advance_row(off, nl, r, t);
                if (r != rl) {
                    load_tab_row(L, J.wl, r, fl);
                    rl = r;
                }
                int32_t fr[HUGE_KMAX];
                load_tab_row(Rs, J.wr, first[r] + (t - off[r]), fr);
                ok = true;
                // the join key itself (the hash only grouped the rows)
                for (int i = 0; i < J.nkey; ++i) {
                    int32_t a = 0, b = 0;
#pragma unroll
                    for (int c = 0; c < HUGE_KMAX; ++c) {
                        if (c == J.kl[i]) a = fl[c];
                        if (c == J.kr[i]) b = fr[c];
                    }
                    ok = ok && a == b;
                }
                // output row: the left columns, then the right-only ones
#pragma unroll
                for (int c = 0; c < HUGE_KMAX; ++c) f[c] = fl[c];
                for (int i = 0; i < J.nro; ++i) {
                    int32_t x = 0;
#pragma unroll
                    for (int c = 0; c < HUGE_KMAX; ++c)
                        if (c == J.ro[i]) x = fr[c];
                    // injectivity: a right-only vertex differs from every left one
#pragma unroll
                    for (int c = 0; c < HUGE_KMAX; ++c)
                        if (c < J.wl) ok = ok && x != fl[c];
#pragma unroll
                    for (int c = 0; c < HUGE_KMAX; ++c)
                        if (c == J.wl + i) f[c] = x;
                }
                // symmetry-breaking constraints across the two sides
                for (int i = 0; i < J.nsb && ok; ++i) {
                    int32_t a = 0, b = 0;
#pragma unroll
                    for (int c = 0; c < HUGE_KMAX; ++c) {
                        if (c == J.sa[i]) a = f[c];
                        if (c == J.sb[i]) b = f[c];
                    }
                    ok = a < b;
                }
            }
            sink_row(sk, ok, f);
        }
    }
}

int grid_for(int64_t n) {
    const int64_t b = (n + kJT - 1) / kJT;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 256 * 64));
}

int grid_items(int64_t items) { return grid_for((items + kChunk - 1) / kChunk); }

Sink make_sink(int mode, int32_t *out, int64_t cap, int w, unsigned long long *acc, int ne, const int8_t *ea,
               const int8_t *eb) {
    Sink s;
    memset(&s, 0, sizeof(s));
    s.mode = mode;
    s.out = out;
    s.cap = cap;
    s.w = w;
    s.acc = acc;
    s.ne = ne;
    for (int e = 0; e < ne && e < 32; ++e) {
        s.ea[e] = ea[e];
        s.eb[e] = eb[e];
    }
    return s;
}

}  // namespace

void launch_tab_prepare(const int32_t *in, int64_t n, const TabStep &S, const GraphDev &g, uint32_t *bound,
                        uint64_t *pinfo, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tab_prepare, dim3(grid_for(n)), dim3(kJT), 0, st, in, n, S, g, bound, pinfo);
    HUGE_HIP(hipGetLastError());
}

void launch_tab_items(const int32_t *in, int64_t n, const int64_t *off, const uint64_t *pinfo, int64_t items,
                      const TabStep &S, const GraphDev &g, int mode, int32_t *out, int64_t cap,
                      unsigned long long *acc, hipStream_t st) {
    if (items <= 0) return;
    const Sink sk = make_sink(mode, out, cap, S.w + (S.add ? 1 : 0), acc, S.ne, S.ea, S.eb);
    hipLaunchKernelGGL(k_tab_items, dim3(grid_items(items)), dim3(kJT), 0, st, in, n, off, pinfo, items, S, g, sk);
    HUGE_HIP(hipGetLastError());
}

void launch_join_keys(const int32_t *R, int64_t nr, const JoinSpec &J, uint32_t *keys, uint32_t *vals,
                      hipStream_t st) {
    if (nr <= 0) return;
    hipLaunchKernelGGL(k_join_keys, dim3(grid_for(nr)), dim3(kJT), 0, st, R, nr, J, keys, vals);
    HUGE_HIP(hipGetLastError());
}

void launch_join_prepare(const int32_t *L, int64_t nl, const JoinSpec &J, const uint32_t *skeys, int64_t nr,
                         uint32_t *bound, int64_t *first, unsigned long long *acc, hipStream_t st) {
    if (nl <= 0) return;
    hipLaunchKernelGGL(k_join_prepare, dim3(grid_for(nl)), dim3(kJT), 0, st, L, nl, J, skeys, nr, bound, first, acc);
    HUGE_HIP(hipGetLastError());
}

void launch_gather_rows(const int32_t *R, int64_t nr, int w, const uint32_t *svals, int32_t *out, hipStream_t st) {
    if (nr <= 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(nr * w)), dim3(kJT), 0, st, R, nr, w, svals, out);
    HUGE_HIP(hipGetLastError());
}

void launch_join_items(const int32_t *L, int64_t nl, const int32_t *Rs, const int64_t *off, const int64_t *first,
                       int64_t items, const JoinSpec &J, int mode, int32_t *out, int64_t cap, unsigned long long *acc,
                       hipStream_t st) {
    if (items <= 0) return;
    const Sink sk = make_sink(mode, out, cap, J.wl + J.nro, acc, J.ne, J.ea, J.eb);
    hipLaunchKernelGGL(k_join_items, dim3(grid_items(items)), dim3(kJT), 0, st, L, nl, Rs, off, first, items, J, sk);
    HUGE_HIP(hipGetLastError());
}

}  // namespace huge
