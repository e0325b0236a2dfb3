// Device helpers shared by the level engine (extend.hip) and the persistent
// engine (persist.hip): hashing, sorted-list search, adjacency tests, row
// loads and wave reductions.
#pragma once
#include "internal.h"

namespace huge {
namespace dev {

constexpr uint64_t kPbMask = (1ull << 56) - 1;  // probe begin in the low 56 bits of a row's probe info

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__device__ __forceinline__ uint64_t edge_key(int32_t a, int32_t b) {
    uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((uint64_t)lo << 32) | hi;
}

// first index in [lo, hi) with col[i] >= key
__device__ __forceinline__ int64_t lower_bound(const int32_t *__restrict__ col, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool contains(const int32_t *__restrict__ col, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        int32_t x = col[mid];
        if (x == key) return true;
        if (x < key) lo = mid + 1; else hi = mid;
    }
    return false;
}

// v in N(x): one bitmap load for a hub, a binary search otherwise
__device__ __forceinline__ bool adj_has(const GraphDev &g, int32_t x, int32_t v) {
    if (x >= g.hub_base) {
        const uint32_t word = g.hub_bm[(int64_t)(x - g.hub_base) * g.hub_words + (v >> 5)];
        return (word >> (v & 31)) & 1u;
    }
    return contains(g.col, g.rp[x], g.rp[x + 1], v);
}

template <int W>
__device__ __forceinline__ void load_row(const int32_t *__restrict__ rows, const GraphDev &g, int64_t r,
                                         int32_t (&f)[W]) {
    if constexpr (W == 2) {
        const int64_t e = g.l2_idx ? g.l2_idx[r] : g.l2_first + r * g.l2_stride;
        f[0] = g.src[e];
        f[1] = g.col[e];
    } else {
#pragma unroll
        for (int p = 0; p < W; ++p) f[p] = rows[r * W + p];
    }
}

// v (a rank) in slice `id` of `count`: by its mix, or by its position in
// degree order (every count-th vertex)
__device__ __forceinline__ bool in_vslice(int32_t v, uint32_t count, uint32_t id, int32_t mode) {
    if (mode) return (uint32_t)v % count == id;
    return (uint32_t)(mix64((uint64_t)(uint32_t)v) % count) == id;
}
__device__ __forceinline__ bool in_slice(int32_t v, const DevPlan &P) {
    return in_vslice(v, P.slice_count, P.slice_id, P.slice_mode);
}
// the vertex slices marked in `bits` (DevStep::slice: bit 0 the slice, bit 1
// the second slice) that apply to v
__device__ __forceinline__ bool slices_ok(int32_t bits, int32_t v, const DevPlan &P) {
    bool ok = true;
    if ((bits & 1) && P.slice_count > 1 && !P.edge_slice) ok &= in_slice(v, P);
    if ((bits & 2) && P.slice2_count > 1 && P.p2a < 0) ok &= in_vslice(v, P.slice2_count, P.slice2_id, P.slice_mode);
    return ok;
}

// Validity of a level-2 row (the SCAN of the first query edge): the
// constraint between positions 0 and 1, and the slices (of the row's ordered
// pair, or of the vertex in position 0 or 1).
// The second slice on a pair of positions (p2a, p2b), checked at the step that
// places the later of them (W is that step's position, v its candidate): the
// pair (x, y) of their images sits at entry e of the relabelled CSR (x's row,
// y's place in it), kept when e % count == id (strided), or by the pair's mix.
template <int W>
__device__ __forceinline__ bool pair2_ok(const GraphDev &g, const DevPlan &P, const int32_t (&f)[W], int32_t v) {
    int32_t x = v, y = v;
#pragma unroll
    for (int p = 0; p < W; ++p) {
        if (p == P.p2a) x = f[p];
        if (p == P.p2b) y = f[p];
    }
    if (P.slice_mode) {
        int64_t lo = g.rp[x], hi = g.rp[x + 1];
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (g.col[mid] < y) lo = mid + 1; else hi = mid;
        }
        return (uint64_t)lo % P.slice2_count == P.slice2_id;
    }
    const uint64_t key = ((uint64_t)(uint32_t)x << 32) | (uint64_t)(uint32_t)y;
    return (uint32_t)(mix64(key) % P.slice2_count) == P.slice2_id;
}

// a -> b is an arc of a directed graph
__device__ __forceinline__ bool arc(const GraphDev &g, int32_t a, int32_t b) {
    return contains(g.dcol, g.drp[a], g.drp[a + 1], b);
}

// directed plans: every query edge between the new vertex v and a matched
// position keeps its direction
template <int W>
__device__ __forceinline__ bool dirs_ok(const GraphDev &g, const DevStep &st, const int32_t (&f)[W], int32_t v) {
    bool ok = true;
#pragma unroll
    for (int p = 0; p < W; ++p) {
        if (ok && ((st.dout >> p) & 1u)) ok = arc(g, f[p], v);
        if (ok && ((st.din >> p) & 1u)) ok = arc(g, v, f[p]);
    }
    return ok;
}

// the label the plan asks of position i's vertex v (labelled plans)
__device__ __forceinline__ bool label_ok(const GraphDev &g, int32_t want, int32_t v) {
    return want < 0 || g.label[v] == want;
}

__device__ __forceinline__ bool level2_ok(const int32_t (&f)[2], const DevPlan &P, const GraphDev &g) {
    const DevStep &s1 = P.st[1];
    if (!label_ok(g, P.st[0].label, f[0]) || !label_ok(g, s1.label, f[1])) return false;
    if ((s1.lo & 1u) && !(f[0] < f[1])) return false;
    if ((s1.hi & 1u) && !(f[1] < f[0])) return false;
    if (P.slice_count > 1 && P.edge_slice == 1) {
        const uint64_t key = ((uint64_t)(uint32_t)f[0] << 32) | (uint64_t)(uint32_t)f[1];
        if ((uint32_t)(mix64(key) % P.slice_count) != P.slice_id) return false;
    }
    if ((s1.slice & 4) && !pair2_ok<1>(g, P, {f[0]}, f[1])) return false;
    if ((s1.dout | s1.din) && !dirs_ok<1>(g, s1, {f[0]}, f[1])) return false;
    return slices_ok(P.st[0].slice, f[0], P) && slices_ok(s1.slice, f[1], P);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}
__device__ __forceinline__ unsigned long long wave_xor_u64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x ^= __shfl_xor(x, d, 64);
    return x;
}

// largest r in [lo, hi] with off[r] <= w
__device__ __forceinline__ int64_t find_row(const int64_t *__restrict__ off, int64_t lo, int64_t hi, int64_t w) {
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}


// first index in [lo, hi) with col[i] > key
__device__ __forceinline__ int64_t upper_bound(const int32_t *__restrict__ col, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// first index in [pos, end) with col[i] >= key; every index before pos holds a smaller value
__device__ __forceinline__ int64_t gallop(const int32_t *__restrict__ col, int64_t pos, int64_t end, int32_t key) {
    if (pos >= end || col[pos] >= key) return pos;
    int64_t lo = pos, step = 1;  // col[lo] < key
    while (lo + step < end && col[lo + step] < key) {
        lo += step;
        step <<= 1;
    }
    int64_t hi = min(lo + step, end);
    lo += 1;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (col[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

}  // namespace dev
}  // namespace huge
