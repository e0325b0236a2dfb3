// Graph loading on the GPU: hygiene checks, degree-rank relabelling, re-sorted
// adjacency lists and the degree sketch used by the planner.
//
// Section 2 of the paper fixes the data-vertex total order used by symmetry
// breaking: vertices are relabelled so that a smaller degree gets a smaller
// ID, ties broken by the original ID.  After relabelling every ID is a rank,
// so the order test in the kernels is a plain integer compare.
//
// Relabelling without a segmented sort: list the pairs (s = rank(w), t =
// rank(u)) for every adjacency entry w of u, grouped by t in increasing t
// (row t of the relabelled graph, unsorted inside the row).  A stable sort
// of these pairs by s groups them by s and keeps t ascending inside each
// group, which is exactly the relabelled CSR with sorted lists: the sorted
// keys are the row of each entry and the sorted values are the column IDs.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

#include "internal.h"
#include "prims.h"

namespace huge {
namespace {

constexpr int kT = 256;

enum : uint32_t {
    BAD_ROWPTR = 1u,
    BAD_ORDER = 2u,     // not strictly ascending (unsorted or duplicate)
    BAD_SELF = 4u,
    BAD_RANGE = 8u,
    BAD_ASYM = 16u,
};

__global__ void k_check_rowptr(const int64_t *__restrict__ rp, int64_t n, int64_t nnz, uint32_t *flags) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    int64_t a = rp[u];
    bool bad = a < 0 || a > nnz;
    if (u == 0 && a != 0) bad = true;
    if (u == n && a != nnz) bad = true;
    if (u < n && rp[u + 1] < a) bad = true;
    if (bad) atomicOr(flags, BAD_ROWPTR);
}

__device__ __forceinline__ bool bsearch_has(const int32_t *__restrict__ col, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        int32_t x = col[mid];
        if (x == key) return true;
        if (x < key) lo = mid + 1; else hi = mid;
    }
    return false;
}

// Visits every adjacency entry of the vertex range [256*b, 256*b+256) with
// the row found by a binary search over the range's row pointers in LDS.
#define EDGE_RANGE_PROLOGUE                                                   \
    __shared__ int64_t srp[kT + 1];                                           \
    int64_t u0 = (int64_t)blockIdx.x * kT;                                    \
    int64_t cnt = n - u0 < kT ? n - u0 : kT;                                  \
    for (int i = threadIdx.x; i <= cnt; i += kT) srp[i] = rp[u0 + i];        \
    __syncthreads();                                                          \
    int64_t e0 = srp[0], e1 = srp[cnt];

__device__ __forceinline__ int64_t row_of(const int64_t *srp, int64_t cnt, int64_t e) {
    // largest r in [0, cnt) with srp[r] <= e
    int64_t lo = 0, hi = cnt;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (srp[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kT) void k_check_edges(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                    int64_t n, uint32_t *flags) {
    EDGE_RANGE_PROLOGUE
    uint32_t f = 0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kT) {
        int64_t r = row_of(srp, cnt, e);
        int64_t u = u0 + r;
        int32_t w = col[e];
        if (w < 0 || (int64_t)w >= n) {
            f |= BAD_RANGE;
            continue;
        }
        if ((int64_t)w == u) f |= BAD_SELF;
        if (e > srp[r] && col[e - 1] >= w) f |= BAD_ORDER;
        if (!bsearch_has(col, rp[w], rp[w + 1], (int32_t)u)) f |= BAD_ASYM;
    }
    if (f) atomicOr(flags, f);
}

constexpr uint32_t kHubMinDegree = 256;

__global__ void k_degree_keys(const int64_t *__restrict__ rp, int64_t n, uint32_t *__restrict__ key,
                              uint32_t *__restrict__ val, uint32_t *dmax, unsigned long long *nhub) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    uint32_t d = (uint32_t)(rp[u + 1] - rp[u]);
    key[u] = d;
    val[u] = (uint32_t)u;
    atomicMax(dmax, d);
    if (d >= kHubMinDegree) atomicAdd(nhub, 1ull);
}

// One n-bit adjacency bitmap per hub (ranks base..n-1): bit w of hub x is
// set iff w is a neighbour of x.
__global__ __launch_bounds__(kT) void k_hub_bitmap(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                   int64_t base, int64_t words, uint32_t *__restrict__ bm) {
    const int64_t x = base + blockIdx.x;
    uint32_t *row = bm + (int64_t)blockIdx.x * words;
    for (int64_t e = rp[x] + threadIdx.x; e < rp[x + 1]; e += kT) {
        const int32_t w = col[e];
        atomicOr(&row[w >> 5], 1u << (w & 31));
    }
}

// inv = vertices sorted by (degree, id); rank[inv[i]] = i; newdeg[i] = deg(inv[i]).
__global__ void k_ranks(const uint32_t *__restrict__ sorted_deg, const uint32_t *__restrict__ inv, int64_t n,
                        int32_t *__restrict__ rank, int32_t *__restrict__ inv_out, uint32_t *__restrict__ newdeg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t u = inv[i];
    rank[u] = (int32_t)i;
    inv_out[i] = (int32_t)u;
    newdeg[i] = sorted_deg[i];
}

__global__ __launch_bounds__(kT) void k_pairs(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                              int64_t n, const int32_t *__restrict__ rank,
                                              const int64_t *__restrict__ nrp, uint32_t *__restrict__ key,
                                              uint32_t *__restrict__ val) {
    EDGE_RANGE_PROLOGUE
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kT) {
        int64_t r = row_of(srp, cnt, e);
        int64_t u = u0 + r;
        int32_t t = rank[u];
        int64_t p = nrp[t] + (e - srp[r]);
        key[p] = (uint32_t)rank[col[e]];
        val[p] = (uint32_t)t;
    }
}

// Degree sketch: log2 histogram (exact integer atomics) and per-block partial
// power sums sum d^p, p = 0..7, reduced in a fixed order afterwards.
__global__ __launch_bounds__(kT) void k_sketch(const int64_t *__restrict__ rp, int64_t n,
                                               unsigned long long *__restrict__ hist,
                                               double *__restrict__ partial) {
    __shared__ unsigned int sh[32];
    __shared__ double sm[8][kT];
    if (threadIdx.x < 32) sh[threadIdx.x] = 0;
    __syncthreads();
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t base = (int64_t)blockIdx.x * kT * 16;
    for (int j = 0; j < 16; ++j) {
        int64_t u = base + j * kT + threadIdx.x;
        if (u >= n) break;
        int64_t d = rp[u + 1] - rp[u];
        int b = d == 0 ? 0 : 64 - __clzll((unsigned long long)d);
        if (b > 31) b = 31;
        atomicAdd(&sh[b], 1u);
        double x = (double)d, p = 1.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            m[q] += p;
            p *= x;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) sm[q][threadIdx.x] = m[q];
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < 8; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 8) partial[(int64_t)blockIdx.x * 8 + threadIdx.x] = sm[threadIdx.x][0];
    if (threadIdx.x < 32 && sh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)sh[threadIdx.x]);
}

__global__ __launch_bounds__(kT) void k_sketch_reduce(const double *__restrict__ partial, int64_t nb,
                                                      double *__restrict__ out) {
    __shared__ double sm[8][kT];
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nb; b += kT)
#pragma unroll
        for (int q = 0; q < 8; ++q) m[q] += partial[b * 8 + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) sm[q][threadIdx.x] = m[q];
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < 8; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = sm[threadIdx.x][0];
}

// Content digest of the relabelled CSR: per-block sums of mixed (index, col)
// words, combined by the host in block order.  Used only as a cache key.
__device__ __forceinline__ uint64_t dmix(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ __launch_bounds__(kT) void k_digest(const int32_t *__restrict__ col, int64_t nnz,
                                               unsigned long long *out) {
    uint64_t s = 0;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kT)
        s += dmix(((uint64_t)e << 32) ^ (uint32_t)col[e]);
    atomicAdd(out, (unsigned long long)s);
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    template <typename T>
    T *alloc(size_t count) {
        HUGE_HIP(hipMalloc(&p, count * sizeof(T) + 16));
        return (T *)p;
    }
    void *release() {
        void *q = p;
        p = nullptr;
        return q;
    }
};

inline unsigned grid_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

huge_graph *graph_load(int64_t n, int64_t nnz, const int64_t *rp_in, const int32_t *col_in, uint32_t flags,
                       hipStream_t st) {
    auto t0 = std::chrono::steady_clock::now();
    if (n < 1 || n >= 0x7FFFFFFF || nnz < 0 || nnz >= (int64_t)0xFFFFFFFF || !rp_in || (nnz > 0 && !col_in))
        HUGE_FAIL(HUGE_EINVAL, "huge_load_csr: bad sizes or NULL pointers (n=%lld nnz=%lld)", (long long)n,
                  (long long)nnz);
    const bool host = (flags & HUGE_HOST_PTRS) != 0;
    const bool dev = (flags & HUGE_DEVICE_PTRS) != 0;
    if (host == dev) HUGE_FAIL(HUGE_EINVAL, "huge_load_csr: exactly one of HUGE_HOST_PTRS / HUGE_DEVICE_PTRS");

    DevBuf b_rp0, b_col0;
    const int64_t *rp0 = rp_in;
    const int32_t *col0 = col_in;
    if (host) {
        int64_t *r = b_rp0.alloc<int64_t>(n + 1);
        int32_t *c = b_col0.alloc<int32_t>(nnz > 0 ? nnz : 1);
        HUGE_HIP(hipMemcpyAsync(r, rp_in, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
        if (nnz) HUGE_HIP(hipMemcpyAsync(c, col_in, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
        rp0 = r;
        col0 = c;
    }

    DevBuf b_small;
    // small control block: flags, dmax, hist[32], moments[8], digest
    char *small = b_small.alloc<char>(1024);
    uint32_t *d_flags = (uint32_t *)small;
    uint32_t *d_dmax = (uint32_t *)(small + 8);
    unsigned long long *d_hist = (unsigned long long *)(small + 64);
    double *d_mom = (double *)(small + 64 + 32 * 8);
    unsigned long long *d_digest = (unsigned long long *)(small + 64 + 32 * 8 + 8 * 8);
    unsigned long long *d_nhub = d_digest + 1;
    HUGE_HIP(hipMemsetAsync(small, 0, 1024, st));

    // ---- hygiene checks
    if (!(flags & HUGE_NO_VALIDATE)) {
        hipLaunchKernelGGL(k_check_rowptr, dim3(grid_for(n + 1, kT)), dim3(kT), 0, st, rp0, n, nnz, d_flags);
        uint32_t hf = 0;
        HUGE_HIP(hipMemcpyAsync(&hf, d_flags, 4, hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        if (hf) HUGE_FAIL(HUGE_EGRAPH, "huge_load_csr: row_ptr is not a valid offset array");
        if (nnz) {
            hipLaunchKernelGGL(k_check_edges, dim3(grid_for(n, kT)), dim3(kT), 0, st, rp0, col0, n, d_flags);
            HUGE_HIP(hipMemcpyAsync(&hf, d_flags, 4, hipMemcpyDeviceToHost, st));
            HUGE_HIP(hipStreamSynchronize(st));
            if (hf) {
                const char *why = (hf & BAD_RANGE)  ? "a column ID is out of range"
                                  : (hf & BAD_SELF) ? "self-loop"
                                  : (hf & BAD_ORDER) ? "an adjacency list is not strictly ascending (unsorted or duplicate)"
                                                     : "the graph is not symmetric";
                HUGE_FAIL(HUGE_EGRAPH, "huge_load_csr: %s", why);
            }
        }
    }

    // ---- degree rank: stable sort of (degree, id) pairs, ids ascending
    int64_t vn = n;
    int64_t hist_n = radix_sort_hist_elems(nnz > vn ? nnz : vn);
    DevBuf b_hist, b_offs, b_stmp;
    uint32_t *hist = b_hist.alloc<uint32_t>(hist_n);
    int64_t *offs = b_offs.alloc<int64_t>(hist_n);
    int64_t stmp_n = scan_tmp_elems(hist_n > vn + 1 ? hist_n : vn + 1);
    int64_t *stmp = b_stmp.alloc<int64_t>(stmp_n);

    DevBuf b_k0, b_v0, b_k1, b_v1;
    uint32_t *vk0 = b_k0.alloc<uint32_t>(vn), *vv0 = b_v0.alloc<uint32_t>(vn);
    uint32_t *vk1 = b_k1.alloc<uint32_t>(vn), *vv1 = b_v1.alloc<uint32_t>(vn);
    hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(vn, kT)), dim3(kT), 0, st, rp0, vn, vk0, vv0, d_dmax, d_nhub);
    uint32_t dmax = 0;
    unsigned long long nhub = 0;
    HUGE_HIP(hipMemcpyAsync(&dmax, d_dmax, 4, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(&nhub, d_nhub, 8, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    int dbits = 0;
    while (dbits < 32 && (dmax >> dbits)) ++dbits;
    bool fl = radix_sort_pairs(vk0, vv0, vk1, vv1, vn, dbits, hist, offs, stmp, st);
    uint32_t *sdeg = fl ? vk1 : vk0, *sinv = fl ? vv1 : vv0;

    DevBuf b_rank, b_inv, b_nrp;
    int32_t *rank = b_rank.alloc<int32_t>(vn);
    int32_t *inv = b_inv.alloc<int32_t>(vn);
    int64_t *nrp = b_nrp.alloc<int64_t>(vn + 1);
    uint32_t *newdeg = fl ? vk0 : vk1;  // free buffer of the ping-pong pair
    hipLaunchKernelGGL(k_ranks, dim3(grid_for(vn, kT)), dim3(kT), 0, st, sdeg, sinv, vn, rank, inv, newdeg);
    scan_excl(newdeg, nrp, vn, nrp + vn, stmp, st);
    HUGE_HIP(hipGetLastError());

    // ---- relabelled, sorted adjacency lists
    DevBuf b_pk0, b_pv0, b_pk1, b_pv1;
    int64_t en = nnz > 0 ? nnz : 1;
    uint32_t *pk0 = b_pk0.alloc<uint32_t>(en), *pv0 = b_pv0.alloc<uint32_t>(en);
    uint32_t *pk1 = b_pk1.alloc<uint32_t>(en), *pv1 = b_pv1.alloc<uint32_t>(en);
    if (nnz) {
        hipLaunchKernelGGL(k_pairs, dim3(grid_for(vn, kT)), dim3(kT), 0, st, rp0, col0, vn, (const int32_t *)rank,
                           (const int64_t *)nrp, pk0, pv0);
    }
    int nbits = 0;
    while (nbits < 32 && ((uint64_t)(vn - 1) >> nbits)) ++nbits;
    bool pf = nnz ? radix_sort_pairs(pk0, pv0, pk1, pv1, nnz, nbits, hist, offs, stmp, st) : false;

    // ---- sketch and digest on the relabelled graph
    int64_t nbs = (vn + kT * 16 - 1) / (kT * 16);
    DevBuf b_part;
    double *part = b_part.alloc<double>(nbs * 8);
    hipLaunchKernelGGL(k_sketch, dim3((unsigned)nbs), dim3(kT), 0, st, (const int64_t *)nrp, vn, d_hist, part);
    hipLaunchKernelGGL(k_sketch_reduce, dim3(1), dim3(kT), 0, st, (const double *)part, nbs, d_mom);
    const int32_t *fcol = (const int32_t *)(pf ? pv1 : pv0);
    if (nnz)
        hipLaunchKernelGGL(k_digest, dim3(1024), dim3(kT), 0, st, fcol, nnz, d_digest);
    HUGE_HIP(hipGetLastError());

    huge_graph *g = new huge_graph();
    unsigned long long hh[32];
    double mom[8];
    unsigned long long dig = 0;
    HUGE_HIP(hipMemcpyAsync(hh, d_hist, sizeof(hh), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(mom, d_mom, sizeof(mom), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(&dig, d_digest, sizeof(dig), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));

    // keep: nrp, inv, final (keys = src, values = col); everything else is freed
    g->rp = (int64_t *)b_nrp.release();
    g->inv_rank = (int32_t *)b_inv.release();
    if (pf) {
        g->src = (int32_t *)b_pk1.release();
        g->col = (int32_t *)b_pv1.release();
    } else {
        g->src = (int32_t *)b_pk0.release();
        g->col = (int32_t *)b_pv0.release();
    }
    g->dev.n = n;
    g->dev.nnz = nnz;
    g->dev.rp = g->rp;
    g->dev.col = g->col;
    g->dev.src = g->src;

    // ---- hub bitmaps for the highest-degree ranks
    int64_t words = ((n + 127) / 128) * 4;  // rows padded to 16 bytes: block-cached readers load 4 words
    int64_t H = 0;
    if (!(flags & HUGE_NO_HUB_BITMAP) && nnz) {
        uint64_t budget = 16ull << 30;
        if (const char *e = getenv("HUGE_HUB_BYTES")) budget = strtoull(e, nullptr, 10);
        size_t fr = 0, tot = 0;
        HUGE_HIP(hipMemGetInfo(&fr, &tot));
        budget = std::min<uint64_t>(budget, fr / 4);
        H = std::min<int64_t>((int64_t)nhub, (int64_t)(budget / (4ull * words)));
    }
    g->dev.hub_words = words;
    g->dev.hub_base = (int32_t)(n - H);
    g->dev.hub_bm = nullptr;
    if (H > 0) {
        HUGE_HIP(hipMalloc(&g->hub_bm, 4ull * words * H));
        HUGE_HIP(hipMemsetAsync(g->hub_bm, 0, 4ull * words * H, st));
        hipLaunchKernelGGL(k_hub_bitmap, dim3((unsigned)H), dim3(kT), 0, st, (const int64_t *)g->rp,
                           (const int32_t *)g->col, (int64_t)(n - H), words, g->hub_bm);
        HUGE_HIP(hipGetLastError());
        int64_t dmin = 0;
        int64_t rp2[2];
        HUGE_HIP(hipMemcpyAsync(rp2, g->rp + (n - H), 16, hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        dmin = rp2[1] - rp2[0];
        g->dev.hub_bm = g->hub_bm;
        g->info.hub_min_degree = dmin;
    }
    g->info.hub_count = H;
    HUGE_HIP(hipGetDevice(&g->device));
    g->info.n = n;
    g->info.nnz = nnz;
    g->info.max_degree = dmax;
    for (int i = 0; i < 32; ++i) g->info.degree_hist[i] = hh[i];
    for (int i = 0; i < 8; ++i) g->info.degree_moments[i] = mom[i];
    g->info.device_bytes = (uint64_t)(n + 1) * 8 + (uint64_t)en * 8 + (uint64_t)n * 4 + 4ull * words * H;
    char buf[64];
    snprintf(buf, sizeof(buf), "%016llx-%lld-%lld", dig, (long long)n, (long long)nnz);
    g->sha = buf;
    auto t1 = std::chrono::steady_clock::now();
    g->info.load_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return g;
}

namespace {
// label of rank r = the label of the original vertex holding rank r
__global__ void k_rank_labels(const int32_t *__restrict__ inv_rank, const int32_t *__restrict__ in, int64_t n,
                              int32_t *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = in[inv_rank[r]];
}
}  // namespace

void graph_set_labels(huge_graph *g, const int32_t *labels, uint32_t flags, hipStream_t st) {
    const int64_t n = g->dev.n;
    if (!labels && n > 0) HUGE_FAIL(HUGE_EINVAL, "labels is NULL");
    HUGE_HIP(hipMalloc(&g->label, sizeof(int32_t) * (size_t)std::max<int64_t>(1, n)));
    if (n > 0) {
        const int32_t *in = labels;
        int32_t *tmp = nullptr;
        if (flags & HUGE_HOST_PTRS) {
            HUGE_HIP(hipMalloc(&tmp, sizeof(int32_t) * (size_t)n));
            HUGE_HIP(hipMemcpyAsync(tmp, labels, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st));
            in = tmp;
        }
        hipLaunchKernelGGL(k_rank_labels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g->inv_rank, in, n,
                           g->label);
        const hipError_t e = hipGetLastError();
        HUGE_HIP(hipStreamSynchronize(st));
        if (tmp) (void)hipFree(tmp);
        HUGE_HIP(e);
    }
    g->dev.label = g->label;
    g->info.device_bytes += 4ull * (uint64_t)n;
}

void graph_free(huge_graph *g) {
    if (!g) return;
    if (g->label) (void)hipFree(g->label);
    if (g->rp) (void)hipFree(g->rp);
    if (g->col) (void)hipFree(g->col);
    if (g->src) (void)hipFree(g->src);
    if (g->inv_rank) (void)hipFree(g->inv_rank);
    if (g->hub_bm) (void)hipFree(g->hub_bm);
    if (g->drp) (void)hipFree(g->drp);
    if (g->dcol) (void)hipFree(g->dcol);
    delete g;
}

}  // namespace huge
