// Directed data graphs (Section 2: the paper's techniques carry over to
// directed graphs).  The matcher runs on the undirected skeleton -- every pair
// joined by an arc in either direction, the graph huge_load_csr builds and
// relabels by degree rank -- and a directed query's edges are kept in their
// direction by looking each one up in the out-lists, relabelled by the same
// ranks, next to the skeleton's intersection.  Built on the host at load time
// (sort and merge per row), then copied to the device once.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace huge {

huge_graph *graph_load_directed(int64_t n, int64_t narcs, const int64_t *rp, const int32_t *col, uint32_t flags,
                                hipStream_t st) {
    if (!(flags & HUGE_HOST_PTRS) || (flags & HUGE_DEVICE_PTRS))
        HUGE_FAIL(HUGE_EINVAL, "huge_load_csr_directed reads host memory (HUGE_HOST_PTRS)");
    if (n < 1 || n >= 0x7FFFFFFF || narcs < 0 || narcs >= (int64_t)0x7FFFFFFF || !rp || (narcs > 0 && !col))
        HUGE_FAIL(HUGE_EINVAL, "huge_load_csr_directed: bad sizes or NULL pointers");
    if (rp[0] != 0 || rp[n] != narcs) HUGE_FAIL(HUGE_EGRAPH, "row_ptr must run from 0 to the arc count");
    for (int64_t u = 0; u < n; ++u) {
        if (rp[u + 1] < rp[u]) HUGE_FAIL(HUGE_EGRAPH, "row_ptr decreases at %lld", (long long)u);
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            const int32_t v = col[e];
            if (v < 0 || v >= n) HUGE_FAIL(HUGE_EGRAPH, "arc %lld: vertex out of range", (long long)e);
            if (v == u) HUGE_FAIL(HUGE_EGRAPH, "arc %lld is a self-loop", (long long)e);
            if (e > rp[u] && col[e - 1] >= v)
                HUGE_FAIL(HUGE_EGRAPH, "out-list of %lld is not strictly ascending", (long long)u);
        }
    }
    // the undirected skeleton: every arc both ways, each list sorted and merged
    std::vector<int64_t> srp((size_t)n + 1, 0);
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            ++srp[(size_t)u + 1];
            ++srp[(size_t)col[e] + 1];
        }
    for (int64_t u = 0; u < n; ++u) srp[(size_t)u + 1] += srp[(size_t)u];
    std::vector<int32_t> scol((size_t)srp[(size_t)n]);
    {
        std::vector<int64_t> fill(srp.begin(), srp.end() - 1);
        for (int64_t u = 0; u < n; ++u)
            for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
                scol[(size_t)fill[(size_t)u]++] = col[e];
                scol[(size_t)fill[(size_t)col[e]]++] = (int32_t)u;
            }
    }
    std::vector<int64_t> crp((size_t)n + 1, 0);
    int64_t w = 0;
    for (int64_t u = 0; u < n; ++u) {
        auto b = scol.begin() + srp[(size_t)u], e = scol.begin() + srp[(size_t)u + 1];
        std::sort(b, e);
        auto last = std::unique(b, e);
        for (auto it = b; it != last; ++it) scol[(size_t)w++] = *it;
        crp[(size_t)u + 1] = w;
    }
    scol.resize((size_t)w);
    huge_graph *g = graph_load(n, w, crp.data(), scol.data(), HUGE_HOST_PTRS | (flags & HUGE_NO_HUB_BITMAP), st);
    try {
        // the out-lists in rank IDs: row r holds the ranks of inv_rank[r]'s out-neighbours, ascending
        std::vector<int32_t> inv((size_t)n), rank((size_t)n);
        HUGE_HIP(hipMemcpyAsync(inv.data(), g->inv_rank, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        for (int64_t r = 0; r < n; ++r) rank[(size_t)inv[(size_t)r]] = (int32_t)r;
        std::vector<int64_t> drp((size_t)n + 1, 0);
        for (int64_t r = 0; r < n; ++r) {
            const int32_t u = inv[(size_t)r];
            drp[(size_t)r + 1] = drp[(size_t)r] + (rp[u + 1] - rp[u]);
        }
        std::vector<int32_t> dcol((size_t)std::max<int64_t>(1, narcs));
        for (int64_t r = 0; r < n; ++r) {
            const int32_t u = inv[(size_t)r];
            int64_t o = drp[(size_t)r];
            for (int64_t e = rp[u]; e < rp[u + 1]; ++e) dcol[(size_t)o++] = rank[(size_t)col[e]];
            std::sort(dcol.begin() + drp[(size_t)r], dcol.begin() + drp[(size_t)r + 1]);
        }
        HUGE_HIP(hipMalloc(&g->drp, sizeof(int64_t) * ((size_t)n + 1)));
        HUGE_HIP(hipMalloc(&g->dcol, sizeof(int32_t) * dcol.size()));
        HUGE_HIP(hipMemcpyAsync(g->drp, drp.data(), sizeof(int64_t) * drp.size(), hipMemcpyHostToDevice, st));
        HUGE_HIP(hipMemcpyAsync(g->dcol, dcol.data(), sizeof(int32_t) * dcol.size(), hipMemcpyHostToDevice, st));
        HUGE_HIP(hipStreamSynchronize(st));
        g->dev.drp = g->drp;
        g->dev.dcol = g->dcol;
        g->directed = true;
        g->info.device_bytes += sizeof(int64_t) * drp.size() + sizeof(int32_t) * dcol.size();
    } catch (...) {
        graph_free(g);
        throw;
    }
    return g;
}

}  // namespace huge
