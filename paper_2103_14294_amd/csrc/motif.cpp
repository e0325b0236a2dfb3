// Motif counting (Section 6's graph-pattern-mining use: subgraph enumeration
// run over every pattern of interest, here every connected k-vertex pattern),
// with both readings of "occurrence" of Section 2: subgraphs isomorphic to the
// pattern (non-induced, what huge_count counts) and induced subgraphs.
//
// The non-induced counts come from one batch of queries (every connected
// k-vertex pattern up to isomorphism).  The induced counts follow from them
// exactly: a k-vertex set X whose induced subgraph G[X] is isomorphic to q
// holds c(p, q) subgraphs isomorphic to p, c(p, q) being the number of
// spanning subgraphs of q isomorphic to p, so
//     noninduced(p) = sum over connected q of c(p, q) * induced(q),
// a triangular system (c(p, q) = 0 unless q has more edges, c(q, q) = 1),
// solved from the densest pattern down in 64-bit integers.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace huge {

namespace {

constexpr int kMotifK = HUGE_MOTIF_KMAX;

struct Classes {
    int k = 0, npairs = 0;
    int pa[15] = {}, pb[15] = {};          // vertex pair of each edge bit
    std::vector<int32_t> cls;              // class of every labelled graph (edge mask), -1 disconnected
    std::vector<uint32_t> rep;             // representative mask of each class
    std::vector<std::vector<uint64_t>> c;  // c[p][q]: spanning subgraphs of q isomorphic to p
};

bool connected_mask(const Classes &C, uint32_t m) {
    int adj[kMotifK] = {};
    for (int e = 0; e < C.npairs; ++e)
        if ((m >> e) & 1u) {
            adj[C.pa[e]] |= 1 << C.pb[e];
            adj[C.pb[e]] |= 1 << C.pa[e];
        }
    int seen = 1, frontier = 1;
    while (frontier) {
        int next = 0;
        for (int v = 0; v < C.k; ++v)
            if ((frontier >> v) & 1) next |= adj[v];
        next &= ~seen;
        seen |= next;
        frontier = next;
    }
    return seen == (1 << C.k) - 1;
}

// Connected graphs on k vertices by isomorphism class: the class of a labelled
// graph is found through its smallest relabelled edge mask over all k!
// permutations; classes are numbered by (edges, smallest mask).
void build_classes(Classes &C, int k) {
    C.k = k;
    C.npairs = 0;
    for (int b = 1; b < k; ++b)
        for (int a = 0; a < b; ++a) {
            C.pa[C.npairs] = a;
            C.pb[C.npairs] = b;
            ++C.npairs;
        }
    int bit[kMotifK][kMotifK] = {};
    for (int e = 0; e < C.npairs; ++e) bit[C.pa[e]][C.pb[e]] = bit[C.pb[e]][C.pa[e]] = e;
    std::vector<int> perm(k);
    std::vector<std::vector<int>> perms;
    for (int i = 0; i < k; ++i) perm[i] = i;
    do perms.push_back(perm);
    while (std::next_permutation(perm.begin(), perm.end()));
    const uint32_t nm = 1u << C.npairs;
    std::vector<uint32_t> canon(nm, 0);
    std::vector<uint32_t> reps;
    for (uint32_t m = 1; m < nm; ++m) {
        if (!connected_mask(C, m)) continue;
        uint32_t best = UINT32_MAX;
        for (auto &p : perms) {
            uint32_t r = 0;
            for (int e = 0; e < C.npairs; ++e)
                if ((m >> e) & 1u) r |= 1u << bit[p[C.pa[e]]][p[C.pb[e]]];
            best = std::min(best, r);
        }
        canon[m] = best;
        if (best == m) reps.push_back(m);
    }
    std::stable_sort(reps.begin(), reps.end(), [](uint32_t a, uint32_t b) {
        const int ea = __builtin_popcount(a), eb = __builtin_popcount(b);
        return ea != eb ? ea < eb : a < b;
    });
    C.rep = reps;
    std::vector<int32_t> idx(nm, -1);
    for (size_t i = 0; i < reps.size(); ++i) idx[reps[i]] = (int32_t)i;
    C.cls.assign(nm, -1);
    if (k == 1) return;
    for (uint32_t m = 1; m < nm; ++m)
        if (canon[m]) C.cls[m] = idx[canon[m]];
    // c[p][q]: the connected spanning subgraphs of q's representative, by class
    const size_t nc = reps.size();
    C.c.assign(nc, std::vector<uint64_t>(nc, 0));
    for (size_t q = 0; q < nc; ++q) {
        const uint32_t mq = reps[q];
        for (uint32_t s = mq;; s = (s - 1) & mq) {  // every subset of q's edges
            if (s && C.cls[s] >= 0) C.c[(size_t)C.cls[s]][q] += 1;
            if (s == 0) break;
        }
    }
}

const Classes &classes(int k) {
    static Classes cache[kMotifK + 1];
    static std::once_flag once[kMotifK + 1];
    std::call_once(once[k], [k] { build_classes(cache[k], k); });
    return cache[k];
}

}  // namespace

int motif_count(const huge_graph *g, int k, const huge_exec_opts &o, huge_motif *out) {
    if (k < 2 || k > kMotifK) HUGE_FAIL(HUGE_EINVAL, "motif counting takes 2..%d vertices (k=%d)", kMotifK, k);
    if (o.slice_count > 1 || o.slice2_count > 1)
        HUGE_FAIL(HUGE_EINVAL, "motif counting needs the whole graph: induced counts mix every pattern's matches");
    if (o.work_limit) HUGE_FAIL(HUGE_EINVAL, "motif counting has no work limit");
    const Classes &C = classes(k);
    const int nc = (int)C.rep.size();
    std::vector<huge_plan> plans(nc);
    std::vector<const huge_plan *> pp(nc);
    for (int i = 0; i < nc; ++i) {
        int32_t qe[2 * 15];
        int ne = 0;
        for (int e = 0; e < C.npairs; ++e)
            if ((C.rep[i] >> e) & 1u) {
                qe[2 * ne] = C.pa[e];
                qe[2 * ne + 1] = C.pb[e];
                ++ne;
            }
        plan_build(g, k, ne, qe, nullptr, HUGE_PLAN_COST_MODEL, nullptr, nullptr, &plans[i]);
        pp[i] = &plans[i];
        memset(&out[i], 0, sizeof(out[i]));
        out[i].k = k;
        out[i].n_edges = ne;
        for (int j = 0; j < 2 * ne; ++j) out[i].edges[j] = qe[j];
    }
    std::vector<huge_result> r(nc);
    if (o.engine == HUGE_ENGINE_GRAPH) {
        for (int i = 0; i < nc; i += kMaxBatch) run_mgraph(g, pp.data() + i, std::min(kMaxBatch, nc - i), o, &r[i]);
    } else {
        run_batch_levels(g, pp.data(), nc, o, r.data());
    }
    for (int i = 0; i < nc; ++i) {
        out[i].noninduced = r[i].count;
        out[i].hash_sum = r[i].hash_sum;
        out[i].hash_xor = r[i].hash_xor;
    }
    // induced counts, densest pattern first (classes are ordered by edge count)
    for (int q = nc - 1; q >= 0; --q) {
        uint64_t v = out[q].noninduced;
        for (int s = q + 1; s < nc; ++s) v -= C.c[(size_t)q][(size_t)s] * out[s].induced;
        out[q].induced = v;
    }
    return nc;
}

}  // namespace huge
