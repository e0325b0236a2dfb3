// Query planning (host): validation, automorphisms, symmetry-breaking
// constraints, matching orders, the PULL-EXTEND step table and the plain
// cost-model plan.
//
// The execution plan is the worst-case-optimal left-deep chain of Section 3.1
// (BiGJoin as complete star joins on induced prefixes, Definition 3.1): for a
// matching order pi, step i extends partial matches of the induced prefix
// {pi_0..pi_{i-1}} by pi_i, intersecting the neighbour lists of the matched
// vertices adjacent to pi_i (Eq. 2, PULL-EXTEND's extend index in Section 4.2).
// Every step is a complete star join, which Eq. 3 sets to (wco join, pull).
//
// Cost model: Algorithm 1's cost of a plan is the sum of the result sizes of
// its joins plus communication; for left-deep wco plans on one device the
// communication term is the same for every order and drops out, leaving
// cost(pi) = sum over prefixes of |R(prefix)|.  The paper leaves the
// cardinality estimator open; this one uses the Chung-Lu expected-degree
// model: the expected number of injective maps of a pattern H is
// prod_v M_{deg_H(v)} / (2m)^{|E_H|} with M_p = sum_u d_u^p, scaled by the
// fraction of vertex orderings of H that satisfy the symmetry-breaking
// constraints inside H.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace huge {

namespace {

void check_query(int k, int ne, const int32_t *qe, huge_plan *p) {
    if (k < 2 || k > HUGE_KMAX) HUGE_FAIL(HUGE_EQUERY, "query must have 2..8 vertices (k=%d)", k);
    if (ne < 1 || ne > k * (k - 1) / 2 || !qe) HUGE_FAIL(HUGE_EQUERY, "bad number of query edges (%d)", ne);
    memset(p->adj, 0, sizeof(p->adj));
    p->edges.clear();
    for (int i = 0; i < ne; ++i) {
        int a = qe[2 * i], b = qe[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k) HUGE_FAIL(HUGE_EQUERY, "query edge %d has a vertex out of range", i);
        if (a == b) HUGE_FAIL(HUGE_EQUERY, "query edge %d is a self-loop", i);
        if (p->adj[a][b]) HUGE_FAIL(HUGE_EQUERY, "query edge %d is a duplicate", i);
        p->adj[a][b] = p->adj[b][a] = 1;
        p->edges.push_back({std::min(a, b), std::max(a, b)});
    }
    // connected?
    int seen = 1, stack[HUGE_KMAX], sp = 0;
    stack[sp++] = 0;
    int mark[HUGE_KMAX] = {1};
    while (sp) {
        int a = stack[--sp];
        for (int b = 0; b < k; ++b)
            if (p->adj[a][b] && !mark[b]) {
                mark[b] = 1;
                ++seen;
                stack[sp++] = b;
            }
    }
    if (seen != k) HUGE_FAIL(HUGE_EQUERY, "query is not connected");
    p->k = k;
}

// Automorphism group by testing every permutation (k <= 8); a labelled query's
// automorphisms also keep every vertex's label (-1 counts as a label of its own),
// a directed query's every edge's direction.
std::vector<std::vector<int8_t>> automorphisms(const huge_plan &p) {
    std::vector<std::vector<int8_t>> out;
    std::vector<int8_t> perm(p.k);
    for (int i = 0; i < p.k; ++i) perm[i] = (int8_t)i;
    do {
        bool ok = true;
        for (auto &e : p.edges)
            if (!p.adj[perm[e.first]][perm[e.second]]) {
                ok = false;
                break;
            }
        for (int v = 0; v < p.k && ok; ++v)
            if (p.qlabel[perm[v]] != p.qlabel[v]) ok = false;
        for (int a = 0; a < p.k && ok && p.directed; ++a)  // a directed query's keep directions
            for (int b = 0; b < p.k && ok; ++b)
                if (p.dadj[perm[a]][perm[b]] != p.dadj[a][b]) ok = false;
        if (ok) out.push_back(perm);
    } while (std::next_permutation(perm.begin(), perm.end()));
    return out;
}

// Grochow-Kellis symmetry breaking (RECOMB 2007): repeatedly pick, among the
// vertices with the largest orbit under the remaining group, the one with the
// smallest ID; constrain it below the rest of its orbit; keep its stabiliser.
void grochow_kellis(huge_plan &p) {
    auto group = automorphisms(p);
    p.naut = (int32_t)group.size();
    p.sb.clear();
    while (group.size() > 1) {
        int best = -1;
        size_t best_sz = 0;
        std::vector<int> best_orbit;
        for (int v = 0; v < p.k; ++v) {
            bool in[HUGE_KMAX] = {};
            for (auto &s : group) in[(int)s[v]] = true;
            std::vector<int> orb;
            for (int w = 0; w < p.k; ++w)
                if (in[w]) orb.push_back(w);
            if (orb.size() > best_sz) {
                best_sz = orb.size();
                best = v;
                best_orbit = orb;
            }
        }
        for (int w : best_orbit)
            if (w != best) p.sb.push_back({best, w});
        std::vector<std::vector<int8_t>> stab;
        for (auto &s : group)
            if (s[best] == best) stab.push_back(s);
        group.swap(stab);
    }
}

// Fraction of the |S|! orderings of the vertex set S that satisfy every
// constraint with both ends in S.
double sb_fraction(const huge_plan &p, const int32_t *verts, int m) {
    std::vector<std::pair<int, int>> cons;
    for (auto &c : p.sb) {
        int ia = -1, ib = -1;
        for (int i = 0; i < m; ++i) {
            if (verts[i] == c.first) ia = i;
            if (verts[i] == c.second) ib = i;
        }
        if (ia >= 0 && ib >= 0) cons.push_back({ia, ib});
    }
    if (cons.empty()) return 1.0;
    std::vector<int> perm(m);  // perm[i] = rank position of local vertex i
    for (int i = 0; i < m; ++i) perm[i] = i;
    long long good = 0, tot = 0;
    do {
        ++tot;
        bool ok = true;
        for (auto &c : cons)
            if (perm[c.first] > perm[c.second]) {
                ok = false;
                break;
            }
        if (ok) ++good;
    } while (std::next_permutation(perm.begin(), perm.end()));
    return (double)good / (double)tot;
}

}  // namespace

bool order_connected(const huge_plan &p, const int32_t *order) {
    bool used[HUGE_KMAX] = {};
    for (int i = 0; i < p.k; ++i) {
        if (order[i] < 0 || order[i] >= p.k || used[order[i]]) return false;
        used[order[i]] = true;
    }
    for (int i = 1; i < p.k; ++i) {
        bool adj = false;
        for (int j = 0; j < i; ++j) adj |= p.adj[order[j]][order[i]] != 0;
        if (!adj) return false;
    }
    return true;
}

void all_connected_orders(const huge_plan &p, std::vector<std::vector<int32_t>> &out) {
    out.clear();
    std::vector<int32_t> perm(p.k);
    for (int i = 0; i < p.k; ++i) perm[i] = i;
    do {
        if (order_connected(p, perm.data())) out.push_back(perm);
    } while (std::next_permutation(perm.begin(), perm.end()));
}

// Estimated partial matches of the induced prefix order[0..size-1].
double estimate_prefix(const huge_graph_info &gi, const huge_plan &p, const int32_t *order, int size) {
    double two_m = (double)gi.nnz;
    if (gi.n <= 0) return 0;  // no graph statistics (host-only planning)
    if (two_m <= 0) return 0;
    double logv = 0;
    int ne = 0;
    for (int i = 0; i < size; ++i) {
        int dv = 0;
        for (int j = 0; j < size; ++j) dv += p.adj[order[i]][order[j]];
        double M = gi.degree_moments[dv < 8 ? dv : 7];
        if (M <= 0) return 0;
        logv += std::log(M);
    }
    for (int i = 0; i < size; ++i)
        for (int j = i + 1; j < size; ++j) ne += p.adj[order[i]][order[j]];
    logv -= ne * std::log(two_m);
    double f = sb_fraction(p, order, size);
    return std::exp(logv) * f;
}

void plan_set_order(huge_plan &p, const int32_t *order) {
    const int k = p.k;
    for (int i = 0; i < k; ++i) p.order[i] = order[i];
    DevPlan &d = p.dev;
    memset(&d, 0, sizeof(d));
    d.k = k;
    int pos[HUGE_KMAX];
    for (int i = 0; i < k; ++i) pos[order[i]] = i;
    for (int v = 0; v < k; ++v) d.pos[v] = (uint8_t)pos[v];
    d.ne = (int32_t)p.edges.size();
    for (size_t e = 0; e < p.edges.size(); ++e) {
        int a = pos[p.edges[e].first], b = pos[p.edges[e].second];
        d.ea[e] = (uint8_t)std::min(a, b);
        d.eb[e] = (uint8_t)std::max(a, b);
    }
    for (int i = 1; i < k; ++i) {
        DevStep &s = d.st[i];
        for (int j = 0; j < i; ++j) {
            if (p.adj[order[j]][order[i]]) s.ext |= 1u << j;
        }
        s.neq = ((1u << i) - 1) & ~s.ext;
        s.nadj = p.induced ? s.neq : 0u;
        if (p.directed)
            for (int j = 0; j < i; ++j) {
                if (p.dadj[order[j]][order[i]]) s.dout |= 1u << j;
                if (p.dadj[order[i]][order[j]]) s.din |= 1u << j;
            }
        s.slice = order[i] == 0 ? 1 : 0;
        for (auto &c : p.sb) {
            int pa = pos[c.first], pb = pos[c.second];
            // constraint f(first) < f(second), checked when the later one is placed
            if (pb == i && pa < i) s.lo |= 1u << pa;
            if (pa == i && pb < i) s.hi |= 1u << pb;
        }
    }
    // position 0's slice flag lives in st[0]
    d.st[0].slice = order[0] == 0 ? 1 : 0;
    for (int i = 0; i < k; ++i) d.st[i].label = p.qlabel[order[i]];
    p.est_cost = 0;
    for (int s = 1; s <= k; ++s) p.est_prefix[s - 1] = 0;
    return;
}

constexpr double kLearnedMargin = 2.0;
constexpr int kVerifyCandidates = 2;                 // the model's best orders measured, besides the cost model's
constexpr int64_t kVerifyWork = 40000000;            // candidates of the cost model's order on the sample
constexpr double kVerifyRelLimit = 3.0;              // other orders stop at this multiple of its candidates
constexpr double kVerifyGain = 1.1;                  // a measured order must be this much faster to be kept

double order_cost(const std::vector<double> &e, size_t o, int k) {
    double c = 0;
    for (int s = 2; s <= k; ++s) c += e[o * k + s - 1];
    return c;
}

// Measured choice among the model's kVerifyCandidates best orders and the cost
// model's order.  Each runs the query on edge slice 0 of S of its own first
// matched pair: the matches whose first two vertices sit at an entry e of the
// relabelled CSR with e % S == 0.  That is every S-th entry of every adjacency
// list, so hubs are sampled in proportion to their degree, the engines read
// only those entries, and the sample is an unbiased 1/S share of that order's
// work.  S is the smallest power of 8 (from 2^9) at which the cost model's
// order examines at most kVerifyWork candidates.  When no edge sample with at
// least 64 entries fits (single hub entries of the query hold more), the
// samples are strided root slices instead (slice 0 of S of the first matched
// vertex by degree rank, at least 4 roots).  The other orders stop (and lose)
// past kVerifyRelLimit times the cost model's candidates.  An order must beat
// the cost model's device time by kVerifyGain; among those within kVerifyGain of
// the fastest (a tie on one sample), the one sharing the longest prefix with the
// cost model's order wins, then the faster.
// About a few milliseconds of device time per order.
size_t verify_orders(const huge_graph *g, const huge_plan &p, const std::vector<std::vector<int32_t>> &orders,
                     const std::vector<double> &est, const huge_graph_info &gi, hipStream_t st) {
    const int k = p.k;
    std::vector<size_t> idx(orders.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](size_t a, size_t b) { return order_cost(est, a, k) < order_cost(est, b, k); });
    std::vector<size_t> cand(idx.begin(), idx.begin() + std::min<size_t>(kVerifyCandidates, idx.size()));
    size_t base = 0;
    double bc = INFINITY;
    for (size_t o = 0; o < orders.size(); ++o) {
        double c = 0;
        for (int s = 2; s <= k; ++s) c += estimate_prefix(gi, p, orders[o].data(), s);
        if (c < bc * (1 - 1e-12)) {
            bc = c;
            base = o;
        }
    }
    // the cost model's order first
    cand.erase(std::remove(cand.begin(), cand.end(), base), cand.end());
    cand.insert(cand.begin(), base);
    if (cand.size() == 1) return base;
    huge_exec_opts o;
    huge_exec_opts_default(&o);
    o.stream = st;
    o.slice_count = 512;
    o.slice_id = 0;
    o.slice_vertex = -2;
    o.slice_mode = HUGE_SLICE_STRIDE;
    o.work_limit = kVerifyWork;
    o.exec_flags = HUGE_EXEC_NO_HASH;
    o.profile = 1;
    std::vector<huge_plan> qs(cand.size(), p);
    for (size_t i = 0; i < cand.size(); ++i) plan_set_order(qs[i], orders[cand[i]].data());
    struct Mem {
        void *p = nullptr;
        ~Mem() {
            if (p) (void)hipFree(p);
        }
    } mem;
    uint64_t wsb = 0;
    auto ensure_ws = [&]() {
        uint64_t need = 256;
        for (size_t i = 0; i < cand.size(); ++i) need = std::max(need, workspace_bytes(g, &qs[i], o));
        if (need > wsb) {
            if (mem.p) HUGE_HIP(hipFree(mem.p));
            mem.p = nullptr;
            HUGE_HIP(hipMalloc(&mem.p, need));
            wsb = need;
        }
        o.workspace = mem.p;
        o.workspace_bytes = wsb;
    };
    auto device_ms = [](const huge_result &r) {
        double ms = 0;
        for (int c = 0; c < 4; ++c) ms += r.kernel_ms[c];
        return ms;
    };
    huge_result r0;
    for (;;) {
        ensure_ws();
        if (!run_levels(g, &qs[0], o, &r0, nullptr)) break;
        if (o.slice_vertex == -2 && (int64_t)o.slice_count * 8 > g->dev.nnz / 64) {
            // single entries hold more than the budget: strided root slices instead
            o.slice_vertex = -1;
            o.slice_count = 512;
            continue;
        }
        if (o.slice_vertex == -1 && (int64_t)o.slice_count * 8 > std::max<int64_t>(gi.n / 4, 1)) return base;
        o.slice_count *= 8;
    }
    double base_work = 0;
    for (int i = 0; i < HUGE_KMAX; ++i) base_work += (double)r0.level_work[i];
    const double base_ms = device_ms(r0);
    o.work_limit = (int64_t)std::max(1.0, std::min(9.0e18, kVerifyRelLimit * base_work));
    // the orders that beat the cost model's by kVerifyGain, with their times
    std::vector<std::pair<size_t, double>> won;
    double best_ms = INFINITY;
    for (size_t i = 1; i < cand.size(); ++i) {
        huge_result r;
        if (run_levels(g, &qs[i], o, &r, nullptr)) continue;
        const double ms = device_ms(r);
        if (ms * kVerifyGain < base_ms) {
            won.push_back({cand[i], ms});
            best_ms = std::min(best_ms, ms);
        }
    }
    // orders within kVerifyGain of the fastest are a tie on this sample: the one
    // sharing the longest prefix with the cost model's order wins it (the least
    // departure from the baseline), then the faster
    size_t best = base;
    int best_pre = -1;
    double best_t = INFINITY;
    for (const auto &w : won) {
        if (w.second > best_ms * kVerifyGain) continue;
        int pre = 0;
        while (pre < k && orders[w.first][pre] == orders[base][pre]) ++pre;
        if (pre > best_pre || (pre == best_pre && w.second < best_t)) {
            best = w.first;
            best_pre = pre;
            best_t = w.second;
        }
    }
    return best;
}

void check_labels(const huge_graph *g, const huge_plan *p) {
    if (p->labelled && !g->label) HUGE_FAIL(HUGE_EINVAL, "a labelled query needs a labelled graph (huge_load_csr_labelled)");
    if (p->directed && !g->directed)
        HUGE_FAIL(HUGE_EINVAL, "a directed query needs a directed graph (huge_load_csr_directed)");
}

void plan_build(const huge_graph *g, int k, int ne, const int32_t *qe, const int32_t *order, uint32_t flags,
                const huge_model *model, hipStream_t st, huge_plan *p, const int32_t *qlabels, int narcs,
                const int32_t *arcs) {
    static const huge_graph_info no_stats{};
    const huge_graph_info &gi = g ? g->info : no_stats;
    const bool learned = (flags & HUGE_PLAN_LEARNED) != 0;
    if (learned && (!model || !g)) HUGE_FAIL(HUGE_EINVAL, "a learned plan needs a graph and a model");
    check_query(k, ne, qe, p);
    for (int i = 0; i < HUGE_KMAX; ++i) p->qlabel[i] = -1;
    p->labelled = false;
    if (qlabels)
        for (int i = 0; i < k; ++i) {
            if (qlabels[i] < -1) HUGE_FAIL(HUGE_EQUERY, "query label %d of vertex %d is below -1", qlabels[i], i);
            p->qlabel[i] = qlabels[i];
            p->labelled |= qlabels[i] >= 0;
        }
    p->directed = arcs != nullptr;
    memset(p->dadj, 0, sizeof(p->dadj));
    for (int i = 0; i < narcs && arcs; ++i) {
        const int a = arcs[2 * i], b = arcs[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || !p->adj[a][b])
            HUGE_FAIL(HUGE_EQUERY, "directed edge %d is not an edge of the skeleton", i);
        if (p->dadj[a][b]) HUGE_FAIL(HUGE_EQUERY, "directed edge %d is a duplicate", i);
        p->dadj[a][b] = 1;
    }
    grochow_kellis(*p);
    if (flags & HUGE_PLAN_ALL_MAPS) p->sb.clear();  // every injective map
    p->flags = flags;
    p->induced = (flags & HUGE_PLAN_INDUCED) != 0;
    std::vector<std::vector<int32_t>> orders;
    if (order) {
        if (!order_connected(*p, order))
            HUGE_FAIL(HUGE_EORDER, "order is not a permutation of 0..k-1 with connected prefixes");
        orders.emplace_back(order, order + k);
    } else {
        all_connected_orders(*p, orders);  // lexicographic
    }
    // estimated |R(prefix_s)| of every candidate order, s = 1..k
    std::vector<double> est(orders.size() * (size_t)k, 0.0);
    if (learned) {
        learned_estimates(g, model, *p, orders, st, est);
    } else {
        for (size_t o = 0; o < orders.size(); ++o)
            for (int s = 1; s <= k; ++s) est[o * k + s - 1] = estimate_prefix(gi, *p, orders[o].data(), s);
    }
    // minimum estimated cost, ties to the lexicographically smallest order
    auto argmin = [&](const std::vector<double> &e) {
        size_t ch = 0;
        double best = INFINITY;
        for (size_t o = 0; o < orders.size(); ++o) {
            double c = 0;
            for (int s = 2; s <= k; ++s) c += e[o * k + s - 1];
            if (c < best * (1 - 1e-12)) {
                best = c;
                ch = o;
            }
        }
        return ch;
    };
    size_t chosen = argmin(est);
    if (learned && (flags & HUGE_PLAN_VERIFY) && orders.size() > 1) {
        chosen = verify_orders(g, *p, orders, est, gi, st);
    } else if (learned && orders.size() > 1) {
        // the learned choice replaces the cost model's only when the model itself
        // predicts at least kLearnedMargin times less work for it: the minimum of many
        // noisy estimates is biased low, so small predicted gains are not trusted
        std::vector<double> cm(orders.size() * (size_t)k, 0.0);
        for (size_t o = 0; o < orders.size(); ++o)
            for (int s = 1; s <= k; ++s) cm[o * k + s - 1] = estimate_prefix(gi, *p, orders[o].data(), s);
        const size_t base = argmin(cm);
        double c_base = 0, c_best = 0;
        for (int s = 2; s <= k; ++s) {
            c_base += est[base * k + s - 1];
            c_best += est[chosen * k + s - 1];
        }
        if (!(c_best * kLearnedMargin < c_base)) chosen = base;
    }
    plan_set_order(*p, orders[chosen].data());
    p->est_cost = 0;
    for (int s = 1; s <= k; ++s) {
        p->est_prefix[s - 1] = est[chosen * k + s - 1];
        if (s >= 2) p->est_cost += p->est_prefix[s - 1];
    }
    p->model_batch = learned;  // est holds the model's predictions for every candidate order
}

void plan_prefix(const huge_plan &p, int size, huge_plan *q) {
    int pos[HUGE_KMAX];
    for (int i = 0; i < p.k; ++i) pos[p.order[i]] = i;
    q->k = size;
    q->flags = p.flags;
    q->induced = p.induced;
    q->labelled = p.labelled;
    for (int i = 0; i < HUGE_KMAX; ++i) q->qlabel[i] = -1;
    for (int v = 0; v < p.k; ++v)
        if (pos[v] < size) q->qlabel[pos[v]] = p.qlabel[v];
    q->naut = 0;
    memset(q->adj, 0, sizeof(q->adj));
    q->directed = p.directed;
    memset(q->dadj, 0, sizeof(q->dadj));
    for (int a = 0; a < p.k; ++a)
        for (int b = 0; b < p.k; ++b)
            if (p.dadj[a][b] && pos[a] < size && pos[b] < size) q->dadj[pos[a]][pos[b]] = 1;
    q->edges.clear();
    for (auto &e : p.edges) {
        const int a = pos[e.first], b = pos[e.second];
        if (a < size && b < size) {
            q->edges.push_back({std::min(a, b), std::max(a, b)});
            q->adj[a][b] = q->adj[b][a] = 1;
        }
    }
    std::sort(q->edges.begin(), q->edges.end());
    q->sb.clear();
    for (auto &c : p.sb) {
        const int a = pos[c.first], b = pos[c.second];
        if (a < size && b < size) q->sb.push_back({a, b});
    }
    int32_t ident[HUGE_KMAX];
    for (int i = 0; i < size; ++i) ident[i] = i;
    plan_set_order(*q, ident);
    q->est_cost = 0;
    for (int s = 1; s <= size; ++s) {
        q->est_prefix[s - 1] = p.est_prefix[s - 1];
        if (s >= 2) q->est_cost += q->est_prefix[s - 1];
    }
}

}  // namespace huge
