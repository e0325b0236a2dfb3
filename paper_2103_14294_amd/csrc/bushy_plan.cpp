// Bushy execution plans: Algorithm 1 (OptimalExecutionPlan, Section 3.3) over
// the join-based framework of Section 3.1, with the physical settings of the
// settings equation (Section 3.3) and stars as the join unit.
//
// A sub-query q' is a connected set of query edges (bit e = the e-th query
// edge).  Stars -- every edge at one centre -- are join units, costed at their
// estimated result size.  Any other q' is a two-way join (q', l, r) of two
// connected, edge-disjoint parts with l | r = q', each part costed by the
// table, plus |R(q')|, plus the join's communication:
//   pulling (r a star (c; L) with L inside V(l), or with c inside V(l)):
//       machines * |E_G|, the graph pulled by every machine (Remark 3.3);
//   pushing (every other join): |R(l)| + |R(r)|, both sides shuffled.
// `machines` is Algorithm 1's k (1 for one GPU).  The table is filled by
// increasing edge count, so both parts of every join are final when a
// sub-query is reached; a later split replaces the kept one only when strictly
// cheaper.  The recovered tree keeps, for every join, the star as the right
// part (joins are commutative, and both orders of every split are tried).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace huge {

namespace {

struct Sub {
    uint32_t vmask = 0;
    bool conn = false;
    int centre = -1;  // stars: the centre (single edges: the lower endpoint); -1 not a star
    double est = 0, cost = INFINITY;
    int kind = -1, root = -1;
    uint32_t left = 0, right = 0;
};

// Chung-Lu estimate of the matches of the edge set `em` that satisfy the
// symmetry-breaking constraints with both ends among its vertices: the product
// over its vertices v of M_{deg(v)} over (2m)^{edges}, times the fraction of
// the vertex orderings that satisfy those constraints.
double estimate_edges(const huge_graph_info &gi, const huge_plan &p, uint32_t em) {
    const double two_m = (double)gi.nnz;
    if (gi.n <= 0 || two_m <= 0) return 0;
    int deg[HUGE_KMAX] = {};
    int ne = 0;
    for (size_t e = 0; e < p.edges.size(); ++e)
        if ((em >> e) & 1u) {
            ++deg[p.edges[e].first];
            ++deg[p.edges[e].second];
            ++ne;
        }
    double logv = 0;
    int32_t verts[HUGE_KMAX];
    int m = 0;
    for (int v = 0; v < p.k; ++v)
        if (deg[v]) {
            const double M = gi.degree_moments[deg[v] < 8 ? deg[v] : 7];
            if (M <= 0) return 0;
            logv += std::log(M);
            verts[m++] = v;
        }
    logv -= ne * std::log(two_m);
    // fraction of orderings of verts satisfying the constraints inside them
    std::vector<std::pair<int, int>> cons;
    for (auto &c : p.sb) {
        int ia = -1, ib = -1;
        for (int i = 0; i < m; ++i) {
            if (verts[i] == c.first) ia = i;
            if (verts[i] == c.second) ib = i;
        }
        if (ia >= 0 && ib >= 0) cons.push_back({ia, ib});
    }
    double frac = 1.0;
    if (!cons.empty()) {
        std::vector<int> perm(m);
        for (int i = 0; i < m; ++i) perm[i] = i;
        long long good = 0, tot = 0;
        do {
            ++tot;
            bool ok = true;
            for (auto &c : cons) ok = ok && perm[c.first] < perm[c.second];
            good += ok;
        } while (std::next_permutation(perm.begin(), perm.end()));
        frac = (double)good / (double)tot;
    }
    return std::exp(logv) * frac;
}

}  // namespace

namespace {

// Every connected edge set of q with its vertices, star centre and estimate.
std::vector<Sub> sub_table(const huge_graph_info &gi, const huge_plan &p) {
    const int ne = (int)p.edges.size();
    const uint32_t full = (1u << ne) - 1;
    std::vector<Sub> t((size_t)full + 1);
    for (uint32_t m = 1; m <= full; ++m) {
        Sub &s = t[m];
        int deg[HUGE_KMAX] = {};
        for (int e = 0; e < ne; ++e)
            if ((m >> e) & 1u) {
                s.vmask |= (1u << p.edges[e].first) | (1u << p.edges[e].second);
                ++deg[p.edges[e].first];
                ++deg[p.edges[e].second];
            }
        // connected: grow from one vertex over the set's edges
        uint32_t seen = s.vmask & (~s.vmask + 1), grow = seen;
        while (grow) {
            uint32_t next = 0;
            for (int e = 0; e < ne; ++e)
                if ((m >> e) & 1u) {
                    const uint32_t ab = (1u << p.edges[e].first) | (1u << p.edges[e].second);
                    if (ab & grow) next |= ab;
                }
            grow = next & ~seen;
            seen |= next;
        }
        s.conn = seen == s.vmask;
        const int edges = __builtin_popcount(m);
        for (int v = 0; v < p.k && s.centre < 0; ++v)
            if (deg[v] == edges) s.centre = v;
        if (s.conn) s.est = estimate_edges(gi, p, m);
    }
    return t;
}

// The physical setting of the join (l | r, l, r) by the settings equation, the
// star read as the right part: a complete star join (centre outside l, leaves
// inside) extends; a star with its centre inside l is a pulled hash join;
// anything else is pushed.  Returns the kind and the star's centre (-1 pushed).
std::pair<int, int> classify(const huge_plan &p, const std::vector<Sub> &t, uint32_t l, uint32_t r) {
    const Sub &L = t[l], &R = t[r];
    if (R.centre < 0) return {HUGE_BUSHY_PUSH, -1};
    // the star's centre; a single edge may be read from either end
    int cands[2] = {R.centre, -1};
    if (__builtin_popcount(r) == 1) {
        const int e = __builtin_ctz(r);
        cands[0] = p.edges[e].first;
        cands[1] = p.edges[e].second;
    }
    for (int c : cands) {
        if (c < 0) continue;
        const uint32_t leaves = R.vmask & ~(1u << c);
        if (!((L.vmask >> c) & 1u) && (leaves & ~L.vmask) == 0) return {HUGE_BUSHY_EXTEND, c};
    }
    for (int c : cands)
        if (c >= 0 && ((L.vmask >> c) & 1u)) return {HUGE_BUSHY_PULL_HASH, c};
    return {HUGE_BUSHY_PUSH, -1};
}

double join_cost(const std::vector<Sub> &t, uint32_t m, uint32_t l, uint32_t r, int kind, double pull) {
    const double comm = kind == HUGE_BUSHY_PUSH ? t[l].est + t[r].est : pull;
    return t[l].cost + t[r].cost + t[m].est + comm;
}

// the tree from the chosen joins, children before parents, the root last
void recover(huge_plan &p, const std::vector<Sub> &t, uint32_t full) {
    p.bushy.clear();
    std::vector<int32_t> id(t.size(), -1);
    struct Rec {
        const std::vector<Sub> &t;
        std::vector<huge_bushy_node> &out;
        std::vector<int32_t> &id;
        int32_t go(uint32_t m) {
            if (id[m] >= 0) return id[m];
            const Sub &s = t[m];
            int32_t l = -1, r = -1;
            if (s.kind != HUGE_BUSHY_UNIT) {
                l = go(s.left);
                r = go(s.right);
            }
            huge_bushy_node nd;
            memset(&nd, 0, sizeof(nd));
            nd.edge_mask = m;
            nd.vertex_mask = s.vmask;
            nd.kind = s.kind;
            nd.left = l;
            nd.right = r;
            nd.star_root = s.kind == HUGE_BUSHY_PUSH ? -1 : s.root;
            nd.est_rows = s.est;
            nd.cost = s.cost;
            out.push_back(nd);
            return id[m] = (int32_t)out.size() - 1;
        }
    } rec{t, p.bushy, id};
    rec.go(full);
    // a pulled join's star: its centre as the unit's root too
    for (auto &nd : p.bushy)
        if (nd.kind == HUGE_BUSHY_EXTEND || nd.kind == HUGE_BUSHY_PULL_HASH) p.bushy[nd.right].star_root = nd.star_root;
}

void check_size(const huge_plan &p, double machines) {
    const int ne = (int)p.edges.size();
    if (ne > HUGE_BUSHY_MAX_EDGES)
        HUGE_FAIL(HUGE_EQUERY, "bushy planning takes at most %d query edges (%d)", HUGE_BUSHY_MAX_EDGES, ne);
    if (!(machines >= 0) || !std::isfinite(machines)) HUGE_FAIL(HUGE_EINVAL, "machines must be finite and >= 0");
}

}  // namespace

void plan_bushy(const huge_graph_info &gi, huge_plan &p, double machines) {
    check_size(p, machines);
    const uint32_t full = (1u << p.edges.size()) - 1;
    std::vector<Sub> t = sub_table(gi, p);
    const double pull = machines * (double)gi.nnz / 2.0;  // k |E_G|
    std::vector<uint32_t> masks;
    for (uint32_t m = 1; m <= full; ++m)
        if (t[m].conn) masks.push_back(m);
    std::stable_sort(masks.begin(), masks.end(),
                     [](uint32_t a, uint32_t b) { return __builtin_popcount(a) < __builtin_popcount(b); });
    for (uint32_t m : masks) {
        Sub &s = t[m];
        if (s.centre >= 0) {  // a join unit
            s.cost = s.est;
            s.kind = HUGE_BUSHY_UNIT;
            s.root = s.centre;
            continue;
        }
        for (uint32_t l = (m - 1) & m; l; l = (l - 1) & m) {
            const uint32_t r = m ^ l;
            if (!t[l].conn || !t[r].conn) continue;
            const auto kr = classify(p, t, l, r);
            const double c = join_cost(t, m, l, r, kr.first, pull);
            if (c < s.cost) {
                s.cost = c;
                s.kind = kr.first;
                s.root = kr.second;
                s.left = l;
                s.right = r;
            }
        }
    }
    recover(p, t, full);
}

void plan_bushy_tree(const huge_graph_info &gi, huge_plan &p, const uint32_t *splits, int nsplits, double machines) {
    check_size(p, machines);
    const uint32_t full = (1u << p.edges.size()) - 1;
    std::vector<Sub> t = sub_table(gi, p);
    const double pull = machines * (double)gi.nnz / 2.0;
    std::vector<std::pair<uint32_t, uint32_t>> sp;
    for (int i = 0; i < nsplits; ++i) {
        const uint32_t l = splits[2 * i], r = splits[2 * i + 1];
        if (!l || !r || (l & r) || ((l | r) & ~full)) HUGE_FAIL(HUGE_EORDER, "join %d: parts must be disjoint, non-empty edge sets", i);
        if (!t[l].conn || !t[r].conn) HUGE_FAIL(HUGE_EORDER, "join %d: both parts must be connected", i);
        for (auto &x : sp)
            if ((x.first | x.second) == (l | r)) HUGE_FAIL(HUGE_EORDER, "join %d splits a part split before", i);
        sp.push_back({l, r});
    }
    // bottom-up over the given tree: children have fewer edges than their parent
    int used = 0;
    struct Walk {
        const huge_plan &p;
        std::vector<Sub> &t;
        const std::vector<std::pair<uint32_t, uint32_t>> &sp;
        double pull;
        int &used;
        void go(uint32_t m) {
            Sub &s = t[m];
            for (auto &x : sp)
                if ((x.first | x.second) == m) {
                    go(x.first);
                    go(x.second);
                    // the star side, if any, on the right
                    auto kr = classify(p, t, x.first, x.second);
                    uint32_t l = x.first, r = x.second;
                    if (kr.first == HUGE_BUSHY_PUSH) {
                        auto k2 = classify(p, t, x.second, x.first);
                        if (k2.first != HUGE_BUSHY_PUSH) {
                            kr = k2;
                            std::swap(l, r);
                        }
                    }
                    s.kind = kr.first;
                    s.root = kr.second;
                    s.left = l;
                    s.right = r;
                    s.cost = join_cost(t, m, l, r, kr.first, pull);
                    ++used;
                    return;
                }
            if (s.centre < 0) HUGE_FAIL(HUGE_EORDER, "a part that no join splits must be a star (edge set 0x%x)", m);
            s.kind = HUGE_BUSHY_UNIT;
            s.root = s.centre;
            s.cost = s.est;
        }
    } w{p, t, sp, pull, used};
    w.go(full);
    if (used != nsplits) HUGE_FAIL(HUGE_EORDER, "%d of the %d joins are not in the tree", nsplits - used, nsplits);
    recover(p, t, full);
}

}  // namespace huge
