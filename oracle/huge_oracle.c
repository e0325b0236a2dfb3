/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct CPU implementation of what the GPU library
 * computes: subgraph enumeration of an unlabelled connected query q in an
 * unlabelled undirected simple data graph G (Section 2, "Subgraph
 * Enumeration"): every subgraph g of G isomorphic to q, non-induced (only the
 * edges of q must be present), reported once.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may call it; the GPU library does
 * not use it and shares no code with it.
 *
 * What it returns for one query:
 *   count       number of subgraphs g of G isomorphic to q;
 *   hash_sum    sum over g of h(g)  (mod 2^64);
 *   hash_xor    xor over g of h(g);
 * where h(g) = mix( sum over query edges (a,b) of mix(edge(f(a), f(b))) ),
 * edge(x, y) = (min(rx, ry) << 32) | max(rx, ry) with r the degree rank
 * below, and mix the SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA 2014).
 * h depends only on the image edge set of g, so both aggregates are
 * independent of the matching order, the symmetry-breaking scheme and the
 * order of enumeration.
 *
 * Data-vertex total order (the symmetry-breaking order of Section 2): vertices
 * ranked by ascending (degree, original ID); r(u) is u's position.
 *
 * Three modes decide which of the |Aut(q)| maps of one subgraph is reported:
 *   ORC_MODE_SB     symmetry breaking (Section 2): the map must satisfy every
 *                   constraint a < b of a partial order on query vertices as
 *                   r(f(a)) < r(f(b)).  The constraints come from the caller,
 *                   or, by default, from the Grochow-Kellis procedure
 *                   (RECOMB 2007) with a lowest-ID tie-break, run here.
 *   ORC_MODE_CANON  no constraints during search; a complete map f is
 *                   reported iff its rank sequence (r f(0), ..., r f(k-1)) is
 *                   lexicographically smallest among f o s for s in Aut(q).
 *                   This is the definition "each subgraph once" written out,
 *                   independent of any symmetry-breaking theory.
 *   ORC_MODE_ALL    every injective edge-preserving map (|Aut(q)| per g).
 *
 * Search: backtracking over query vertices in the oracle's own order (BFS
 * from query vertex 0, smallest ID first) unless an order is given.  The
 * candidates of a query vertex are the neighbours of its earliest matched
 * neighbour; adjacency to every other matched neighbour is checked by binary
 * search in sorted adjacency lists (Eq. 2 computed one candidate at a time).
 * Injectivity is checked against every matched vertex (Algorithm 4's filter).
 *
 * level_counts[d] (d = 0..k-1) counts the accepted partial maps of the first
 * d+1 vertices of the order: injective, edge-preserving on that induced
 * prefix, satisfying the constraints (mode SB) whose two ends are both in the
 * prefix, and the root slice when query vertex 0 is in the prefix.
 *
 * Root slice (slice_count S, slice_id s, slice_vertex a): only maps with
 * mix(r(f(a))) mod S == s are kept (a = query vertex 0 by default).  The
 * slices of any fixed query vertex partition the results, so
 * counts and sums add and xors combine over s.
 *
 * Pair slice (slice_vertex a and slice_vertex2 b >= 0): only maps with
 * mix(r(f(a)) * 2^32 + r(f(b))) mod S == s are kept, checked when the later
 * of a and b is matched; slices of a fixed ordered pair also partition the
 * results.
 *
 * Strided slices (slice_mode 1): a vertex slice keeps r(f(a)) mod S == s
 * instead of the mix; a pair slice keeps the maps whose pair (f(a), f(b)) (a, b
 * adjacent in q) sits at an entry e of the rank-relabelled CSR with
 * e mod S == s, where e(x, y) = (sum of the degrees of the vertices ranked below
 * x) + #{z in N(x) : r(z) < r(y)}.  A second slice (vertex c, or pair (c, d);
 * count S2, id s2, same mode) can be applied on top of the first: only maps in
 * both are kept.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORC_MODE_SB 0
#define ORC_MODE_CANON 1
#define ORC_MODE_ALL 2
#define ORC_INDUCED 4 /* or'ed into the mode: only induced occurrences (non-edges of q absent too) */
#define ORC_KMAX 8

typedef struct {
    uint64_t count, hash_sum, hash_xor;
    uint64_t level_counts[ORC_KMAX];
} orc_result;

static inline uint64_t orc_mix(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

uint64_t orc_mix64(uint64_t x) { return orc_mix(x); }

/* ------------------------------------------------------------------ */
/* query graph                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    int k;
    int adj[ORC_KMAX][ORC_KMAX];
    int ne;
    int ea[28], eb[28];
    int naut;
    int8_t *aut; /* naut * k */
    int nsb;
    int sba[28], sbb[28]; /* constraint sba < sbb (query vertex IDs) */
    int label[ORC_KMAX];  /* labelled queries: the label each query vertex's image must carry, -1 any */
    int directed;         /* directed queries: dadj[a][b] = 1 for every query edge a -> b */
    int dadj[ORC_KMAX][ORC_KMAX];
} orc_query;

/* Returns 0 on success, -1 on malformed query (k out of range, bad edge,
 * duplicate edge, self-loop, or disconnected). */
static int orc_query_init(orc_query *q, int k, int ne, const int32_t *e) {
    memset(q, 0, sizeof(*q));
    if (k < 2 || k > ORC_KMAX || ne < 1 || ne > 28) return -1;
    q->k = k;
    for (int i = 0; i < ne; ++i) {
        int a = e[2 * i], b = e[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b || q->adj[a][b]) return -1;
        q->adj[a][b] = q->adj[b][a] = 1;
        q->ea[q->ne] = a < b ? a : b;
        q->eb[q->ne] = a < b ? b : a;
        q->ne++;
    }
    /* connectivity by flood fill from vertex 0 */
    int seen[ORC_KMAX] = {0}, stack[ORC_KMAX], sp = 0, cnt = 1;
    seen[0] = 1;
    stack[sp++] = 0;
    while (sp) {
        int a = stack[--sp];
        for (int b = 0; b < k; ++b)
            if (q->adj[a][b] && !seen[b]) {
                seen[b] = 1;
                cnt++;
                stack[sp++] = b;
            }
    }
    if (cnt != k) return -1;
    return 0;
}

/* A directed query: edges a -> b (a pair may hold both directions).  Its
 * undirected skeleton (one edge per adjacent pair) must be connected; the
 * skeleton drives the search, the directions filter it. */
static int orc_query_init_directed(orc_query *q, int k, int ne, const int32_t *e) {
    memset(q, 0, sizeof(*q));
    if (k < 2 || k > ORC_KMAX || ne < 1 || ne > 56) return -1;
    int32_t sk[2 * 28];
    int nsk = 0;
    int dadj[ORC_KMAX][ORC_KMAX];
    memset(dadj, 0, sizeof(dadj));
    for (int i = 0; i < ne; ++i) {
        int a = e[2 * i], b = e[2 * i + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b || dadj[a][b]) return -1;
        dadj[a][b] = 1;
        if (!dadj[b][a]) {
            sk[2 * nsk] = a;
            sk[2 * nsk + 1] = b;
            ++nsk;
        }
    }
    if (orc_query_init(q, k, nsk, sk) != 0) return -1;
    q->directed = 1;
    memcpy(q->dadj, dadj, sizeof(dadj));
    return 0;
}

/* All automorphisms by trying every permutation (k <= 8: at most 40320). */
static void orc_query_aut(orc_query *q) {
    int k = q->k;
    int cap = 1;
    for (int i = 2; i <= k; ++i) cap *= i;
    q->aut = (int8_t *)malloc((size_t)cap * (size_t)k);
    q->naut = 0;
    int p[ORC_KMAX];
    for (int i = 0; i < k; ++i) p[i] = i;
    for (;;) {
        int ok = 1;
        for (int i = 0; i < q->ne && ok; ++i)
            if (!q->adj[p[q->ea[i]]][p[q->eb[i]]]) ok = 0;
        for (int i = 0; i < k && ok; ++i) /* automorphisms of a labelled query keep labels */
            if (q->label[p[i]] != q->label[i]) ok = 0;
        for (int a = 0; a < k && ok && q->directed; ++a) /* ... and of a directed one, directions */
            for (int b = 0; b < k && ok; ++b)
                if (q->dadj[p[a]][p[b]] != q->dadj[a][b]) ok = 0;
        if (ok) {
            for (int i = 0; i < k; ++i) q->aut[q->naut * k + i] = (int8_t)p[i];
            q->naut++;
        }
        /* next permutation in lexicographic order */
        int i = k - 2;
        while (i >= 0 && p[i] > p[i + 1]) --i;
        if (i < 0) break;
        int j = k - 1;
        while (p[j] < p[i]) --j;
        int t = p[i];
        p[i] = p[j];
        p[j] = t;
        for (int a = i + 1, b = k - 1; a < b; ++a, --b) {
            t = p[a];
            p[a] = p[b];
            p[b] = t;
        }
    }
}

/*
 * Grochow-Kellis symmetry breaking: while the group G (initially Aut(q)) is
 * not trivial, take the vertex v of smallest ID among those whose orbit under
 * G is largest, require v < w for every other w of that orbit, and replace G
 * by the stabiliser of v.
 */
static void orc_query_gk(orc_query *q) {
    int k = q->k;
    int8_t *alive = (int8_t *)malloc((size_t)q->naut);
    for (int i = 0; i < q->naut; ++i) alive[i] = 1;
    q->nsb = 0;
    for (;;) {
        int nalive = 0;
        for (int i = 0; i < q->naut; ++i) nalive += alive[i];
        if (nalive <= 1) break;
        int best = -1, bestsz = 0;
        int orbit[ORC_KMAX][ORC_KMAX];
        int osz[ORC_KMAX];
        for (int v = 0; v < k; ++v) {
            osz[v] = 0;
            int in[ORC_KMAX] = {0};
            for (int s = 0; s < q->naut; ++s)
                if (alive[s]) in[q->aut[s * k + v]] = 1;
            for (int w = 0; w < k; ++w)
                if (in[w]) orbit[v][osz[v]++] = w;
            if (osz[v] > bestsz) {
                bestsz = osz[v];
                best = v;
            }
        }
        for (int i = 0; i < osz[best]; ++i) {
            int w = orbit[best][i];
            if (w != best) {
                q->sba[q->nsb] = best;
                q->sbb[q->nsb] = w;
                q->nsb++;
            }
        }
        for (int s = 0; s < q->naut; ++s)
            if (alive[s] && q->aut[s * k + best] != best) alive[s] = 0;
    }
    free(alive);
}

/* ------------------------------------------------------------------ */
/* data graph view + ranks                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const int64_t *rp;
    const int32_t *col;
    int32_t *rank;
    const int32_t *label; /* vertex labels (original IDs), or NULL */
    const int64_t *drp;   /* directed graphs: out-lists (original IDs, ascending), or NULL */
    const int32_t *dcol;
} orc_graph;

static const int64_t *orc_sort_deg;
static int orc_cmp_vertex(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    int64_t dx = orc_sort_deg[x], dy = orc_sort_deg[y];
    if (dx != dy) return dx < dy ? -1 : 1;
    return (x > y) - (x < y);
}

static pthread_mutex_t orc_sort_mu = PTHREAD_MUTEX_INITIALIZER;

/* rank[u] = position of u in ascending (degree, ID) order. */
int orc_ranks(int64_t n, const int64_t *rp, int32_t *rank) {
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t u = 0; u < n; ++u) {
        deg[u] = rp[u + 1] - rp[u];
        ord[u] = (int32_t)u;
    }
    pthread_mutex_lock(&orc_sort_mu);
    orc_sort_deg = deg;
    qsort(ord, (size_t)n, sizeof(int32_t), orc_cmp_vertex);
    pthread_mutex_unlock(&orc_sort_mu);
    for (int64_t i = 0; i < n; ++i) rank[ord[i]] = (int32_t)i;
    free(ord);
    free(deg);
    return 0;
}

static int orc_adjacent(const orc_graph *g, int32_t a, int32_t b) {
    int64_t lo = g->rp[a], hi = g->rp[a + 1];
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        int32_t x = g->col[mid];
        if (x == b) return 1;
        if (x < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* a -> b in a directed graph's out-lists */
static int orc_arc(const orc_graph *g, int32_t a, int32_t b) {
    int64_t lo = g->drp[a], hi = g->drp[a + 1];
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        int32_t x = g->dcol[mid];
        if (x == b) return 1;
        if (x < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* search plan                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_query *q;
    const orc_graph *g;
    int mode;
    int order[ORC_KMAX];
    int pos[ORC_KMAX];          /* pos[v] = position of query vertex v */
    int pivot[ORC_KMAX];        /* position of the earliest matched neighbour */
    int nchk[ORC_KMAX];         /* other matched neighbours to check */
    int chk[ORC_KMAX][ORC_KMAX];
    int nlt[ORC_KMAX], ngt[ORC_KMAX];
    int lt[ORC_KMAX][28];       /* positions p: need r(f[p]) < r(new) */
    int gt[ORC_KMAX][28];       /* positions p: need r(new) < r(f[p]) */
    uint32_t slice_count, slice_id;
    int slice_pos;              /* position of the sliced query vertex */
    int pair_a, pair_b;         /* pair slice: positions of the two query vertices, or -1 */
    int slice_mode;             /* vertex slices: 0 by mix of the rank, 1 by the rank itself */
    uint32_t slice2_count, slice2_id;
    int slice2_pos;             /* position of the second sliced query vertex, or -1 */
    int pair2_a, pair2_b;       /* second slice on a pair of positions (or -1) */
    const int64_t *roff;        /* strided pair slices: first entry of each rank's row in the relabelled CSR */
    int induced;                /* 1: the image of every non-edge of q must be a non-edge of G */
    int nnon[ORC_KMAX];
    int non[ORC_KMAX][ORC_KMAX]; /* earlier positions not adjacent to position i in q */
} orc_plan;

struct orc_worker_s {
    const orc_plan *P;
    orc_result res;
    int32_t f[ORC_KMAX];
};
typedef struct orc_worker_s orc_worker;

/* rank r in slice id of count (vertex slices) */
static int orc_in_vslice(int32_t r, uint32_t count, uint32_t id, int mode) {
    uint64_t x = mode ? (uint64_t)(uint32_t)r : orc_mix((uint64_t)(uint32_t)r);
    return x % count == id;
}

static int orc_plan_init(orc_plan *P, const orc_query *q, const orc_graph *g, int mode,
                         const int32_t *order, uint32_t sc, uint32_t sid, int slice_vertex, int slice_vertex2,
                         int slice_mode, int slice2_vertex, int slice2_vertex2, uint32_t sc2, uint32_t sid2) {
    memset(P, 0, sizeof(*P));
    P->q = q;
    P->g = g;
    P->induced = (mode & ORC_INDUCED) != 0;
    mode &= ~ORC_INDUCED;
    P->mode = mode;
    int k = q->k;
    if (order) {
        int used[ORC_KMAX] = {0};
        for (int i = 0; i < k; ++i) {
            if (order[i] < 0 || order[i] >= k || used[order[i]]) return -1;
            used[order[i]] = 1;
            P->order[i] = order[i];
        }
    } else {
        /* BFS from query vertex 0, neighbours in increasing ID */
        int seen[ORC_KMAX] = {0}, head = 0, tail = 0;
        P->order[tail++] = 0;
        seen[0] = 1;
        while (head < tail) {
            int a = P->order[head++];
            for (int b = 0; b < k; ++b)
                if (q->adj[a][b] && !seen[b]) {
                    seen[b] = 1;
                    P->order[tail++] = b;
                }
        }
    }
    for (int i = 0; i < k; ++i) P->pos[P->order[i]] = i;
    for (int i = 1; i < k; ++i) {
        int v = P->order[i];
        P->pivot[i] = -1;
        P->nchk[i] = 0;
        for (int p = 0; p < i; ++p)
            if (q->adj[P->order[p]][v]) {
                if (P->pivot[i] < 0) P->pivot[i] = p;
                else P->chk[i][P->nchk[i]++] = p;
            }
        if (P->pivot[i] < 0) return -1; /* prefix not connected */
        P->nnon[i] = 0;
        for (int p = 0; p < i; ++p)
            if (!q->adj[P->order[p]][v]) P->non[i][P->nnon[i]++] = p;
    }
    if (mode == ORC_MODE_SB) {
        for (int c = 0; c < q->nsb; ++c) {
            int pa = P->pos[q->sba[c]], pb = P->pos[q->sbb[c]];
            /* constraint r(f(sba)) < r(f(sbb)); checked at the later position */
            if (pa < pb) P->lt[pb][P->nlt[pb]++] = pa;
            else P->gt[pa][P->ngt[pa]++] = pb;
        }
    }
    P->slice_count = sc ? sc : 1;
    P->slice_id = sid;
    if (slice_vertex < 0 || slice_vertex >= k) return -1;
    P->slice_pos = P->pos[slice_vertex];
    P->pair_a = P->pair_b = -1;
    if (slice_vertex2 >= 0) {
        if (slice_vertex2 >= k || slice_vertex2 == slice_vertex) return -1;
        P->pair_a = P->pos[slice_vertex];
        P->pair_b = P->pos[slice_vertex2];
        P->slice_pos = -1; /* no vertex slice */
    }
    if (slice_mode != 0 && slice_mode != 1) return -1;
    P->slice_mode = slice_mode;
    P->slice2_count = sc2 > 1 ? sc2 : 1;
    P->slice2_id = sc2 > 1 ? sid2 : 0;
    P->slice2_pos = -1;
    P->pair2_a = P->pair2_b = -1;
    if (P->slice2_count > 1) {
        if (slice2_vertex < 0 || slice2_vertex >= k || P->slice2_id >= P->slice2_count) return -1;
        if (slice2_vertex2 >= 0) {
            if (slice2_vertex2 >= k || slice2_vertex2 == slice2_vertex) return -1;
            P->pair2_a = P->pos[slice2_vertex];
            P->pair2_b = P->pos[slice2_vertex2];
        } else {
            P->slice2_pos = P->pos[slice2_vertex];
        }
    }
    /* strided pair slices need adjacent ends (their pair is an edge of G) */
    if (slice_mode == 1 && P->pair_a >= 0 && !q->adj[slice_vertex][slice_vertex2]) return -1;
    if (slice_mode == 1 && P->pair2_a >= 0 && !q->adj[slice2_vertex][slice2_vertex2]) return -1;
    return 0;
}

/* e(x, y) of a strided pair slice: x's first entry in the relabelled CSR plus
 * the number of x's neighbours ranked below y */
static int64_t orc_entry(const orc_plan *P, int32_t x, int32_t y) {
    const orc_graph *g = P->g;
    int64_t e = P->roff[g->rank[x]];
    const int32_t ry = g->rank[y];
    for (int64_t t = g->rp[x]; t < g->rp[x + 1]; ++t) e += g->rank[g->col[t]] < ry;
    return e;
}

/* the pair slice (positions a, b; count, id; mode) at position i with candidate c */
static int orc_pair_ok(const struct orc_worker_s *w, int i, int32_t c, int a, int b, uint32_t count, uint32_t id) {
    const orc_plan *P = w->P;
    if (count <= 1 || a < 0 || i != (a > b ? a : b)) return 1;
    const int32_t x = i == a ? c : w->f[a], y = i == b ? c : w->f[b];
    if (P->slice_mode == 1) return (uint64_t)orc_entry(P, x, y) % count == id;
    const uint32_t ra = (uint32_t)P->g->rank[x], rb = (uint32_t)P->g->rank[y];
    return orc_mix(((uint64_t)ra << 32) | rb) % count == id;
}

/* the vertex slices that apply at position i to the vertex of rank r */
static int orc_slices_ok(const orc_plan *P, int i, int32_t r) {
    if (P->slice_count > 1 && i == P->slice_pos &&
        !orc_in_vslice(r, P->slice_count, P->slice_id, P->slice_mode))
        return 0;
    if (P->slice2_count > 1 && i == P->slice2_pos &&
        !orc_in_vslice(r, P->slice2_count, P->slice2_id, P->slice_mode))
        return 0;
    return 1;
}


static void orc_emit(orc_worker *w) {
    const orc_plan *P = w->P;
    const orc_query *q = P->q;
    const int32_t *rank = P->g->rank;
    int k = q->k;
    if (P->mode == ORC_MODE_CANON) {
        int32_t seq[ORC_KMAX];
        for (int v = 0; v < k; ++v) seq[v] = rank[w->f[P->pos[v]]];
        for (int s = 1; s < q->naut; ++s) {
            const int8_t *sg = q->aut + s * k;
            for (int v = 0; v < k; ++v) {
                int32_t a = seq[(int)sg[v]];
                if (a < seq[v]) return; /* f o s is smaller: not the representative */
                if (a > seq[v]) break;
            }
        }
    }
    uint64_t s = 0;
    for (int e = 0; e < q->ne; ++e) {
        uint64_t ra = (uint64_t)(uint32_t)rank[w->f[P->pos[q->ea[e]]]];
        uint64_t rb = (uint64_t)(uint32_t)rank[w->f[P->pos[q->eb[e]]]];
        uint64_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        s += orc_mix((lo << 32) | hi);
    }
    uint64_t h = orc_mix(s);
    w->res.count++;
    w->res.hash_sum += h;
    w->res.hash_xor ^= h;
}

static int orc_accept(orc_worker *w, int i, int32_t c) {
    const orc_plan *P = w->P;
    const orc_graph *g = P->g;
    for (int p = 0; p < i; ++p)
        if (w->f[p] == c) return 0; /* injectivity */
    if (P->q->label[P->order[i]] >= 0 && (!g->label || g->label[c] != P->q->label[P->order[i]])) return 0;
    for (int t = 0; t < P->nchk[i]; ++t)
        if (!orc_adjacent(g, w->f[P->chk[i][t]], c)) return 0;
    if (P->induced)
        for (int t = 0; t < P->nnon[i]; ++t)
            if (orc_adjacent(g, w->f[P->non[i][t]], c)) return 0;
    if (P->q->directed) /* every query edge between an earlier vertex and this one, in its direction */
        for (int p = 0; p < i; ++p) {
            const int u = P->order[p], v = P->order[i];
            if (P->q->dadj[u][v] && !orc_arc(g, w->f[p], c)) return 0;
            if (P->q->dadj[v][u] && !orc_arc(g, c, w->f[p])) return 0;
        }
    int32_t rc = g->rank[c];
    for (int t = 0; t < P->nlt[i]; ++t)
        if (!(g->rank[w->f[P->lt[i][t]]] < rc)) return 0;
    for (int t = 0; t < P->ngt[i]; ++t)
        if (!(rc < g->rank[w->f[P->gt[i][t]]])) return 0;
    if (!orc_slices_ok(P, i, rc)) return 0;
    if (!orc_pair_ok(w, i, c, P->pair_a, P->pair_b, P->slice_count, P->slice_id)) return 0;
    if (!orc_pair_ok(w, i, c, P->pair2_a, P->pair2_b, P->slice2_count, P->slice2_id)) return 0;
    return 1;
}

static int orc_cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static void orc_search(orc_worker *w, int i);

/* Position 1 under a strided pair slice on positions (0, 1): only the entries
 * e = base + j of f[0]'s row in the relabelled CSR with e mod S == s, j being
 * the rank order of the neighbour in N(f[0]). */
static void orc_search_pair_slice(orc_worker *w) {
    const orc_plan *P = w->P;
    const orc_graph *g = P->g;
    const int32_t x = w->f[0];
    const int64_t d = g->rp[x + 1] - g->rp[x];
    const int64_t base = P->roff[g->rank[x]];
    const int64_t S = P->slice_count;
    const int64_t j0 = ((int64_t)P->slice_id - base % S + S) % S;
    if (j0 >= d) return;
    uint64_t *nb = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)d);
    for (int64_t t = 0; t < d; ++t) {
        const int32_t z = g->col[g->rp[x] + t];
        nb[t] = ((uint64_t)(uint32_t)g->rank[z] << 32) | (uint32_t)z;
    }
    qsort(nb, (size_t)d, sizeof(uint64_t), orc_cmp_u64);
    for (int64_t j = j0; j < d; j += S) {
        const int32_t c = (int32_t)(uint32_t)nb[j];
        if (!orc_accept(w, 1, c)) continue;
        w->res.level_counts[1]++;
        w->f[1] = c;
        orc_search(w, 2);
    }
    free(nb);
}

static void orc_search(orc_worker *w, int i) {
    const orc_plan *P = w->P;
    int k = P->q->k;
    if (i == k) {
        orc_emit(w);
        return;
    }
    if (i == 1 && P->slice_mode == 1 && P->slice_count > 1 && P->pair_a == 0 && P->pair_b == 1) {
        orc_search_pair_slice(w);
        return;
    }
    const orc_graph *g = P->g;
    int32_t piv = w->f[P->pivot[i]];
    for (int64_t e = g->rp[piv]; e < g->rp[piv + 1]; ++e) {
        int32_t c = g->col[e];
        if (!orc_accept(w, i, c)) continue;
        w->res.level_counts[i]++;
        w->f[i] = c;
        orc_search(w, i + 1);
    }
}

typedef struct {
    const orc_plan *P;
    int64_t *next;
    int64_t n, chunk;
    orc_result res;
} orc_thread_arg;

static void *orc_thread(void *arg) {
    orc_thread_arg *a = (orc_thread_arg *)arg;
    orc_worker w;
    memset(&w, 0, sizeof(w));
    w.P = a->P;
    const orc_plan *P = a->P;
    for (;;) {
        int64_t lo = __atomic_fetch_add(a->next, a->chunk, __ATOMIC_RELAXED);
        if (lo >= a->n) break;
        int64_t hi = lo + a->chunk < a->n ? lo + a->chunk : a->n;
        for (int64_t u = lo; u < hi; ++u) {
            if (!orc_slices_ok(P, 0, P->g->rank[u])) continue;
            {
                const int want = P->q->label[P->order[0]];
                if (want >= 0 && (!P->g->label || P->g->label[u] != want)) continue;
            }
            w.res.level_counts[0]++;
            w.f[0] = (int32_t)u;
            orc_search(&w, 1);
        }
    }
    a->res = w.res;
    return NULL;
}

/*
 * Enumerate one query.  Inputs: a clean CSR (see orc_check_csr) in original
 * IDs; k query vertices; nqe edges as 2*nqe ints; mode; optional order
 * (k entries, every prefix connected); optional caller SB pairs (nsb pairs as
 * 2*nsb ints a<b; used by ORC_MODE_SB when nsb >= 0, nsb < 0 = compute
 * Grochow-Kellis here); root slice; optional ranks of an earlier orc_ranks
 * call on the same graph (NULL = computed here); thread count (0 = all
 * online CPUs).
 * Returns 0, or -1 for a malformed query/order.
 */
static int orc_enumerate_impl(int64_t n, const int64_t *rp, const int32_t *col, int k, int nqe,
                              const int32_t *qedges, int mode, const int32_t *order, int nsb,
                              const int32_t *sb_pairs, uint32_t slice_count, uint32_t slice_id, int slice_vertex,
                              int slice_vertex2, int slice_mode, int slice2_vertex, int slice2_vertex2,
                              uint32_t slice2_count, uint32_t slice2_id, const int32_t *rank_in,
                              const int32_t *vlabels, const int32_t *qlabels, int nthreads, orc_result *out,
                              const int64_t *drp, const int32_t *dcol) {
    orc_query q;
    if ((drp ? orc_query_init_directed(&q, k, nqe, qedges) : orc_query_init(&q, k, nqe, qedges)) != 0) return -1;
    for (int i = 0; i < k; ++i) q.label[i] = qlabels ? qlabels[i] : -1;
    orc_query_aut(&q);
    if (nsb >= 0) {
        if (nsb > 28) {
            free(q.aut);
            return -1;
        }
        q.nsb = nsb;
        for (int i = 0; i < nsb; ++i) {
            q.sba[i] = sb_pairs[2 * i];
            q.sbb[i] = sb_pairs[2 * i + 1];
            if (q.sba[i] < 0 || q.sba[i] >= k || q.sbb[i] < 0 || q.sbb[i] >= k) {
                free(q.aut);
                return -1;
            }
        }
    } else {
        orc_query_gk(&q);
    }
    orc_graph g;
    g.n = n;
    g.rp = rp;
    g.col = col;
    g.label = vlabels;
    g.drp = drp;
    g.dcol = dcol;
    g.rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (rank_in) /* ranks from an earlier orc_ranks call on the same graph */
        memcpy(g.rank, rank_in, sizeof(int32_t) * (size_t)n);
    else
        orc_ranks(n, rp, g.rank);
    orc_plan P;
    if (orc_plan_init(&P, &q, &g, mode, order, slice_count, slice_id, slice_vertex, slice_vertex2, slice_mode,
                      slice2_vertex, slice2_vertex2, slice2_count, slice2_id) != 0) {
        free(g.rank);
        free(q.aut);
        return -1;
    }
    int64_t *roff = NULL;
    if (slice_mode == 1 && (P.pair_a >= 0 || P.pair2_a >= 0)) {
        /* first entry of each rank's row in the relabelled CSR */
        roff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        for (int64_t u = 0; u < n; ++u) roff[g.rank[u] + 1] = rp[u + 1] - rp[u];
        roff[0] = 0;
        for (int64_t r = 0; r < n; ++r) roff[r + 1] += roff[r];
        P.roff = roff;
    }
    if (nthreads <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        nthreads = c > 0 ? (int)c : 1;
    }
    if (nthreads > 256) nthreads = 256;
    int64_t next = 0;
    orc_thread_arg *args = (orc_thread_arg *)calloc((size_t)nthreads, sizeof(orc_thread_arg));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        args[t].P = &P;
        args[t].next = &next;
        args[t].n = n;
        args[t].chunk = 16;
        if (t) pthread_create(&th[t], NULL, orc_thread, &args[t]);
    }
    orc_thread(&args[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    orc_result r;
    memset(&r, 0, sizeof(r));
    for (int t = 0; t < nthreads; ++t) {
        r.count += args[t].res.count;
        r.hash_sum += args[t].res.hash_sum;
        r.hash_xor ^= args[t].res.hash_xor;
        for (int i = 0; i < ORC_KMAX; ++i) r.level_counts[i] += args[t].res.level_counts[i];
    }
    *out = r;
    free(args);
    free(th);
    free(roff);
    free(g.rank);
    free(q.aut);
    return 0;
}

int orc_enumerate(int64_t n, const int64_t *rp, const int32_t *col, int k, int nqe,
                  const int32_t *qedges, int mode, const int32_t *order, int nsb,
                  const int32_t *sb_pairs, uint32_t slice_count, uint32_t slice_id, int slice_vertex,
                  int slice_vertex2, int slice_mode, int slice2_vertex, int slice2_vertex2, uint32_t slice2_count,
                  uint32_t slice2_id, const int32_t *rank_in, const int32_t *vlabels, const int32_t *qlabels,
                  int nthreads, orc_result *out) {
    return orc_enumerate_impl(n, rp, col, k, nqe, qedges, mode, order, nsb, sb_pairs, slice_count, slice_id,
                              slice_vertex, slice_vertex2, slice_mode, slice2_vertex, slice2_vertex2, slice2_count,
                              slice2_id, rank_in, vlabels, qlabels, nthreads, out, NULL, NULL);
}

/*
 * The same for a directed graph and a directed query: rp/col is the graph's
 * undirected skeleton (every adjacent pair both ways), drp/dcol its out-lists
 * (original IDs, ascending); qedges are the query's directed edges a -> b.  A
 * match is an injective map keeping every query edge's direction, reported
 * once per class of the automorphisms that keep directions (and labels).
 */
int orc_enumerate_directed(int64_t n, const int64_t *rp, const int32_t *col, const int64_t *drp,
                           const int32_t *dcol, int k, int nqe, const int32_t *qedges, int mode,
                           const int32_t *order, uint32_t slice_count, uint32_t slice_id, int slice_vertex,
                           int slice_mode, const int32_t *vlabels, const int32_t *qlabels, int nthreads,
                           orc_result *out) {
    if (!drp || !dcol) return -1;
    return orc_enumerate_impl(n, rp, col, k, nqe, qedges, mode, order, -1, NULL, slice_count, slice_id,
                              slice_vertex, -1, slice_mode, -1, -1, 1, 0, NULL, vlabels, qlabels, nthreads, out,
                              drp, dcol);
}

/* |Aut(q)| of a directed query (automorphisms keep directions), or -1. */
int orc_automorphisms_directed(int k, int nqe, const int32_t *qedges) {
    orc_query q;
    if (orc_query_init_directed(&q, k, nqe, qedges) != 0) return -1;
    orc_query_aut(&q);
    int n = q.naut;
    free(q.aut);
    return n;
}

/* |Aut(q)|, or -1 for a malformed query; perms (if not NULL) receives naut*k entries. */
int orc_automorphisms(int k, int nqe, const int32_t *qedges, int32_t *perms, int cap) {
    orc_query q;
    if (orc_query_init(&q, k, nqe, qedges) != 0) return -1;
    orc_query_aut(&q);
    int n = q.naut;
    if (perms)
        for (int s = 0; s < n && s < cap; ++s)
            for (int i = 0; i < k; ++i) perms[s * k + i] = q.aut[s * k + i];
    free(q.aut);
    return n;
}

/* Grochow-Kellis constraints (pairs a<b); returns their number, -1 if malformed. */
int orc_sb_pairs(int k, int nqe, const int32_t *qedges, int32_t *pairs) {
    orc_query q;
    if (orc_query_init(&q, k, nqe, qedges) != 0) return -1;
    orc_query_aut(&q);
    orc_query_gk(&q);
    for (int i = 0; i < q.nsb; ++i) {
        pairs[2 * i] = q.sba[i];
        pairs[2 * i + 1] = q.sbb[i];
    }
    free(q.aut);
    return q.nsb;
}

/*
 * CSR hygiene check: 0 = clean; 1 = a list is not strictly ascending
 * (unsorted or duplicate); 2 = self-loop; 3 = ID out of range;
 * 4 = not symmetric; 5 = bad row_ptr.
 */
int orc_check_csr(int64_t n, const int64_t *rp, const int32_t *col) {
    if (rp[0] != 0) return 5;
    for (int64_t u = 0; u < n; ++u)
        if (rp[u + 1] < rp[u]) return 5;
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t v = col[e];
            if (v < 0 || v >= n) return 3;
            if (v == u) return 2;
            if (e > rp[u] && col[e - 1] >= v) return 1;
        }
    orc_graph g;
    g.n = n;
    g.rp = rp;
    g.col = col;
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e)
            if (!orc_adjacent(&g, col[e], (int32_t)u)) return 4;
    return 0;
}
