/*
 * huge.h -- C ABI of a single-GPU (MI355X, gfx950) subgraph enumeration
 * library built around the PULL-EXTEND operator of HUGE (Yang, Lai, Lin, Hao,
 * Zhang, "HUGE: An Efficient and Scalable Subgraph Enumeration System").
 *
 * Problem (Section 2, "Subgraph Enumeration"): given an unlabelled, undirected,
 * connected query q and an unlabelled undirected data graph G, find every
 * subgraph g of G isomorphic to q.  Subgraphs are non-induced: only q's edges
 * must be present.  Symmetry breaking (Section 2) reports each g exactly once.
 *
 * The computation is the left-deep chain of complete star joins on induced
 * prefixes (Section 3.1, Definition 3.1 and the BiGJoin discussion): a SCAN of
 * the first query edge followed by one PULL-EXTEND per further query vertex
 * (Section 4.2), whose candidate set is the intersection of the neighbour
 * lists of the already-matched neighbours (Eq. 2), filtered by injectivity
 * (Algorithm 4, intersect stage) and by the symmetry-breaking order, and a
 * counting SINK (Section 4.2).  Execution follows the DFS/BFS-adaptive
 * scheduler (Section 5.2, Algorithm 5) with a bounded device frontier, and
 * work stealing (Section 5.3) inside the GPU.
 *
 * Conventions for every function:
 *   - returns huge_status; no exception crosses the ABI;
 *   - out-parameters are written only on HUGE_OK (or HUGE_STOPPED where
 *     stated);
 *   - huge_last_error() gives a thread-local message for the last failure
 *     on the calling thread, valid until the next call on that thread;
 *   - handles are immutable after creation and may be shared between threads;
 *     two concurrent exec calls need two workspaces (or NULL workspaces).
 *
 * IDs: vertex IDs in and out of the library are the caller's original IDs.
 * Internally the graph is relabelled by degree rank (ascending degree, ties by
 * original ID), the data-vertex total order of Section 2's symmetry breaking.
 */
#ifndef HUGE_H
#define HUGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HUGE_KMAX 8 /* largest query: 8 vertices */

typedef enum {
    HUGE_OK = 0,
    HUGE_STOPPED = 1,    /* huge_enumerate: the callback asked to stop */
    HUGE_EINVAL = -1,    /* NULL pointer, bad size, bad option */
    HUGE_ENOMEM = -2,    /* device or host allocation failed, or workspace too small */
    HUGE_EDEVICE = -3,   /* a HIP runtime call or kernel failed */
    HUGE_EGRAPH = -4,    /* CSR not sorted, duplicate, self-loop, asymmetric, ID out of range */
    HUGE_EQUERY = -5,    /* k < 2, k > 8, bad/duplicate/self edge, or disconnected query */
    HUGE_EORDER = -6,    /* order is not a permutation, or a prefix is disconnected */
    HUGE_EOVERFLOW = -7  /* a 64-bit count overflowed */
} huge_status;

typedef struct huge_graph huge_graph;
typedef struct huge_plan huge_plan;

/* huge_load_csr flags */
#define HUGE_HOST_PTRS 0x1u   /* row_ptr / col are host memory (copied) */
#define HUGE_DEVICE_PTRS 0x2u /* row_ptr / col are device memory (read, not kept) */
#define HUGE_NO_VALIDATE 0x4u /* skip the hygiene checks (caller guarantees a clean CSR) */
#define HUGE_NO_HUB_BITMAP 0x8u /* do not build adjacency bitmaps for the highest-degree vertices */

/* huge_plan flags */
#define HUGE_PLAN_COST_MODEL 0x0u /* order from the cost model (Algorithm 1, wco plans) */
#define HUGE_PLAN_LEARNED 0x1u    /* order from the learned cost model (huge_plan_create_learned) */
#define HUGE_PLAN_VERIFY 0x2u     /* learned plans: measure the model's best orders on a small sample */
/* Induced matching (Section 2's induced subgraphs): keep only the matches whose
 * image is an induced subgraph, i.e. every non-edge of q maps to a non-edge of
 * G.  Each step also tests the new vertex against the lists of the matched
 * vertices it is NOT adjacent to in q and keeps it only when it is absent from
 * all of them (a set difference next to Eq. 2's intersection).  Level and
 * graph engines and batches (the persistent engine: HUGE_EINVAL).  The cost
 * model's estimate stays the non-induced one, an upper bound. */
#define HUGE_PLAN_INDUCED 0x4u
/* Every injective map counted: no symmetry breaking, so each subgraph is
 * reported once per automorphism of q (Section 2's matches before the
 * automorphism classes are taken; used for queries with pinned vertices). */
#define HUGE_PLAN_ALL_MAPS 0x8u

/* huge_exec_opts.engine */
#define HUGE_ENGINE_AUTO 0
#define HUGE_ENGINE_LEVELS 1     /* host-driven Algorithm 5, one grid-wide launch per chunk */
#define HUGE_ENGINE_PERSISTENT 2 /* one persistent launch: per-workgroup Algorithm 5 + stealing */
/* Algorithm 5 with its scheduler on the device: one round (a one-thread
 * scheduler launch, then fixed-grid prepare / scan / extend launches of every
 * level, idle unless the round's action is theirs) is recorded once in a
 * hipGraph and replayed until a device flag says the query is done; the host
 * reads that flag once per 8 replays of 4 rounds.  huge_count and
 * huge_count_batch only (huge_enumerate: HUGE_EINVAL).  Strategies as on the
 * level engine: a tune table with strategy AUTO gives the per-bucket dispatch
 * (and its rows per segment), a fixed strategy runs everywhere, and AUTO
 * without a table runs HUGE_STRAT_BLOCK_MERGE_LONG.  work_limit must be 0.
 * Segments are capped at 2^24 rows.  Results equal the other engines' bit for
 * bit; huge_result.launches counts graph launches, and profile gives no
 * per-launch timing (kernel_ms stays 0). */
#define HUGE_ENGINE_GRAPH 3
#define HUGE_PERSIST_KMAX 4      /* largest query the persistent engine runs (HUGE_EINVAL above) */

typedef struct {
    uint64_t count;                    /* subgraphs found (in the selected slice) */
    uint64_t hash_sum;                 /* sum of h(g) mod 2^64, see below */
    uint64_t hash_xor;                 /* xor of h(g) */
    uint64_t level_counts[HUGE_KMAX];  /* [i]: partial matches of the first i+1 order vertices */
    double query_ms;                   /* wall time of the call (planning excluded, D2H included) */
    uint64_t peak_frontier_bytes;      /* largest device bytes held by intermediate partial matches */
    uint64_t launches;                 /* kernel launches issued */
    uint64_t steals;                   /* successful steals (persistent engine) */
    /* filled when huge_exec_opts.profile != 0 (HIP events on the exec stream),
       per kernel class HUGE_KC_*: summed device time, launches, and the
       algorithmic bytes of the work those launches did: an intersection of
       symmetry-breaking-trimmed lists must read, per input row of width i with
       j intersected lists, 4i + 16j bytes, the shortest window P whole and of
       every other window W at least 4 * min(|W|, |P|) bytes (one element per
       candidate, or the whole window if shorter), plus 4(i+1) bytes per
       emitted row */
    double kernel_ms[4];
    uint64_t kernel_launches[4];
    double alg_bytes[4];
    /* level engine: level_work[i] = candidates examined (probe-list elements inside
       the symmetry-breaking window) while extending the partial matches of level i
       (i+1 order vertices) by one vertex; 0 on the persistent engine */
    uint64_t level_work[HUGE_KMAX];
    /* persistent engine: its workgroups, and the mean and standard deviation over
       them of the time each spent in tiles and prepare passes (how evenly the
       load was spread, Section 7.3); 0 on the other engines */
    uint64_t workgroups;
    double wg_busy_ms_mean, wg_busy_ms_std;
} huge_result;
#define HUGE_KC_PREPARE 0 /* SB window trim + probe choice */
#define HUGE_KC_SCAN 1    /* exclusive scan of per-row bounds */
#define HUGE_KC_EXTEND 2  /* intersection + filters + compaction into the next level */
#define HUGE_KC_SINK 3    /* last-level intersection + filters + counting SINK (or output) */
/*
 * h(g) = mix( sum over query edges (a,b) of mix(edge(f(a), f(b))) ) with
 * edge(x, y) = (min(rx, ry) << 32) | max(rx, ry), rx the degree rank of x,
 * mix the SplitMix64 finalizer; all arithmetic mod 2^64.  h depends only on
 * the image edge set of g, so hash_sum / hash_xor do not depend on the plan,
 * the schedule or the symmetry-breaking scheme.
 */

/* intersection strategies (huge_exec_opts.strategy, huge_tune_table.strategy) */
#define HUGE_STRAT_AUTO -1        /* the tuned table's choice if one is given, else lane merge */
#define HUGE_STRAT_BSEARCH 0      /* a thread per candidate, binary search (or bitmap) per other list */
#define HUGE_STRAT_WAVE_STAGED 1  /* a wave stages each row's list windows in LDS, then searches there */
#define HUGE_STRAT_LANE_MERGE 2   /* a lane per 16 consecutive candidates, galloping cursors per list */
#define HUGE_STRAT_MERGE_SHORT 3  /* lane merge with 4 candidates per lane */
#define HUGE_STRAT_MERGE_LONG 4   /* lane merge with 64 candidates per lane (16 when rows are emitted) */
#define HUGE_STRAT_BLOCK_MERGE 5  /* lane merge, 16 per lane, every list read as register-cached 16-byte blocks */
#define HUGE_STRAT_BLOCK_MERGE_LONG 6 /* the same with 64 candidates per lane (16 when rows are emitted) */
#define HUGE_STRAT_COUNT 7

/*
 * Autotuned dispatch (Section 7.3's batch-size knob, and the choice of
 * intersection kernel): for each number j of intersected lists and each
 * bucket of the probe (shortest trimmed) list length
 *     bucket 0: < 2^6, 1: < 2^9, 2: < 2^12, 3: < 2^15, 4: >= 2^15,
 * a strategy; and per j the rows per scheduling segment.  When a table is
 * given and strategy is HUGE_STRAT_AUTO, every segment is partitioned by
 * bucket (a stable counting partition of its rows) and each bucket's work
 * runs with its own kernel.  Results never depend on the table.
 */
#define HUGE_TUNE_BUCKETS 5
typedef struct {
    int32_t strategy[HUGE_KMAX + 1][HUGE_TUNE_BUCKETS]; /* [j][bucket]; HUGE_STRAT_AUTO = library default */
    int64_t chunk_rows[HUGE_KMAX + 1];                  /* [j]; 0 = library default */
    double ms[HUGE_KMAX + 1][HUGE_TUNE_BUCKETS];        /* huge_autotune: sample time of the chosen strategy */
    int64_t items[HUGE_KMAX + 1][HUGE_TUNE_BUCKETS];    /* huge_autotune: sample work items (0 = not seen) */
} huge_tune_table;

typedef struct {
    uint64_t frontier_cap_bytes; /* device bytes for intermediate partial matches;
                                    0 = smallest workable (DFS-like), UINT64_MAX = as large as fits */
    int64_t chunk_rows;          /* rows per scheduling segment; 0 = autotuned / default */
    int32_t strategy;            /* HUGE_STRAT_*; HUGE_STRAT_AUTO = per the tune table, else lane merge */
    int32_t engine;              /* HUGE_ENGINE_* */
    int32_t work_stealing;       /* persistent engine: 1 = steal, 0 = static root split only */
    int32_t reserved0;           /* must be 0 */
    uint32_t slice_count;        /* root slice: keep matches with mix(rank(f(s))) % slice_count == slice_id, */
    uint32_t slice_id;           /* s = slice_vertex; slice_count 0 or 1 = everything (see slice_mode) */
    void *stream;                /* hipStream_t; NULL = the null stream */
    void *workspace;             /* caller-owned device memory, or NULL = library allocates */
    uint64_t workspace_bytes;
    int32_t profile;             /* 1 = time every launch with HIP events (kernel_ms etc.) */
    int32_t slice_vertex;        /* query vertex whose image is sliced (default 0; -1 = the plan's first
                                    matched vertex, order[0]; -2 = edge slice: keep the matches whose
                                    first two matched vertices (x, y) = (f(order[0]), f(order[1])), as
                                    ranks, have mix(x << 32 | y) % slice_count == slice_id, or with
                                    HUGE_SLICE_STRIDE whose entry index e (x's row, y's place in it) in
                                    the relabelled CSR has e % slice_count == slice_id: the engines then
                                    read only entries slice_id, slice_id + slice_count, ..., a sample of
                                    every vertex's list in proportion to its degree); slices of any
                                    fixed vertex, or edge slices of one plan, partition the matches,
                                    so counts add and hashes add / xor */
    uint32_t exec_flags;         /* HUGE_EXEC_* bits */
    uint32_t slice_mode;         /* how every slice selects (edge slices: see slice_vertex -2):
                                    HUGE_SLICE_MIX keeps mix(rank) % count == id, HUGE_SLICE_STRIDE keeps
                                    rank % count == id: every count-th vertex in degree order, so every
                                    slice holds the same share of each degree class.  A strided slice of
                                    the plan's first matched vertex (slice_vertex -1, or the vertex in
                                    order[0]) reads only the edge-array entries of the slice's vertices:
                                    the level engine and the graph engine gather them into the workspace
                                    first (about 8 * (nnz / count + max degree) bytes) instead of
                                    scanning every entry.  The persistent engine takes HUGE_SLICE_MIX
                                    only. */
    const huge_tune_table *tune; /* per-bucket dispatch table, or NULL (read during the call only) */
    int64_t work_limit;          /* huge_count on the level engine: stop with HUGE_STOPPED once more than this
                                    many candidates were examined (the result then covers part of the work
                                    only); 0 = no limit */
    int32_t slice2_vertex;       /* a second vertex slice, applied with the first: keep the matches whose
                                    query vertex slice2_vertex has its image in slice slice2_id of
                                    slice2_count (same slice_mode); slice2_count 0 or 1 = none.  Two plans
                                    with different first vertices a and b can then run the same sample:
                                    (a, s1 of S1) and (b, s2 of S2) in either role select the same
                                    matches, and each plan still reads only its own slice's entries.
                                    With HUGE_EXEC_SLICE2_PAIR the second slice is on a pair of
                                    adjacent query vertices (slice2_vertex, slice2_vertex2), read as an
                                    edge slice of that pair, so two plans with different first pairs
                                    can share an edge-slice sample the same way.
                                    Not on the persistent engine. */
    uint32_t slice2_count;
    uint32_t slice2_id;
    int32_t slice2_vertex2;      /* the pair's other query vertex (with HUGE_EXEC_SLICE2_PAIR), else unused */
} huge_exec_opts;
#define HUGE_SLICE_MIX 0u
#define HUGE_SLICE_STRIDE 1u
#define HUGE_EXEC_NO_HASH 0x1u /* count only: hash_sum / hash_xor are left 0 */
/* the second slice is on the pair (slice2_vertex, slice2_vertex2) of adjacent
   query vertices, read like an edge slice of that pair (its mix, or with
   HUGE_SLICE_STRIDE its entry index in the relabelled CSR) */
#define HUGE_EXEC_SLICE2_PAIR 0x2u

/* Default options: frontier cap 4 GiB, autotuned chunk and strategy, AUTO engine, no slice. */
huge_status huge_exec_opts_default(huge_exec_opts *opts);

/*
 * huge_load_csr -- load an undirected simple graph (Section 2, "Graph
 * Storage": each vertex with its adjacency list; here all on one device).
 *   n, nnz   : vertices, directed adjacency entries (= 2|E|); n < 2^31, nnz < 2^32
 *   row_ptr  : int64[n+1], row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz
 *   col      : int32[nnz], each list strictly ascending, symmetric, no self-loops
 *   flags    : HUGE_HOST_PTRS or HUGE_DEVICE_PTRS, optionally | HUGE_NO_VALIDATE
 *   stream   : hipStream_t for the load kernels (NULL = null stream)
 * The library relabels by degree rank on the GPU, re-sorts every list and
 * builds a degree sketch; the inputs are not retained.  Unless
 * HUGE_NO_HUB_BITMAP is given it also keeps an n-bit adjacency bitmap for each
 * of the highest-degree vertices (degree >= 256, at most HUGE_HUB_BYTES bytes
 * in total, environment variable, default 16 GiB, and at most a quarter of the
 * free device memory), so that a membership test
 * against a hub's list is one load.  Errors: HUGE_EGRAPH
 * (hygiene), HUGE_ENOMEM, HUGE_EDEVICE, HUGE_EINVAL.
 */
huge_status huge_load_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                          void *stream, huge_graph **out);
/*
 * huge_load_csr_directed -- a directed graph (Section 2: the techniques carry
 * over to directed graphs) from out-lists: row_ptr int64[n+1], col int32[n_arcs]
 * in host memory (HUGE_HOST_PTRS; copied), each list strictly ascending, no
 * self-loops.  The graph the engines search is the undirected skeleton (every
 * pair joined by an arc in either direction, relabelled by degree rank as by
 * huge_load_csr); the out-lists are kept beside it in rank IDs, and a directed
 * query's edges are checked in their direction by lookups in them.  Undirected
 * queries on a directed graph match its skeleton.  Errors: HUGE_EGRAPH,
 * HUGE_EINVAL, HUGE_ENOMEM, HUGE_EDEVICE.
 */
huge_status huge_load_csr_directed(int64_t n, int64_t n_arcs, const int64_t *row_ptr, const int32_t *col,
                                   uint32_t flags, void *stream, huge_graph **out);
void huge_graph_free(huge_graph *g);

/*
 * huge_load_csr_labelled -- huge_load_csr for a vertex-labelled graph (the
 * labelled graphs the paper's techniques extend to, Section 2): labels[u] is
 * the label of vertex u (original IDs), in host or device memory as flags
 * say; read, not kept.  Labelled queries (huge_plan_create_labelled) need such
 * a graph; unlabelled queries ignore the labels.
 */
huge_status huge_load_csr_labelled(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                                   const int32_t *labels, uint32_t flags, void *stream, huge_graph **out);

typedef struct {
    int64_t n, nnz;
    int64_t max_degree;
    uint64_t degree_hist[32];   /* [0]: degree 0; [b>0]: 2^(b-1) <= degree < 2^b */
    double degree_moments[8];   /* sum_u d_u^p, p = 0..7 */
    double load_ms;
    uint64_t device_bytes;      /* device memory held by the graph */
    int64_t hub_count;          /* vertices with an adjacency bitmap (the highest degree ranks) */
    int64_t hub_min_degree;     /* smallest degree among them */
} huge_graph_info;
huge_status huge_graph_get_info(const huge_graph *g, huge_graph_info *out);

/*
 * Copy the relabelled device graph back to the host (for inspection / tests).
 * row_ptr int64[n+1], col int32[nnz], inv_rank int32[n] (rank -> original ID);
 * any pointer may be NULL to skip it.
 */
huge_status huge_graph_export(const huge_graph *g, int64_t *row_ptr, int32_t *col, int32_t *inv_rank);

/*
 * huge_plan -- build the execution plan of one query (host only).
 *   g        : the graph whose degree sketch drives the cost model; NULL plans
 *              without statistics (the lexicographically first connected
 *              order unless one is given)
 *   k        : query vertices 0..k-1, 2 <= k <= 8
 *   qedges   : 2*n_qedges ints, undirected, no self/duplicate edges; q connected
 *   order    : k entries, a matching order whose every prefix is connected
 *              (user-supplied logical plan, Remark 3.2), or NULL: the planner
 *              picks one (cost model of Algorithm 1 restricted to left-deep
 *              worst-case-optimal plans, or the learned model per flags)
 * Symmetry-breaking constraints come from q alone (Grochow-Kellis with a
 * lowest-ID tie-break), never from the order, so every order gives the same
 * matches.  Errors: HUGE_EQUERY, HUGE_EORDER, HUGE_EINVAL.
 */
huge_status huge_plan_create(const huge_graph *g, int32_t k, int32_t n_qedges, const int32_t *qedges,
                             const int32_t *order, uint32_t flags, huge_plan **out);
void huge_plan_free(huge_plan *p);

/*
 * huge_plan_create_labelled -- huge_plan_create for a labelled query:
 * qlabels[v] (k ints) is the label the image of query vertex v must carry, -1
 * for any label.  A match is an injective map that keeps q's edges and these
 * labels; matches are reported once per class under the automorphisms of q
 * that also keep its labels (-1 counting as a label of its own), which is what
 * the symmetry-breaking constraints are computed from.  Each step filters its
 * candidates by label (next to the injectivity filter of Algorithm 4).  flags:
 * HUGE_PLAN_INDUCED or 0 (cost model; the estimate ignores labels).  Runs on
 * a graph from huge_load_csr_labelled (HUGE_EINVAL otherwise) on the level and
 * graph engines and in batches (the persistent engine: HUGE_EINVAL).
 */
huge_status huge_plan_create_labelled(const huge_graph *g, int32_t k, int32_t n_qedges, const int32_t *qedges,
                                      const int32_t *qlabels, const int32_t *order, uint32_t flags, huge_plan **out);

/*
 * huge_plan_create_directed -- a directed query: arcs holds n_arcs directed
 * edges a -> b over vertices 0..k-1 (both directions of a pair may be given);
 * its undirected skeleton must be connected.  A match is an injective map
 * that keeps every edge's direction (and labels, with qlabels as in
 * huge_plan_create_labelled, or NULL), counted once per class of the
 * automorphisms of q that keep directions (and labels), from which the
 * symmetry-breaking constraints come.  The order (or the cost model's, on the
 * skeleton) and Eq. 2's intersections run on the skeleton; each step then
 * looks up its directed edges to matched vertices in the out-lists.  The
 * set-hash hashes the image's skeleton edges.  Needs a graph from
 * huge_load_csr_directed (HUGE_EINVAL otherwise).  Level and graph engines and
 * batches (the persistent engine and bushy plans: HUGE_EINVAL).
 */
huge_status huge_plan_create_directed(const huge_graph *g, int32_t k, int32_t n_arcs, const int32_t *arcs,
                                      const int32_t *qlabels, const int32_t *order, huge_plan **out);

/*
 * huge_plan_prefix -- the plan of the first `size` vertices (2..k) of p's
 * order: the induced prefix, numbered by order position, with p's
 * symmetry-breaking constraints restricted to it.  Its count is p's
 * level_counts[size-1] (the partial matches that p's run holds at that level).
 */
huge_status huge_plan_prefix(const huge_plan *p, int32_t size, huge_plan **out);

/*
 * Plan details: order_out int32[k]; n_sb number of constraints; sb_pairs
 * int32[2*28] as (a, b) meaning rank(f(a)) < rank(f(b)); est_cost: the
 * model's estimated total partial matches (sum over prefixes).  NULL skips.
 */
huge_status huge_plan_info(const huge_plan *p, int32_t *k, int32_t *order_out, int32_t *n_sb, int32_t *sb_pairs,
                           double *est_cost);

/*
 * The estimator behind the plan's order, per prefix of that order: est[s-1]
 * (s = 1..k) is the estimated number of partial matches of the induced prefix
 * of the first s order vertices that satisfy the symmetry-breaking constraints
 * inside it (Algorithm 1's |R(q')|).  Cost model: the Chung-Lu estimate
 * prod over prefix vertices v of M_{deg(v)} / (2m)^{edges}, M_p = sum over data
 * vertices u of d_u^p, times the fraction of the prefix's vertex orderings that
 * satisfy its constraints; learned plans: the model's predictions.  Entries
 * past k are 0; all are 0 without graph statistics.  est holds HUGE_KMAX doubles.
 */
huge_status huge_plan_estimates(const huge_plan *p, double *est);

/*
 * Bushy plans: Algorithm 1 (OptimalExecutionPlan, Section 3.3) over the
 * join-based framework of Section 3.1 (Eq. 1), stars as the join unit, with
 * each join's physical setting from the settings equation of Section 3.3.
 * A sub-query is a connected set of query edges; a star (every edge at one
 * centre) is a join unit, costed at its estimated result size; any other
 * sub-query q' is a two-way join (q', l, r) of two connected edge-disjoint
 * parts, costed M(l) + M(r) + |R(q')| plus its communication:
 *   machines * |E_G| when it pulls (r a star (c; L) with L inside V(l) --
 *   a complete star join -- or with c inside V(l)), else |R(l)| + |R(r)|.
 * |R| is the Chung-Lu estimate of huge_plan_estimates over the part's edges
 * and vertices, with the symmetry-breaking constraints inside it.  Kinds:
 */
#define HUGE_BUSHY_UNIT 0      /* a star join unit: SCAN of one edge, EXTENDs from the centre (Section 5.1) */
#define HUGE_BUSHY_EXTEND 1    /* complete star join, right = star (c; L), c new, L in V(left): one PULL-EXTEND
                                  of c intersecting the lists of L (Eq. 2) */
#define HUGE_BUSHY_PULL_HASH 2 /* pulled hash join, right = star (c; L) with c in V(left): the edges from c to
                                  L inside V(left) verified by lookup (the verify-only EXTEND with its hint),
                                  then one EXTEND from c per other leaf (Section 5.1) */
#define HUGE_BUSHY_PUSH 3      /* PUSH-JOIN (Section 4.3): both parts materialised, hash-joined on their shared
                                  vertices */
#define HUGE_BUSHY_MAX_EDGES 15
#define HUGE_BUSHY_MAX_NODES 29 /* 2 * HUGE_BUSHY_MAX_EDGES - 1 */

typedef struct {
    uint32_t edge_mask;   /* bit e: query edge e, in the order given at creation */
    uint32_t vertex_mask; /* its query vertices */
    int32_t kind;         /* HUGE_BUSHY_* */
    int32_t left, right;  /* children (node indices), -1 for units; pulled joins keep the star on the right */
    int32_t star_root;    /* units and pulled joins: the star's centre; PUSH-JOIN: -1 */
    int32_t reserved;
    double est_rows;      /* estimated |R(q')| */
    double cost;          /* Algorithm 1's M_cost[q'] */
} huge_bushy_node;

/*
 * huge_plan_create_bushy -- a bushy plan by Algorithm 1.  stats: the degree
 * statistics the estimates use (NULL: g's; g may be NULL when stats is given,
 * for planning only); machines: Algorithm 1's k (1 for one GPU; 0 makes every
 * pull free, large values make pulling dear); qlabels: as
 * huge_plan_create_labelled, or NULL.  At most HUGE_BUSHY_MAX_EDGES query
 * edges (HUGE_EQUERY).  Symmetry breaking is q's, as for every plan, and
 * each part of the tree applies the constraints inside it.  The plan runs
 * through huge_count (level engine; HUGE_EINVAL for other engines, for edge
 * slices, second slices, work limits and induced matching): chains of pulled
 * joins over a SCAN run on the level engine with a bounded frontier; the
 * parts below and around a PUSH-JOIN are materialised in device memory that
 * the call allocates (sized exactly by a counting pass) and frees.
 */
huge_status huge_plan_create_bushy(const huge_graph *g, const huge_graph_info *stats, int32_t k, int32_t n_qedges,
                                   const int32_t *qedges, const int32_t *qlabels, double machines, huge_plan **out);
/*
 * huge_plan_create_bushy_tree -- a bushy plan from a logical plan the caller
 * gives (Remark 3.2: existing logical plans plug into the optimiser, which
 * only configures each join's physical setting).  joins: n_joins pairs of edge
 * masks (left, right) over the query edges in the order given; the pairs must
 * form one tree whose root splits the whole query: each part connected, the
 * two parts of a join disjoint and non-empty, every part that no join splits
 * a star.  Each join's setting follows the settings equation (a star side is
 * read as the right part); costs are computed as Algorithm 1's for the report.
 * Errors: HUGE_EORDER for a malformed tree, otherwise as huge_plan_create_bushy.
 */
huge_status huge_plan_create_bushy_tree(const huge_graph *g, const huge_graph_info *stats, int32_t k,
                                        int32_t n_qedges, const int32_t *qedges, const int32_t *qlabels,
                                        const uint32_t *joins, int32_t n_joins, double machines, huge_plan **out);
/* The join tree of a bushy plan, children before parents, the root last
   (HUGE_EINVAL for other plans).  nodes may be NULL to read the count. */
huge_status huge_plan_bushy_nodes(const huge_plan *p, huge_bushy_node *nodes, int32_t max_nodes, int32_t *n_nodes);

/* Device workspace needed by huge_count / huge_enumerate for these options
 * (engine included: the graph engine also keeps its scheduler state there,
 * and the persistent engine its per-workgroup buffers, boards and counters). */
huge_status huge_workspace_size(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts,
                                uint64_t *bytes);

/*
 * huge_count -- enumerate and count (SINK by counting, Section 4.2).  Fills
 * count, hash_sum, hash_xor, level_counts, timing and frontier statistics.
 * opts NULL = huge_exec_opts_default.  Blocks until the result is on the host.
 * Returns HUGE_STOPPED (out filled, partial) when opts->work_limit ended the run.
 */
huge_status huge_count(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, huge_result *out);
/* The rows of one scheduling segment (the batch of input rows a level's operator
   takes per scheduling, Sections 5.2 and 7.3) that the level engine uses at each
   level w = 2..k-1 under these options: rows[w], HUGE_KMAX entries, 0 elsewhere.
   Precedence: opts->chunk_rows; for learned plans the model's choice -- enough
   rows that one segment's predicted output (the model's estimate of the step's
   fan-out) fills the next level's queue once, 2^12..2^22, the last level excepted;
   the tune table's choice per |Ext|; 2^22.  Each is capped by the level's queue
   (and level 2 by its rows). */
huge_status huge_segment_rows(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, int64_t *rows);
/*
 * huge_count_paths -- hop-constrained path queries (Section 6 lists them among
 * the applications): counts[L] (L = 1..max_hops, max_hops <= 7; counts[0] = 0)
 * is the number of simple paths of exactly L edges from s to t (original IDs,
 * s != t).  Each length runs as the path query 0 - 1 - ... - L in that order,
 * every map counted (HUGE_PLAN_ALL_MAPS), with query vertex 0 pinned to s by a
 * strided root slice of count n (one root: s's rank) and vertex L pinned to t
 * by a second strided slice; the options' engine, cap and tune table apply
 * (slice options must be unset).  counts holds max_hops + 1 entries.
 */
huge_status huge_count_paths(const huge_graph *g, int32_t s, int32_t t, int32_t max_hops,
                             const huge_exec_opts *opts, uint64_t *counts);
/* huge_count of a bushy plan that also reports, per tree node, the rows its
   part produced (node_rows[i] for node i < max_nodes; the root's is the
   count). */
huge_status huge_count_bushy(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, huge_result *out,
                             int64_t *node_rows, int32_t max_nodes);

/*
 * huge_count_noalloc -- huge_count for callers that cannot allocate memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It runs the level engine with every device buffer it needs
 * (counters, segment buffers, queues, scan scratch, a gathered level 2) in one
 * file-scope device array of 256 MiB (huge_noalloc_capacity), which each
 * device that runs it holds until the process ends, and its host read-backs
 * in a static host block: it calls no allocator of any kind.  Options as
 * huge_count, except: no workspace (HUGE_EINVAL), profile 0, engine AUTO or
 * LEVELS, a finite frontier_cap_bytes; options whose workspace
 * (huge_workspace_size) exceeds the array fail with HUGE_ENOMEM: lower
 * frontier_cap_bytes or chunk_rows (frontier_cap_bytes = 64 MiB with
 * chunk_rows = 2^18 fits every query of up to 8 vertices, tuned or not; a
 * strided slice adds 8 * (nnz / slice_count + max degree) bytes).  The array keeps the last call's
 * contents; each call clears its counters first.  Calls on one device take
 * turns (one lock per device): they are serialised, never interleaved.
 * Results equal huge_count's bit for bit.
 */
huge_status huge_count_noalloc(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, huge_result *out);
/* Bytes of the device array huge_count_noalloc runs in. */
huge_status huge_noalloc_capacity(uint64_t *bytes);

/*
 * huge_enumerate -- enumerate and deliver every match.  Matches are written to
 * host_buf (buf_rows rows of k int32, row = f(0), ..., f(k-1) indexed by query
 * vertex, original IDs) and cb(user, host_buf, nrows, k) is called on the
 * calling thread each time the buffer is full and once at the end.  A nonzero
 * return from cb stops the run with HUGE_STOPPED; out->count is then the
 * number of rows delivered.  Row order is unspecified.  Runs on the level
 * engine (HUGE_ENGINE_GRAPH: HUGE_EINVAL).
 */
typedef int (*huge_emit_fn)(void *user, const int32_t *rows, int64_t nrows, int32_t k);
huge_status huge_enumerate(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, int32_t *host_buf,
                           int64_t buf_rows, huge_emit_fn cb, void *user, huge_result *out);

/*
 * huge_count_batch -- count np queries (the batching of Section 4.2, and
 * Section 5.3's sharing of the workers between queries); outs[np], in the
 * order of plans.  Results equal np separate huge_count calls bit for bit.
 *
 * engine GRAPH (batched rounds): every query keeps its own Algorithm 5 state,
 * queues (an equal share of frontier_cap_bytes) and segment buffers on the
 * device.  One round advances every query by one action (a one-workgroup
 * scheduler launch, one thread per query), then runs one prepare launch, one
 * batched bounds scan and one extend launch per (level, last level or not)
 * for all queries together: their workgroups claim tiles in order across the
 * queries, so many small queries fill the chip together.  Rounds are recorded
 * once in a hipGraph and replayed on opts->stream until no query is active.
 * Queries of 2 vertices run first on the level engine.  At most 256 queries
 * share a round (larger batches run 256 at a time).  Strategy: a fixed
 * strategy for every query (2..6 a lane merge; 0 and 1 binary-search tiles),
 * or AUTO: with a tune table, a query's level runs binary-search tiles when the
 * table's buckets at its Ext size give more work items to strategies 0 and 1
 * than to the lane merges, and lane merges otherwise, in the same extend launch
 * (each tile belongs to one query); the launch's lane merge is the one the
 * table gives most work to over the merging queries (searches count as
 * HUGE_STRAT_MERGE_SHORT); without a table every level merges,
 * HUGE_STRAT_BLOCK_MERGE_LONG for last levels and HUGE_STRAT_BLOCK_MERGE
 * otherwise; segments hold chunk_rows rows (default 2^20, or a learned plan's
 * choice; a tune table's segment rows apply to the level engine only).  work_limit must be 0.  Workspace:
 * opts->workspace when it holds huge_batch_workspace_size bytes, else
 * allocated for the call.  Each result's query_ms is the whole batch's wall
 * time and launches counts graph launches.
 *
 * engine AUTO or LEVELS: a few host workers (environment variable
 * HUGE_BATCH_STREAMS, default 4), each with its own HIP stream, workspace
 * (sized for the largest query; opts->workspace is not used; kept allocated
 * between calls, one pool per device, until the process ends) and an equal
 * share of frontier_cap_bytes, run the queries on the level engine
 * concurrently; work queued on opts->stream before the call runs first;
 * batch calls on one device take turns.  engine PERSISTENT: the queries of
 * 3..HUGE_PERSIST_KMAX vertices run in one persistent launch (they share the
 * workgroups, the frontier budget and the stealing pool, Section 5.3), the
 * others on the level engine one after another on opts->stream.
 */
huge_status huge_count_batch(const huge_graph *g, const huge_plan *const *plans, int32_t np,
                             const huge_exec_opts *opts, huge_result *outs);

/* Device workspace huge_count_batch needs on the graph engine for these plans
 * and options (HUGE_EINVAL for another engine). */
huge_status huge_batch_workspace_size(const huge_graph *g, const huge_plan *const *plans, int32_t np,
                                      const huge_exec_opts *opts, uint64_t *bytes);

/*
 * huge_motif_count -- motif counting over every connected pattern of k
 * vertices (2 <= k <= HUGE_MOTIF_KMAX): the graph-pattern-mining use of
 * Section 6, which runs subgraph enumeration over every pattern of interest,
 * with both readings of an occurrence from Section 2.  For each connected
 * k-vertex graph up to isomorphism (1, 1, 2, 6, 21 and 112 of them for k = 1..6;
 * ordered by edge count, then by the representative's edge bits), out[i] gets
 * the representative (query vertices 0..k-1, edges), `noninduced`, the number
 * of subgraphs of G isomorphic to it with their set-hashes (huge_count's
 * count, hash_sum, hash_xor), and `induced`, the number of k-vertex sets X
 * whose induced subgraph G[X] is isomorphic to it.  The induced counts follow
 * exactly from the non-induced ones: X with G[X] isomorphic to q holds
 * c(p, q) subgraphs isomorphic to p, c(p, q) the number of spanning subgraphs
 * of q isomorphic to p, and the triangular system is solved from the densest
 * pattern down.  The patterns run as one batch (huge_count_batch with the same
 * options: engine GRAPH gives batched rounds).  No slices or work limit
 * (HUGE_EINVAL): induced counts need every pattern's whole count.  out holds
 * HUGE_MOTIF_MAX entries; *n_out receives the number of patterns.
 */
#define HUGE_MOTIF_KMAX 6
#define HUGE_MOTIF_MAX 112
typedef struct {
    int32_t k, n_edges;
    int32_t edges[30];           /* 2 * n_edges query-vertex IDs */
    uint64_t noninduced;         /* subgraphs of G isomorphic to the pattern */
    uint64_t induced;            /* vertex sets whose induced subgraph is isomorphic to it */
    uint64_t hash_sum, hash_xor; /* set-hashes of the non-induced matches */
} huge_motif;
huge_status huge_motif_count(const huge_graph *g, int32_t k, const huge_exec_opts *opts, huge_motif *out,
                             int32_t *n_out);

/* ------------------------------------------------------------------------
 * Learned cost model.  The optimiser of Section 3.3 (Algorithm 1) ranks
 * plans by estimated sizes and leaves the estimator open; this is a 2-layer
 * MLP that predicts, for the step that produces prefix s of an order,
 * log(1 + W_s) with W_s the candidates that step examines (the engine's
 * level_work[s-2]), from HUGE_MLP_F features of the prefix and of the graph's
 * degree sketch:
 *     y = b2 + sum_h W2[h] relu(b1[h] + sum_f W1[f][h] xn[f]),
 *     xn[f] = (x[f] - xmean[f]) * xinv[f],  label = y * tstd + tmean.
 * Parameters (float, HUGE_MLP_PARAMS of them) are laid out as
 * W1[f * HUGE_MLP_H + h] | b1[HUGE_MLP_H] | W2[HUGE_MLP_H] | b2.  The library
 * keeps FP32 master weights and computes with their BF16 (round to nearest
 * even) copies, accumulating in FP32.  A model lives on the device that was
 * current when it was created; its calls must run there.
 * ------------------------------------------------------------------------ */
#define HUGE_MLP_F 128
#define HUGE_MLP_H 256
#define HUGE_MLP_PARAMS (HUGE_MLP_F * HUGE_MLP_H + 2 * HUGE_MLP_H + 1)
typedef struct huge_model huge_model;

/* A model with zero weights, xmean 0, xinv 1, tmean 0, tstd 1.  Errors: HUGE_ENOMEM, HUGE_EDEVICE. */
huge_status huge_model_create(huge_model **out);
void huge_model_free(huge_model *m);

/*
 * Set host-side values; NULL leaves that part unchanged.  Setting params also
 * resets the Adam state.  Errors: HUGE_EINVAL (non-finite parameter, tstd <= 0).
 */
huge_status huge_model_set(huge_model *m, const float *params, const float *xmean, const float *xinv, float tmean,
                           float tstd);
huge_status huge_model_get(const huge_model *m, float *params, float *xmean, float *xinv, float *tmean, float *tstd);

/* y[B] = predicted label (log(1 + W_s)) for x[B][HUGE_MLP_F]; device pointers, asynchronous on stream. */
huge_status huge_model_forward(const huge_model *m, const float *x, int64_t B, float *y, void *stream);

/*
 * Gradient of L = (1/B) sum_r (yn_r - (t_r - tmean)/tstd)^2, yn the network
 * output before de-standardisation, at the current BF16 weights.  x, t device;
 * grad host float[HUGE_MLP_PARAMS] (or NULL); loss host (or NULL).  Blocks.
 */
huge_status huge_model_grad(const huge_model *m, const float *x, const float *t, int64_t B, float *grad, double *loss,
                            void *stream);

/*
 * Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) on n
 * samples x[n][HUGE_MLP_F], t[n] (device), `epochs` passes of minibatches of
 * `batch` samples, reshuffled each pass from `seed`.  loss_out (host
 * float[epochs] or NULL) receives each pass's mean squared error in
 * standardised units.  Blocks.  Errors: HUGE_EINVAL, HUGE_ENOMEM, HUGE_EDEVICE.
 */
huge_status huge_model_train(huge_model *m, const float *x, const float *t, int64_t n, int32_t epochs, int64_t batch,
                             float lr, uint64_t seed, float *loss_out, void *stream);

/*
 * The model's input for prefix `size` (2..k) of `order` (NULL = the plan's
 * order) of plan p's query on graph g: out host float[HUGE_MLP_F].
 */
huge_status huge_plan_features(const huge_graph *g, const huge_plan *p, const int32_t *order, int32_t size,
                               float *out);

/*
 * huge_plan_create with the learned model as the estimator: every connected
 * order is scored in one batched forward pass on `stream`; the order with the
 * smallest estimated sum over steps s = 3..k of W_s (ties to the
 * lexicographically smallest) replaces the cost model's order only when its
 * predicted sum is less than half of the cost model's order's; the plan's
 * est_cost is the predicted sum of the order kept.  The plan only decides the order (and chunk sizes): counts are
 * exact whatever it picks.  huge_plan_create with HUGE_PLAN_LEARNED and no
 * model returns HUGE_EINVAL.
 */
huge_status huge_plan_create_learned(const huge_graph *g, const huge_model *m, int32_t k, int32_t n_qedges,
                                     const int32_t *qedges, const int32_t *order, void *stream, huge_plan **out);
/*
 * As huge_plan_create_learned, with flags: HUGE_PLAN_VERIFY runs the cost
 * model's order and the model's two best orders on a strided edge slice of
 * each order's own first matched pair (slice 0 of S: every S-th entry of the
 * relabelled CSR, so each order reads only its own sample's entries), S the
 * smallest power of 8 from 512 at which the cost model's order examines at
 * most 4e7 candidates (when no edge sample of 64 entries or more fits, strided
 * root slices of the first matched vertex, at least 4 roots); the others stop
 * at 3 times its candidates.  The order with the
 * least device time wins; the cost model's order keeps ties within 10%.  This
 * costs a few milliseconds of device time per order, on `stream`.
 */
huge_status huge_plan_create_learned2(const huge_graph *g, const huge_model *m, int32_t k, int32_t n_qedges,
                                      const int32_t *qedges, const int32_t *order, uint32_t flags, void *stream,
                                      huge_plan **out);

/*
 * huge_autotune -- fill a dispatch table by timing, on the graph itself, the
 * work of the given plans on one root slice (opts->slice_count /
 * slice_id / slice_vertex choose the sample; slice_count <= 1 means the
 * whole graph): every strategy is run on the same sample and, per (j,
 * bucket), the fastest is kept; then per j the segment size among
 * {2^18, 2^20, 2^22} rows.  Uses the level engine on opts->stream with HIP
 * events around every launch.  Buckets or j never seen keep
 * HUGE_STRAT_AUTO.  Errors: as huge_count.
 */
huge_status huge_autotune(const huge_graph *g, const huge_plan *const *plans, int32_t np, const huge_exec_opts *opts,
                          huge_tune_table *out);

/*
 * Content digest of the relabelled graph, the tune cache key: a 64-bit digest
 * of the CSR computed on the device at load, with n and nnz, as text of at
 * most 64 characters + NUL.
 */
huge_status huge_graph_digest(const huge_graph *g, char *out65);

/* The current device's architecture name and compute-unit count, e.g. "gfx950:sramecc+:xnack- 256CU"
   (at most len-1 characters + NUL): the GPU part of the tune cache key. */
huge_status huge_device_name(char *out, int32_t len);

const char *huge_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HUGE_H */
