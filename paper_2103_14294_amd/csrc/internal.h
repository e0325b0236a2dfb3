// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/huge.h"

namespace huge {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
std::string last_error_text();  // this thread's last error message

struct Error {
    huge_status st;
};

#define HUGE_HIP(call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            ::huge::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            throw ::huge::Error{e_ == hipErrorOutOfMemory ? HUGE_ENOMEM : HUGE_EDEVICE};              \
        }                                                                                           \
    } while (0)

#define HUGE_FAIL(status, ...)                 \
    do {                                       \
        ::huge::set_error(__VA_ARGS__);        \
        throw ::huge::Error{status};           \
    } while (0)

// ---------------------------------------------------------------------------
// device graph (relabelled by degree rank: vertex IDs are ranks)
// ---------------------------------------------------------------------------
struct GraphDev {
    int64_t n;
    int64_t nnz;
    const int64_t *rp;   // [n+1]
    const int32_t *col;  // [nnz], each list strictly ascending
    const int32_t *src;  // [nnz], src[e] = the row that holds entry e
    const uint32_t *hub_bm;  // adjacency bitmaps of vertices hub_base..n-1, hub_words words each
    int64_t hub_words;
    int32_t hub_base;        // first vertex (rank) with a bitmap; n when there is none
    int32_t pad;
    // level-2 rows of one execution: row r is edge-array entry l2_idx[r], or
    // entry r when l2_idx is NULL (every entry)
    const int64_t *l2_idx = nullptr;
    int64_t l2_first = 0, l2_stride = 1;  // without l2_idx: row r is entry l2_first + r * l2_stride
    const int32_t *label = nullptr;  // vertex labels by rank (labelled graphs), or NULL
    // directed graphs: out-lists by rank, each ascending (the lists above are the
    // undirected skeleton); NULL for undirected graphs
    const int64_t *drp = nullptr;
    const int32_t *dcol = nullptr;
};

}  // namespace huge

struct huge_graph {
    huge::GraphDev dev;
    int64_t *rp = nullptr;
    int32_t *col = nullptr;
    int32_t *src = nullptr;
    int32_t *inv_rank = nullptr;  // rank -> original ID
    uint32_t *hub_bm = nullptr;
    int32_t *label = nullptr;     // vertex labels by rank, or NULL (unlabelled)
    int64_t *drp = nullptr;       // directed graphs: out-lists by rank (dev.drp / dev.dcol)
    int32_t *dcol = nullptr;
    bool directed = false;
    huge_graph_info info{};
    int device = 0;
    std::string sha;  // content digest of the relabelled CSR (autotune cache key)
};

namespace huge {

// ---------------------------------------------------------------------------
// plan: one PULL-EXTEND step per new query-vertex position i = 1..k-1
// ---------------------------------------------------------------------------
struct DevStep {
    uint32_t ext;   // positions p < i adjacent to position i in q (lists to intersect)
    uint32_t lo;    // positions p with constraint f[p] < v
    uint32_t hi;    // positions p with constraint v < f[p]
    uint32_t neq;   // positions p < i not in ext (injectivity checks)
    int32_t slice;  // slice filters on position i's vertex: bit 0 the slice, bit 1 the second slice
    uint32_t nadj;  // induced plans: positions p < i not adjacent to position i in q (v must not be in N(f[p]))
    int32_t label;  // labelled plans: the label position i's vertex must carry, -1 any
    uint32_t vadj;  // positions p < i whose lists must hold position i's vertex, looked up only (never the
                    // probe): the verify-only edges of a bushy plan's pulled hash joins
    uint32_t dout;  // directed plans: positions p < i with a query edge p -> i (f[p] -> v must be an arc)
    uint32_t din;   // ... and with an edge i -> p (v -> f[p] must be an arc)
};

struct DevPlan {
    int32_t k;
    int32_t ne;                 // query edges, as position pairs ea < eb
    uint8_t ea[32], eb[32];
    uint8_t pos[HUGE_KMAX];     // pos[v] = position of query vertex v
    DevStep st[HUGE_KMAX];      // st[i], i = 1..k-1; st[i].slice marks the sliced vertices' positions
    uint32_t slice_count, slice_id;
    int32_t edge_slice;         // slice the level-2 rows (ordered pairs f[0], f[1]) instead of a vertex:
                                // 1 by the pair's mix, 2 by its entry index (rows pre-selected by stride)
    int32_t slice_mode;         // vertex slices: 0 mix(v) % count, 1 v % count (v a rank)
    uint32_t slice2_count, slice2_id;  // second slice (1, 0 = none)
    int32_t p2a, p2b;           // second slice on the pair of these positions (-1: a vertex slice)
};

}  // namespace huge

struct huge_plan {
    int32_t k = 0;
    std::vector<std::pair<int, int>> edges;  // query edges (a < b)
    int adj[HUGE_KMAX][HUGE_KMAX] = {};
    std::vector<std::pair<int, int>> sb;     // a < b constraints (query vertex IDs)
    int32_t naut = 0;
    int32_t order[HUGE_KMAX] = {};
    double est_cost = 0;                     // sum over prefixes of estimated partial matches
    double est_prefix[HUGE_KMAX] = {};       // estimated partial matches per prefix size
    uint32_t flags = 0;
    bool induced = false;                    // HUGE_PLAN_INDUCED: non-edges of q must map to non-edges
    int32_t qlabel[HUGE_KMAX] = {-1, -1, -1, -1, -1, -1, -1, -1};  // labelled queries: label per query vertex
    bool labelled = false;
    huge::DevPlan dev{};
    std::vector<huge_bushy_node> bushy;      // bushy plans (Algorithm 1): the join tree, root last; else empty
    bool model_batch = false;                // learned plans: segment rows from the predicted fan-outs
    bool directed = false;                   // directed query: dadj[a][b] for every edge a -> b; `edges` is
    int dadj[HUGE_KMAX][HUGE_KMAX] = {};     // its undirected skeleton
};

namespace huge {
// Learned plans choose the input rows of each scheduling segment (the batch
// size of Section 7.3) from the model's predicted fan-out of the step: enough
// rows that one segment's predicted output fills the next level's queue once,
// between 2^12 and 2^22.  0: no choice (other plans, the last level, no
// prediction).  est_prefix[s - 1] predicts the partial matches of s vertices.
inline int64_t model_segment_rows(const huge_plan *p, int W, int64_t out_queue_rows) {
    if (!p->model_batch || W < 2 || W >= p->k - 1) return 0;
    const double a = p->est_prefix[W - 1], b = p->est_prefix[W];
    if (!(a > 0) || !(b > 0)) return 0;
    const double rows = (double)out_queue_rows * a / b;
    return (int64_t)(rows < 4096.0 ? 4096.0 : rows > 4194304.0 ? 4194304.0 : rows);
}
}  // namespace huge

// learned cardinality model (mlp.hip): FP32 master weights, BF16 copies used
// by the kernels, Adam moments and the feature / target standardisation
struct huge_model {
    void *mem = nullptr;
    float *w = nullptr, *m = nullptr, *v = nullptr;  // [HUGE_MLP_PARAMS] each
    uint16_t *wb = nullptr;                          // BF16 copy of w
    float *xmean = nullptr, *xinv = nullptr;         // [HUGE_MLP_F]
    float tmean = 0.f, tstd = 1.f;
    int64_t step = 0;  // Adam steps taken
    int device = 0;
};

namespace huge {

// plan.cpp
void plan_build(const huge_graph *g, int k, int ne, const int32_t *qe, const int32_t *order, uint32_t flags,
                const huge_model *model, hipStream_t st, huge_plan *out, const int32_t *qlabels = nullptr,
                int narcs = 0, const int32_t *arcs = nullptr);
// graph.hip: a directed graph from out-lists (host memory): the skeleton loaded as usual,
// the out-lists relabelled by rank beside it
huge_graph *graph_load_directed(int64_t n, int64_t narcs, const int64_t *rp, const int32_t *col, uint32_t flags,
                                hipStream_t stream);
// a labelled plan needs a labelled graph, a directed plan a directed graph (HUGE_EINVAL otherwise)
void check_labels(const huge_graph *g, const huge_plan *p);
bool order_connected(const huge_plan &p, const int32_t *order);
void plan_set_order(huge_plan &p, const int32_t *order);
double estimate_prefix(const huge_graph_info &gi, const huge_plan &p, const int32_t *order, int size);
void plan_prefix(const huge_plan &p, int size, huge_plan *q);
void all_connected_orders(const huge_plan &p, std::vector<std::vector<int32_t>> &out);

// learn.cpp
void plan_features(const huge_graph_info &gi, const huge_plan &p, const int32_t *order, int size, float *out);
void learned_estimates(const huge_graph *g, const huge_model *m, const huge_plan &p,
                       const std::vector<std::vector<int32_t>> &orders, hipStream_t st, std::vector<double> &est);

// mlp.hip
huge_model *model_create();
void model_free(huge_model *m);
void model_set(huge_model *m, const float *params, const float *xmean, const float *xinv, float tmean, float tstd);
void model_get(const huge_model *m, float *params, float *xmean, float *xinv, float *tmean, float *tstd);
void model_forward(const huge_model *m, const float *x, int64_t B, float *y, hipStream_t st);
void model_grad(const huge_model *m, const float *x, const float *t, int64_t B, float *grad_host, double *loss,
                hipStream_t st);
void model_train(huge_model *m, const float *x, const float *t, int64_t N, int epochs, int64_t batch, float lr,
                 uint64_t seed, float *loss_out, hipStream_t st);

// graph.hip
huge_graph *graph_load(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *col, uint32_t flags,
                       hipStream_t stream);
// labels[u] by original ID (host or device memory per flags) -> g->label by rank
void graph_set_labels(huge_graph *g, const int32_t *labels, uint32_t flags, hipStream_t stream);
void graph_free(huge_graph *g);

// engine.cpp
// per-(j, bucket) device time of tuning runs
struct TuneProbe {
    double ms[HUGE_KMAX + 1][HUGE_TUNE_BUCKETS] = {};
    double other_ms[HUGE_KMAX + 1] = {};  // prepare, partition and scan launches, per j
    int64_t items[HUGE_KMAX + 1][HUGE_TUNE_BUCKETS] = {};
};
struct ExecStats {
    uint64_t launches = 0;
    uint64_t steals = 0;
    uint64_t peak_frontier_bytes = 0;
};
struct EmitSink {
    int32_t *dev_out = nullptr;  // rows go to this device table (ranks, no callback) instead of host_buf
    int64_t dev_cap = 0;         // its capacity in rows
    int32_t *host_buf = nullptr;
    int64_t buf_rows = 0;
    huge_emit_fn cb = nullptr;
    void *user = nullptr;
    bool stopped = false;
    uint64_t delivered = 0;
};
uint64_t workspace_bytes(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o);
// the level engine's rows per scheduling segment of every level w = 2..k-1 (rows[w])
void segment_rows(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, int64_t *rows);
// the plan as one execution sees it (slice options applied); HUGE_EINVAL on bad options
DevPlan exec_plan(const huge_plan *p, const huge_exec_opts &o);
bool root_sliced(const DevPlan &P);       // level_counts[0] is the number of roots in the slices
bool gathers_level2(const DevPlan &P);
// level_counts[0] of a root slice whose only filter is a rank stride (false: needs k_root_count)
bool strided_root_count(const DevPlan &P, int64_t n, uint64_t *count);    // level 2 is the gathered entries of a strided root slice
int64_t gathered_rows_bound(const huge_graph *g, const DevPlan &P);
int64_t gathered_roots(const huge_graph *g, const DevPlan &P);
int64_t strided_l2_rows(const huge_graph *g, const DevPlan &P);  // rows of a strided edge slice
// returns true when the run stopped at o.work_limit; host_stage: a host block of
// kHostStageBytes for the scheduler's read-backs (NULL: pinned memory is allocated)
bool run_levels(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, huge_result *out, EmitSink *emit,
                TuneProbe *probe = nullptr, unsigned char *host_stage = nullptr);
// counting through replays of a recorded round (HUGE_ENGINE_GRAPH)
void run_graph(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, huge_result *out);
void autotune(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
              huge_tune_table *out);
// batch.cpp
void run_batch_levels(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                      huge_result *outs);
void run_persistent(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                    huge_result *outs);
uint64_t persist_workspace_bytes(const huge_plan *const *plans, int np, const huge_exec_opts &o);
// motif.cpp: every connected k-vertex pattern, non-induced and induced counts; returns the pattern count
int motif_count(const huge_graph *g, int k, const huge_exec_opts &o, huge_motif *out);
// bushy_plan.cpp: Algorithm 1 over connected edge sets (p.bushy); machines = the k of k |E_G|
void plan_bushy(const huge_graph_info &gi, huge_plan &p, double machines);
// the same tables for a given tree: splits[2i], splits[2i+1] = the parts of join i
void plan_bushy_tree(const huge_graph_info &gi, huge_plan &p, const uint32_t *splits, int nsplits, double machines);
// bushy.cpp: run a bushy plan (level engine for chains from a SCAN, join.hip for the rest)
void run_bushy(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, huge_result *out,
               int64_t *node_rows, int max_nodes);
// noalloc.hip: huge_count on the level engine inside the file-scope device array
uint64_t noalloc_scratch_bytes();
void run_count_noalloc(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, huge_result *out,
                       bool *limited);
// mbatch.cpp: the batch in batched rounds (HUGE_ENGINE_GRAPH)
void run_mgraph(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                huge_result *outs);
uint64_t mgraph_workspace_bytes(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o);

// ---------------------------------------------------------------------------
// kernel launchers (extend.hip)
// ---------------------------------------------------------------------------
struct SegBufs {
    int64_t *off;       // [cap+1] exclusive scan of bounds, then total
    uint64_t *pinfo;    // [cap] probe begin (low 56 bits) | probe position << 56
    uint64_t *hpre;     // [cap] prefix hash (last level only)
    int32_t *bound;     // [cap]
    int64_t cap;
    // probe-length bucket partition (tuned runs): the prepare pass writes the
    // *_in arrays, the partition moves them into bucket order above, and
    // rid[r] is the input row of segment row r
    int32_t *bound_in;
    uint64_t *pinfo_in, *hpre_in;
    int32_t *rid;
    int32_t *bcnt;      // [HUGE_TUNE_BUCKETS * blocks]
    int64_t *bscan;     // [HUGE_TUNE_BUCKETS * blocks + 1]
};

struct Ctrl {                      // device-resident counters
    unsigned long long qcount[HUGE_KMAX + 1];   // rows in the queue of level i
    unsigned long long level[HUGE_KMAX];        // level_counts
    unsigned long long acc[4];                  // count, hash_sum, hash_xor, overflow flag
    unsigned long long segbytes[HUGE_KMAX];     // algorithmic bytes of the current segment, per width
    long long scratch[8];
};

constexpr size_t kHostStageBytes = sizeof(Ctrl) + 64;  // the level engine's host read-back block

void launch_prepare(int width, bool last, const GraphDev &g, const DevPlan &P, const int32_t *rows, int64_t row0,
                    int64_t nrows, const SegBufs &s, Ctrl *ctrl, hipStream_t st);
void launch_scan_bounds(const SegBufs &s, int64_t nrows, int64_t *tmp, hipStream_t st);
void launch_extend(int width, int mode, int strategy, const GraphDev &g, const DevPlan &P, const int32_t *rows,
                   int64_t row0, const SegBufs &s, int64_t nrows, int64_t w0, int64_t w1, int32_t *out_rows,
                   Ctrl *ctrl, const int32_t *inv_rank, hipStream_t st, bool partitioned);
void launch_bucket_partition(const SegBufs &s, int64_t nrows, bool last, int64_t *scan_tmp, Ctrl *ctrl,
                             hipStream_t st);
// ctrl->scratch[c] = first work item of bucket c, scratch[HUGE_TUNE_BUCKETS] = total
void launch_bucket_bounds(const SegBufs &s, int64_t nrows, Ctrl *ctrl, hipStream_t st);
void launch_edge_sink(const GraphDev &g, const DevPlan &P, int64_t e0, int64_t e1, int mode, int32_t *out,
                      const int32_t *inv_rank, Ctrl *ctrl, hipStream_t st);
void launch_root_count(const GraphDev &g, const DevPlan &P, Ctrl *ctrl, hipStream_t st);
// Level 2 of a strided slice of the first matched vertex (ranks s, s + S, ...):
// the edge-array entries of those roots, in order, into idx (at most cap
// entries; the count lands in off[roots]).  deg int32[roots], off int64[roots + 1].
void launch_gather_level2(const GraphDev &g, const DevPlan &P, int64_t roots, int32_t *deg, int64_t *off,
                          int64_t *idx, int64_t cap, int64_t *scan_tmp, hipStream_t st);
int64_t scan_tmp_elems(int64_t n);

// ---------------------------------------------------------------------------
// device-driven rounds (graph engine): Algorithm 5's scheduler runs on the
// device, one action per round, so that a round of fixed launches can be
// recorded once in a hipGraph and replayed until the query is done
// ---------------------------------------------------------------------------
struct GLevel {
    int64_t nrows;      // rows in this level's input (queue rows; level 2: the edge array)
    int64_t next;       // first row not yet taken into a segment
    int64_t seg_row0, seg_n;        // current segment's rows
    int64_t seg_total, seg_done;    // its work items, and those already extended
};
enum { GACT_NONE = 0, GACT_PREPARE = 1, GACT_EMIT = 2, GACT_SINK = 3 };
struct GState {
    GLevel lv[HUGE_KMAX + 1];
    int64_t n_prep[HUGE_KMAX + 1];  // this round: rows to prepare at level W (0: none)
    int64_t n_part[HUGE_KMAX + 1];  // this round: per-block bucket counts of level W's partition
    int64_t bw[HUGE_KMAX + 1][HUGE_TUNE_BUCKETS + 1];  // level W's segment: first work item per bucket, total
    unsigned long long tile_next[HUGE_KMAX + 1][HUGE_TUNE_BUCKETS + 1];  // this round: next tile to claim,
                                                                        // per level and bucket (+1; 0: unpartitioned)
    int64_t ext_w0[HUGE_KMAX + 1];  // this round: work items [w0, w1) to extend at level W
    int64_t ext_w1[HUGE_KMAX + 1];
    int64_t work[HUGE_KMAX];        // work items per level (huge_result.level_work)
    int64_t cur_bytes, peak_bytes;  // frontier bytes held in queues
    int64_t rounds;                 // rounds that took an action
    int32_t W;                      // level the scheduler is on
    int32_t inner;                  // 1: inside level W's run (its input was checked on entry)
    int32_t last_kind, last_W;      // the previous round's action
    int32_t done, error;
};
struct GConst {                      // fixed for a query (kernel argument)
    int32_t k, lastW;
    int64_t seg_cap[HUGE_KMAX + 1];
    int64_t q_cap[HUGE_KMAX + 1];
    const int64_t *off[HUGE_KMAX + 1];  // each level's scanned bounds (off[seg_n] = segment total)
};
void launch_round_sched(GState *s, const GConst &c, Ctrl *ctrl, hipStream_t st);
void launch_round_prepare(int width, bool last, const GraphDev &g, const DevPlan &P, const int32_t *rows,
                          const SegBufs &s, Ctrl *ctrl, GState *gs, int64_t seg_cap, hipStream_t st);
void launch_round_scan(int width, const SegBufs &s, GState *gs, int64_t seg_cap, int64_t *tmp, hipStream_t st);
// tuned dispatch: the probe-length partition of the prepared segment (reads
// the *_in arrays, like launch_bucket_partition) and its bucket bounds
// (after the scan), into gs->bw[width]
void launch_round_partition(int width, bool last, const SegBufs &s, GState *gs, int64_t seg_cap, int64_t *tmp,
                            hipStream_t st);
void launch_round_bucket_bounds(int width, const SegBufs &s, GState *gs, hipStream_t st);
// extend this round's work items of level `width` with `strategy`; bucket >= 0
// restricts them to that probe-length bucket of a partitioned segment
void launch_round_extend(int width, int mode, int strategy, const GraphDev &g, const DevPlan &P, const int32_t *rows,
                         const SegBufs &s, int32_t *out_rows, Ctrl *ctrl, const int32_t *inv_rank, GState *gs,
                         int bucket, hipStream_t st);

// ---------------------------------------------------------------------------
// batched rounds (huge_count_batch on the graph engine): every query of a
// batch keeps its own Algorithm 5 state, queues and segment buffers; one round
// advances each query by one action (round_sched_step, one thread per query)
// and then runs ONE prepare launch, one batched scan and one extend launch per
// (level, last-level-or-not) for all queries together, each workgroup claiming
// tiles of whichever query comes next.  Recorded once in a hipGraph, replayed.
// ---------------------------------------------------------------------------
constexpr int kMaxBatch = 256;                 // queries in one batched round
constexpr int kMLaunches = 2 * (HUGE_KMAX - 1);  // extend launch id (W - 2) * 2 + (W is the last level)
struct MPat {                      // one query of the batch (fixed for the call)
    GConst gc;                     // its scheduler constants (off[W] = sb[W].off)
    DevPlan P;
    GraphDev g;                    // with the batch's level-2 rows
    Ctrl *ctrl;
    GState *gs;
    int32_t *q[HUGE_KMAX + 1];     // queues of levels 3..k-1
    SegBufs sb[HUGE_KMAX + 1];     // segment buffers of levels 2..k-1
    int64_t *scan_part;            // tile sums of its segment scan (<= 4096 tiles)
    const int32_t *inv_rank;
    int32_t search[HUGE_KMAX + 1]; // 1: level W runs binary-search tiles (kTile items), 0: lane merges
};
struct MRound {                    // written by the round's scheduler launch
    int64_t prep_pre[kMaxBatch + 1];            // prepare workgroups: exclusive prefix over queries
    int64_t scan_pre[kMaxBatch + 1];            // scan tiles
    int64_t ext_pre[kMLaunches][kMaxBatch + 1]; // extend tiles of each launch
    unsigned long long claim[kMLaunches];       // next tile of each extend launch
    int32_t prep_W[kMaxBatch];                  // level each query prepares (0: none)
    int32_t active;                             // queries not done
    int32_t error;                              // a query's scheduler found no action
};
struct MConst {                    // kernel argument of the scheduler
    int32_t np;
    uint32_t lids;                   // the extend launches the batch uses
    int32_t tile_items[kMLaunches];  // work items per lane-merge tile of each extend launch's kernel
};
void launch_mround_sched(MPat *mp, MRound *mr, const MConst &mc, hipStream_t st);
void launch_mround_prepare(const MPat *mp, const MRound *mr, int np, hipStream_t st);
void launch_mround_scan(const MPat *mp, MRound *mr, int np, int64_t max_tiles, hipStream_t st);
// extend launch `lid` (level W = lid / 2 + 2, last level when lid is odd) with
// `strategy` (a lane-merge strategy) for the queries whose level W merges, and,
// with `search`, binary-search tiles for those whose level W searches
// (MPat::search); mround_tile_items gives the work items per lane-merge tile
int mround_tile_items(int lid, int strategy);
void launch_mround_extend(int lid, int count_mode, int strategy, bool search, const MPat *mp, MRound *mr, int np,
                          hipStream_t st);

// extend modes
enum { MODE_EMIT = 0, MODE_COUNT = 1, MODE_OUTPUT = 2, MODE_COUNT_NOHASH = 3 };
// intersection strategies (huge_exec_opts.strategy, HUGE_STRAT_*)
enum {
    STRAT_BSEARCH = HUGE_STRAT_BSEARCH,
    STRAT_WAVE_STAGED = HUGE_STRAT_WAVE_STAGED,
    STRAT_LANE_MERGE = HUGE_STRAT_LANE_MERGE,
    STRAT_MERGE_SHORT = HUGE_STRAT_MERGE_SHORT,
    STRAT_MERGE_LONG = HUGE_STRAT_MERGE_LONG,
    STRAT_BLOCK_MERGE = HUGE_STRAT_BLOCK_MERGE,
    STRAT_BLOCK_MERGE_LONG = HUGE_STRAT_BLOCK_MERGE_LONG,
    STRAT_COUNT = HUGE_STRAT_COUNT
};


}  // namespace huge
