// A batch of queries in batched rounds (huge_count_batch, HUGE_ENGINE_GRAPH).
//
// Section 4.2 batches the input of an operator so that all workers share it;
// Section 5.3 lets idle workers take over the work of busy ones.  On one GPU
// the batch is the set of queries itself: each query runs Algorithm 5 (its own
// device state, queues and segment buffers, an equal share of the frontier
// budget), and every round advances all of them by one action in a fixed
// sequence of launches whose workgroups claim tiles across the queries.  The
// round is recorded once in a hipGraph and replayed until every query is done;
// the host only reads one "queries still active" word per few replays.
//
// Queries of two vertices are a single edge-array pass each and run on the
// level engine first.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <list>
#include <mutex>
#include <vector>

#include "internal.h"
#include "prims.h"

namespace huge {

namespace {

constexpr int kRounds = 4;                  // rounds recorded in the graph
constexpr int kBatchReplays = 8;            // most graph launches between reads of the active count
constexpr int64_t kMaxRounds = 1ll << 26;
constexpr int64_t kDefaultSegRows = 1 << 20;
constexpr int64_t kMinQueueRows = 1 << 12;
constexpr int64_t kScanPartElems = 4096 + 8;  // tile sums of a segment of up to 4096 tiles

inline uint64_t align_up(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct PatLayout {
    int64_t seg_cap[HUGE_KMAX + 1] = {};
    int64_t q_cap[HUGE_KMAX + 1] = {};
    bool gathered = false;  // level 2 is the gathered strided slice
    uint64_t bytes = 0;
};

struct BatchLayout {
    std::vector<int> idx;        // batch positions of the queries with 3 or more vertices
    std::vector<DevPlan> P;
    std::vector<PatLayout> pl;
    int64_t l2_roots = 0, l2_rows = 0, scan_tmp = 0;
    uint64_t total = 0;
};

// Rows per segment of a query's level W: the caller's, the learned model's, or
// kDefaultSegRows.  A tune table's segment rows are left to the level engine:
// they are measured there, while a batched round pays its fixed launches once
// per segment, so smaller segments only add rounds.
int64_t seg_rows_for(const huge_plan *p, int W, const huge_exec_opts &o, int64_t out_queue_rows) {
    if (o.chunk_rows > 0) return o.chunk_rows;
    const int64_t m = model_segment_rows(p, W, out_queue_rows);
    if (m > 0) return m;
    return kDefaultSegRows;
}

BatchLayout make_batch_layout(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o) {
    BatchLayout B;
    for (int i = 0; i < np; ++i)
        if (plans[i]->k >= 3) B.idx.push_back(i);
    const int nb = (int)B.idx.size();
    if (nb == 0) return B;
    uint64_t cap = o.frontier_cap_bytes;
    if (cap == UINT64_MAX) {
        size_t fr = 0, tot = 0;
        HUGE_HIP(hipMemGetInfo(&fr, &tot));
        cap = (uint64_t)(fr * 0.5);
    }
    const uint64_t share = cap / (uint64_t)nb;
    uint64_t t = 0;
    for (int b = 0; b < nb; ++b) {
        const huge_plan *p = plans[B.idx[b]];
        const DevPlan P = exec_plan(p, o);
        B.P.push_back(P);
        PatLayout L;
        const int k = p->k, nq = std::max(0, k - 3);
        L.gathered = gathers_level2(P);
        if (L.gathered) {
            B.l2_roots = gathered_roots(g, P);
            B.l2_rows = gathered_rows_bound(g, P);
        }
        for (int w = 3; w <= k - 1; ++w)
            L.q_cap[w] = std::max<int64_t>(kMinQueueRows, (int64_t)((nq ? share / nq : 0) / (4ull * w)));
        const int64_t l2 = L.gathered ? gathered_rows_bound(g, P) : P.edge_slice == 2 ? strided_l2_rows(g, P)
                                                                                      : g->dev.nnz;
        L.seg_cap[2] = std::min<int64_t>(std::min(seg_rows_for(p, 2, o, L.q_cap[3]), scan_devn_max()),
                                         std::max<int64_t>(1, l2));
        for (int w = 3; w <= k - 1; ++w)
            L.seg_cap[w] = std::min<int64_t>(std::min(seg_rows_for(p, w, o, L.q_cap[w + 1]), scan_devn_max()),
                                             L.q_cap[w]);
        uint64_t b2 = 0;
        for (int w = 2; w <= k - 1; ++w) {
            const int64_t c = L.seg_cap[w];
            b2 += align_up(8ull * (c + 1)) + align_up(8ull * c) * 2 + align_up(4ull * c);
        }
        for (int w = 3; w <= k - 1; ++w) b2 += align_up(4ull * w * L.q_cap[w]);
        b2 += align_up(8ull * kScanPartElems);
        L.bytes = b2;
        t += b2;
        B.pl.push_back(L);
    }
    t += align_up(sizeof(Ctrl) * nb) + align_up(sizeof(GState) * nb) + align_up(sizeof(MPat) * nb) +
         align_up(sizeof(MRound));
    if (B.l2_rows) {
        B.scan_tmp = scan_tmp_elems(B.l2_roots + 1);
        t += align_up(8ull * B.l2_rows) + align_up(4ull * B.l2_roots) + align_up(8ull * (B.l2_roots + 1)) +
             align_up(8ull * B.scan_tmp);
    }
    B.total = t;
    return B;
}

struct Carver {
    char *base;
    uint64_t off = 0;
    template <typename T>
    T *take(uint64_t count) {
        T *p = (T *)(base + off);
        off += align_up(sizeof(T) * count);
        return p;
    }
};

// A recorded round reads everything that changes between calls (query
// plans, slices, scheduler states, counters) from device memory that each call
// rewrites before the replays; its launches capture only the addresses of
// that memory, the batch size, the scan grid, the per-launch strategies and
// tile sizes, the count mode and the device.  Calls that agree on all of these
// replay the same instantiated graph, so a call records and instantiates only
// when its key is new.  The cache keeps the 16 most recent graphs.
struct GraphKey {
    int device;
    const void *mp, *mr;
    int nb, count_mode;
    int64_t max_scan_tiles;
    int strat[kMLaunches];
    int64_t tile_items[kMLaunches];
    uint32_t lids, search_lids;
    bool operator==(const GraphKey &o) const { return memcmp(this, &o, sizeof(*this)) == 0; }
};

struct GraphCache {
    std::mutex mu;
    std::list<std::pair<GraphKey, hipGraphExec_t>> lru;  // most recent first
    static constexpr size_t kCap = 16;
    hipGraphExec_t find(const GraphKey &k) {
        for (auto it = lru.begin(); it != lru.end(); ++it)
            if (it->first == k) {
                lru.splice(lru.begin(), lru, it);
                return lru.front().second;
            }
        return nullptr;
    }
    void put(const GraphKey &k, hipGraphExec_t e) {
        lru.emplace_front(k, e);
        while (lru.size() > kCap) {
            (void)hipGraphExecDestroy(lru.back().second);
            lru.pop_back();
        }
    }
};

GraphCache &graph_cache() {
    static GraphCache *c = new GraphCache();  // lives until the process ends
    return *c;
}

struct Res {
    void *mem = nullptr;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;  // owned by the cache once stored there
    bool cached = false;
    ~Res() {
        if (exec && !cached) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) {
            hipStreamCaptureStatus status = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(cs, &status) == hipSuccess && status != hipStreamCaptureStatusNone) {
                hipGraph_t partial = nullptr;
                (void)hipStreamEndCapture(cs, &partial);
                if (partial) (void)hipGraphDestroy(partial);
            }
            (void)hipStreamDestroy(cs);
        }
        if (mem) (void)hipFree(mem);
    }
};

// Whether a query's level W runs binary-search tiles rather than lane merges:
// a forced strategy decides for every query (0 and 1 search); a tune table by
// the work items its buckets at the level's Ext count give to each kind;
// without either, lane merges.
bool level_searches(const huge_plan *p, int W, const huge_exec_opts &o) {
    if (o.strategy >= 0 && o.strategy < STRAT_COUNT) return o.strategy < STRAT_LANE_MERGE;
    if (!o.tune) return false;
    const int j = __builtin_popcount(p->dev.st[W].ext);
    int64_t search = 0, merge = 0;
    for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) {
        const int s = o.tune->strategy[j][c];
        if (s < 0 || s >= STRAT_COUNT) continue;
        (s < STRAT_LANE_MERGE ? search : merge) += std::max<int64_t>(1, o.tune->items[j][c]);
    }
    return search > merge;
}

// The lane merge of each extend launch, for the queries whose level merges: a
// forced lane-merge strategy, or the one the tune table gives most work to at
// the Ext sizes of those queries (searches count as the short lane merge, the
// nearest of its kernels), or without a table the block-cached merges.
int launch_strategy(int lid, const huge_exec_opts &o, const std::vector<const huge_plan *> &ps,
                    const std::vector<MPat> &hm) {
    const bool last = (lid & 1) != 0;
    const int dflt = last ? STRAT_BLOCK_MERGE_LONG : STRAT_BLOCK_MERGE;
    if (o.strategy >= STRAT_LANE_MERGE && o.strategy < STRAT_COUNT) return o.strategy;
    if (!o.tune) return dflt;
    const int W = lid / 2 + 2;
    int64_t items[STRAT_COUNT] = {};
    for (size_t b = 0; b < ps.size(); ++b) {
        const huge_plan *p = ps[b];
        if (W > p->k - 1 || (W == p->k - 1) != last || hm[b].search[W]) continue;
        const int j = __builtin_popcount(p->dev.st[W].ext);
        for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) {
            int s = o.tune->strategy[j][c];
            if (s < 0 || s >= STRAT_COUNT) continue;
            if (s < STRAT_LANE_MERGE) s = STRAT_MERGE_SHORT;
            items[s] += std::max<int64_t>(1, o.tune->items[j][c]);
        }
    }
    int best = dflt;
    for (int s = STRAT_LANE_MERGE; s < STRAT_COUNT; ++s)
        if (items[s] > items[best]) best = s;
    return best;
}

}  // namespace

uint64_t mgraph_workspace_bytes(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o) {
    if (np > kMaxBatch) HUGE_FAIL(HUGE_EINVAL, "batched rounds take at most %d queries per call", kMaxBatch);
    return make_batch_layout(g, plans, np, o).total;
}

void run_mgraph(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                huge_result *outs) {
    auto t0 = std::chrono::steady_clock::now();
    if (np > kMaxBatch) HUGE_FAIL(HUGE_EINVAL, "batched rounds take at most %d queries per call", kMaxBatch);
    if (o.work_limit > 0) HUGE_FAIL(HUGE_EINVAL, "batched rounds have no work limit");
    hipStream_t st = (hipStream_t)o.stream;
    // two-vertex queries: one edge-array pass each
    for (int i = 0; i < np; ++i)
        if (plans[i]->k < 3) {
            huge_exec_opts lo = o;
            lo.engine = HUGE_ENGINE_LEVELS;
            lo.tune = nullptr;
            lo.workspace = nullptr;
            lo.workspace_bytes = 0;
            run_levels(g, plans[i], lo, &outs[i], nullptr);
        }
    BatchLayout B = make_batch_layout(g, plans, np, o);
    const int nb = (int)B.idx.size();
    if (nb == 0) return;
    Res res;
    char *ws = (char *)o.workspace;
    if (ws) {
        if (o.workspace_bytes < B.total)
            HUGE_FAIL(HUGE_ENOMEM, "workspace too small: %llu bytes given, %llu needed",
                      (unsigned long long)o.workspace_bytes, (unsigned long long)B.total);
    } else {
        HUGE_HIP(hipMalloc(&res.mem, B.total));
        ws = (char *)res.mem;
    }
    Carver cv{ws};
    Ctrl *ctrl = cv.take<Ctrl>(nb);
    GState *gs = cv.take<GState>(nb);
    MPat *mp = cv.take<MPat>(nb);
    MRound *mr = cv.take<MRound>(1);
    GraphDev G = g->dev;
    GraphDev Gg = g->dev;  // with the gathered level 2
    int64_t l2_gathered = 0;
    if (B.l2_rows) {
        int64_t *idx = cv.take<int64_t>(B.l2_rows);
        int32_t *deg = cv.take<int32_t>(B.l2_roots);
        int64_t *off = cv.take<int64_t>(B.l2_roots + 1);
        int64_t *tmp = cv.take<int64_t>(B.scan_tmp);
        const int first = [&] {
            for (int b = 0; b < nb; ++b)
                if (B.pl[b].gathered) return b;
            return 0;
        }();
        launch_gather_level2(G, B.P[first], B.l2_roots, deg, off, idx, B.l2_rows, tmp, st);
        HUGE_HIP(hipMemcpyAsync(&l2_gathered, off + B.l2_roots, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        if (l2_gathered > B.l2_rows) HUGE_FAIL(HUGE_EDEVICE, "gathered level 2 exceeds its bound");
        Gg.l2_idx = idx;
    }
    std::vector<MPat> hm(nb);
    std::vector<GState> hs(nb);
    std::vector<const huge_plan *> ps;
    int64_t max_scan_tiles = 0;
    bool use_lid[kMLaunches] = {}, search_lid[kMLaunches] = {};
    for (int b = 0; b < nb; ++b) {
        const huge_plan *p = plans[B.idx[b]];
        ps.push_back(p);
        const PatLayout &L = B.pl[b];
        const int k = p->k;
        MPat &m = hm[b];
        memset((void *)&m, 0, sizeof(m));
        m.gc.k = k;
        m.gc.lastW = k - 1;
        m.P = B.P[b];
        m.g = L.gathered ? Gg : G;
        if (m.P.edge_slice == 2) {
            m.g.l2_first = m.P.slice_id;
            m.g.l2_stride = m.P.slice_count;
        }
        m.ctrl = ctrl + b;
        m.gs = gs + b;
        m.inv_rank = g->inv_rank;
        for (int w = 2; w <= k - 1; ++w) {
            const int64_t c = L.seg_cap[w];
            m.sb[w].off = cv.take<int64_t>(c + 1);
            m.sb[w].pinfo = cv.take<uint64_t>(c);
            m.sb[w].hpre = cv.take<uint64_t>(c);
            m.sb[w].bound = cv.take<int32_t>(c);
            m.sb[w].cap = c;
            m.gc.seg_cap[w] = c;
            m.gc.off[w] = m.sb[w].off;
            max_scan_tiles += (c + 4095) / 4096;
            const int lid = (w - 2) * 2 + (w == k - 1 ? 1 : 0);
            m.search[w] = level_searches(p, w, o) ? 1 : 0;
            use_lid[lid] = true;
            search_lid[lid] |= m.search[w] != 0;
        }
        for (int w = 3; w <= k - 1; ++w) {
            m.q[w] = cv.take<int32_t>((uint64_t)w * L.q_cap[w]);
            m.gc.q_cap[w] = L.q_cap[w];
        }
        m.scan_part = cv.take<int64_t>(kScanPartElems);
        GState &s = hs[b];
        memset((void *)&s, 0, sizeof(s));
        s.W = 2;
        s.lv[2].nrows = L.gathered ? l2_gathered : m.P.edge_slice == 2 ? strided_l2_rows(g, m.P) : g->dev.nnz;
    }
    if (cv.off > B.total) HUGE_FAIL(HUGE_EDEVICE, "batched round layout overflow");
    HUGE_HIP(hipMemsetAsync(ctrl, 0, sizeof(Ctrl) * nb, st));
    HUGE_HIP(hipMemsetAsync(mr, 0, sizeof(MRound), st));
    HUGE_HIP(hipMemcpyAsync(gs, hs.data(), sizeof(GState) * nb, hipMemcpyHostToDevice, st));
    HUGE_HIP(hipMemcpyAsync(mp, hm.data(), sizeof(MPat) * nb, hipMemcpyHostToDevice, st));
    std::vector<uint64_t> roots_known(nb, UINT64_MAX);
    for (int b = 0; b < nb; ++b)
        if (root_sliced(hm[b].P) && !strided_root_count(hm[b].P, g->dev.n, &roots_known[b]))
            launch_root_count(hm[b].g, hm[b].P, hm[b].ctrl, st);
    const int count_mode = (o.exec_flags & HUGE_EXEC_NO_HASH) ? MODE_COUNT_NOHASH : MODE_COUNT;
    MConst mc{};
    mc.np = nb;
    int strat[kMLaunches];
    for (int l = 0; l < kMLaunches; ++l) {
        strat[l] = use_lid[l] ? launch_strategy(l, o, ps, hm) : STRAT_BLOCK_MERGE;
        mc.tile_items[l] = mround_tile_items(l, strat[l]);
        if (use_lid[l]) mc.lids |= 1u << l;
    }
    // the host copies above come from pageable memory: finish them before recording
    HUGE_HIP(hipStreamSynchronize(st));

    GraphKey key;
    memset(&key, 0, sizeof(key));
    HUGE_HIP(hipGetDevice(&key.device));
    key.mp = mp;
    key.mr = mr;
    key.nb = nb;
    key.count_mode = count_mode;
    key.max_scan_tiles = max_scan_tiles;
    for (int l = 0; l < kMLaunches; ++l) {
        key.strat[l] = strat[l];
        key.tile_items[l] = mc.tile_items[l];
        if (use_lid[l]) key.lids |= 1u << l;
        if (search_lid[l]) key.search_lids |= 1u << l;
    }
    // the cache lock is held from lookup to the last replay: two calls with one
    // key would share one workspace anyway, and a graph is not replayed while
    // another call could evict and destroy it
    std::lock_guard<std::mutex> lock(graph_cache().mu);
    res.exec = graph_cache().find(key);
    res.cached = res.exec != nullptr;
    if (!res.exec) {
        HUGE_HIP(hipStreamCreateWithFlags(&res.cs, hipStreamNonBlocking));
        HUGE_HIP(hipStreamBeginCapture(res.cs, hipStreamCaptureModeRelaxed));  // occupancy queries run while recording
        for (int r = 0; r < kRounds; ++r) {
            launch_mround_sched(mp, mr, mc, res.cs);
            launch_mround_prepare(mp, mr, nb, res.cs);
            launch_mround_scan(mp, mr, nb, max_scan_tiles, res.cs);
            for (int l = 0; l < kMLaunches; ++l)
                if (use_lid[l]) launch_mround_extend(l, count_mode, strat[l], search_lid[l], mp, mr, nb, res.cs);
        }
        HUGE_HIP(hipStreamEndCapture(res.cs, &res.graph));
        HUGE_HIP(hipGraphInstantiate(&res.exec, res.graph, nullptr, nullptr, 0));
        graph_cache().put(key, res.exec);
        res.cached = true;
    }

    int32_t hdr[2] = {1, 0};  // active, error
    int64_t replays = 0;
    // replays between reads of the active count: 1, 2, 4, ... up to kBatchReplays,
    // so that a batch of light queries does not run rounds after it is done
    int burst = 1;
    while (hdr[0] > 0) {
        for (int i = 0; i < burst; ++i) HUGE_HIP(hipGraphLaunch(res.exec, st));
        replays += burst;
        burst = std::min(2 * burst, kBatchReplays);
        HUGE_HIP(hipMemcpyAsync(hdr, &mr->active, sizeof(hdr), hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        if (hdr[1]) HUGE_FAIL(HUGE_EINVAL, "batched rounds: a query's scheduler found no action");
        if (hdr[0] > 0 && replays * kRounds > kMaxRounds)
            HUGE_FAIL(HUGE_EINVAL, "batched rounds: no end after %lld rounds", (long long)(replays * kRounds));
    }
    std::vector<Ctrl> hc(nb);
    HUGE_HIP(hipMemcpyAsync(hc.data(), ctrl, sizeof(Ctrl) * nb, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(hs.data(), gs, sizeof(GState) * nb, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    auto t1 = std::chrono::steady_clock::now();
    const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    for (int b = 0; b < nb; ++b) {
        huge_result &out = outs[B.idx[b]];
        memset(&out, 0, sizeof(out));
        if (hs[b].error) HUGE_FAIL(HUGE_EINVAL, "batched rounds: the device scheduler found no action");
        out.count = hc[b].acc[0];
        out.hash_sum = hc[b].acc[1];
        out.hash_xor = hc[b].acc[2];
        for (int i = 0; i < HUGE_KMAX; ++i) out.level_counts[i] = hc[b].level[i];
        if (!root_sliced(hm[b].P)) out.level_counts[0] = (uint64_t)g->dev.n;
        if (roots_known[b] != UINT64_MAX) out.level_counts[0] = roots_known[b];
        out.peak_frontier_bytes = (uint64_t)hs[b].peak_bytes;
        for (int i = 0; i < HUGE_KMAX; ++i) out.level_work[i] = (uint64_t)hs[b].work[i];
        out.launches = (uint64_t)replays;
        out.query_ms = ms;
    }
}

}  // namespace huge
