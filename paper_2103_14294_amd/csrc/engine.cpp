// The level engine: Algorithm 5 (DFS/BFS-adaptive scheduling, Section 5.2)
// driven from the host, one grid-wide launch per chunk.
//
// Operators form a line: SCAN (level-2 rows, read straight from the CSR edge
// array, never materialised) -> EXTEND at widths 2..k-2 -> EXTEND+SINK at
// width k-1 (counting fused in, never materialised).  Every materialised
// level W (3..k-1) owns a fixed-capacity queue.  The scheduler keeps running
// the current operator until its output queue is full or its input is empty,
// then moves to the successor; an operator with no input hands control back
// to its precursor, and the fused SINK always does.
//
// Bounded memory, stricter than Lemma 5.1: a chunk never produces more rows
// than the free space of the output queue, because each launch covers at
// most `free` work items and a work item (one probe element) emits at most
// one row.  A single hub row larger than the queue is simply split across
// launches.  So the frontier never exceeds the configured capacity.
//
// Two drivers of the same scheduler live here: run_levels takes every
// decision on the host (one read-back per segment and per emitting chunk);
// run_graph (the graph engine, at the end of this file) takes them in a
// one-thread device kernel and replays a recorded round of launches.
#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "prims.h"

namespace huge {

namespace {

constexpr int64_t kDefaultSeg = 1 << 22;
constexpr int64_t kMinQueueRows = 1 << 12;
constexpr int64_t kMaxItems = 1ll << 30;
constexpr int kSegTotalSlot = 7;  // Ctrl::scratch slot for the segment total (0..5: bucket bounds)
static_assert(kSegTotalSlot > HUGE_TUNE_BUCKETS, "segment total must not overlap the bucket bounds");
constexpr uint64_t kDefaultCap = 4ull << 30;

inline int ext_count(const huge_plan *p, int W) { return __builtin_popcount(p->dev.st[W].ext); }

// per-bucket dispatch: a tune table and no fixed strategy
inline bool partitioned(const huge_exec_opts &o) { return o.tune && (o.strategy < 0 || o.strategy >= STRAT_COUNT); }

struct Layout {
    int64_t l2_rows = 0, l2_roots = 0;  // gathered level 2 (strided slice of the first vertex): bound, roots
    int64_t seg_cap[HUGE_KMAX] = {};
    int64_t q_cap[HUGE_KMAX + 1] = {};
    int64_t stage_rows = 0;
    int64_t scan_tmp = 0;
    uint64_t total = 0;
};

inline uint64_t align_up(uint64_t x) { return (x + 255) & ~uint64_t(255); }

Layout make_layout(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, int64_t stage_rows,
                   int64_t seg_limit = INT64_MAX) {
    Layout L;
    const int k = p->k;
    const DevPlan P = exec_plan(p, o);
    if (gathers_level2(P)) {
        L.l2_roots = gathered_roots(g, P);
        L.l2_rows = gathered_rows_bound(g, P);
    }
    const int64_t l2_all = L.l2_rows ? L.l2_rows : P.edge_slice == 2 ? strided_l2_rows(g, P) : g->dev.nnz;
    int64_t seg = o.chunk_rows > 0 ? o.chunk_rows : kDefaultSeg;
    const int nq = std::max(0, k - 3);
    uint64_t cap = o.frontier_cap_bytes;
    if (cap == UINT64_MAX) {
        size_t fr = 0, tot = 0;
        HUGE_HIP(hipMemGetInfo(&fr, &tot));
        cap = (uint64_t)(fr * 0.6);
    }
    for (int w = 3; w <= k - 1; ++w) {
        uint64_t share = nq ? cap / nq : 0;
        L.q_cap[w] = std::max<int64_t>(kMinQueueRows, (int64_t)(share / (4ull * w)));
    }
    auto seg_for = [&](int w) {
        if (o.chunk_rows <= 0 && w + 1 <= k - 1) {
            const int64_t m = model_segment_rows(p, w, L.q_cap[w + 1]);
            if (m > 0) return std::min(m, seg_limit);
        }
        if (o.chunk_rows <= 0 && o.tune) {
            const int64_t c = o.tune->chunk_rows[ext_count(p, w)];
            if (c > 0) return std::min(c, seg_limit);
        }
        return std::min(seg, seg_limit);
    };
    L.seg_cap[2] = std::min<int64_t>(seg_for(2), std::max<int64_t>(1, l2_all));
    for (int w = 3; w <= k - 1; ++w) L.seg_cap[w] = std::min<int64_t>(seg_for(w), L.q_cap[w]);
    L.stage_rows = stage_rows;
    int64_t maxseg = 1;
    for (int w = 2; w <= k - 1; ++w) maxseg = std::max(maxseg, L.seg_cap[w]);
    const bool part = partitioned(o);
    const int64_t maxblk = (maxseg + 255) / 256;
    L.scan_tmp = scan_tmp_elems(std::max(std::max(maxseg + 1, HUGE_TUNE_BUCKETS * maxblk + 1), L.l2_roots + 1));
    uint64_t t = align_up(sizeof(Ctrl));
    if (L.l2_rows) t += align_up(8ull * L.l2_rows) + align_up(4ull * L.l2_roots) + align_up(8ull * (L.l2_roots + 1));
    if (k >= 3)
        for (int w = 2; w <= k - 1; ++w) {
            int64_t c = L.seg_cap[w];
            t += align_up(8ull * (c + 1)) + align_up(8ull * c) * 2 + align_up(4ull * c);
            if (part) {
                const int64_t nb = (c + 255) / 256;
                t += align_up(4ull * c) * 2 + align_up(8ull * c) * 2 + align_up(4ull * HUGE_TUNE_BUCKETS * nb) +
                     align_up(8ull * (HUGE_TUNE_BUCKETS * nb + 1));
            }
        }
    for (int w = 3; w <= k - 1; ++w) t += align_up(4ull * w * L.q_cap[w]);
    t += align_up(4ull * k * std::max<int64_t>(1, stage_rows));
    t += align_up(8ull * L.scan_tmp);
    L.total = t;
    return L;
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

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

// The plan as one execution sees it: the slice options of o applied to its steps.
DevPlan exec_plan(const huge_plan *p, const huge_exec_opts &o) {
    const int k = p->k;
    DevPlan P = p->dev;
    if (o.reserved0) HUGE_FAIL(HUGE_EINVAL, "reserved option fields must be 0");
    if (!p->bushy.empty()) HUGE_FAIL(HUGE_EINVAL, "a bushy plan runs through huge_count / huge_count_bushy only");
    if (o.slice_mode > HUGE_SLICE_STRIDE) HUGE_FAIL(HUGE_EINVAL, "unknown slice_mode %u", o.slice_mode);
    P.slice_count = o.slice_count > 1 ? o.slice_count : 1;
    P.slice_id = o.slice_count > 1 ? o.slice_id : 0;
    if (P.slice_count > 1 && P.slice_id >= P.slice_count) HUGE_FAIL(HUGE_EINVAL, "slice_id >= slice_count");
    if (o.slice_vertex < -2 || o.slice_vertex >= k) HUGE_FAIL(HUGE_EINVAL, "slice_vertex out of range");
    P.slice_mode = (int32_t)o.slice_mode;
    P.slice2_count = o.slice2_count > 1 ? o.slice2_count : 1;
    P.slice2_id = o.slice2_count > 1 ? o.slice2_id : 0;
    P.p2a = P.p2b = -1;
    const bool pair2 = (o.exec_flags & HUGE_EXEC_SLICE2_PAIR) != 0;
    int pos[HUGE_KMAX];
    for (int i = 0; i < k; ++i) pos[p->order[i]] = i;
    if (P.slice2_count > 1) {
        if (P.slice2_id >= P.slice2_count) HUGE_FAIL(HUGE_EINVAL, "slice2_id >= slice2_count");
        if (o.slice2_vertex < 0 || o.slice2_vertex >= k) HUGE_FAIL(HUGE_EINVAL, "slice2_vertex out of range");
        if (pair2) {
            const int b = o.slice2_vertex2;
            if (b < 0 || b >= k || b == o.slice2_vertex) HUGE_FAIL(HUGE_EINVAL, "slice2_vertex2 out of range");
            if (!p->adj[o.slice2_vertex][b]) HUGE_FAIL(HUGE_EINVAL, "a pair slice needs adjacent query vertices");
            P.p2a = pos[o.slice2_vertex];
            P.p2b = pos[b];
        }
    }
    const int sv = o.slice_vertex == -1 ? p->order[0] : o.slice_vertex;  // -2: edge slice, no vertex
    for (int i = 0; i < k; ++i)
        P.st[i].slice = (p->order[i] == sv ? 1 : 0) |
                        (P.slice2_count > 1 && !pair2 && p->order[i] == o.slice2_vertex ? 2 : 0) |
                        (P.p2a >= 0 && i == std::max(P.p2a, P.p2b) ? 4 : 0);
    P.edge_slice = (o.slice_vertex == -2 && P.slice_count > 1) ? (o.slice_mode == HUGE_SLICE_STRIDE ? 2 : 1) : 0;
    return P;
}

// Level-2 rows of a strided edge slice: entries slice_id, slice_id + S, ...
int64_t strided_l2_rows(const huge_graph *g, const DevPlan &P) {
    const int64_t nnz = g->dev.nnz, s = P.slice_id, S = P.slice_count;
    return nnz > s ? (nnz - s + S - 1) / S : 0;
}

// level_counts[0] counts the roots in the slices, and with the label, that apply to position 0
bool root_sliced(const DevPlan &P) {
    return ((P.st[0].slice & 1) && P.slice_count > 1 && !P.edge_slice) || ((P.st[0].slice & 2) && P.slice2_count > 1) ||
           P.st[0].label >= 0;
}

// The first matched vertex's count when its only filter is a strided slice
// (ranks s, s + S, ... below n): known without a pass over the vertices.
bool strided_root_count(const DevPlan &P, int64_t n, uint64_t *count) {
    if (P.st[0].label >= 0 || P.slice_mode != (int32_t)HUGE_SLICE_STRIDE || P.edge_slice) return false;
    if ((P.st[0].slice & 2) && P.slice2_count > 1) return false;
    if (!((P.st[0].slice & 1) && P.slice_count > 1)) return false;
    *count = n > (int64_t)P.slice_id ? (uint64_t)((n - P.slice_id + P.slice_count - 1) / P.slice_count) : 0;
    return true;
}

// A strided slice of the first matched vertex: level 2 is gathered, not scanned.
bool gathers_level2(const DevPlan &P) {
    return P.slice_mode == (int32_t)HUGE_SLICE_STRIDE && P.slice_count > 1 && (P.st[0].slice & 1) && !P.edge_slice;
}

// Rows in the slice's gathered level 2: slice s of S keeps ranks s, s + S, ...,
// and ranks ascend with degree, so every selected rank but the last has at most
// the mean degree of the S ranks from it on: at most nnz / S + max degree entries.
int64_t gathered_rows_bound(const huge_graph *g, const DevPlan &P) {
    return g->dev.nnz / (int64_t)P.slice_count + g->info.max_degree + 1;
}
int64_t gathered_roots(const huge_graph *g, const DevPlan &P) {
    const int64_t n = g->dev.n, s = P.slice_id, S = P.slice_count;
    return s < n ? (n - s + S - 1) / S : 0;
}

namespace {

// Pinned host memory for the scheduler's read-backs: a device-to-host copy lands
// there directly instead of through a staging copy.  Blocks come from a process
// pool (a call takes one and gives it back; the pool holds as many as calls ever
// ran at once and is never freed), so a call does not pay for an allocation;
// callers that must not allocate hand in a host block of their own instead.
struct PinnedPool {
    std::mutex mu;
    std::vector<unsigned char *> free_blocks;
};
PinnedPool &pinned_pool() {
    static PinnedPool *pool = new PinnedPool();  // never destroyed: blocks outlive static teardown
    return *pool;
}
struct PinnedBuf {
    unsigned char *p = nullptr;
    bool pooled = false;
    PinnedBuf(size_t bytes, unsigned char *given) {
        if (given) {
            p = given;
            return;
        }
        PinnedPool &pool = pinned_pool();
        {
            std::lock_guard<std::mutex> lock(pool.mu);
            if (!pool.free_blocks.empty()) {
                p = pool.free_blocks.back();
                pool.free_blocks.pop_back();
            }
        }
        if (!p) HUGE_HIP(hipHostMalloc((void **)&p, bytes, hipHostMallocDefault));
        pooled = true;
    }
    ~PinnedBuf() {
        if (!pooled) return;
        PinnedPool &pool = pinned_pool();
        std::lock_guard<std::mutex> lock(pool.mu);
        pool.free_blocks.push_back(p);
    }
};

int64_t read_i64(const void *dev, hipStream_t st, int64_t *pinned) {
    HUGE_HIP(hipMemcpyAsync(pinned, dev, 8, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    return *pinned;
}


}  // namespace

// Per-kernel-class device timing with HIP events recorded on the exec stream
// around each launch (only when profiling is requested).
struct Profiler {
    bool on = false;
    hipStream_t st = nullptr;
    TuneProbe *probe = nullptr;  // per-(j, bucket) attribution of tagged launches
    struct Ev {
        int cls, tag;
        hipEvent_t a, b;
    };
    std::vector<Ev> ev;
    uint64_t launches[4] = {0, 0, 0, 0};
    double bytes[4] = {0, 0, 0, 0};
    // tag = j * 8 + bucket for intersection launches, j * 8 + 7 for the
    // segment's other launches, -1 untagged
    template <typename F>
    void run(int cls, F &&launch, int tag = -1) {
        launches[cls]++;
        if (!on) {
            launch();
            return;
        }
        hipEvent_t a, b;
        HUGE_HIP(hipEventCreate(&a));
        HUGE_HIP(hipEventCreate(&b));
        ev.push_back({cls, tag, a, b});
        HUGE_HIP(hipEventRecord(a, st));
        launch();
        HUGE_HIP(hipEventRecord(b, st));
    }
    void finish(huge_result *out) {
        for (int c = 0; c < 4; ++c) {
            out->kernel_ms[c] = 0;
            out->kernel_launches[c] = launches[c];
            out->alg_bytes[c] = bytes[c];
        }
        if (on) HUGE_HIP(hipStreamSynchronize(st));
        for (auto &e : ev) {
            float ms = 0;
            if (on) HUGE_HIP(hipEventElapsedTime(&ms, e.a, e.b));
            out->kernel_ms[e.cls] += ms;
            if (probe && e.tag >= 0) {
                const int j = e.tag / 8, c = e.tag % 8;
                if (c < HUGE_TUNE_BUCKETS)
                    probe->ms[j][c] += ms;
                else
                    probe->other_ms[j] += ms;
            }
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        ev.clear();
    }
    ~Profiler() {
        for (auto &e : ev) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    }
};

uint64_t workspace_bytes(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o) {
    if (o.engine == HUGE_ENGINE_PERSISTENT) {
        const huge_plan *pl[1] = {p};
        return persist_workspace_bytes(pl, 1, o);
    }
    if (o.engine == HUGE_ENGINE_GRAPH) return make_layout(g, p, o, 0, scan_devn_max()).total + align_up(sizeof(GState));
    return make_layout(g, p, o, 1 << 16).total;
}

void segment_rows(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, int64_t *rows) {
    const Layout L = make_layout(g, p, o, 0);
    for (int w = 0; w < HUGE_KMAX; ++w) rows[w] = (w >= 2 && w <= p->k - 1) ? L.seg_cap[w] : 0;
}

bool run_levels(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, huge_result *out, EmitSink *emit,
                TuneProbe *probe, unsigned char *host_stage) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)o.stream;
    const int k = p->k;
    const DevPlan P = exec_plan(p, o);

    int64_t stage_rows = 0;
    if (emit) {
        if ((!emit->dev_out && (!emit->host_buf || !emit->cb)) || emit->buf_rows <= 0)
            HUGE_FAIL(HUGE_EINVAL, "huge_enumerate: host_buf, buf_rows and cb are required");
        stage_rows = std::min<int64_t>(emit->buf_rows, 1 << 22);
    }
    // rows for a device table are written in place, as ranks; for the host, staged and mapped to original IDs
    const int32_t *inv_rank = (emit && emit->dev_out) ? nullptr : g->inv_rank;
    auto out_rows = [&](int32_t *stage_buf, int64_t chunk) -> int32_t * {
        if (!emit->dev_out) return stage_buf;
        if ((int64_t)emit->delivered + chunk > emit->dev_cap) HUGE_FAIL(HUGE_EDEVICE, "device table overflow");
        return emit->dev_out + (int64_t)emit->delivered * k;
    };
    Layout L = make_layout(g, p, o, stage_rows);
    PinnedBuf pinned(kHostStageBytes, host_stage);
    int64_t *pin64 = (int64_t *)(pinned.p + sizeof(Ctrl));
    DevMem own;
    char *ws = (char *)o.workspace;
    if (ws) {
        if (o.workspace_bytes < L.total)
            HUGE_FAIL(HUGE_ENOMEM, "workspace too small: %llu bytes given, %llu needed",
                      (unsigned long long)o.workspace_bytes, (unsigned long long)L.total);
    } else {
        HUGE_HIP(hipMalloc(&own.p, L.total));
        ws = (char *)own.p;
    }
    Carver cv{ws};
    Ctrl *ctrl = cv.take<Ctrl>(1);
    const bool part = partitioned(o);
    struct Lv {
        int64_t nrows = 0, next = 0;
        int64_t seg_row0 = 0, seg_n = 0, seg_total = 0, seg_done = 0;
        int64_t bw[HUGE_TUNE_BUCKETS + 1] = {};  // partitioned segment: first work item of each bucket, total
        double seg_bytes = 0;
        SegBufs s{};
        int32_t *q = nullptr;
        int64_t qcap = 0;
    } lv[HUGE_KMAX + 1];
    if (k >= 3)
        for (int w = 2; w <= k - 1; ++w) {
            int64_t c = L.seg_cap[w];
            lv[w].s.off = cv.take<int64_t>(c + 1);
            lv[w].s.pinfo = cv.take<uint64_t>(c);
            lv[w].s.hpre = cv.take<uint64_t>(c);
            lv[w].s.bound = cv.take<int32_t>(c);
            lv[w].s.cap = c;
            if (part) {
                const int64_t nb = (c + 255) / 256;
                lv[w].s.bound_in = cv.take<int32_t>(c);
                lv[w].s.rid = cv.take<int32_t>(c);
                lv[w].s.pinfo_in = cv.take<uint64_t>(c);
                lv[w].s.hpre_in = cv.take<uint64_t>(c);
                lv[w].s.bcnt = cv.take<int32_t>(HUGE_TUNE_BUCKETS * nb);
                lv[w].s.bscan = cv.take<int64_t>(HUGE_TUNE_BUCKETS * nb + 1);
            }
        }
    for (int w = 3; w <= k - 1; ++w) {
        lv[w].q = cv.take<int32_t>((uint64_t)w * L.q_cap[w]);
        lv[w].qcap = L.q_cap[w];
    }
    int32_t *stage = cv.take<int32_t>((uint64_t)k * std::max<int64_t>(1, stage_rows));
    int64_t *scan_tmp = cv.take<int64_t>(L.scan_tmp);

    HUGE_HIP(hipMemsetAsync(ctrl, 0, sizeof(Ctrl), st));
    ExecStats stats;
    Profiler prof;
    prof.on = o.profile != 0 || probe;
    prof.probe = probe;
    prof.st = st;
    GraphDev G = g->dev;
    int64_t l2_rows = G.nnz;  // level-2 rows: every edge-array entry, a strided edge slice, or the gathered slice
    if (P.edge_slice == 2) {
        G.l2_first = P.slice_id;
        G.l2_stride = P.slice_count;
        l2_rows = strided_l2_rows(g, P);
    }
    if (L.l2_rows) {
        int64_t *idx = cv.take<int64_t>(L.l2_rows);
        int32_t *deg = cv.take<int32_t>(L.l2_roots);
        int64_t *off = cv.take<int64_t>(L.l2_roots + 1);
        launch_gather_level2(G, P, L.l2_roots, deg, off, idx, L.l2_rows, scan_tmp, st);
        stats.launches += 4;
        l2_rows = read_i64(off + L.l2_roots, st, pin64);
        if (l2_rows > L.l2_rows) HUGE_FAIL(HUGE_EDEVICE, "gathered level 2 exceeds its bound");
        G.l2_idx = idx;
    }
    const int strat = (o.strategy >= 0 && o.strategy < STRAT_COUNT) ? o.strategy : STRAT_LANE_MERGE;
    const int count_mode = (o.exec_flags & HUGE_EXEC_NO_HASH) ? MODE_COUNT_NOHASH : MODE_COUNT;
    const bool root_slice = root_sliced(P);
    bool limited = false;
    uint64_t level_work[HUGE_KMAX] = {};
    uint64_t roots_known = 0;
    const bool roots_closed = root_slice && strided_root_count(P, G.n, &roots_known);
    if (root_slice && !roots_closed) {
        launch_root_count(G, P, ctrl, st);
        stats.launches++;
    }

    auto deliver = [&](int64_t nout) {
        if (nout <= 0) return;
        if (emit->dev_out) {  // already in place
            emit->delivered += (uint64_t)nout;
            return;
        }
        HUGE_HIP(hipMemcpyAsync(emit->host_buf, stage, sizeof(int32_t) * k * nout, hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        emit->delivered += (uint64_t)nout;
        if (emit->cb(emit->user, emit->host_buf, nout, k) != 0) emit->stopped = true;
    };

    // intersection launches over work items [w0, w1) of level l's segment: one
    // launch, or one per probe-length bucket with the tuned strategy
    auto extend_range = [&](int cls, int W, int mode, Lv &l, int64_t w0, int64_t w1, int32_t *outp) {
        const int jW = ext_count(p, W);
        if (!part) {
            prof.run(cls, [&] {
                launch_extend(W, mode, strat, G, P, l.q, l.seg_row0, l.s, l.seg_n, w0, w1, outp, ctrl, inv_rank,
                              st, false);
            });
            stats.launches++;
            return;
        }
        for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) {
            const int64_t a = std::max(w0, l.bw[c]), b = std::min(w1, l.bw[c + 1]);
            if (a >= b) continue;
            int sc = o.tune->strategy[jW][c];
            if (sc < 0 || sc >= STRAT_COUNT) sc = STRAT_LANE_MERGE;
            prof.run(cls, [&] {
                launch_extend(W, mode, sc, G, P, l.q, l.seg_row0, l.s, l.seg_n, a, b, outp, ctrl, inv_rank, st,
                              true);
            }, jW * 8 + c);
            if (probe) probe->items[jW][c] += b - a;
            stats.launches++;
        }
    };

    if (k == 2) {
        const int64_t nnz = l2_rows;
        if (!emit) {
            for (int64_t e = 0; e < nnz; e += kMaxItems) {
                launch_edge_sink(G, P, e, std::min(nnz, e + kMaxItems), MODE_COUNT, nullptr, g->inv_rank, ctrl, st);
                stats.launches++;
            }
        } else {
            for (int64_t e = 0; e < nnz && !emit->stopped; e += stage_rows) {
                const int64_t e1 = std::min(nnz, e + stage_rows);
                launch_edge_sink(G, P, e, e1, MODE_OUTPUT, out_rows(stage, e1 - e), inv_rank, ctrl, st);
                stats.launches++;
                int64_t nout = read_i64(&ctrl->qcount[HUGE_KMAX], st, pin64);
                deliver(nout);
                HUGE_HIP(hipMemsetAsync(&ctrl->qcount[HUGE_KMAX], 0, 8, st));
            }
        }
    } else {
        const int lastW = k - 1;
        lv[2].nrows = l2_rows;
        int64_t work_done = 0;  // candidates examined (work items launched)
        int W = 2;
        uint64_t cur_bytes = 0;
        auto has_input = [](const Lv &l) { return l.seg_done < l.seg_total || l.next < l.nrows; };
        bool stop = false;
        while (!stop) {
            Lv &l = lv[W];
            if (!has_input(l)) {
                if (W == 2) break;
                cur_bytes -= (uint64_t)l.nrows * 4ull * W;
                l.nrows = l.next = 0;
                l.seg_total = l.seg_done = 0;
                HUGE_HIP(hipMemsetAsync(&ctrl->qcount[W], 0, 8, st));
                --W;
                continue;
            }
            // Schedule(O): run until the output queue is full or the input is empty
            for (;;) {
                if (l.seg_done == l.seg_total) {
                    if (l.next == l.nrows) break;
                    int64_t cnt = std::min(l.s.cap, l.nrows - l.next);
                    HUGE_HIP(hipMemsetAsync(&ctrl->segbytes[W], 0, 8, st));
                    const int otag = ext_count(p, W) * 8 + 7;
                    SegBufs pre = l.s;
                    if (part) {
                        pre.bound = l.s.bound_in;
                        pre.pinfo = l.s.pinfo_in;
                        pre.hpre = l.s.hpre_in;
                    }
                    prof.run(HUGE_KC_PREPARE,
                             [&] { launch_prepare(W, W == lastW, G, P, lv[W].q, l.next, cnt, pre, ctrl, st); }, otag);
                    if (part) {
                        prof.run(HUGE_KC_SCAN,
                                 [&] { launch_bucket_partition(l.s, cnt, W == lastW, scan_tmp, ctrl, st); }, otag);
                        stats.launches += 3;
                    }
                    prof.run(HUGE_KC_SCAN, [&] { launch_scan_bounds(l.s, cnt, scan_tmp, st); }, otag);
                    stats.launches += 2;
                    if (part) {
                        launch_bucket_bounds(l.s, cnt, ctrl, st);
                        stats.launches += 1;
                    }
                    l.seg_row0 = l.next;
                    l.seg_n = cnt;
                    // one read-back per segment: the segment total goes next to the
                    // bucket bounds (a device-side copy), then segbytes[W] .. scratch[]
                    // come back in one copy
                    HUGE_HIP(hipMemcpyAsync(&ctrl->scratch[kSegTotalSlot], l.s.off + cnt, 8, hipMemcpyDeviceToDevice,
                                            st));
                    const size_t first = offsetof(Ctrl, segbytes) + sizeof(unsigned long long) * W;
                    unsigned char *hb = pinned.p;
                    HUGE_HIP(hipMemcpyAsync(hb, (const unsigned char *)ctrl + first, sizeof(Ctrl) - first,
                                            hipMemcpyDeviceToHost, st));
                    HUGE_HIP(hipStreamSynchronize(st));
                    Ctrl hc;
                    memcpy((unsigned char *)&hc + first, hb, sizeof(Ctrl) - first);
                    l.seg_total = hc.scratch[kSegTotalSlot];
                    level_work[W - 1] += (uint64_t)l.seg_total;
                    l.seg_bytes = (double)hc.segbytes[W];
                    for (int c = 0; c <= HUGE_TUNE_BUCKETS; ++c) l.bw[c] = part ? hc.scratch[c] : 0;
                    l.seg_done = 0;
                    l.next += cnt;
                    if (l.seg_total == 0) continue;
                }
                const int64_t remaining = l.seg_total - l.seg_done;
                if (W == lastW) {
                    if (!emit) {
                        int64_t chunk = std::min(remaining, kMaxItems);
                        // under a work limit, stop soon after crossing it
                        if (o.work_limit > 0)
                            chunk = std::min(chunk, std::max<int64_t>(1 << 20, o.work_limit - work_done + 1));
                        extend_range(HUGE_KC_SINK, W, count_mode, l, l.seg_done, l.seg_done + chunk, nullptr);
                        prof.bytes[HUGE_KC_SINK] += l.seg_bytes * (double)chunk / (double)l.seg_total;
                        l.seg_done += chunk;
                        work_done += chunk;
                        if (o.work_limit > 0 && work_done > o.work_limit) {
                            stop = limited = true;
                            break;
                        }
                    } else {
                        int64_t chunk = std::min(remaining, stage_rows);
                        extend_range(HUGE_KC_SINK, W, MODE_OUTPUT, l, l.seg_done, l.seg_done + chunk,
                                     out_rows(stage, chunk));
                        l.seg_done += chunk;
                        int64_t nout = read_i64(&ctrl->qcount[HUGE_KMAX], st, pin64);
                        deliver(nout);
                        HUGE_HIP(hipMemsetAsync(&ctrl->qcount[HUGE_KMAX], 0, 8, st));
                        if (emit->stopped) {
                            stop = true;
                            break;
                        }
                    }
                } else {
                    Lv &q = lv[W + 1];
                    const int64_t free = q.qcap - q.nrows;
                    if (free <= 0 || (free < remaining && free < q.qcap / 8)) break;  // Q_O full: yield
                    const int64_t chunk = std::min(std::min(free, remaining), kMaxItems);
                    extend_range(HUGE_KC_EXTEND, W, MODE_EMIT, l, l.seg_done, l.seg_done + chunk, q.q);
                    l.seg_done += chunk;
                    work_done += chunk;
                    int64_t nr = read_i64(&ctrl->qcount[W + 1], st, pin64);
                    prof.bytes[HUGE_KC_EXTEND] +=
                        l.seg_bytes * (double)chunk / (double)l.seg_total + 4.0 * (W + 1) * (double)(nr - q.nrows);
                    cur_bytes += (uint64_t)(nr - q.nrows) * 4ull * (W + 1);
                    q.nrows = nr;
                    stats.peak_frontier_bytes = std::max(stats.peak_frontier_bytes, cur_bytes);
                    if (o.work_limit > 0 && work_done > o.work_limit) {
                        stop = limited = true;
                        break;
                    }
                }
            }
            if (W == lastW) {
                if (W > 2) --W;
            } else {
                ++W;
            }
        }
    }

    Ctrl h;
    HUGE_HIP(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    memset(out, 0, sizeof(*out));
    out->count = emit ? emit->delivered : h.acc[0];
    out->hash_sum = h.acc[1];
    out->hash_xor = h.acc[2];
    for (int i = 0; i < HUGE_KMAX; ++i) out->level_counts[i] = h.level[i];
    if (!root_slice) out->level_counts[0] = (uint64_t)G.n;
    if (roots_closed) out->level_counts[0] = roots_known;
    out->peak_frontier_bytes = stats.peak_frontier_bytes;
    for (int i = 0; i < HUGE_KMAX; ++i) out->level_work[i] = level_work[i];
    out->launches = stats.launches;
    prof.finish(out);
    auto t1 = std::chrono::steady_clock::now();
    out->query_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return limited;
}


// ---------------------------------------------------------------------------
// Graph engine: the same Algorithm 5, with its scheduler on the device
// (k_round_sched) so that no host decision sits between launches.  One round
// is: the scheduler picks one action (prepare + scan a segment of level W, or
// extend a range of its work items), then every level's fixed-grid prepare,
// scan and extend launches run, idle unless the action is theirs.  kRounds
// rounds are recorded once in a hipGraph; the host replays it and reads the
// done flag every kBatch replays.  Rounds after the end are idle.  No memset
// or copy is recorded: counters are cleared by the scheduler kernel itself.
// ---------------------------------------------------------------------------
namespace {
constexpr int kRounds = 4;                 // rounds recorded in the graph
constexpr int kBatch = 8;                  // graph launches between done checks
constexpr int64_t kMaxRoundsTotal = 1ll << 26;

struct GraphRes {
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphRes() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) {
            // an error while recording leaves the stream capturing: close that first
            hipStreamCaptureStatus status = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(cs, &status) == hipSuccess && status != hipStreamCaptureStatusNone) {
                hipGraph_t partial = nullptr;
                (void)hipStreamEndCapture(cs, &partial);
                if (partial) (void)hipGraphDestroy(partial);
            }
            (void)hipStreamDestroy(cs);
        }
    }
};
}  // namespace

void run_graph(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o_in, huge_result *out) {
    auto t0 = std::chrono::steady_clock::now();
    if (o_in.work_limit > 0) HUGE_FAIL(HUGE_EINVAL, "the graph engine has no work limit");
    const bool part = partitioned(o_in);
    const int strat = (o_in.strategy >= 0 && o_in.strategy < STRAT_COUNT) ? o_in.strategy : STRAT_BLOCK_MERGE_LONG;
    const int k = p->k;
    if (k < 3) {  // one edge-array launch: nothing to replay
        huge_exec_opts o = o_in;
        o.engine = HUGE_ENGINE_LEVELS;
        o.tune = nullptr;
        run_levels(g, p, o, out, nullptr, nullptr);
        return;
    }
    const huge_exec_opts &o = o_in;
    hipStream_t st = (hipStream_t)o.stream;
    const DevPlan P = exec_plan(p, o);
    const bool root_slice = root_sliced(P);

    Layout L = make_layout(g, p, o, 0, scan_devn_max());  // segments within the device-count scan's limit
    const uint64_t gs_off = L.total;
    const uint64_t total = gs_off + align_up(sizeof(GState));
    DevMem own;
    char *ws = (char *)o.workspace;
    if (ws) {
        if (o.workspace_bytes < total)
            HUGE_FAIL(HUGE_ENOMEM, "workspace too small: %llu bytes given, %llu needed",
                      (unsigned long long)o.workspace_bytes, (unsigned long long)total);
    } else {
        HUGE_HIP(hipMalloc(&own.p, total));
        ws = (char *)own.p;
    }
    Carver cv{ws};
    Ctrl *ctrl = cv.take<Ctrl>(1);
    SegBufs sb[HUGE_KMAX + 1] = {};
    int32_t *q[HUGE_KMAX + 1] = {};
    for (int w = 2; w <= k - 1; ++w) {
        const int64_t c = L.seg_cap[w];
        sb[w].off = cv.take<int64_t>(c + 1);
        sb[w].pinfo = cv.take<uint64_t>(c);
        sb[w].hpre = cv.take<uint64_t>(c);
        sb[w].bound = cv.take<int32_t>(c);
        sb[w].cap = c;
        if (part) {
            const int64_t nb = (c + 255) / 256;
            sb[w].bound_in = cv.take<int32_t>(c);
            sb[w].rid = cv.take<int32_t>(c);
            sb[w].pinfo_in = cv.take<uint64_t>(c);
            sb[w].hpre_in = cv.take<uint64_t>(c);
            sb[w].bcnt = cv.take<int32_t>(HUGE_TUNE_BUCKETS * nb);
            sb[w].bscan = cv.take<int64_t>(HUGE_TUNE_BUCKETS * nb + 1);
        }
    }
    for (int w = 3; w <= k - 1; ++w) q[w] = cv.take<int32_t>((uint64_t)w * L.q_cap[w]);
    (void)cv.take<int32_t>((uint64_t)k);  // staging (unused here): the level engine's layout
    int64_t *scan_tmp = cv.take<int64_t>(L.scan_tmp);
    GState *gs = (GState *)(ws + gs_off);

    GConst gc{};
    gc.k = k;
    gc.lastW = k - 1;
    for (int w = 2; w <= k - 1; ++w) {
        gc.seg_cap[w] = L.seg_cap[w];
        gc.off[w] = sb[w].off;
    }
    for (int w = 3; w <= k - 1; ++w) gc.q_cap[w] = L.q_cap[w];
    GraphDev G = g->dev;
    int64_t l2_rows = G.nnz;
    if (P.edge_slice == 2) {
        G.l2_first = P.slice_id;
        G.l2_stride = P.slice_count;
        l2_rows = strided_l2_rows(g, P);
    }
    if (L.l2_rows) {  // a strided root slice: gather its level-2 entries first
        int64_t *idx = cv.take<int64_t>(L.l2_rows);
        int32_t *deg = cv.take<int32_t>(L.l2_roots);
        int64_t *off = cv.take<int64_t>(L.l2_roots + 1);
        launch_gather_level2(G, P, L.l2_roots, deg, off, idx, L.l2_rows, scan_tmp, st);
        HUGE_HIP(hipMemcpyAsync(&l2_rows, off + L.l2_roots, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        if (l2_rows > L.l2_rows) HUGE_FAIL(HUGE_EDEVICE, "gathered level 2 exceeds its bound");
        G.l2_idx = idx;
    }
    GState init{};
    init.W = 2;
    init.lv[2].nrows = l2_rows;
    HUGE_HIP(hipMemsetAsync(ctrl, 0, sizeof(Ctrl), st));
    HUGE_HIP(hipMemcpyAsync(gs, &init, sizeof(GState), hipMemcpyHostToDevice, st));
    uint64_t roots_known = 0;
    const bool roots_closed = root_slice && strided_root_count(P, G.n, &roots_known);
    if (root_slice && !roots_closed) launch_root_count(G, P, ctrl, st);
    const int count_mode = (o.exec_flags & HUGE_EXEC_NO_HASH) ? MODE_COUNT_NOHASH : MODE_COUNT;

    // record kRounds rounds on a private stream
    GraphRes gr;
    HUGE_HIP(hipStreamCreateWithFlags(&gr.cs, hipStreamNonBlocking));
    HUGE_HIP(hipStreamBeginCapture(gr.cs, hipStreamCaptureModeRelaxed));  // occupancy queries run while recording
    for (int r = 0; r < kRounds; ++r) {
        launch_round_sched(gs, gc, ctrl, gr.cs);
        for (int w = 2; w <= k - 1; ++w) {
            const bool last = w == k - 1;
            const int mode = last ? count_mode : MODE_EMIT;
            int32_t *outq = last ? nullptr : q[w + 1];
            if (!part) {
                launch_round_prepare(w, last, G, P, q[w], sb[w], ctrl, gs, L.seg_cap[w], gr.cs);
                launch_round_scan(w, sb[w], gs, L.seg_cap[w], scan_tmp, gr.cs);
                launch_round_extend(w, mode, strat, G, P, q[w], sb[w], outq, ctrl, g->inv_rank, gs, -1, gr.cs);
                continue;
            }
            // tuned dispatch, as in the level engine: prepare into the *_in
            // arrays, partition by probe-length bucket, scan, one launch per bucket
            SegBufs pre = sb[w];
            pre.bound = sb[w].bound_in;
            pre.pinfo = sb[w].pinfo_in;
            pre.hpre = sb[w].hpre_in;
            launch_round_prepare(w, last, G, P, q[w], pre, ctrl, gs, L.seg_cap[w], gr.cs);
            launch_round_partition(w, last, sb[w], gs, L.seg_cap[w], scan_tmp, gr.cs);
            launch_round_scan(w, sb[w], gs, L.seg_cap[w], scan_tmp, gr.cs);
            launch_round_bucket_bounds(w, sb[w], gs, gr.cs);
            const int jW = ext_count(p, w);
            for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) {
                int sc = o.tune->strategy[jW][c];
                if (sc < 0 || sc >= STRAT_COUNT) sc = STRAT_LANE_MERGE;
                launch_round_extend(w, mode, sc, G, P, q[w], sb[w], outq, ctrl, g->inv_rank, gs, c, gr.cs);
            }
        }
    }
    HUGE_HIP(hipStreamEndCapture(gr.cs, &gr.graph));
    HUGE_HIP(hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0));

    int32_t done = 0;
    int64_t replays = 0;
    while (!done) {
        for (int b = 0; b < kBatch; ++b) HUGE_HIP(hipGraphLaunch(gr.exec, st));
        replays += kBatch;
        HUGE_HIP(hipMemcpyAsync(&done, &gs->done, sizeof(done), hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        if (!done && replays * kRounds > kMaxRoundsTotal)
            HUGE_FAIL(HUGE_EINVAL, "graph engine: no end after %lld rounds", (long long)(replays * kRounds));
    }
    Ctrl h;
    GState hs;
    HUGE_HIP(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipMemcpyAsync(&hs, gs, sizeof(GState), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    if (hs.error) HUGE_FAIL(HUGE_EINVAL, "graph engine: the device scheduler found no action");
    memset(out, 0, sizeof(*out));
    out->count = h.acc[0];
    out->hash_sum = h.acc[1];
    out->hash_xor = h.acc[2];
    for (int i = 0; i < HUGE_KMAX; ++i) out->level_counts[i] = h.level[i];
    if (!root_slice) out->level_counts[0] = (uint64_t)G.n;
    if (roots_closed) out->level_counts[0] = roots_known;
    out->peak_frontier_bytes = (uint64_t)hs.peak_bytes;
    for (int i = 0; i < HUGE_KMAX; ++i) out->level_work[i] = (uint64_t)hs.work[i];
    out->launches = (uint64_t)replays;  // graph launches
    auto t1 = std::chrono::steady_clock::now();
    out->query_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

}  // namespace huge
