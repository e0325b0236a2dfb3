// Autotuner for the per-bucket dispatch (Section 7.3 studies the batch size
// as the knob of the scheduler; on the GPU the choice of intersection kernel
// per probe length matters as much).
//
// The sample is the real work: the given plans on one root slice of the
// graph.  Every strategy runs the same sample with the table forcing it for
// all buckets; HIP events around every launch attribute device time to
// (j, bucket), j = |Ext| of the step.  Per (j, bucket) the fastest strategy
// wins.  Then, with those strategies, each candidate segment size runs the
// sample and per j the fastest total (intersections plus the segment's
// prepare, partition and scan launches) wins.  Because every run counts the
// same matches, the tuner also checks that all runs agree.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace huge {

namespace {

void blank(huge_tune_table &t) {
    memset(&t, 0, sizeof(t));
    for (int j = 0; j <= HUGE_KMAX; ++j)
        for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) t.strategy[j][c] = HUGE_STRAT_AUTO;
}

struct Key {
    uint64_t count, hs, hx;
    bool operator!=(const Key &o) const { return count != o.count || hs != o.hs || hx != o.hx; }
};

void run_sample(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &base,
                const huge_tune_table &t, TuneProbe *probe, std::vector<Key> &keys) {
    huge_exec_opts o = base;
    o.tune = &t;
    o.strategy = HUGE_STRAT_AUTO;
    o.engine = HUGE_ENGINE_LEVELS;
    o.profile = 0;
    keys.resize(np);
    for (int i = 0; i < np; ++i) {
        huge_result r;
        run_levels(g, plans[i], o, &r, nullptr, probe);
        keys[i] = {r.count, r.hash_sum, r.hash_xor};
    }
}

}  // namespace

void autotune(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &opts,
              huge_tune_table *out) {
    const int64_t cands[3] = {1 << 18, 1 << 20, 1 << 22};  // segment rows tried in pass 2
    // one workspace for every run: the largest any plan needs under any table tried
    struct Mem {
        void *p = nullptr;
        ~Mem() {
            if (p) (void)hipFree(p);
        }
    } mem;
    huge_exec_opts o = opts;
    if (!o.workspace) {
        huge_tune_table t;
        blank(t);
        huge_exec_opts oo = o;
        oo.tune = &t;
        oo.strategy = HUGE_STRAT_AUTO;
        oo.engine = HUGE_ENGINE_LEVELS;
        uint64_t need = 256;
        for (int i = 0; i < np; ++i) need = std::max(need, workspace_bytes(g, plans[i], oo));
        oo.chunk_rows = 0;
        for (int64_t c : cands) {
            for (int j = 0; j <= HUGE_KMAX; ++j) t.chunk_rows[j] = c;
            for (int i = 0; i < np; ++i) need = std::max(need, workspace_bytes(g, plans[i], oo));
        }
        HUGE_HIP(hipMalloc(&mem.p, need));
        o.workspace = mem.p;
        o.workspace_bytes = need;
    }
    huge_tune_table best;
    blank(best);
    std::vector<Key> ref, keys;
    // 1. strategy per (j, bucket)
    TuneProbe pr[STRAT_COUNT];
    for (int s = 0; s < STRAT_COUNT; ++s) {
        huge_tune_table forced;
        blank(forced);
        for (int j = 0; j <= HUGE_KMAX; ++j)
            for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) forced.strategy[j][c] = s;
        run_sample(g, plans, np, o, forced, &pr[s], s == 0 ? ref : keys);
        if (s > 0)
            for (int i = 0; i < np; ++i)
                if (keys[i] != ref[i]) HUGE_FAIL(HUGE_EDEVICE, "autotune: strategy %d disagrees on plan %d", s, i);
    }
    for (int j = 0; j <= HUGE_KMAX; ++j)
        for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) {
            if (pr[0].items[j][c] == 0) continue;  // same work under every strategy
            int b = 0;
            for (int s = 1; s < STRAT_COUNT; ++s)
                if (pr[s].ms[j][c] < pr[b].ms[j][c]) b = s;
            best.strategy[j][c] = b;
            best.ms[j][c] = pr[b].ms[j][c];
            best.items[j][c] = pr[b].items[j][c];
        }
    // 2. segment rows per j, with the chosen strategies
    TuneProbe pc[3];
    for (int i = 0; i < 3; ++i) {
        huge_tune_table t = best;
        for (int j = 0; j <= HUGE_KMAX; ++j) t.chunk_rows[j] = cands[i];
        huge_exec_opts oo = o;
        oo.chunk_rows = 0;
        run_sample(g, plans, np, oo, t, &pc[i], keys);
        for (int q = 0; q < np; ++q)
            if (keys[q] != ref[q]) HUGE_FAIL(HUGE_EDEVICE, "autotune: segment size %lld disagrees on plan %d",
                                             (long long)cands[i], q);
    }
    for (int j = 0; j <= HUGE_KMAX; ++j) {
        double tb = 0;
        int b = -1;
        for (int i = 0; i < 3; ++i) {
            double tot = pc[i].other_ms[j];
            for (int c = 0; c < HUGE_TUNE_BUCKETS; ++c) tot += pc[i].ms[j][c];
            if (tot <= 0) continue;
            if (b < 0 || tot < tb) {
                tb = tot;
                b = i;
            }
        }
        if (b >= 0) best.chunk_rows[j] = cands[b];
    }
    *out = best;
}

}  // namespace huge
