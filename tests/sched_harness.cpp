// Test harness (CPU): drives the graph engine's scheduler step, the same
// source the device runs (round_sched.h), over a synthetic query tree, next to
// a model of the level engine's host loop, with the same simulated kernels.
// Prints the two action counts, whether the sequences agree, the SINK count of
// each, the count from a direct recursion over the tree, and the largest
// queue fill seen against its capacity.
//
// usage: sched_harness k nnz bmax emit_mod seed seg_cap q_cap
//        sched_harness trace k nnz seg_cap q_cap b_2 .. b_{k-1}
// The trace form uses a fixed model (every row of level W has b_W candidates,
// all of them kept) and prints the device scheduler's actions in order, as
// "kind:W" tokens (P prepare, E emit, S sink), after the count comparison.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "round_sched.h"

using namespace huge;

namespace {

uint64_t mixh(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

struct Synth {
    int k = 4, lastW = 3;
    int64_t nnz = 0;
    uint64_t seed = 1;
    int bmax = 8, emit_mod = 3;
    int64_t fixed[HUGE_KMAX + 1] = {};  // trace form: fixed bound per level, every candidate kept
    bool use_fixed = false;
    int64_t bound(int W, uint64_t id) const {
        if (use_fixed) return fixed[W];
        return (int64_t)(mixh(id ^ seed ^ ((uint64_t)W << 56)) % (uint64_t)(bmax + 1));
    }
    bool emits(int W, uint64_t id, int64_t i) const {
        if (use_fixed) return true;
        return mixh(id * 0x100000001B3ull + (uint64_t)i + ((uint64_t)W << 48) + seed) % (uint64_t)emit_mod == 0;
    }
    uint64_t child(uint64_t id, int64_t i) const { return mixh(id ^ ((uint64_t)(i + 1) * 0xD6E8FEB86659FD93ull)); }
    int64_t ground(int W, uint64_t id) const {
        const int64_t b = bound(W, id);
        if (W == lastW) return b;
        int64_t t = 0;
        for (int64_t i = 0; i < b; ++i)
            if (emits(W, id, i)) t += ground(W + 1, child(id, i));
        return t;
    }
};

struct Action {
    int kind, W;
    int64_t a, b;
    bool operator!=(const Action &o) const { return kind != o.kind || W != o.W || a != o.a || b != o.b; }
};

// The simulated device: queues, scanned segment bounds, emission counters.
struct Sim {
    const Synth &S;
    std::vector<std::vector<uint64_t>> q;   // [W] row ids by queue position (level 2: the row index)
    std::vector<std::vector<int64_t>> off;  // [W] exclusive scan of the current segment's bounds
    std::vector<int64_t> seg_row0;
    unsigned long long qcount[HUGE_KMAX + 1] = {};
    std::vector<int64_t> qcap;
    int64_t count = 0, max_fill_over_cap = 0;
    bool overflow = false;
    Sim(const Synth &s, int64_t seg_cap, const std::vector<int64_t> &qc)
        : S(s), q(HUGE_KMAX + 1), off(HUGE_KMAX + 1, std::vector<int64_t>(seg_cap + 1)), seg_row0(HUGE_KMAX + 1),
          qcap(qc) {
        for (int w = 3; w <= s.lastW; ++w) q[w].assign(qc[w], 0);
    }
    uint64_t row_id(int W, int64_t r) const { return W == 2 ? (uint64_t)r : q[W][r]; }
    void prepare(int W, int64_t row0, int64_t n) {
        seg_row0[W] = row0;
        off[W][0] = 0;
        for (int64_t i = 0; i < n; ++i) off[W][i + 1] = off[W][i] + S.bound(W, row_id(W, row0 + i));
    }
    void extend(int W, int64_t w0, int64_t w1) {
        int64_t r = 0;
        for (int64_t w = w0; w < w1; ++w) {
            while (off[W][r + 1] <= w) ++r;
            const int64_t i = w - off[W][r];
            const uint64_t id = row_id(W, seg_row0[W] + r);
            if (W == S.lastW) {
                ++count;
            } else if (S.emits(W, id, i)) {
                const int64_t pos = (int64_t)qcount[W + 1]++;
                if (pos >= qcap[W + 1]) {
                    overflow = true;
                    return;
                }
                q[W + 1][pos] = S.child(id, i);
            }
        }
    }
};

// Model of the level engine's host loop (its control flow, not its kernels).
std::vector<Action> host_loop(Sim &sim, const std::vector<int64_t> &seg_cap, const std::vector<int64_t> &qcap) {
    const Synth &S = sim.S;
    struct Lv {
        int64_t nrows = 0, next = 0, seg_row0 = 0, seg_n = 0, seg_total = 0, seg_done = 0;
    } lv[HUGE_KMAX + 1];
    std::vector<Action> log;
    lv[2].nrows = S.nnz;
    int W = 2;
    auto has_input = [](const Lv &l) { return l.seg_done < l.seg_total || l.next < l.nrows; };
    for (;;) {
        Lv &l = lv[W];
        if (!has_input(l)) {
            if (W == 2) break;
            l = Lv{};
            sim.qcount[W] = 0;
            --W;
            continue;
        }
        for (;;) {
            if (l.seg_done == l.seg_total) {
                if (l.next == l.nrows) break;
                const int64_t cnt = std::min(seg_cap[W], l.nrows - l.next);
                log.push_back({GACT_PREPARE, W, l.next, cnt});
                sim.prepare(W, l.next, cnt);
                l.seg_row0 = l.next;
                l.seg_n = cnt;
                l.seg_total = sim.off[W][cnt];
                l.seg_done = 0;
                l.next += cnt;
                if (l.seg_total == 0) continue;
            }
            const int64_t rem = l.seg_total - l.seg_done;
            if (W == S.lastW) {
                log.push_back({GACT_SINK, W, l.seg_done, l.seg_total});
                sim.extend(W, l.seg_done, l.seg_total);
                l.seg_done = l.seg_total;
            } else {
                Lv &nq = lv[W + 1];
                const int64_t fr = qcap[W + 1] - nq.nrows;
                if (fr <= 0 || (fr < rem && fr < qcap[W + 1] / 8)) break;
                const int64_t chunk = std::min(fr, rem);
                log.push_back({GACT_EMIT, W, l.seg_done, l.seg_done + chunk});
                sim.extend(W, l.seg_done, l.seg_done + chunk);
                l.seg_done += chunk;
                nq.nrows = (int64_t)sim.qcount[W + 1];
            }
        }
        if (W == S.lastW) {
            if (W > 2) --W;
        } else {
            ++W;
        }
    }
    return log;
}

std::vector<Action> device_steps(Sim &sim, const std::vector<int64_t> &seg_cap, const std::vector<int64_t> &qcap,
                                 bool &error) {
    const Synth &S = sim.S;
    GState s{};
    s.W = 2;
    s.lv[2].nrows = S.nnz;
    GConst c{};
    c.k = S.k;
    c.lastW = S.lastW;
    for (int w = 2; w <= S.lastW; ++w) {
        c.seg_cap[w] = seg_cap[w];
        c.q_cap[w] = qcap[w];
        c.off[w] = sim.off[w].data();
    }
    std::vector<Action> log;
    for (int64_t guard = 0; guard < 100000000 && !s.done; ++guard) {
        round_sched_step(s, c, sim.qcount, 1ll << 30);
        for (int w = 2; w <= S.lastW; ++w) {
            if (s.n_prep[w] > 0) {
                log.push_back({GACT_PREPARE, w, s.lv[w].seg_row0, s.n_prep[w]});
                sim.prepare(w, s.lv[w].seg_row0, s.n_prep[w]);
            }
            if (s.ext_w1[w] > s.ext_w0[w]) {
                log.push_back({w == S.lastW ? GACT_SINK : GACT_EMIT, w, s.ext_w0[w], s.ext_w1[w]});
                sim.extend(w, s.ext_w0[w], s.ext_w1[w]);
            }
        }
    }
    error = s.error != 0 || !s.done;
    return log;
}

}  // namespace

int main(int argc, char **argv) {
    const bool trace = argc >= 2 && std::string(argv[1]) == "trace";
    Synth S;
    int64_t seg = 0, qc = 0;
    if (trace) {
        if (argc < 6) {
            std::fprintf(stderr, "usage: %s trace k nnz seg_cap q_cap b_2 .. b_{k-1}\n", argv[0]);
            return 2;
        }
        S.k = std::atoi(argv[2]);
        S.lastW = S.k - 1;
        S.nnz = std::atoll(argv[3]);
        seg = std::atoll(argv[4]);
        qc = std::atoll(argv[5]);
        if (argc != 6 + (S.k - 2)) {
            std::fprintf(stderr, "trace: need k - 2 bounds\n");
            return 2;
        }
        S.use_fixed = true;
        for (int w = 2; w <= S.lastW; ++w) S.fixed[w] = std::atoll(argv[6 + (w - 2)]);
    } else {
        if (argc != 8) {
            std::fprintf(stderr, "usage: %s k nnz bmax emit_mod seed seg_cap q_cap\n", argv[0]);
            return 2;
        }
        S.k = std::atoi(argv[1]);
        S.lastW = S.k - 1;
        S.nnz = std::atoll(argv[2]);
        S.bmax = std::atoi(argv[3]);
        S.emit_mod = std::atoi(argv[4]);
        S.seed = std::strtoull(argv[5], nullptr, 10);
        seg = std::atoll(argv[6]);
        qc = std::atoll(argv[7]);
    }
    std::vector<int64_t> seg_cap(HUGE_KMAX + 1, seg), qcap(HUGE_KMAX + 1, qc);
    int64_t ground = 0;
    for (int64_t r = 0; r < S.nnz; ++r) ground += S.ground(2, (uint64_t)r);
    Sim a(S, seg, qcap), b(S, seg, qcap);
    const std::vector<Action> la = host_loop(a, seg_cap, qcap);
    bool err = false;
    const std::vector<Action> lb = device_steps(b, seg_cap, qcap, err);
    bool same = la.size() == lb.size();
    for (size_t i = 0; same && i < la.size(); ++i) same = !(la[i] != lb[i]);
    std::printf("host_actions %zu device_actions %zu same %d host_count %lld device_count %lld ground %lld "
                "overflow %d error %d\n",
                la.size(), lb.size(), same ? 1 : 0, (long long)a.count, (long long)b.count, (long long)ground,
                (a.overflow || b.overflow) ? 1 : 0, err ? 1 : 0);
    if (trace) {
        std::printf("trace");
        for (const Action &x : lb)
            std::printf(" %c:%d", x.kind == GACT_PREPARE ? 'P' : x.kind == GACT_EMIT ? 'E' : 'S', x.W);
        std::printf("\n");
    }
    return 0;
}
