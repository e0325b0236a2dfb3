// Test harness (CPU): a model of the persistent engine's scheduling protocol
// (Section 5.2's Algorithm 5 per workgroup, Section 5.3's stealing), run by host
// threads that stand in for workgroups.  Each thread keeps the engine's
// per-level deques (head | tail | query in one word), the pending counts a thief
// holds while it copies rows out of a victim's level, a tile board (generation
// | tiles | next claim, and a done count) on which an owner publishes a large
// last-level chunk for idle threads to help with, and the busy count that ends
// the run.  Its steps follow the kernel's control flow; the intersections are
// replaced by a synthetic query tree (every row of level W has a seeded number
// of children), the last level counting them.
//
// Random yields between the shared operations vary the interleavings.  Every
// wait is bounded; a wait past its limit is reported with its site.  The run
// checks that it ends, that no wait timed out, and that the leaves counted
// equal a direct count of the tree (a row overwritten while still in use, or a
// row lost or taken twice, changes that count).
//
// usage: persist_harness k nwg edges bmax cap tile chunk steal seed yield_per_mille
// prints: count <n> ground <n> error <0|1> site <s> steals <n> helped <n>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <thread>
#include <vector>

namespace {

constexpr int kLv = 8;

uint64_t mixh(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

struct Tree {
    int k = 4;
    uint64_t seed = 1;
    int bmax = 4;
    // children of a row of level W (the row's id encodes its path)
    int64_t bound(int W, uint64_t id) const {
        return (int64_t)(mixh(id ^ (seed * 0x100000001B3ull) ^ ((uint64_t)W << 56)) % (uint64_t)(bmax + 1));
    }
    uint64_t child(uint64_t id, int64_t i) const { return mixh(id * 31 + (uint64_t)i + 7) | 1ull; }
    // leaves under a row of level W (the last level W = k - 1 counts its children)
    uint64_t leaves(int W, uint64_t id) const {
        const int64_t b = bound(W, id);
        if (W == k - 1) return (uint64_t)b;
        uint64_t s = 0;
        for (int64_t i = 0; i < b; ++i) s += leaves(W + 1, child(id, i));
        return s;
    }
};

// deque word: head | tail << 24 | plan << 48
uint32_t dq_head(uint64_t x) { return (uint32_t)(x & 0xFFFFFFull); }
uint32_t dq_tail(uint64_t x) { return (uint32_t)((x >> 24) & 0xFFFFFFull); }
uint64_t dq_make(uint32_t h, uint32_t t, int plan) {
    return (uint64_t)h | ((uint64_t)t << 24) | ((uint64_t)plan << 48);
}
// board word: next | tiles << 24 | gen << 48
uint32_t bw_next(uint64_t x) { return (uint32_t)(x & 0xFFFFFFull); }
uint32_t bw_tiles(uint64_t x) { return (uint32_t)((x >> 24) & 0xFFFFFFull); }

struct Board {
    std::atomic<uint64_t> word{0}, done{0};
    // the published chunk (plain data, written before the word is released)
    std::atomic<int> W{0};
    std::atomic<int64_t> row0{0}, nrows{0}, total{0};
    std::vector<std::atomic<int64_t>> off;
};

struct Shared {
    Tree tree;
    int nwg = 4, cap = 64, tile = 8, chunk = 8;
    bool steal = true;
    int64_t edges = 0;
    int yield_pm = 100;
    std::vector<std::atomic<uint64_t>> deq;      // [nwg][kLv]
    std::vector<std::atomic<int>> pending;       // [nwg][kLv]
    std::vector<std::atomic<uint64_t>> bufs;     // [nwg][kLv][cap] row ids
    std::vector<Board> boards;
    std::atomic<uint64_t> cursor{0};
    std::atomic<int> busy{0};
    std::atomic<uint64_t> leaves{0}, steals{0}, helped{0};
    std::atomic<int> error{0};
    std::atomic<int> site{0};
    std::chrono::steady_clock::time_point start;
    double limit_s = 20.0;
    std::atomic<uint64_t> &dq(int wg, int W) { return deq[(size_t)wg * kLv + W]; }
    std::atomic<int> &pend(int wg, int W) { return pending[(size_t)wg * kLv + W]; }
    std::atomic<uint64_t> &row(int wg, int W, int64_t r) { return bufs[((size_t)wg * kLv + W) * cap + (size_t)r]; }
    bool past() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - start).count() > limit_s;
    }
};

struct Chunk {
    int64_t row0 = 0, nrows = 0, total = 0, done = 0;
    std::vector<int64_t> off;  // nrows + 1 offsets of the rows' children
};

struct Wg {
    Shared &S;
    int id;
    std::mt19937_64 rng;
    Chunk lv[kLv];
    int W = 2;
    uint32_t gen = 0;
    bool counted = true;

    void maybe_yield() {
        if ((int)(rng() % 1000) < S.yield_pm) std::this_thread::yield();
    }
    void fail(int site) {
        S.error.store(1);
        S.site.store(site);
    }
    uint64_t row_id(int Wl, int64_t r) {
        if (Wl == 2) return mixh((uint64_t)r + 12345);  // level-2 rows are edges: ids from their index
        return S.row(id, Wl, r).load(std::memory_order_relaxed);
    }

    void prepare(int Wl) {
        Chunk &L = lv[Wl];
        L.off.assign((size_t)L.nrows + 1, 0);
        for (int64_t i = 0; i < L.nrows; ++i) {
            const uint64_t rid = row_id(Wl, L.row0 + i);
            L.off[(size_t)i + 1] = L.off[(size_t)i] + S.tree.bound(Wl, rid);
        }
        L.total = L.off[(size_t)L.nrows];
        L.done = 0;
    }

    // items [w0, w1) of a chunk of level Wl whose rows sit in workgroup `src`'s buffer
    uint64_t run_tile(int src, int Wl, int64_t row0, const std::vector<int64_t> &off, int64_t w0, int64_t w1,
                      int64_t out_base, int64_t &emitted) {
        uint64_t cnt = 0;
        int64_t r = 0;
        while (off[(size_t)r + 1] <= w0) ++r;
        for (int64_t w = w0; w < w1; ++w) {
            while (off[(size_t)r + 1] <= w) ++r;
            const uint64_t rid =
                Wl == 2 ? mixh((uint64_t)(row0 + r) + 12345) : S.row(src, Wl, row0 + r).load(std::memory_order_relaxed);
            if (Wl == S.tree.k - 1) {
                ++cnt;
            } else {
                const uint64_t c = S.tree.child(rid, w - off[(size_t)r]);
                S.row(id, Wl + 1, out_base + emitted).store(c, std::memory_order_relaxed);
                ++emitted;
            }
        }
        return cnt;
    }

    // owner side: publish rows appended at the tail
    void dq_push(int Wl, uint32_t add) {
        auto &d = S.dq(id, Wl);
        for (;;) {
            uint64_t o = d.load();
            maybe_yield();
            if (d.compare_exchange_strong(o, dq_make(dq_head(o), dq_tail(o) + add, (int)(o >> 48)))) return;
        }
    }
    int dq_pop(int Wl, int64_t &row0) {
        auto &d = S.dq(id, Wl);
        for (;;) {
            uint64_t o = d.load();
            const uint32_t h = dq_head(o), t = dq_tail(o);
            if (t <= h) return 0;
            const uint32_t c = std::min<uint32_t>(t - h, (uint32_t)S.chunk);
            maybe_yield();
            if (d.compare_exchange_strong(o, dq_make(h, t - c, (int)(o >> 48)))) {
                row0 = t - c;
                return (int)c;
            }
        }
    }
    uint32_t dq_prepare_append(int Wl) {
        auto &d = S.dq(id, Wl);
        for (;;) {
            uint64_t o = d.load();
            const uint32_t h = dq_head(o), t = dq_tail(o);
            if (h != t || t == 0) return t;
            const uint32_t pos = S.pend(id, Wl).load() == 0 ? 0u : t;
            maybe_yield();
            if (d.compare_exchange_strong(o, dq_make(pos, pos, 0))) return pos;
        }
    }

    // a tile of another workgroup's published chunk, claimed at next = tile
    void help(int v, uint32_t tile) {
        Board &b = S.boards[(size_t)v];
        const int Wl = b.W.load();
        const int64_t row0 = b.row0.load(), nrows = b.nrows.load(), total = b.total.load();
        std::vector<int64_t> off((size_t)nrows + 1);
        for (int64_t i = 0; i <= nrows; ++i) off[(size_t)i] = b.off[(size_t)i].load();
        const int64_t w0 = (int64_t)tile * S.tile, w1 = std::min<int64_t>(w0 + S.tile, total);
        int64_t e = 0;
        S.leaves += run_tile(v, Wl, row0, off, w0, w1, 0, e);
        maybe_yield();
        b.done.fetch_add(1);
        S.helped.fetch_add(1);
    }

    // the last level's chunk: alone when it is one tile, else published for helpers
    bool sink_chunk(int Wl) {
        Chunk &L = lv[Wl];
        const int64_t ntiles = (L.total + S.tile - 1) / S.tile;
        if (ntiles <= 1) {
            int64_t e = 0;
            S.leaves += run_tile(id, Wl, L.row0, L.off, 0, L.total, 0, e);
            return true;
        }
        Board &b = S.boards[(size_t)id];
        for (int64_t i = 0; i <= L.nrows; ++i) b.off[(size_t)i].store(L.off[(size_t)i]);
        b.W.store(Wl);
        b.row0.store(L.row0);
        b.nrows.store(L.nrows);
        b.total.store(L.total);
        b.done.store(0);
        gen = (gen + 1) & 0xFFFF;
        maybe_yield();
        b.word.store(dq_make(0, (uint32_t)ntiles, (int)gen));
        for (;;) {
            const uint64_t x = b.word.fetch_add(1);
            if (bw_next(x) >= bw_tiles(x)) break;
            const int64_t w0 = (int64_t)bw_next(x) * S.tile, w1 = std::min<int64_t>(w0 + S.tile, L.total);
            int64_t e = 0;
            S.leaves += run_tile(id, Wl, L.row0, L.off, w0, w1, 0, e);
            b.done.fetch_add(1);
            maybe_yield();
        }
        while (b.done.load() < (uint64_t)ntiles) {
            if (S.past()) {
                fail(1);  // the owner's wait for its helpers
                return false;
            }
            std::this_thread::yield();
        }
        return true;
    }

    void run() {
        const int k = S.tree.k;
        S.busy.fetch_add(1);
        for (;;) {
            // ---- a level-2 chunk from the cursor
            bool got = false;
            if (S.cursor.load() < (uint64_t)S.edges) {
                const uint64_t e0 = S.cursor.fetch_add((uint64_t)S.chunk);
                if (e0 < (uint64_t)S.edges) {
                    lv[2].row0 = (int64_t)e0;
                    lv[2].nrows = std::min<int64_t>(S.chunk, S.edges - (int64_t)e0);
                    got = true;
                }
            }
            if (got) {
                for (int q = 2; q < kLv; ++q) lv[q].total = lv[q].done = 0;
                W = 2;
                prepare(2);
            } else {
                if (counted) {
                    S.busy.fetch_sub(1);
                    counted = false;
                }
                int action = 0, victim = -1, vlevel = 0;
                uint32_t vhead = 0, vcount = 0, tile = 0;
                for (;;) {
                    action = 0;
                    for (int tries = 0; tries < 16 && !action && S.nwg > 1; ++tries) {
                        const int v = (int)(rng() % (uint64_t)S.nwg);
                        if (v == id) continue;
                        Board &b = S.boards[(size_t)v];
                        const uint64_t o = b.word.load();
                        if (bw_next(o) >= bw_tiles(o)) continue;
                        maybe_yield();
                        const uint64_t x = b.word.fetch_add(1);
                        if (bw_next(x) < bw_tiles(x)) {
                            action = 5;
                            victim = v;
                            tile = bw_next(x);
                        }
                    }
                    if (!action && S.steal) {
                        for (int tries = 0; tries < 8 && !action && S.nwg > 1; ++tries) {
                            const int v = (int)(rng() % (uint64_t)S.nwg);
                            if (v == id) continue;
                            for (int Wl = 3; Wl <= k - 1 && !action; ++Wl) {
                                auto &d = S.dq(v, Wl);
                                uint64_t o = d.load();
                                const uint32_t h = dq_head(o), t = dq_tail(o);
                                if (t < h + 2) continue;
                                S.busy.fetch_add(1);
                                S.pend(v, Wl).fetch_add(1);
                                const uint32_t kk = std::min<uint32_t>((t - h) / 2, (uint32_t)S.cap);
                                maybe_yield();
                                if (d.compare_exchange_strong(o, dq_make(h + kk, t, (int)(o >> 48)))) {
                                    action = 3;
                                    victim = v;
                                    vlevel = Wl;
                                    vhead = h;
                                    vcount = kk;
                                    counted = true;
                                } else {
                                    S.pend(v, Wl).fetch_sub(1);
                                    S.busy.fetch_sub(1);
                                }
                            }
                        }
                    }
                    if (!action) {
                        if (S.busy.load() == 0) {
                            action = 4;
                        } else if (S.past()) {
                            fail(2);  // an idle workgroup's wait for the end
                            action = 4;
                        } else {
                            std::this_thread::yield();
                        }
                    }
                    if (action == 0) continue;
                    if (action == 4) break;
                    if (action == 5) {
                        help(victim, tile);
                        continue;
                    }
                    break;  // action 3: stolen rows
                }
                if (action != 3) break;
                // ---- take the stolen rows into our own (empty) level
                const int Wl = vlevel;
                while (S.pend(id, Wl).load() != 0) {
                    if (S.past()) {
                        fail(3);  // a thief's wait for its own level's copiers
                        return;
                    }
                    std::this_thread::yield();
                }
                S.dq(id, Wl).store(dq_make(0, 0, 0));
                for (uint32_t i = 0; i < vcount; ++i) {
                    S.row(id, Wl, i).store(S.row(victim, Wl, (int64_t)vhead + i).load(std::memory_order_relaxed),
                                           std::memory_order_relaxed);
                    if (i % 4 == 0) maybe_yield();
                }
                S.pend(victim, Wl).fetch_sub(1);
                S.steals.fetch_add(1);
                for (int q = 2; q < kLv; ++q) lv[q].total = lv[q].done = 0;
                W = Wl;
                dq_push(Wl, vcount);
            }

            // ---- Algorithm 5 on this workgroup's levels
            for (;;) {
                Chunk &L = lv[W];
                if (L.done < L.total) {
                    if (W == k - 1) {
                        if (!sink_chunk(W)) return;
                        L.done = L.total;
                        continue;
                    }
                    const uint32_t base = dq_prepare_append(W + 1);
                    const bool room = (int64_t)S.cap - (int64_t)base >= S.tile;
                    if (room) {
                        const int64_t w0 = L.done, w1 = std::min<int64_t>(L.done + S.tile, L.total);
                        int64_t e = 0;
                        run_tile(id, W, L.row0, L.off, w0, w1, base, e);
                        L.done = w1;
                        if (e) dq_push(W + 1, (uint32_t)e);
                    }
                    const uint64_t o = S.dq(id, W + 1).load();
                    if (dq_tail(o) > dq_head(o)) {
                        W = W + 1;
                    } else if (!room) {
                        if (S.past()) {
                            fail(4);  // an owner's wait for thieves to leave a full, empty level
                            return;
                        }
                        std::this_thread::yield();
                    }
                    continue;
                }
                if (W == 2) {
                    bool more = false;
                    if (S.cursor.load() < (uint64_t)S.edges) {
                        const uint64_t e0 = S.cursor.fetch_add((uint64_t)S.chunk);
                        if (e0 < (uint64_t)S.edges) {
                            lv[2].row0 = (int64_t)e0;
                            lv[2].nrows = std::min<int64_t>(S.chunk, S.edges - (int64_t)e0);
                            more = true;
                        }
                    }
                    if (!more) break;
                    prepare(2);
                    continue;
                }
                int64_t row0 = 0;
                const int c = dq_pop(W, row0);
                if (c) {
                    L.row0 = row0;
                    L.nrows = c;
                    prepare(W);
                } else {
                    W = W - 1;
                }
            }
        }
        if (counted) S.busy.fetch_sub(1);
    }
};

}  // namespace

int main(int argc, char **argv) {
    if (argc != 11) {
        fprintf(stderr, "usage: persist_harness k nwg edges bmax cap tile chunk steal seed yield_per_mille\n");
        return 2;
    }
    Shared S;
    S.tree.k = atoi(argv[1]);
    S.nwg = atoi(argv[2]);
    S.edges = atoll(argv[3]);
    S.tree.bmax = atoi(argv[4]);
    S.cap = atoi(argv[5]);
    S.tile = atoi(argv[6]);
    S.chunk = atoi(argv[7]);
    S.steal = atoi(argv[8]) != 0;
    S.tree.seed = strtoull(argv[9], nullptr, 10);
    S.yield_pm = atoi(argv[10]);
    if (S.tree.k < 3 || S.tree.k > kLv - 1 || S.nwg < 1 || S.cap < 2 * S.tile || S.tile < 1 || S.chunk < 1 ||
        S.chunk > S.cap) {
        fprintf(stderr, "bad arguments\n");
        return 2;
    }
    S.deq = std::vector<std::atomic<uint64_t>>((size_t)S.nwg * kLv);
    S.pending = std::vector<std::atomic<int>>((size_t)S.nwg * kLv);
    S.bufs = std::vector<std::atomic<uint64_t>>((size_t)S.nwg * kLv * S.cap);
    S.boards = std::vector<Board>((size_t)S.nwg);
    for (auto &b : S.boards) b.off = std::vector<std::atomic<int64_t>>((size_t)S.chunk + 1);
    uint64_t ground = 0;
    for (int64_t e = 0; e < S.edges; ++e) ground += S.tree.leaves(2, mixh((uint64_t)e + 12345));
    S.start = std::chrono::steady_clock::now();
    std::vector<std::thread> th;
    std::vector<Wg *> wgs;
    for (int i = 0; i < S.nwg; ++i) {
        Wg *w = new Wg{S, i, std::mt19937_64(S.tree.seed * 1000003ull + (uint64_t)i)};
        wgs.push_back(w);
        th.emplace_back([w] { w->run(); });
    }
    for (auto &t : th) t.join();
    for (auto *w : wgs) delete w;
    printf("count %llu ground %llu error %d site %d steals %llu helped %llu\n", (unsigned long long)S.leaves.load(),
           (unsigned long long)ground, S.error.load(), S.site.load(), (unsigned long long)S.steals.load(),
           (unsigned long long)S.helped.load());
    return 0;
}
