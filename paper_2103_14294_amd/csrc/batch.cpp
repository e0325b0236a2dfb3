// Batched queries on the level engine: several queries in flight at once.
//
// Each query of a batch is an independent run of Algorithm 5 (Section 5.2);
// run one after another, a batch of many small queries is dominated by
// launch and synchronisation latency, and a large query's tail leaves the GPU
// idle.  Here a few host workers, each with its own HIP stream (default
// priority) and its own workspace sized for the largest query, take queries
// from a shared counter, so the queries' kernels overlap on the device.
// Results land in the caller's array by query index, so they do not depend on
// the interleaving.  The frontier budget is split evenly between the workers,
// and their workspaces stay allocated between calls (one grow-only pool per
// device, held until the process ends); batch calls on one device take turns.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace huge {

namespace {
constexpr int kDefaultWorkers = 4;  // HIP's default number of hardware queues per process
constexpr int kMaxWorkers = 16;
constexpr int kMaxDevices = 64;

struct Pool {
    std::mutex mu;
    void *buf[kMaxWorkers] = {};
    uint64_t bytes[kMaxWorkers] = {};
};
Pool g_pool[kMaxDevices];
}  // namespace

void run_batch_levels(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                      huge_result *outs) {
    int nw = kDefaultWorkers;
    if (const char *e = getenv("HUGE_BATCH_STREAMS")) nw = std::max(1, std::min(kMaxWorkers, atoi(e)));
    nw = std::min(nw, np);
    huge_exec_opts base = o;
    base.engine = HUGE_ENGINE_LEVELS;
    base.workspace = nullptr;
    base.workspace_bytes = 0;
    if (base.frontier_cap_bytes != UINT64_MAX) base.frontier_cap_bytes /= (uint64_t)nw;
    uint64_t ws_bytes = 256;
    for (int i = 0; i < np; ++i) ws_bytes = std::max(ws_bytes, workspace_bytes(g, plans[i], base));
    int dev = 0;
    HUGE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) HUGE_FAIL(HUGE_EDEVICE, "device %d out of range", dev);
    Pool &pool = g_pool[dev];
    std::lock_guard<std::mutex> lock(pool.mu);
    for (int w = 0; w < nw; ++w) {
        if (pool.bytes[w] >= ws_bytes) continue;
        if (pool.buf[w]) HUGE_HIP(hipFree(pool.buf[w]));
        pool.buf[w] = nullptr;
        pool.bytes[w] = 0;
        HUGE_HIP(hipMalloc(&pool.buf[w], ws_bytes));
        pool.bytes[w] = ws_bytes;
    }
    // work already queued on the caller's stream comes first
    HUGE_HIP(hipStreamSynchronize((hipStream_t)o.stream));
    std::atomic<int> next{0};
    std::atomic<bool> failed{false};
    std::vector<huge_status> st(nw, HUGE_OK);
    std::vector<std::string> msg(nw);
    auto worker = [&](int w) {
        hipStream_t s = nullptr;
        try {
            HUGE_HIP(hipSetDevice(dev));
            HUGE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            huge_exec_opts oo = base;
            oo.stream = s;
            oo.workspace = pool.buf[w];
            oo.workspace_bytes = pool.bytes[w];
            for (;;) {
                if (failed.load()) break;
                const int i = next.fetch_add(1);
                if (i >= np) break;
                run_levels(g, plans[i], oo, &outs[i], nullptr);
            }
        } catch (const Error &e) {
            st[w] = e.st;
            msg[w] = last_error_text();
            failed.store(true);
        } catch (...) {
            st[w] = HUGE_EDEVICE;
            msg[w] = "unexpected internal error in a batch worker";
            failed.store(true);
        }
        if (s) (void)hipStreamSynchronize(s);
        if (s) (void)hipStreamDestroy(s);
    };
    std::vector<std::thread> th;
    for (int w = 1; w < nw; ++w) th.emplace_back(worker, w);
    worker(0);
    for (auto &t : th) t.join();
    for (int w = 0; w < nw; ++w)
        if (st[w] != HUGE_OK) HUGE_FAIL(st[w], "%s", msg[w].c_str());
}

}  // namespace huge
