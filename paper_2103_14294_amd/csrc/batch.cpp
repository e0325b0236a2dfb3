// Batched queries on the level engine: several queries in flight at once.
//
// Each query of a batch is an independent run of Algorithm 5 (Section 5.2);
// run one after another, a batch of many small queries is dominated by
// launch and synchronisation latency, and a large query's tail leaves the GPU
// idle.  Here a few host workers, each with its own HIP stream (default
// priority) and its own workspace sized for the largest query, take queries
// from a shared counter, so the queries' kernels overlap on the device.
// Results land in the caller's array by query index, so they do not depend on
// the interleaving.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <thread>
#include <vector>

#include "internal.h"

namespace huge {

namespace {
constexpr int kDefaultWorkers = 4;  // HIP's default number of hardware queues per process
}

void run_batch_levels(const huge_graph *g, const huge_plan *const *plans, int np, const huge_exec_opts &o,
                      huge_result *outs) {
    int nw = kDefaultWorkers;
    if (const char *e = getenv("HUGE_BATCH_STREAMS")) nw = std::max(1, std::min(16, atoi(e)));
    nw = std::min(nw, np);
    huge_exec_opts base = o;
    base.engine = HUGE_ENGINE_LEVELS;
    base.workspace = nullptr;
    base.workspace_bytes = 0;
    uint64_t ws_bytes = 256;
    for (int i = 0; i < np; ++i) ws_bytes = std::max(ws_bytes, workspace_bytes(g, plans[i], base));
    int dev = 0;
    HUGE_HIP(hipGetDevice(&dev));
    // work already queued on the caller's stream comes first
    HUGE_HIP(hipStreamSynchronize((hipStream_t)o.stream));
    std::atomic<int> next{0};
    std::atomic<bool> failed{false};
    std::vector<huge_status> st(nw, HUGE_OK);
    std::vector<std::string> msg(nw);
    auto worker = [&](int w) {
        hipStream_t s = nullptr;
        void *ws = nullptr;
        try {
            HUGE_HIP(hipSetDevice(dev));
            HUGE_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            HUGE_HIP(hipMalloc(&ws, ws_bytes));
            huge_exec_opts oo = base;
            oo.stream = s;
            oo.workspace = ws;
            oo.workspace_bytes = ws_bytes;
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
        if (ws) (void)hipFree(ws);
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
