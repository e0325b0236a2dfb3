// Device memory for huge_count_noalloc: one file-scope array per device,
// reached through its device address, so that the entry point never calls an
// allocator.  The level engine carves its workspace (counters, segment
// buffers, queues, scan scratch, a gathered level 2) out of it and clears its
// counters at the start of every call.
#include <mutex>

#include "internal.h"

namespace huge {

namespace {

constexpr uint64_t kScratchBytes = 256ull << 20;
constexpr int kMaxDevices = 64;

// Each device that runs the library holds its own copy until the process ends.
// In host code this name stands for the array but is not its device address:
// host code uses the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    std::mutex mu;              // calls on one device take turns
    void *ptr = nullptr;        // this device's copy of `scratch`
    alignas(64) unsigned char host_stage[kHostStageBytes];  // the engine's read-backs land here
};
DeviceScratch g_scratch[kMaxDevices];

}  // namespace

uint64_t noalloc_scratch_bytes() { return kScratchBytes; }

void run_count_noalloc(const huge_graph *g, const huge_plan *p, const huge_exec_opts &opts, huge_result *out,
                       bool *limited) {
    int dev = 0;
    HUGE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) HUGE_FAIL(HUGE_EDEVICE, "device %d out of range", dev);
    if (dev != g->device) HUGE_FAIL(HUGE_EINVAL, "the graph lives on device %d, the current device is %d", g->device, dev);
    DeviceScratch &d = g_scratch[dev];
    std::lock_guard<std::mutex> lock(d.mu);
    if (!d.ptr) {  // once per device, with that device current
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            HUGE_FAIL(HUGE_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        d.ptr = ptr;
    }
    huge_exec_opts o = opts;
    o.engine = HUGE_ENGINE_LEVELS;
    const uint64_t need = workspace_bytes(g, p, o);
    if (need > kScratchBytes)
        HUGE_FAIL(HUGE_ENOMEM, "huge_count_noalloc: these options need %llu bytes of device memory, the array holds "
                               "%llu; lower frontier_cap_bytes or chunk_rows",
                  (unsigned long long)need, (unsigned long long)kScratchBytes);
    o.workspace = d.ptr;
    o.workspace_bytes = kScratchBytes;
    *limited = run_levels(g, p, o, out, nullptr, nullptr, d.host_stage);
}

}  // namespace huge
