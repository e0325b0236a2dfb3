// Features of an order prefix for the learned cost model, and order
// selection with it.
//
// The optimiser of Section 3.3 ranks candidate orders by estimates over their
// induced prefixes; the paper leaves the estimator pluggable.  The learned
// estimator reads, for prefix size s of order pi on graph G:
//   [0..5]    k one-hot (3..8)              [6..12]  s one-hot (2..8)
//   [13..40]  prefix adjacency, position pairs a < b < 8 (index b(b-1)/2 + a)
//   [41..68]  symmetry-breaking constraints between prefix positions, same
//             pair index: +1 when the earlier position's image is the smaller,
//             -1 when it is the larger
//   [69..75]  Ext mask of the last step (positions adjacent to position s-1)
//   [76..77]  constraints of the last step: "f[p] < v" count, "v < f[p]" count
//   [78..85]  degree of each prefix position inside the prefix, / 7
//   [86..117] the graph's log2 degree histogram, as fractions of n
//   [118..123] log(1 + M_p), M_p = sum_u d_u^p, p = 1..6
//   [124..125] log(1 + n), log(1 + 2m)
//   [126]     log(1 + the Chung-Lu estimate of the prefix)
//   [127]     prefix edges / 28
// and predicts log(1 + W_s), W_s the number of candidates the step that
// produces prefix s examines: the probe-list elements inside the symmetry-
// breaking window, summed over the partial matches of prefix s-1 (the
// engine's level_work).  Time is spent per candidate, so the learned cost of
// an order is sum over s = 3..k of W_s (producing prefix 2 scans the edge
// array whatever the order).  The plain cost model instead sums |R(prefix)|,
// which cannot tell apart orders whose prefixes have equal sizes (all orders
// of a clique) but whose steps search very different lists.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace huge {

namespace {
inline int pair_index(int a, int b) { return b * (b - 1) / 2 + a; }  // a < b
}  // namespace

void plan_features(const huge_graph_info &gi, const huge_plan &p, const int32_t *order, int size, float *out) {
    static_assert(HUGE_MLP_F == 128, "feature layout is for 128 inputs");
    memset(out, 0, sizeof(float) * HUGE_MLP_F);
    const int k = p.k;
    if (k >= 3 && k <= 8) out[k - 3] = 1.f;
    if (size >= 2 && size <= 8) out[6 + size - 2] = 1.f;
    int pos[HUGE_KMAX];
    for (int v = 0; v < k; ++v) pos[v] = HUGE_KMAX;
    for (int i = 0; i < k; ++i) pos[order[i]] = i;
    int nedge = 0;
    for (int b = 1; b < size; ++b)
        for (int a = 0; a < b; ++a)
            if (p.adj[order[a]][order[b]]) {
                out[13 + pair_index(a, b)] = 1.f;
                ++nedge;
            }
    int lo = 0, hi = 0;
    for (auto &c : p.sb) {
        const int pa = pos[c.first], pb = pos[c.second];  // rank f(first) < rank f(second)
        if (pa >= size || pb >= size) continue;
        const int a = std::min(pa, pb), b = std::max(pa, pb);
        out[41 + pair_index(a, b)] = pa < pb ? 1.f : -1.f;
        if (b == size - 1) {
            if (pb == size - 1) ++lo;  // earlier image < new vertex
            else ++hi;                 // new vertex < earlier image
        }
    }
    for (int a = 0; a + 1 < size; ++a)
        if (p.adj[order[a]][order[size - 1]]) out[69 + a] = 1.f;
    out[76] = (float)lo;
    out[77] = (float)hi;
    for (int a = 0; a < size; ++a) {
        int d = 0;
        for (int b = 0; b < size; ++b) d += p.adj[order[a]][order[b]];
        out[78 + a] = (float)d / 7.f;
    }
    const double n = gi.n > 0 ? (double)gi.n : 1.0;
    for (int b = 0; b < 32; ++b) out[86 + b] = (float)((double)gi.degree_hist[b] / n);
    for (int q = 1; q <= 6; ++q) out[118 + q - 1] = (float)std::log1p(std::max(0.0, gi.degree_moments[q]));
    out[124] = (float)std::log1p((double)std::max<int64_t>(0, gi.n));
    out[125] = (float)std::log1p((double)std::max<int64_t>(0, gi.nnz));
    out[126] = (float)std::log1p(std::max(0.0, estimate_prefix(gi, p, order, size)));
    out[127] = (float)nedge / 28.f;
}

// Learned estimates for every order, with one batched forward pass:
// est[o * k + s - 1] = estimated W_s for s = 3..k, 0 for s = 2, n for s = 1.
void learned_estimates(const huge_graph *g, const huge_model *m, const huge_plan &p,
                       const std::vector<std::vector<int32_t>> &orders, hipStream_t st, std::vector<double> &est) {
    const int k = p.k;
    const int64_t rows = (int64_t)orders.size() * std::max(0, k - 2);
    est.assign(orders.size() * (size_t)k, 0.0);
    for (size_t o = 0; o < orders.size(); ++o) est[o * k + 0] = (double)g->info.n;
    if (rows == 0) return;
    std::vector<float> x((size_t)rows * HUGE_MLP_F);
    int64_t r = 0;
    for (auto &o : orders)
        for (int s = 3; s <= k; ++s) plan_features(g->info, p, o.data(), s, &x[(size_t)(r++) * HUGE_MLP_F]);
    int dev = 0;
    HUGE_HIP(hipGetDevice(&dev));
    if (dev != m->device) HUGE_FAIL(HUGE_EINVAL, "the model lives on device %d, the current device is %d", m->device, dev);
    struct Mem {
        void *p = nullptr;
        ~Mem() {
            if (p) (void)hipFree(p);
        }
    } mem;
    const uint64_t xb = (4ull * rows * HUGE_MLP_F + 255) & ~255ull;
    HUGE_HIP(hipMalloc(&mem.p, xb + 4ull * rows));
    float *dx = (float *)mem.p, *dy = (float *)((char *)mem.p + xb);
    HUGE_HIP(hipMemcpyAsync(dx, x.data(), 4ull * rows * HUGE_MLP_F, hipMemcpyHostToDevice, st));
    model_forward(m, dx, rows, dy, st);
    std::vector<float> y((size_t)rows);
    HUGE_HIP(hipMemcpyAsync(y.data(), dy, 4ull * rows, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    r = 0;
    for (size_t o = 0; o < orders.size(); ++o)
        for (int s = 3; s <= k; ++s) est[o * k + s - 1] = std::max(0.0, std::expm1((double)y[(size_t)(r++)]));
}

}  // namespace huge
