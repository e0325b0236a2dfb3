// The C ABI (include/huge.h): argument checks, error capture, dispatch.
#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstring>

#include <vector>

#include "internal.h"

namespace huge {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

std::string last_error_text() { return g_last_error; }

template <typename F>
static huge_status guard(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        return e.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return HUGE_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return HUGE_EDEVICE;
    }
}

static huge_exec_opts resolve_opts(const huge_exec_opts *o) {
    huge_exec_opts r;
    huge_exec_opts_default(&r);
    if (o) r = *o;
    return r;
}

}  // namespace huge

using namespace huge;

extern "C" {

huge_status huge_exec_opts_default(huge_exec_opts *o) {
    if (!o) return HUGE_EINVAL;
    memset(o, 0, sizeof(*o));
    o->frontier_cap_bytes = 4ull << 30;
    o->chunk_rows = 0;
    o->strategy = -1;
    o->engine = HUGE_ENGINE_AUTO;
    o->work_stealing = 1;
    o->slice_count = 1;
    return HUGE_OK;
}

huge_status huge_load_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                          void *stream, huge_graph **out) {
    return guard([&] {
        if (!out) HUGE_FAIL(HUGE_EINVAL, "out is NULL");
        huge_graph *g = graph_load(n, nnz, row_ptr, col, flags, (hipStream_t)stream);
        *out = g;
        return HUGE_OK;
    });
}

huge_status huge_load_csr_labelled(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                                   const int32_t *labels, uint32_t flags, void *stream, huge_graph **out) {
    return guard([&] {
        if (!out) HUGE_FAIL(HUGE_EINVAL, "out is NULL");
        huge_graph *g = graph_load(n, nnz, row_ptr, col, flags, (hipStream_t)stream);
        try {
            graph_set_labels(g, labels, flags, (hipStream_t)stream);
        } catch (...) {
            graph_free(g);
            throw;
        }
        *out = g;
        return HUGE_OK;
    });
}

huge_status huge_load_csr_directed(int64_t n, int64_t narcs, const int64_t *row_ptr, const int32_t *col,
                                   uint32_t flags, void *stream, huge_graph **out) {
    return guard([&] {
        if (!out) HUGE_FAIL(HUGE_EINVAL, "out is NULL");
        *out = graph_load_directed(n, narcs, row_ptr, col, flags, (hipStream_t)stream);
        return HUGE_OK;
    });
}

huge_status huge_plan_create_directed(const huge_graph *g, int32_t k, int32_t n_arcs, const int32_t *arcs,
                                      const int32_t *qlabels, const int32_t *order, huge_plan **out) {
    return guard([&] {
        if (!out || !arcs) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (n_arcs < 1 || n_arcs > 56) HUGE_FAIL(HUGE_EQUERY, "bad number of directed edges (%d)", n_arcs);
        // the undirected skeleton: one edge per pair joined in either direction
        std::vector<int32_t> sk;
        for (int i = 0; i < n_arcs; ++i) {
            const int a = arcs[2 * i], b = arcs[2 * i + 1];
            bool seen = false;
            for (size_t j = 0; j < sk.size(); j += 2)
                seen |= (sk[j] == a && sk[j + 1] == b) || (sk[j] == b && sk[j + 1] == a);
            if (!seen) {
                sk.push_back(a);
                sk.push_back(b);
            }
        }
        huge_plan *p = new huge_plan();
        try {
            plan_build(g, k, (int)sk.size() / 2, sk.data(), order, 0, nullptr, nullptr, p, qlabels, n_arcs, arcs);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return HUGE_OK;
    });
}

huge_status huge_count_paths(const huge_graph *g, int32_t s, int32_t t, int32_t max_hops,
                             const huge_exec_opts *opts, uint64_t *counts) {
    return guard([&] {
        if (!g || !counts) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        const int64_t n = g->dev.n;
        if (s < 0 || t < 0 || s >= n || t >= n || s == t) HUGE_FAIL(HUGE_EINVAL, "s and t must be distinct vertices");
        if (max_hops < 1 || max_hops > HUGE_KMAX - 1) HUGE_FAIL(HUGE_EINVAL, "max_hops must be 1..%d", HUGE_KMAX - 1);
        huge_exec_opts o = resolve_opts(opts);
        if (o.slice_count > 1 || o.slice2_count > 1) HUGE_FAIL(HUGE_EINVAL, "huge_count_paths sets the slices itself");
        if (o.engine == HUGE_ENGINE_PERSISTENT) HUGE_FAIL(HUGE_EINVAL, "huge_count_paths runs on the level or graph engine");
        o.workspace = nullptr;  // each length sizes its own
        o.workspace_bytes = 0;
        // the ranks of s and t
        std::vector<int32_t> inv((size_t)n);
        HUGE_HIP(hipMemcpy(inv.data(), g->inv_rank, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
        int32_t rs = -1, rt = -1;
        for (int64_t r = 0; r < n; ++r) {
            if (inv[(size_t)r] == s) rs = (int32_t)r;
            if (inv[(size_t)r] == t) rt = (int32_t)r;
        }
        o.slice_count = (uint32_t)n;
        o.slice_id = (uint32_t)rs;
        o.slice_vertex = 0;
        o.slice_mode = HUGE_SLICE_STRIDE;
        o.slice2_count = (uint32_t)n;
        o.slice2_id = (uint32_t)rt;
        o.exec_flags &= ~(uint32_t)HUGE_EXEC_SLICE2_PAIR;
        counts[0] = 0;
        for (int L = 1; L <= max_hops; ++L) {
            int32_t qe[2 * (HUGE_KMAX - 1)], order[HUGE_KMAX];
            for (int i = 0; i < L; ++i) {
                qe[2 * i] = i;
                qe[2 * i + 1] = i + 1;
            }
            for (int i = 0; i <= L; ++i) order[i] = i;
            huge_plan p;
            plan_build(g, L + 1, L, qe, order, HUGE_PLAN_ALL_MAPS, nullptr, nullptr, &p);
            huge_exec_opts ol = o;
            ol.slice2_vertex = L;
            huge_result r;
            if (ol.engine == HUGE_ENGINE_GRAPH && L + 1 >= 3) {
                run_graph(g, &p, ol, &r);
            } else {
                ol.engine = HUGE_ENGINE_LEVELS;
                run_levels(g, &p, ol, &r, nullptr);
            }
            counts[L] = r.count;
        }
        return HUGE_OK;
    });
}

void huge_graph_free(huge_graph *g) { graph_free(g); }

huge_status huge_graph_get_info(const huge_graph *g, huge_graph_info *out) {
    return guard([&] {
        if (!g || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        *out = g->info;
        return HUGE_OK;
    });
}

huge_status huge_graph_export(const huge_graph *g, int64_t *row_ptr, int32_t *col, int32_t *inv_rank) {
    return guard([&] {
        if (!g) HUGE_FAIL(HUGE_EINVAL, "NULL graph");
        if (row_ptr) HUGE_HIP(hipMemcpy(row_ptr, g->rp, sizeof(int64_t) * (g->dev.n + 1), hipMemcpyDeviceToHost));
        if (col && g->dev.nnz)
            HUGE_HIP(hipMemcpy(col, g->col, sizeof(int32_t) * g->dev.nnz, hipMemcpyDeviceToHost));
        if (inv_rank) HUGE_HIP(hipMemcpy(inv_rank, g->inv_rank, sizeof(int32_t) * g->dev.n, hipMemcpyDeviceToHost));
        return HUGE_OK;
    });
}

huge_status huge_plan_create(const huge_graph *g, int32_t k, int32_t n_qedges, const int32_t *qedges,
                             const int32_t *order, uint32_t flags, huge_plan **out) {
    return guard([&] {
        if (!out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        huge_plan *p = new huge_plan();
        try {
            if (flags & HUGE_PLAN_LEARNED) HUGE_FAIL(HUGE_EINVAL, "a learned plan needs a model: use huge_plan_create_learned");
            if (flags & ~(uint32_t)(HUGE_PLAN_INDUCED | HUGE_PLAN_ALL_MAPS))
                HUGE_FAIL(HUGE_EINVAL, "unknown plan flags 0x%x", flags);
            plan_build(g, k, n_qedges, qedges, order, flags, nullptr, nullptr, p);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return HUGE_OK;
    });
}

huge_status huge_plan_create_labelled(const huge_graph *g, int32_t k, int32_t n_qedges, const int32_t *qedges,
                                      const int32_t *qlabels, const int32_t *order, uint32_t flags, huge_plan **out) {
    return guard([&] {
        if (!out || !qlabels) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (flags & ~(uint32_t)(HUGE_PLAN_INDUCED | HUGE_PLAN_ALL_MAPS))
            HUGE_FAIL(HUGE_EINVAL, "unknown plan flags 0x%x", flags);
        huge_plan *p = new huge_plan();
        try {
            plan_build(g, k, n_qedges, qedges, order, flags, nullptr, nullptr, p, qlabels);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return HUGE_OK;
    });
}

void huge_plan_free(huge_plan *p) { delete p; }

huge_status huge_plan_prefix(const huge_plan *p, int32_t size, huge_plan **out) {
    return guard([&] {
        if (!p || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (size < 2 || size > p->k) HUGE_FAIL(HUGE_EINVAL, "prefix size %d outside 2..%d", size, p->k);
        huge_plan *q = new huge_plan();
        plan_prefix(*p, size, q);
        *out = q;
        return HUGE_OK;
    });
}

huge_status huge_plan_info(const huge_plan *p, int32_t *k, int32_t *order_out, int32_t *n_sb, int32_t *sb_pairs,
                           double *est_cost) {
    return guard([&] {
        if (!p) HUGE_FAIL(HUGE_EINVAL, "NULL plan");
        if (k) *k = p->k;
        if (order_out)
            for (int i = 0; i < p->k; ++i) order_out[i] = p->order[i];
        if (n_sb) *n_sb = (int32_t)p->sb.size();
        if (sb_pairs)
            for (size_t i = 0; i < p->sb.size(); ++i) {
                sb_pairs[2 * i] = p->sb[i].first;
                sb_pairs[2 * i + 1] = p->sb[i].second;
            }
        if (est_cost) *est_cost = p->est_cost;
        return HUGE_OK;
    });
}

huge_status huge_plan_estimates(const huge_plan *p, double *est) {
    return guard([&] {
        if (!p || !est) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        for (int i = 0; i < HUGE_KMAX; ++i) est[i] = i < p->k ? p->est_prefix[i] : 0.0;
        return HUGE_OK;
    });
}

huge_status huge_workspace_size(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts,
                                uint64_t *bytes) {
    return guard([&] {
        if (!g || !p || !bytes) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        huge_exec_opts o = resolve_opts(opts);
        *bytes = workspace_bytes(g, p, o);
        return HUGE_OK;
    });
}

huge_status huge_segment_rows(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, int64_t *rows) {
    return guard([&] {
        if (!g || !p || !rows) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        huge_exec_opts o = resolve_opts(opts);
        segment_rows(g, p, o, rows);
        return HUGE_OK;
    });
}

huge_status huge_count(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, huge_result *out) {
    return guard([&] {
        if (!g || !p || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        huge_exec_opts o = resolve_opts(opts);
        if (o.work_limit < 0) HUGE_FAIL(HUGE_EINVAL, "work_limit < 0");
        check_labels(g, p);
        huge_result r;
        bool limited = false;
        if (!p->bushy.empty()) {
            run_bushy(g, p, o, &r, nullptr, 0);
        } else if (o.engine == HUGE_ENGINE_PERSISTENT) {
            const huge_plan *pl[1] = {p};
            run_persistent(g, pl, 1, o, &r);
        } else if (o.engine == HUGE_ENGINE_GRAPH) {
            run_graph(g, p, o, &r);
        } else {
            limited = run_levels(g, p, o, &r, nullptr);
        }
        *out = r;
        return limited ? HUGE_STOPPED : HUGE_OK;
    });
}

huge_status huge_count_bushy(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, huge_result *out,
                             int64_t *node_rows, int32_t max_nodes) {
    return guard([&] {
        if (!g || !p || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (max_nodes < 0 || (max_nodes > 0 && !node_rows)) HUGE_FAIL(HUGE_EINVAL, "bad node_rows");
        huge_exec_opts o = resolve_opts(opts);
        check_labels(g, p);
        huge_result r;
        run_bushy(g, p, o, &r, node_rows, max_nodes);
        *out = r;
        return HUGE_OK;
    });
}

huge_status huge_plan_create_bushy(const huge_graph *g, const huge_graph_info *stats, int32_t k, int32_t n_qedges,
                                   const int32_t *qedges, const int32_t *qlabels, double machines, huge_plan **out) {
    return guard([&] {
        if (!out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (!g && !stats) HUGE_FAIL(HUGE_EINVAL, "a bushy plan needs a graph or its statistics");
        huge_plan *p = new huge_plan();
        try {
            plan_build(g, k, n_qedges, qedges, nullptr, 0, nullptr, nullptr, p, qlabels);
            plan_bushy(stats ? *stats : g->info, *p, machines);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return HUGE_OK;
    });
}

huge_status huge_plan_create_bushy_tree(const huge_graph *g, const huge_graph_info *stats, int32_t k,
                                        int32_t n_qedges, const int32_t *qedges, const int32_t *qlabels,
                                        const uint32_t *joins, int32_t n_joins, double machines, huge_plan **out) {
    return guard([&] {
        if (!out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (!g && !stats) HUGE_FAIL(HUGE_EINVAL, "a bushy plan needs a graph or its statistics");
        if (n_joins < 0 || (n_joins > 0 && !joins)) HUGE_FAIL(HUGE_EINVAL, "bad joins");
        huge_plan *p = new huge_plan();
        try {
            plan_build(g, k, n_qedges, qedges, nullptr, 0, nullptr, nullptr, p, qlabels);
            plan_bushy_tree(stats ? *stats : g->info, *p, joins, n_joins, machines);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return HUGE_OK;
    });
}

huge_status huge_plan_bushy_nodes(const huge_plan *p, huge_bushy_node *nodes, int32_t max_nodes, int32_t *n_nodes) {
    return guard([&] {
        if (!p || !n_nodes) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (p->bushy.empty()) HUGE_FAIL(HUGE_EINVAL, "not a bushy plan");
        *n_nodes = (int32_t)p->bushy.size();
        if (nodes)
            for (int i = 0; i < max_nodes && i < (int)p->bushy.size(); ++i) nodes[i] = p->bushy[(size_t)i];
        return HUGE_OK;
    });
}

huge_status huge_count_noalloc(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, huge_result *out) {
    return guard([&] {
        if (!g || !p || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        huge_exec_opts o = resolve_opts(opts);
        if (o.workspace || o.workspace_bytes) HUGE_FAIL(HUGE_EINVAL, "huge_count_noalloc takes no workspace");
        if (o.profile) HUGE_FAIL(HUGE_EINVAL, "huge_count_noalloc does not profile (events would be created)");
        if (o.engine != HUGE_ENGINE_AUTO && o.engine != HUGE_ENGINE_LEVELS)
            HUGE_FAIL(HUGE_EINVAL, "huge_count_noalloc runs on the level engine");
        if (o.work_limit < 0) HUGE_FAIL(HUGE_EINVAL, "work_limit < 0");
        if (o.frontier_cap_bytes == UINT64_MAX) HUGE_FAIL(HUGE_EINVAL, "huge_count_noalloc needs a finite frontier cap");
        check_labels(g, p);
        huge_result r;
        bool limited = false;
        run_count_noalloc(g, p, o, &r, &limited);
        *out = r;
        return limited ? HUGE_STOPPED : HUGE_OK;
    });
}

huge_status huge_noalloc_capacity(uint64_t *bytes) {
    return guard([&] {
        if (!bytes) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        *bytes = noalloc_scratch_bytes();
        return HUGE_OK;
    });
}

huge_status huge_enumerate(const huge_graph *g, const huge_plan *p, const huge_exec_opts *opts, int32_t *host_buf,
                           int64_t buf_rows, huge_emit_fn cb, void *user, huge_result *out) {
    return guard([&] {
        if (!g || !p || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        huge_exec_opts o = resolve_opts(opts);
        if (o.engine == HUGE_ENGINE_GRAPH) HUGE_FAIL(HUGE_EINVAL, "huge_enumerate does not run on the graph engine");
        check_labels(g, p);
        EmitSink sink;
        sink.host_buf = host_buf;
        sink.buf_rows = buf_rows;
        sink.cb = cb;
        sink.user = user;
        huge_result r;
        run_levels(g, p, o, &r, &sink);
        *out = r;
        return sink.stopped ? HUGE_STOPPED : HUGE_OK;
    });
}

huge_status huge_count_batch(const huge_graph *g, const huge_plan *const *plans, int32_t np,
                             const huge_exec_opts *opts, huge_result *outs) {
    return guard([&] {
        if (!g || !plans || np <= 0 || !outs) HUGE_FAIL(HUGE_EINVAL, "bad arguments");
        for (int i = 0; i < np; ++i) {
            if (!plans[i]) HUGE_FAIL(HUGE_EINVAL, "plan %d is NULL", i);
            check_labels(g, plans[i]);
        }
        huge_exec_opts o = resolve_opts(opts);
        std::vector<huge_result> r(np);
        if (o.engine == HUGE_ENGINE_GRAPH) {  // batched rounds, kMaxBatch queries at a time
            for (int i = 0; i < np; i += kMaxBatch)
                run_mgraph(g, plans + i, std::min(kMaxBatch, np - i), o, r.data() + i);
            for (int i = 0; i < np; ++i) outs[i] = r[i];
            return HUGE_OK;
        }
        if (o.engine != HUGE_ENGINE_PERSISTENT) {
            run_batch_levels(g, plans, np, o, r.data());
            for (int i = 0; i < np; ++i) outs[i] = r[i];
            return HUGE_OK;
        }
        // queries the persistent kernel is built for share one launch; the
        // others run on the level engine, one after another, on the same stream
        std::vector<const huge_plan *> pers;
        std::vector<int> idx;
        for (int i = 0; i < np; ++i) {
            if (plans[i]->k >= 3 && plans[i]->k <= HUGE_PERSIST_KMAX) {
                pers.push_back(plans[i]);
                idx.push_back(i);
            }
        }
        if (!pers.empty()) {
            std::vector<huge_result> rp(pers.size());
            run_persistent(g, pers.data(), (int)pers.size(), o, rp.data());
            for (size_t j = 0; j < pers.size(); ++j) r[idx[j]] = rp[j];
        }
        huge_exec_opts lo = o;
        lo.engine = HUGE_ENGINE_LEVELS;
        for (int i = 0; i < np; ++i)
            if (!(plans[i]->k >= 3 && plans[i]->k <= HUGE_PERSIST_KMAX)) run_levels(g, plans[i], lo, &r[i], nullptr);
        for (int i = 0; i < np; ++i) outs[i] = r[i];
        return HUGE_OK;
    });
}

huge_status huge_batch_workspace_size(const huge_graph *g, const huge_plan *const *plans, int32_t np,
                                      const huge_exec_opts *opts, uint64_t *bytes) {
    return guard([&] {
        if (!g || !plans || np <= 0 || !bytes) HUGE_FAIL(HUGE_EINVAL, "bad arguments");
        for (int i = 0; i < np; ++i)
            if (!plans[i]) HUGE_FAIL(HUGE_EINVAL, "plan %d is NULL", i);
        huge_exec_opts o = resolve_opts(opts);
        if (o.engine != HUGE_ENGINE_GRAPH) HUGE_FAIL(HUGE_EINVAL, "a batch workspace is for HUGE_ENGINE_GRAPH");
        uint64_t b = 0;
        for (int i = 0; i < np; i += kMaxBatch)
            b = std::max(b, mgraph_workspace_bytes(g, plans + i, std::min(kMaxBatch, np - i), o));
        *bytes = b;
        return HUGE_OK;
    });
}

huge_status huge_motif_count(const huge_graph *g, int32_t k, const huge_exec_opts *opts, huge_motif *out,
                             int32_t *n_out) {
    return guard([&] {
        if (!g || !out || !n_out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        huge_exec_opts o = resolve_opts(opts);
        std::vector<huge_motif> r(HUGE_MOTIF_MAX);
        const int n = motif_count(g, k, o, r.data());
        for (int i = 0; i < n; ++i) out[i] = r[i];
        *n_out = n;
        return HUGE_OK;
    });
}

huge_status huge_model_create(huge_model **out) {
    return guard([&] {
        if (!out) HUGE_FAIL(HUGE_EINVAL, "out is NULL");
        *out = model_create();
        return HUGE_OK;
    });
}

void huge_model_free(huge_model *m) { model_free(m); }

huge_status huge_model_set(huge_model *m, const float *params, const float *xmean, const float *xinv, float tmean,
                           float tstd) {
    return guard([&] {
        if (!m) HUGE_FAIL(HUGE_EINVAL, "NULL model");
        model_set(m, params, xmean, xinv, tmean, tstd);
        return HUGE_OK;
    });
}

huge_status huge_model_get(const huge_model *m, float *params, float *xmean, float *xinv, float *tmean, float *tstd) {
    return guard([&] {
        if (!m) HUGE_FAIL(HUGE_EINVAL, "NULL model");
        model_get(m, params, xmean, xinv, tmean, tstd);
        return HUGE_OK;
    });
}

huge_status huge_model_forward(const huge_model *m, const float *x, int64_t B, float *y, void *stream) {
    return guard([&] {
        if (!m || B < 0 || (B > 0 && (!x || !y))) HUGE_FAIL(HUGE_EINVAL, "bad arguments");
        model_forward(m, x, B, y, (hipStream_t)stream);
        return HUGE_OK;
    });
}

huge_status huge_model_grad(const huge_model *m, const float *x, const float *t, int64_t B, float *grad, double *loss,
                            void *stream) {
    return guard([&] {
        if (!m || !x || !t || B <= 0) HUGE_FAIL(HUGE_EINVAL, "bad arguments");
        model_grad(m, x, t, B, grad, loss, (hipStream_t)stream);
        return HUGE_OK;
    });
}

huge_status huge_model_train(huge_model *m, const float *x, const float *t, int64_t n, int32_t epochs, int64_t batch,
                             float lr, uint64_t seed, float *loss_out, void *stream) {
    return guard([&] {
        if (!m || !x || !t || !(lr > 0.f)) HUGE_FAIL(HUGE_EINVAL, "bad arguments");
        model_train(m, x, t, n, epochs, batch, lr, seed, loss_out, (hipStream_t)stream);
        return HUGE_OK;
    });
}

huge_status huge_plan_features(const huge_graph *g, const huge_plan *p, const int32_t *order, int32_t size,
                               float *out) {
    return guard([&] {
        if (!g || !p || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (size < 2 || size > p->k) HUGE_FAIL(HUGE_EINVAL, "prefix size %d outside 2..%d", size, p->k);
        if (order && !order_connected(*p, order))
            HUGE_FAIL(HUGE_EORDER, "order is not a permutation of 0..k-1 with connected prefixes");
        plan_features(g->info, *p, order ? order : p->order, size, out);
        return HUGE_OK;
    });
}

huge_status huge_plan_create_learned(const huge_graph *g, const huge_model *m, int32_t k, int32_t n_qedges,
                                     const int32_t *qedges, const int32_t *order, void *stream, huge_plan **out) {
    return huge_plan_create_learned2(g, m, k, n_qedges, qedges, order, 0, stream, out);
}

huge_status huge_plan_create_learned2(const huge_graph *g, const huge_model *m, int32_t k, int32_t n_qedges,
                                      const int32_t *qedges, const int32_t *order, uint32_t flags, void *stream,
                                      huge_plan **out) {
    return guard([&] {
        if (!g || !m || !out) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        if (flags & ~(uint32_t)(HUGE_PLAN_VERIFY | HUGE_PLAN_INDUCED)) HUGE_FAIL(HUGE_EINVAL, "unknown flags 0x%x", flags);
        huge_plan *p = new huge_plan();
        try {
            plan_build(g, k, n_qedges, qedges, order, HUGE_PLAN_LEARNED | flags, m, (hipStream_t)stream, p);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return HUGE_OK;
    });
}

huge_status huge_autotune(const huge_graph *g, const huge_plan *const *plans, int32_t np, const huge_exec_opts *opts,
                          huge_tune_table *out) {
    return guard([&] {
        if (!g || !plans || np <= 0 || !out) HUGE_FAIL(HUGE_EINVAL, "bad arguments");
        for (int i = 0; i < np; ++i) {
            if (!plans[i]) HUGE_FAIL(HUGE_EINVAL, "plan %d is NULL", i);
            check_labels(g, plans[i]);
        }
        huge_exec_opts o = resolve_opts(opts);
        huge_tune_table t;
        autotune(g, plans, np, o, &t);
        *out = t;
        return HUGE_OK;
    });
}

huge_status huge_graph_digest(const huge_graph *g, char *out65) {
    return guard([&] {
        if (!g || !out65) HUGE_FAIL(HUGE_EINVAL, "NULL argument");
        const size_t n = std::min<size_t>(64, g->sha.size());
        memcpy(out65, g->sha.data(), n);
        out65[n] = 0;
        return HUGE_OK;
    });
}

huge_status huge_device_name(char *out, int32_t len) {
    return guard([&] {
        if (!out || len <= 0) HUGE_FAIL(HUGE_EINVAL, "bad buffer");
        int dev = 0;
        HUGE_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        HUGE_HIP(hipGetDeviceProperties(&prop, dev));
        snprintf(out, (size_t)len, "%s %dCU", prop.gcnArchName, prop.multiProcessorCount);
        return HUGE_OK;
    });
}

const char *huge_last_error(void) { return huge::g_last_error.c_str(); }

}  // extern "C"
