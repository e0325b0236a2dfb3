// Running a bushy plan (Algorithm 1's join tree) on one GPU.
//
// The tree is evaluated bottom-up.  A pulled join (a complete star join, or a
// pulled hash join) extends its left part, so a run of pulled joins over one
// star unit is one chain of PULL-EXTEND steps from a SCAN (Section 5.1): it
// runs on the level engine as a left-deep plan of its own whose steps
// intersect only the lists their star names, while the edges a pulled hash
// join verifies (the verify-only EXTEND and its hint) are looked up, never
// probed, at the step that places the later of their ends -- a filter on the
// final rows, applied as early as it can be.  A PUSH-JOIN materialises both of
// its parts as device tables (a counting pass sizes each exactly) and joins
// them on their shared vertices (join.hip); pulled joins above a PUSH-JOIN
// extend its table step by step.  The root counts its rows with the set-hash
// of the query's edges instead of storing them.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.h"
#include "join.h"
#include "prims.h"

namespace huge {

namespace {

// device memory of one table or scratch array; `live` / `peak` (when given)
// track the bytes the run holds at once
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    uint64_t *live = nullptr;
    Buf(size_t b, uint64_t *live_ = nullptr, uint64_t *peak = nullptr) : bytes(std::max<size_t>(b, 256)), live(live_) {
        HUGE_HIP(hipMalloc(&p, bytes));
        if (live) {
            *live += bytes;
            *peak = std::max(*peak, *live);
        }
    }
    ~Buf() {
        if (p) (void)hipFree(p);
        if (live) *live -= bytes;
    }
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    template <typename T>
    T *as() const {
        return (T *)p;
    }
};

struct Table {
    std::shared_ptr<Buf> mem;
    const int32_t *rows = nullptr;
    int64_t n = 0;
    int w = 0;
    int8_t vert[HUGE_KMAX] = {};  // query vertex of each column
    int col_of(int v) const {
        for (int c = 0; c < w; ++c)
            if (vert[c] == v) return c;
        return -1;
    }
};

struct Exec {
    const huge_graph *g;
    const huge_plan *p;
    huge_exec_opts o;
    hipStream_t st;
    std::vector<int64_t> rows;  // per node: rows produced (-1 inside a chain)
    huge_result res{};
    uint64_t live = 0, peak = 0;
    std::unique_ptr<Buf> acc;   // 4 x u64 counters of the table operators

    std::shared_ptr<Buf> table_mem(size_t bytes) { return std::make_shared<Buf>(bytes, &live, &peak); }

    void read_acc(unsigned long long (&h)[4]) {
        HUGE_HIP(hipMemcpyAsync(h, acc->p, sizeof(h), hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
    }
    void clear_acc() { HUGE_HIP(hipMemsetAsync(acc->p, 0, 4 * sizeof(unsigned long long), st)); }
    int64_t read_i64(const int64_t *d) {
        int64_t v = 0;
        HUGE_HIP(hipMemcpyAsync(&v, d, 8, hipMemcpyDeviceToHost, st));
        HUGE_HIP(hipStreamSynchronize(st));
        return v;
    }

    const huge_bushy_node &node(int i) const { return p->bushy[(size_t)i]; }

    // the query's edges / constraints restricted to a vertex -> column map
    void edges_as_cols(const int8_t *colv, int w, int32_t &ne, int8_t *ea, int8_t *eb) const {
        auto col = [&](int v) {
            for (int c = 0; c < w; ++c)
                if (colv[c] == v) return c;
            return -1;
        };
        ne = 0;
        for (auto &e : p->edges) {
            const int a = col(e.first), b = col(e.second);
            if (a >= 0 && b >= 0) {
                ea[ne] = (int8_t)a;
                eb[ne] = (int8_t)b;
                ++ne;
            }
        }
    }

    bool sliced(int v) const { return o.slice_count > 1 && o.slice_vertex == v; }

    // ---- a chain of pulled joins over a star unit: the level engine ----
    // steps: the pulled join nodes above the unit, bottom-up
    Table run_scan_chain(int unit, const std::vector<int> &steps, bool root) {
        const huge_bushy_node &u = node(unit);
        std::vector<int> order;             // query vertices in placement order
        std::vector<uint32_t> ext;          // per position: positions whose lists are intersected
        int pos[HUGE_KMAX];
        for (int v = 0; v < HUGE_KMAX; ++v) pos[v] = -1;
        auto place = [&](int v, uint32_t e) {
            pos[v] = (int)order.size();
            order.push_back(v);
            ext.push_back(e);
        };
        const int c0 = u.star_root >= 0 ? u.star_root : __builtin_ctz(u.vertex_mask);
        place(c0, 0);
        for (int v = 0; v < p->k; ++v)
            if (v != c0 && ((u.vertex_mask >> v) & 1u)) place(v, 1u << pos[c0]);
        uint32_t chain_edges = u.edge_mask;
        for (int s : steps) {
            const huge_bushy_node &j = node(s);
            const huge_bushy_node &r = node(j.right);
            const int c = j.star_root;
            chain_edges |= r.edge_mask;
            const uint32_t leaves = r.vertex_mask & ~(1u << c);
            if (j.kind == HUGE_BUSHY_EXTEND) {
                uint32_t e = 0;
                for (int v = 0; v < p->k; ++v)
                    if ((leaves >> v) & 1u) e |= 1u << pos[v];
                place(c, e);
            } else {  // pulled hash join: the leaves not yet placed grow from c
                for (int v = 0; v < p->k; ++v)
                    if (((leaves >> v) & 1u) && pos[v] < 0) place(v, 1u << pos[c]);
            }
        }
        // the chain as a plan of its own: local vertex i = position i
        const int kk = (int)order.size();
        huge_plan cp;
        cp.k = kk;
        for (size_t e = 0; e < p->edges.size(); ++e)
            if ((chain_edges >> e) & 1u) {
                const int a = pos[p->edges[e].first], b = pos[p->edges[e].second];
                cp.edges.push_back({std::min(a, b), std::max(a, b)});
                cp.adj[a][b] = cp.adj[b][a] = 1;
            }
        for (auto &c : p->sb)
            if (pos[c.first] >= 0 && pos[c.second] >= 0) cp.sb.push_back({pos[c.first], pos[c.second]});
        for (int i = 0; i < kk; ++i) cp.qlabel[i] = p->qlabel[order[(size_t)i]];
        cp.labelled = p->labelled;
        std::vector<int32_t> ident(kk);
        for (int i = 0; i < kk; ++i) ident[i] = i;
        plan_set_order(cp, ident.data());
        for (int i = 1; i < kk; ++i) {
            DevStep &s = cp.dev.st[i];
            uint32_t adj = 0;
            for (int j = 0; j < i; ++j)
                if (cp.adj[j][i]) adj |= 1u << j;
            s.ext = ext[(size_t)i];
            s.vadj = adj & ~s.ext;  // verified edges: looked up at the later end's step
            s.neq = ((1u << i) - 1) & ~s.ext;
        }
        huge_exec_opts oc = o;
        oc.workspace = nullptr;
        oc.workspace_bytes = 0;
        oc.profile = 0;
        oc.slice_vertex = 0;
        if (o.slice_count > 1 && o.slice_vertex >= 0 && pos[o.slice_vertex] >= 0) {
            oc.slice_vertex = pos[o.slice_vertex];
        } else {
            oc.slice_count = 0;
            oc.slice_id = 0;
        }
        Table t;
        t.w = kk;
        for (int i = 0; i < kk; ++i) t.vert[i] = (int8_t)order[(size_t)i];
        huge_result r;
        if (root) {
            run_levels(g, &cp, oc, &r, nullptr);
            res.count = r.count;
            res.hash_sum = r.hash_sum;
            res.hash_xor = r.hash_xor;
            peak = std::max(peak, live + r.peak_frontier_bytes);  // the engine's frontier beside the tables
            t.n = (int64_t)r.count;
            return t;
        }
        oc.exec_flags |= HUGE_EXEC_NO_HASH;
        run_levels(g, &cp, oc, &r, nullptr);
        const int64_t n = (int64_t)r.count;
        const int64_t stage = 1 << 20;
        t.mem = table_mem((size_t)(n + stage) * kk * sizeof(int32_t));
        EmitSink e;
        e.dev_out = t.mem->as<int32_t>();
        e.dev_cap = n + stage;
        e.buf_rows = stage;
        run_levels(g, &cp, oc, &r, &e);
        if ((int64_t)e.delivered != n) HUGE_FAIL(HUGE_EDEVICE, "chain materialised %llu rows, counted %lld",
                                                 (unsigned long long)e.delivered, (long long)n);
        t.rows = t.mem->as<int32_t>();
        t.n = n;
        return t;
    }

    // ---- one step over a table ----
    Table tab_step(const Table &in, const TabStep &S, bool root, int add_vertex) {
        const int64_t n = in.n;
        Table out;
        out.w = in.w + (S.add ? 1 : 0);
        memcpy(out.vert, in.vert, sizeof(out.vert));
        if (S.add) out.vert[in.w] = (int8_t)add_vertex;
        Buf bound((size_t)std::max<int64_t>(1, n) * 4), pinfo((size_t)std::max<int64_t>(1, n) * 8),
            off((size_t)(std::max<int64_t>(1, n) + 1) * 8), tmp((size_t)scan_tmp_elems(std::max<int64_t>(1, n)) * 8);
        launch_tab_prepare(in.rows, n, S, g->dev, bound.as<uint32_t>(), pinfo.as<uint64_t>(), st);
        int64_t items = 0;
        if (n > 0) {
            scan_excl(bound.as<uint32_t>(), off.as<int64_t>(), n, off.as<int64_t>() + n, tmp.as<int64_t>(), st);
            items = read_i64(off.as<int64_t>() + n);
        }
        return sink(out, root, items, [&](int mode, int32_t *dst, int64_t cap) {
            launch_tab_items(in.rows, n, off.as<int64_t>(), pinfo.as<uint64_t>(), items, S, g->dev, mode, dst, cap,
                             acc->as<unsigned long long>(), st);
        });
    }

    // the item pass: root count, or count then write into an exact table
    template <typename F>
    Table sink(Table out, bool root, int64_t items, F &&run) {
        unsigned long long h[4];
        clear_acc();
        if (root) {
            run(TAB_ROOT, nullptr, 0);
            read_acc(h);
            if (h[3]) HUGE_FAIL(HUGE_EDEVICE, "table operator overflow (flags %llu)", h[3]);
            res.count = h[0];
            res.hash_sum = h[1];
            res.hash_xor = h[2];
            out.n = (int64_t)h[0];
            return out;
        }
        run(TAB_COUNT, nullptr, 0);
        read_acc(h);
        if (h[3]) HUGE_FAIL(HUGE_EDEVICE, "table operator overflow (flags %llu)", h[3]);
        const int64_t n = (int64_t)h[0];
        out.mem = table_mem((size_t)std::max<int64_t>(1, n) * out.w * sizeof(int32_t));
        clear_acc();
        run(TAB_WRITE, out.mem->as<int32_t>(), n);
        read_acc(h);
        if (h[3] || (int64_t)h[0] != n) HUGE_FAIL(HUGE_EDEVICE, "table operator wrote %llu rows, counted %lld",
                                                  h[0], (long long)n);
        out.rows = out.mem->as<int32_t>();
        out.n = n;
        (void)items;
        return out;
    }

    // the constraints of q between a new vertex c and the table's vertices
    void window(const Table &t, int c, TabStep &S) const {
        for (auto &x : p->sb) {
            if (x.second == c) {
                const int a = t.col_of(x.first);
                if (a >= 0) S.lo |= 1u << a;  // f(first) < f(c)
            }
            if (x.first == c) {
                const int b = t.col_of(x.second);
                if (b >= 0) S.hi |= 1u << b;
            }
        }
    }

    TabStep add_step(const Table &t, int c, uint32_t ext_cols) const {
        TabStep S;
        S.w = t.w;
        S.add = 1;
        S.ext = ext_cols;
        window(t, c, S);
        if (sliced(c)) {
            S.slice = 1;
            S.slice_count = o.slice_count;
            S.slice_id = o.slice_id;
            S.slice_mode = (int32_t)o.slice_mode;
        }
        S.label = p->qlabel[c];
        return S;
    }

    // ---- pulled joins over a table ----
    Table run_table_chain(Table t, const std::vector<int> &steps, bool root) {
        for (size_t si = 0; si < steps.size(); ++si) {
            const huge_bushy_node &j = node(steps[si]);
            const int c = j.star_root;
            const uint32_t leaves = node(j.right).vertex_mask & ~(1u << c);
            const bool last_node = si + 1 == steps.size();
            // one operation over the current table; the root's last one counts
            auto op = [&](TabStep S, int add_vertex, bool last_op) {
                const bool is_root = root && last_node && last_op;
                if (is_root) {
                    Table shape = t;
                    if (S.add) shape.vert[shape.w++] = (int8_t)add_vertex;
                    edges_as_cols(shape.vert, shape.w, S.ne, S.ea, S.eb);
                }
                t = tab_step(t, S, is_root, add_vertex);
            };
            if (j.kind == HUGE_BUSHY_EXTEND) {
                uint32_t e = 0;
                for (int v = 0; v < p->k; ++v)
                    if ((leaves >> v) & 1u) e |= 1u << t.col_of(v);
                op(add_step(t, c, e), c, true);
            } else {
                // the verify-only EXTEND: edges from c to the leaves already in the table
                const int cc = t.col_of(c);
                TabStep ver;
                ver.w = t.w;
                std::vector<int> grow;
                for (int v = 0; v < p->k; ++v) {
                    if (!((leaves >> v) & 1u)) continue;
                    if (t.col_of(v) >= 0) {
                        ver.va[ver.nver] = (int8_t)cc;
                        ver.vb[ver.nver] = (int8_t)t.col_of(v);
                        ++ver.nver;
                    } else {
                        grow.push_back(v);
                    }
                }
                if (grow.empty()) op(ver, -1, true);
                for (size_t q = 0; q < grow.size(); ++q) {
                    TabStep S = add_step(t, grow[q], 1u << t.col_of(c));
                    if (q == 0) {  // the verify pairs filter the rows before the first leaf grows
                        S.nver = ver.nver;
                        memcpy(S.va, ver.va, sizeof(S.va));
                        memcpy(S.vb, ver.vb, sizeof(S.vb));
                    }
                    op(S, grow[q], q + 1 == grow.size());
                }
            }
            rows[(size_t)steps[si]] = t.n;
        }
        return t;
    }

    // ---- PUSH-JOIN ----
    Table push_join(Table L, Table R, bool root) {
        JoinSpec J;
        J.wl = L.w;
        J.wr = R.w;
        for (int c = 0; c < R.w; ++c) {
            const int lc = L.col_of(R.vert[c]);
            if (lc >= 0) {
                J.kl[J.nkey] = (int8_t)lc;
                J.kr[J.nkey] = (int8_t)c;
                ++J.nkey;
            } else {
                J.ro[J.nro++] = (int8_t)c;
            }
        }
        Table out;
        out.w = L.w + J.nro;
        memcpy(out.vert, L.vert, sizeof(out.vert));
        for (int i = 0; i < J.nro; ++i) out.vert[L.w + i] = R.vert[J.ro[i]];
        for (auto &x : p->sb) {
            const int a = out.col_of(x.first), b = out.col_of(x.second);
            if (a >= 0 && b >= 0) {
                J.sa[J.nsb] = (int8_t)a;
                J.sb[J.nsb] = (int8_t)b;
                ++J.nsb;
            }
        }
        if (root) edges_as_cols(out.vert, out.w, J.ne, J.ea, J.eb);
        if (R.n >= (int64_t)0xFFFFFFFFll) HUGE_FAIL(HUGE_ENOMEM, "PUSH-JOIN: the right part has 2^32 rows or more");
        const int64_t nr = R.n, nl = L.n;
        const int64_t nr1 = std::max<int64_t>(1, nr), nl1 = std::max<int64_t>(1, nl);
        Buf k0((size_t)nr1 * 4), v0((size_t)nr1 * 4), k1((size_t)nr1 * 4), v1((size_t)nr1 * 4);
        Buf hist((size_t)radix_sort_hist_elems(nr1) * 4), offs((size_t)radix_sort_hist_elems(nr1) * 8),
            stmp((size_t)scan_tmp_elems(std::max<int64_t>(radix_sort_hist_elems(nr1), nl1)) * 8);
        const uint32_t *skeys = k0.as<uint32_t>(), *svals = v0.as<uint32_t>();
        if (nr > 0) {
            launch_join_keys(R.rows, nr, J, k0.as<uint32_t>(), v0.as<uint32_t>(), st);
            const bool in1 = radix_sort_pairs(k0.as<uint32_t>(), v0.as<uint32_t>(), k1.as<uint32_t>(),
                                              v1.as<uint32_t>(), nr, 32, hist.as<uint32_t>(), offs.as<int64_t>(),
                                              stmp.as<int64_t>(), st);
            if (in1) {
                skeys = k1.as<uint32_t>();
                svals = v1.as<uint32_t>();
            }
        }
        // R's rows in key order, so that every left row meets a run of adjacent rows
        Buf rs((size_t)nr1 * std::max(1, R.w) * 4, &live, &peak);
        launch_gather_rows(R.rows, nr, R.w, svals, rs.as<int32_t>(), st);
        Buf bound((size_t)nl1 * 4), first((size_t)nl1 * 8), off((size_t)(nl1 + 1) * 8);
        clear_acc();
        int64_t items = 0;
        if (nl > 0 && nr > 0) {
            launch_join_prepare(L.rows, nl, J, skeys, nr, bound.as<uint32_t>(), first.as<int64_t>(),
                                acc->as<unsigned long long>(), st);
            unsigned long long h[4];
            read_acc(h);
            if (h[3]) HUGE_FAIL(HUGE_ENOMEM, "PUSH-JOIN: a key holds 2^32 right rows or more");
            scan_excl(bound.as<uint32_t>(), off.as<int64_t>(), nl, off.as<int64_t>() + nl, stmp.as<int64_t>(), st);
            items = read_i64(off.as<int64_t>() + nl);
        }
        return sink(out, root, items, [&](int mode, int32_t *dst, int64_t cap) {
            launch_join_items(L.rows, nl, rs.as<int32_t>(), off.as<int64_t>(), first.as<int64_t>(), items, J, mode,
                              dst, cap, acc->as<unsigned long long>(), st);
        });
    }

    Table eval(int id, bool root) {
        const huge_bushy_node &nd = node(id);
        if (nd.kind == HUGE_BUSHY_PUSH) {
            Table L = eval(nd.left, false);
            Table R = eval(nd.right, false);
            Table t = push_join(L, R, root);
            rows[(size_t)id] = t.n;
            return t;
        }
        std::vector<int> steps;
        int cur = id;
        while (node(cur).kind == HUGE_BUSHY_EXTEND || node(cur).kind == HUGE_BUSHY_PULL_HASH) {
            steps.insert(steps.begin(), cur);
            cur = node(cur).left;
        }
        if (node(cur).kind == HUGE_BUSHY_UNIT) {
            Table t = run_scan_chain(cur, steps, root);
            rows[(size_t)id] = t.n;
            return t;
        }
        Table base = eval(cur, false);
        Table t = run_table_chain(base, steps, root);
        rows[(size_t)id] = t.n;
        return t;
    }
};

}  // namespace

void run_bushy(const huge_graph *g, const huge_plan *p, const huge_exec_opts &o, huge_result *out, int64_t *node_rows,
               int max_nodes) {
    if (p->bushy.empty()) HUGE_FAIL(HUGE_EINVAL, "not a bushy plan");
    if (o.engine != HUGE_ENGINE_AUTO && o.engine != HUGE_ENGINE_LEVELS)
        HUGE_FAIL(HUGE_EINVAL, "bushy plans run on the level engine");
    if (o.work_limit) HUGE_FAIL(HUGE_EINVAL, "bushy plans take no work limit");
    if (o.slice2_count > 1) HUGE_FAIL(HUGE_EINVAL, "bushy plans take no second slice");
    if (o.profile) HUGE_FAIL(HUGE_EINVAL, "bushy plans are not profiled");
    if (o.slice_count > 1 && (o.slice_vertex < 0 || o.slice_vertex >= p->k))
        HUGE_FAIL(HUGE_EINVAL, "bushy plans slice a query vertex (slice_vertex 0..k-1)");
    if (o.slice_count > 1 && o.slice_id >= o.slice_count) HUGE_FAIL(HUGE_EINVAL, "slice_id >= slice_count");
    if (o.slice_mode > HUGE_SLICE_STRIDE) HUGE_FAIL(HUGE_EINVAL, "unknown slice_mode %u", o.slice_mode);
    if (p->induced) HUGE_FAIL(HUGE_EINVAL, "bushy plans do not run induced matching");
    if (p->directed) HUGE_FAIL(HUGE_EINVAL, "bushy plans take undirected queries");
    const auto t0 = std::chrono::steady_clock::now();
    Exec ex{g, p, o, (hipStream_t)o.stream};
    ex.rows.assign(p->bushy.size(), -1);
    ex.acc = std::make_unique<Buf>(4 * sizeof(unsigned long long));
    ex.eval((int)p->bushy.size() - 1, true);
    HUGE_HIP(hipStreamSynchronize(ex.st));
    huge_result r = ex.res;
    r.peak_frontier_bytes = ex.peak;
    r.query_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = r;
    if (node_rows)
        for (int i = 0; i < max_nodes; ++i) node_rows[i] = i < (int)ex.rows.size() ? ex.rows[(size_t)i] : -1;
}

}  // namespace huge
