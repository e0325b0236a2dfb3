"""Training of the learned cost model on counts the engine produces.

Labels: for a query q and a matching order pi, the step that produces
prefix s (s = 3..k) examines W_s candidates: the engine's level_work[s-2]
when it runs the prefix plan of size s (huge_plan_prefix), whose count is
|R(prefix_s)|.  --target work (the planner's model, mlp_work.npz) learns
log(1 + W_s); --target count (a cardinality estimator, mlp_count.npz)
learns log(1 + |R(prefix_s)|) for s = 2..k.  Each prefix is run on one root slice of S (matches whose
first matched vertex u has mix(rank u) mod S == s0), scaled by S; S is
sized from the previous prefix's count and raised when a run hits its work
limit, so that every run stays short.  Each labelled pattern is run on one
training graph (every labelled 4-vertex pattern on every graph), with the
cost-model order and random connected orders, and every prefix s >= 3
becomes one sample
    x = huge_plan_features(graph, plan, s, order),  t = log(1 + S * level_work[s-2]).
Prefixes that repeat (same edges and constraints in order positions) are
run once per graph.

Training runs in the library's HIP kernels (huge_model_train: minibatch Adam
on the BF16/FP32 MLP).  This module only orchestrates.

    python -m paper_2103_14294_amd.learn --target work --out paper_2103_14294_amd/mlp_work.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import random
import sys
import time

import numpy as np

import paper_2103_14294_amd as huge

# training graphs: the power-law and R-MAT configurations plus smaller members
# of the same families, so that the graph sketch features vary
TRAIN_GRAPHS = [
    ("rmat18", ("rmat", dict(scale=18, edge_factor=16, seed=11))),
    ("rmat20", ("rmat", dict(scale=20, edge_factor=16, seed=12))),
    ("rmat22", ("rmat", dict(scale=22, edge_factor=16, seed=2))),
    ("cl500k", ("chung_lu", dict(n=500_000, dbar=20, gamma=2.5, seed=13))),
    ("cl1m", ("chung_lu", dict(n=1_000_000, dbar=40, gamma=2.2, seed=14))),
    ("cl3m", ("chung_lu", dict(n=3_072_441, dbar=76, gamma=2.2, seed=3))),
    ("rmat24", ("rmat", dict(scale=24, edge_factor=16, seed=4))),
]


def log(*a):
    print(*a, flush=True)


def make_graph(spec):
    import graphgen as gg

    kind, kw = spec
    if kind == "rmat":
        return gg.rmat(kw["scale"], kw["edge_factor"], seed=kw["seed"])
    return gg.chung_lu(kw["n"], kw["dbar"], kw["gamma"], seed=kw["seed"], exact=kw.get("exact", False))


def random_connected_order(k, edges, rng):
    adj = [[0] * k for _ in range(k)]
    for a, b in edges:
        adj[a][b] = adj[b][a] = 1
    while True:
        o = list(range(k))
        rng.shuffle(o)
        if all(any(adj[o[i]][o[j]] for j in range(i)) for i in range(1, k)):
            return o


def pow2_at_least(x):
    return 1 << max(0, math.ceil(math.log2(max(1.0, x))))


def prefix_key(p_info, k, edges, order, size):
    """The labelled prefix in order positions: its edges and symmetry-breaking pairs."""
    pos = {v: i for i, v in enumerate(order)}
    pe = tuple(sorted((min(pos[a], pos[b]), max(pos[a], pos[b])) for a, b in edges
                      if pos[a] < size and pos[b] < size))
    sb = tuple(sorted((pos[a], pos[b]) for a, b in p_info["sb_pairs"] if pos[a] < size and pos[b] < size))
    return size, pe, sb


def measure_prefix(G, q, size, prev_count, avg_deg, work_target, rng, ws, n):
    """Prefix plan q on a root slice sized from the previous prefix's count; returns the
    full-graph estimates (|R(prefix)|, candidates of its last step, slices used), or None
    when every try hits the work limit."""
    S = pow2_at_least(prev_count * max(1.0, avg_deg) * 4.0 / work_target) if size > 2 else 1
    s_max = max(1, pow2_at_least(n / 16.0) // 2)
    for _ in range(4):
        S = min(S, s_max)
        sid = rng.randrange(S)
        r = huge.count(G, q, slice_count=S, slice_id=sid, slice_vertex=0, workspace=ws, hash=False,
                       work_limit=int(work_target))
        if not r["stopped"]:
            return float(r["count"]) * S, float(r["level_work"][size - 2]) * S, S
        if S >= s_max:
            return None
        S *= 32
    return None


def labelled_connected(k):
    """Every connected labelled graph on vertices 0..k-1 (as edge lists)."""
    from graphgen import patterns as P

    pairs = [(a, b) for a in range(k) for b in range(a + 1, k)]
    out = []
    for mask in range(1, 1 << len(pairs)):
        e = [pairs[i] for i in range(len(pairs)) if (mask >> i) & 1]
        if P.is_connected(k, e):
            out.append({"k": k, "edges": e, "family": "all%d" % k})
    return out


def label_runs(G, patterns, rng, work_target, deadline, ws, n, m, orders_per_pattern=6, orders_small=None,
               target="work"):
    """Label every prefix of every pattern under several orders (the cost model's and
    random connected ones, so that the model sees good and bad orders alike); returns
    feature rows, targets and per-sample records."""
    X, T, recs = [], [], []
    cache = {}
    avg_deg = 2.0 * m / max(1, n)
    runs = 0
    for i, q in enumerate(patterns):
        if time.time() > deadline:
            log("  label budget reached after %d patterns" % i)
            break
        k, e = q["k"], q["edges"]
        p0 = huge.plan(G, k, e)
        orders = [p0.info()["order"]]
        want = orders_small if (orders_small and k == 4) else orders_per_pattern
        for _ in range(8 * want):
            if len(orders) >= want:
                break
            ro = random_connected_order(k, e, rng)
            if ro not in orders:
                orders.append(ro)
        for o in orders:
            p = huge.plan(G, k, e, order=o)
            info = p.info()
            prev = float(n)
            for s in range(2, k + 1):
                key = prefix_key(info, k, e, o, s)
                if key not in cache:
                    runs += 1
                    cache[key] = measure_prefix(G, huge.plan_prefix(p, s), s, prev, avg_deg, work_target, rng, ws, n)
                got = cache[key]
                if got is None:
                    break  # deeper prefixes are at least as expensive
                cnt, work, S = got
                if target == "count" or s >= 3:
                    X.append(huge.plan_features(G, p, s, order=o))
                    T.append(math.log1p(cnt if target == "count" else work))
                    recs.append({"pattern": i, "size": s, "count": cnt, "work": work, "S": S})
                prev = max(cnt, 1.0)
        if (i + 1) % 50 == 0:
            log("  %d patterns, %d prefix runs, %d samples" % (i + 1, runs, len(T)))
    return X, T, recs


def q_error(est, true):
    a, b = np.maximum(1.0, est), np.maximum(1.0, true)
    return np.maximum(a / b, b / a)


def he_init(seed):
    rng = np.random.default_rng(seed)
    F, H = huge.MLP_F, huge.MLP_H
    w1 = rng.normal(0, math.sqrt(2.0 / F), F * H)
    w2 = rng.normal(0, math.sqrt(1.0 / H), H)
    return np.concatenate([w1, np.zeros(H), w2, [0.0]]).astype(np.float32)


def fit(X, T, groups, epochs, lr, batch, seed, val_frac=0.1, residual=False):
    """Standardise, split by pattern group, train on the GPU; returns the model and a report.
    residual: the network learns the correction to the Chung-Lu log-estimate (feature 126),
    so that an estimate is expm1(feature 126 + output)."""
    X = np.asarray(X, np.float32)
    T = np.asarray(T, np.float32)
    base = X[:, 126].astype(np.float32) if residual else np.zeros(len(T), np.float32)
    T = T - base
    ug = np.unique(groups)
    rng = np.random.default_rng(seed)
    val_g = set(rng.choice(ug, max(1, int(len(ug) * val_frac)), replace=False).tolist())
    val = np.array([g in val_g for g in groups])
    xm = X[~val].mean(axis=0)
    xs = X[~val].std(axis=0)
    xinv = np.where(xs > 1e-6, 1.0 / np.maximum(xs, 1e-6), 0.0).astype(np.float32)
    tm, ts = float(T[~val].mean()), float(max(T[~val].std(), 1e-3))
    m = huge.Model().set(he_init(seed), xm.astype(np.float32), xinv, tm, ts)
    t0 = time.perf_counter()
    losses = m.train(X[~val], T[~val], epochs=epochs, batch=batch, lr=lr, seed=seed)
    train_s = time.perf_counter() - t0
    pv = (m.forward(X[val]) if val.any() else np.zeros(0)) + base[val]
    true = np.expm1((T[val] + base[val]).astype(np.float64))
    qe_mlp = q_error(np.expm1(pv.astype(np.float64)), true)
    qe_cl = q_error(np.expm1(X[val][:, 126].astype(np.float64)), true)
    rep = {"samples_train": int((~val).sum()), "samples_val": int(val.sum()), "patterns_val": len(val_g),
           "epochs": epochs, "lr": lr, "batch": batch, "train_s": round(train_s, 2),
           "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
           "residual": bool(residual),
           "val_rmse_log": float(np.sqrt(np.mean((pv - T[val] - base[val]) ** 2))) if val.any() else None,
           "val_qerror_mlp": {"median": float(np.median(qe_mlp)), "p90": float(np.percentile(qe_mlp, 90)),
                              "geomean": float(np.exp(np.mean(np.log(qe_mlp))))},
           "val_qerror_chung_lu_feature": {"median": float(np.median(qe_cl)), "p90": float(np.percentile(qe_cl, 90)),
                                           "geomean": float(np.exp(np.mean(np.log(qe_cl))))}}
    return m, rep, losses


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="model file (.npz)")
    ap.add_argument("--labels", default=None, help="write / reuse labelled samples (.npz)")
    ap.add_argument("--patterns", type=int, default=2100)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--work-target", type=float, default=5e8, help="candidates examined per labelling run, at most")
    ap.add_argument("--label-minutes", type=float, default=12.0)
    ap.add_argument("--graphs", default=",".join(n for n, _ in TRAIN_GRAPHS))
    ap.add_argument("--orders", type=int, default=6, help="orders per pattern (cost model's + random)")
    ap.add_argument("--target", choices=["work", "count"], default="work",
                    help="work: candidates of the step producing each prefix (the planner's cost); "
                         "count: |R(prefix)| (cardinality estimation)")
    ap.add_argument("--residual", action="store_true",
                    help="learn the correction to the Chung-Lu log-estimate (feature 126)")
    ap.add_argument("--epochs", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=256)
    args = ap.parse_args(argv)

    import torch

    torch.cuda.set_device(0)
    if args.labels and os.path.exists(args.labels):
        with np.load(args.labels, allow_pickle=False) as z:
            X, T, groups = z["X"], z["T"], z["groups"]
        log("reusing %d samples from %s" % (len(T), args.labels))
        meta = {"labels": args.labels}
    else:
        from graphgen import patterns as P

        names = args.graphs.split(",")
        specs = dict(TRAIN_GRAPHS)
        # every labelled connected 4-vertex pattern runs on every graph (there are only 38);
        # random labelled 5- and 6-vertex patterns are spread over the graphs
        small = labelled_connected(4)
        pats = P.random_patterns(args.patterns, seed=args.seed, kmin=5, kmax=6, distinct="labelled")
        log("%d labelled 4-vertex patterns on every graph, %d random 5-6-vertex patterns (k: %s)" % (
            len(small), len(pats), {k: sum(p["k"] == k for p in pats) for k in (5, 6)}))
        rng = random.Random(args.seed)
        X, T, groups, meta = [], [], [], {"graphs": {}, "patterns": len(pats)}
        ws = huge.Workspace()
        t_all = time.time()
        per_graph = args.label_minutes * 60.0 / len(names)
        for gi, name in enumerate(names):
            mine = small + [p for j, p in enumerate(pats) if j % len(names) == gi]
            t0 = time.perf_counter()
            g = make_graph(specs[name])
            G = huge.load(g.row_ptr, g.col)
            log("graph %s: n=%d m=%d (%.1f s); %d patterns" % (name, g.n, g.m, time.perf_counter() - t0, len(mine)))
            x, t, recs = label_runs(G, mine, rng, args.work_target, time.time() + per_graph, ws, g.n, g.m,
                                    args.orders, orders_small=12, target=args.target)
            # samples of one pattern share a group (the validation split is by pattern)
            groups.extend([gi * 100000 + r["pattern"] for r in recs])
            X.extend(x)
            T.extend(t)
            meta["graphs"][name] = {"n": g.n, "m": g.m, "samples": len(t),
                                    "patterns": len({r["pattern"] for r in recs}),
                                    "label_s": round(time.perf_counter() - t0, 1)}
            G.free()
            del g
            log("  %s: %d samples, %.1f s" % (name, len(t), time.perf_counter() - t0))
        X = np.asarray(X, np.float32)
        T = np.asarray(T, np.float32)
        groups = np.asarray(groups, np.int64)
        meta["label_s"] = round(time.time() - t_all, 1)
        if args.labels:
            np.savez(args.labels, X=X, T=T, groups=groups)
    m, rep, losses = fit(X, T, groups, args.epochs, args.lr, args.batch, args.seed, residual=args.residual)
    rep["target"] = args.target
    m.save(args.out)
    rep.update(meta)
    rep["loss_curve"] = [float(x) for x in losses[:: max(1, len(losses) // 30)]]
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(rep, f, indent=1)
    log(json.dumps({k: v for k, v in rep.items() if k != "loss_curve"}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
