"""Benchmark: subgraph enumeration throughput on one MI355X.

Default workload (the plain PULL-EXTEND configuration): 4-clique, diamond and
4-cycle counted on an R-MAT graph of scale 22, edge factor 16,
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05), symmetrised and deduplicated, seed 2.
The whole-graph counts are of order 10^11 to 10^12, so the input is processed
in 64 root batches: batch s holds the matches whose first matched vertex u
has mix(rank(u)) mod 64 == s (the batches partition the matches).  One step =
one batch of all three queries, each a huge_count call with the graph already
resident in HBM (planning excluded; every kernel, the count, the set-hash and
the result read-back included).  value = embeddings / timed seconds.

Prints one JSON line.  Also reports, for the kernel class with the most device
time, the algorithmic bytes it moved per second against the 8 TB/s HBM peak
(timed with HIP events on the exec stream during the timed steps), and the
CPU oracle's throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KC_NAMES = ["prepare", "scan", "extend", "extend_sink"]
KC_KERNELS = ["k_prepare", "k_tile_scan/k_tile_reduce", "k_extend*<W,EMIT>", "k_extend*<W,COUNT>"]
STRAT_KERNEL = {0: "k_extend", 1: "k_extend", 2: "k_extend_merge", -1: "k_extend_merge"}

WORKLOADS = {
    "c2": {
        "desc": "R-MAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), seed 2: 4-clique, diamond, 4-cycle",
        "graph": ("rmat", dict(scale=22, edge_factor=16, seed=2)),
        "queries": ["4-clique", "diamond", "4-cycle"],
        "cap": 4 << 30,
        "batches": 64,
    },
    "c1": {
        "desc": "Chung-Lu n=16384, mean degree 16, gamma 2.5, exact, seed 1: triangle, 4-cycle",
        "graph": ("chung_lu", dict(n=16384, dbar=16, gamma=2.5, seed=1, exact=True)),
        "queries": ["triangle", "4-cycle"],
        "cap": 4 << 30,
        "batches": 1,
    },
    "c3": {
        "desc": "Chung-Lu n=3072441, mean degree 76, gamma 2.2, seed 3: 5-clique, house, frontier cap 32 GiB",
        "graph": ("chung_lu", dict(n=3072441, dbar=76, gamma=2.2, seed=3)),
        "queries": ["5-clique", "house"],
        "cap": 32 << 30,
        "batches": 16,
    },
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(spec):
    import graphgen as gg

    kind, kw = spec
    if kind == "rmat":
        return gg.rmat(kw["scale"], kw["edge_factor"], seed=kw["seed"])
    return gg.chung_lu(kw["n"], kw["dbar"], kw["gamma"], seed=kw["seed"], exact=kw.get("exact", False))


def cpu_baseline(g, queries, budget_s, threads):
    """The oracle, as it stands, on root slices of the same graph and queries."""
    import oracle
    from graphgen import patterns as P

    S = 1 << 20
    per_q = budget_s / len(queries)
    tot_cnt, tot_t, slices = 0, 0.0, {}
    for name in queries:
        k, e = P.NAMED[name]
        t_q, s = 0.0, 0
        while t_q < per_q and s < S:
            t0 = time.perf_counter()
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, slice_count=S, slice_id=s, threads=threads)
            dt = time.perf_counter() - t0
            t_q += dt
            tot_cnt += r["count"]
            s += 1
        tot_t += t_q
        slices[name] = s
    return {
        "value": tot_cnt / tot_t if tot_t > 0 else 0.0,
        "unit": "embeddings/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "root slices s=0..R-1 of %d (query vertex 0's image, mix(rank) mod %d); R per query = %s; "
                  "%d embeddings in %.1f s" % (S, S, json.dumps(slices), tot_cnt, tot_t),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--learned", action="store_true", help="plan with the learned cardinality model")
    ap.add_argument("--strategy", type=int, default=-1, help="intersection strategy (-1 = library default)")
    ap.add_argument("--no-hash", action="store_true", help="count only (no set-hash)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see the sharding design); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2103_14294_amd as huge
    from graphgen import patterns as P

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    W = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = make_graph(W["graph"])
    log("graph %s: n=%d m=%d (%.1f s to generate)" % (args.workload, g.n, g.m, time.perf_counter() - t0))
    G = huge.load(g.row_ptr, g.col)
    info = G.info()
    log("loaded on GPU in %.1f ms (max degree %d)" % (info["load_ms"], info["max_degree"]))
    plans = []
    for name in W["queries"]:
        k, e = P.NAMED[name]
        p = huge.plan(G, k, e, learned=args.learned)
        plans.append((name, p))
        log("plan %s: order %s est_cost %.3g" % (name, p.info()["order"], p.info()["est_cost"]))
    ws = huge.Workspace()
    nb = W["batches"]
    kw = dict(cap=W["cap"], workspace=ws, strategy=args.strategy, hash=not args.no_hash)

    def batch_kw(name, p, b):
        if nb <= 1:
            return {}
        return dict(slice_count=nb, slice_id=b % nb, slice_vertex=p.info()["order"][0])

    # warmup on the last batches, time the first ones: no batch is seen twice
    for i in range(args.warmup):
        b = nb - 1 - i
        for name, p in plans:
            r = huge.count(G, p, **kw, **batch_kw(name, p, b))
            log("warmup batch %d %s: count=%d %.1f ms launches=%d peak_frontier=%.2f GB" % (
                b, name, r["count"], r["query_ms"], r["launches"], r["peak_frontier_bytes"] / 1e9))

    kms = [0.0] * 4
    kl = [0] * 4
    kb = [0.0] * 4
    total = 0
    per_q = {name: [] for name, _ in plans}
    counts = {name: [] for name, _ in plans}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        for name, p in plans:
            r = huge.count(G, p, profile=True, **kw, **batch_kw(name, p, s))
            total += r["count"]
            counts[name].append(r["count"])
            per_q[name].append(r["query_ms"])
            for c in range(4):
                kms[c] += r["kernel_ms"][c]
                kl[c] += r["kernel_launches"][c]
                kb[c] += r["alg_bytes"][c]
        log("step %d (batch %d) done" % (s, s % max(1, nb)))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    dom = max(range(4), key=lambda c: kms[c])
    avg_ms = kms[dom] / max(1, kl[dom])
    bytes_per_launch = kb[dom] / max(1, kl[dom])
    achieved = (bytes_per_launch / (avg_ms * 1e-3)) / 1e9 if avg_ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": KC_KERNELS[dom].replace("k_extend*", STRAT_KERNEL.get(args.strategy, "k_extend")),
            "avg_launch_ms": round(avg_ms, 4),
            "alg_bytes_per_launch": bytes_per_launch, "launches": kl[dom],
            "kernel_ms_by_class": {KC_NAMES[c]: round(kms[c], 3) for c in range(4)}}

    out = {
        "metric": "embeddings/sec + query time, learned/batched vs cost-model plan, 1 GPU",
        "value": total / elapsed,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": W["desc"], "plan": "learned" if args.learned else "cost-model",
                   "batches": "%d root batches (first matched vertex), batch i timed at step i" % nb
                   if nb > 1 else "whole graph per step",
                   "engine": "levels", "strategy": args.strategy, "hash": not args.no_hash,
                   "frontier_cap_bytes": W["cap"],
                   "counts": counts,
                   "query_ms_median": {k: sorted(v)[len(v) // 2] for k, v in per_q.items()},
                   "graph_load_ms": info["load_ms"], "n": g.n, "m": g.m},
        "roofline": roof,
    }
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        log("cpu baseline: oracle on root slices, %d threads, budget %.0f s" % (threads, args.cpu_budget))
        out["cpu_baseline"] = cpu_baseline(g, W["queries"], args.cpu_budget, threads)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
