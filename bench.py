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
        "batches": 1 << 14,
    },
    "c4": {
        "desc": "R-MAT scale 24, edge factor 16, (0.57,0.19,0.19,0.05), seed 4: 64 random connected 3-6 vertex "
                "patterns (seed 4; at most 4e9 candidates per 1/2^20 edge batch)",
        "graph": ("rmat", dict(scale=24, edge_factor=16, seed=4)),
        "queries": ("random", dict(count=64, seed=4, kmin=3, kmax=6, max_work=4e9)),
        "cap": 8 << 30,
        "batches": 1 << 20,
        "slice": "edge",
    },
    "c5": {
        "desc": "R-MAT scale 26, edge factor 16, (0.57,0.19,0.19,0.05), seed 5: 32 held-out random 4-6 vertex "
                "patterns (seed 5; at most 2e10 candidates per 1/2^16 edge batch)",
        "graph": ("rmat", dict(scale=26, edge_factor=16, seed=5)),
        "queries": ("random", dict(count=32, seed=5, kmin=4, kmax=6, max_work=2e10)),
        "cap": 16 << 30,
        "batches": 1 << 16,
        "slice": "edge",
    },
}
MODEL_PATH = os.path.join(ROOT, "paper_2103_14294_amd", "mlp_work.npz")

# HBM traffic of the last-level intersection class on the default workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of this benchmark,
# scaled by what the same counters read for the benchmark's own 4 GiB device copy
# (FETCH_SIZE x2.0, WRITE_SIZE x1.0).  Recorded per algorithmic byte, because the tuned
# table (which kernel runs each probe-length bucket, hence the launches per step) can
# differ between tuning runs: a run's traffic per launch is that ratio times its own
# algorithmic bytes per launch (bytes_per_launch: the profiled run's own figure).  Valid
# for the kernel and graph-load sources (hub bitmaps change the traffic) whose digest is
# given; null for any other sources or workload.
TRAFFIC = {"c2": {"sources_sha256_16": "e659cd17d4841fef", "bytes_per_launch": 3.079e9,
                  "per_alg_byte": 0.3166}}
KERNEL_SOURCES = ["paper_2103_14294_amd/csrc/extend.hip", "paper_2103_14294_amd/csrc/devfuncs.h",
                  "paper_2103_14294_amd/csrc/graph.hip"]


def recorded_traffic(workload, alg_bytes_per_launch):
    import hashlib

    rec = TRAFFIC.get(workload)
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["sources_sha256_16"]:
        return None
    return rec["per_alg_byte"] * alg_bytes_per_launch


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

    S = 1 if g.n <= (1 << 17) else 1 << 20  # small graphs: the whole graph at once
    per_q = budget_s / len(queries)
    tot_cnt, tot_t, slices = 0, 0.0, {}
    for name, k, e in queries:
        t_q, s = 0.0, 0
        while t_q < per_q and (s < S or S == 1):  # a whole-graph sample repeats to fill the budget
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
        "sample": ("whole graph, repeated (runs per query %s); " % json.dumps(slices) if S == 1 else
                   "root slices s=0..R-1 of %d (query vertex 0's image, mix(rank) mod %d); R per query = %s; "
                   % (S, S, json.dumps(slices))) + "%d embeddings in %.1f s" % (tot_cnt, tot_t),
    }


def build_queries(W, G, huge, P, ws):
    """[(name, k, edges)] for the workload: named queries, or seeded random patterns
    whose cost-model plan finishes one batch (the last, never timed) within the
    workload's work budget (candidates examined)."""
    q = W["queries"]
    if isinstance(q, list):
        return [(n,) + tuple(P.NAMED[n]) for n in q]
    kw = dict(q[1])
    budget = kw.pop("max_work")
    nb = W["batches"]
    out, tried = [], 0
    for pat in P.random_patterns(kw["count"] * 8, seed=kw["seed"], kmin=kw["kmin"], kmax=kw["kmax"]):
        if len(out) == kw["count"]:
            break
        tried += 1
        p = huge.plan(G, pat["k"], pat["edges"])
        r = huge.count(G, p, slice_count=nb, slice_id=nb - 1, slice_vertex=-2 if W.get("slice") == "edge" else -1,
                       work_limit=int(budget),
                       workspace=ws, hash=False, cap=W["cap"])
        if not r["stopped"]:
            out.append(("%s-k%d-%d" % (pat["family"], pat["k"], len(out)), pat["k"], pat["edges"]))
    log("%d of %d random patterns within %.3g candidates per batch" % (len(out), tried, budget))
    return out


def copy_bandwidth(torch, nbytes=4 << 30, reps=5):
    """Device-to-device copy of nbytes (torch's copy kernel): achieved GB/s counting the
    read and the write, and the bytes one copy moves."""
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        b.copy_(a)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, 2 * nbytes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--learned", nargs="?", const=MODEL_PATH, default=None,
                    help="plan with the learned cost model, its best orders verified on a root sample "
                         "(default model file if no path)")
    ap.add_argument("--compare", action="store_true",
                    help="time the cost-model plans and the learned plans on the same batches")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip autotuning the per-bucket dispatch before timing (library default kernels)")
    ap.add_argument("--batched", action="store_true", help="one huge_count_batch call per step")
    ap.add_argument("--engine", choices=["levels", "graph"], default="levels",
                    help="levels: host-driven scheduler (default); graph: device scheduler, rounds replayed "
                         "from a hipGraph")
    ap.add_argument("--cap", type=float, default=None, help="frontier cap in bytes (default: the workload's)")
    ap.add_argument("--strategy", type=int, default=-1, help="intersection strategy (-1 = library default)")
    ap.add_argument("--no-hash", action="store_true", help="count only (no set-hash)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the 4 GiB device copy (counter calibration) and print its bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (see the sharding design); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2103_14294_amd as huge
    from graphgen import patterns as P

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    if args.copy_only:
        gbs, moved = copy_bandwidth(torch)
        print(json.dumps({"copy_gbs": round(gbs, 1), "bytes_per_copy": moved, "copies": 6}), flush=True)
        return
    W = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = make_graph(W["graph"])
    log("graph %s: n=%d m=%d (%.1f s to generate)" % (args.workload, g.n, g.m, time.perf_counter() - t0))
    G = huge.load(g.row_ptr, g.col)
    info = G.info()
    log("loaded on GPU in %.1f ms (max degree %d)" % (info["load_ms"], info["max_degree"]))
    ws = huge.Workspace()
    queries = build_queries(W, G, huge, P, ws)
    model = huge.Model.load(args.learned if args.learned else MODEL_PATH) \
        if (args.learned or args.compare) else None
    modes = ["cost-model", "learned"] if args.compare else (["learned"] if args.learned else ["cost-model"])
    plans = {m: [] for m in modes}
    for name, k, e in queries:
        for m in modes:
            t_p = time.perf_counter()
            p = huge.plan(G, k, e, learned=model if m == "learned" else None, verify=m == "learned")
            plan_ms = (time.perf_counter() - t_p) * 1e3
            plans[m].append((name, k, p, plan_ms))
            log("plan %s [%s]: order %s est_cost %.3g (%.1f ms)" % (name, m, p.info()["order"],
                                                                   p.info()["est_cost"], plan_ms))
    nb = W["batches"]
    cap = int(args.cap) if args.cap is not None else W["cap"]
    kw = dict(cap=cap, workspace=ws, strategy=args.strategy, hash=not args.no_hash)
    if args.engine == "graph":
        kw["engine"] = huge.ENGINE_GRAPH
    # batches slice on each plan's first matched vertex, or on its level-2 rows (edge
    # slices, which reach hubs in proportion to their degree): an unbiased 1/nb sample of
    # that plan's work, the same in sequential and batched runs

    def batch_kw(p, b):
        if nb <= 1:
            return {}
        return dict(slice_count=nb, slice_id=b % nb, slice_vertex=sv_mode)

    sv_mode = -2 if W.get("slice") == "edge" else -1
    tune_info = None
    if args.tune:
        t_t = time.perf_counter()
        sample = [p for _, _, p, _ in plans[modes[-1]]]
        # the sample: the largest slice on which every plan examines at most 2e9 candidates
        S = max(4 * nb, 256)
        while S < (1 << 30):
            if all(not huge.count(G, p, slice_count=S, slice_id=S - 1, slice_vertex=sv_mode, work_limit=int(2e9),
                                  cap=cap, workspace=ws, hash=False)["stopped"] for p in sample):
                break
            S *= 4
            log("tuning sample: trying 1/%d" % S)
        log("autotuning the per-bucket dispatch on a 1/%d sample" % S)
        table = huge.autotune(G, sample, cache=os.environ.get("HUGE_TUNE_CACHE"),
                              slice_count=S, slice_id=S - 1, slice_vertex=sv_mode, cap=cap)
        kw["tune"] = table
        tune_info = {"tune_s": round(time.perf_counter() - t_t, 2),
                     "strategy": {str(j): table.to_dict()["strategy"][j] for j in range(huge.KMAX + 1)
                                  if any(table.items[j][c] for c in range(huge.TUNE_BUCKETS))},
                     "chunk_rows": {str(j): table.chunk_rows[j] for j in range(huge.KMAX + 1) if table.chunk_rows[j]}}
        log("autotuned in %.1f s: %s" % (tune_info["tune_s"], json.dumps(tune_info)))

    def run_step(m, b, profile, acc):
        pl = plans[m]
        if args.batched:
            rs = huge.count_batch(G, [p for _, _, p, _ in pl], **{k2: v for k2, v in kw.items() if k2 != "workspace"},
                                  profile=profile, **batch_kw(pl[0][2], b))
        else:
            rs = []
            for name, _, p, _ in pl:
                rs.append(huge.count(G, p, profile=profile, **kw, **batch_kw(p, b)))
                if len(pl) > 4 or rs[-1]["query_ms"] > 2000:
                    log("  [%s] batch %d %s: %.1f ms" % (m, b, name, rs[-1]["query_ms"]))
        for (name, k, p, _), r in zip(pl, rs):
            acc["_peak"] = max(acc.get("_peak", 0), r["peak_frontier_bytes"])
            a = acc.setdefault(name, {"count": 0, "ms": [], "keys": []})
            a["count"] += r["count"]
            a["ms"].append(r["query_ms"])
            a["keys"].append((r["count"], r["hash_sum"], r["hash_xor"]))
            for c in range(4):
                acc["_kms"][c] += r["kernel_ms"][c]
                acc["_kl"][c] += r["kernel_launches"][c]
                acc["_kb"][c] += r["alg_bytes"][c]

    results = {}
    for m in modes:
        # warmup on the last batches, time the first ones: no batch is seen twice
        for i in range(args.warmup):
            run_step(m, nb - 1 - i, False, {"_kms": [0.0] * 4, "_kl": [0] * 4, "_kb": [0.0] * 4})
            log("warmup [%s] batch %d done" % (m, nb - 1 - i))
        acc = {"_kms": [0.0] * 4, "_kl": [0] * 4, "_kb": [0.0] * 4}
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            run_step(m, s_, True, acc)
            log("step %d [%s] (batch %d) done" % (s_, m, s_ % max(1, nb)))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        results[m] = (acc, elapsed)
    checked = 0
    if args.compare:
        # exactness: where both plans start from the same query vertex they ran the same
        # batches; otherwise the learned plan runs the cost-model plan's first batch (bounded)
        a0, a1 = results["cost-model"][0], results["learned"][0]
        for (name, k, p0, _), (_, _, p1, _) in zip(plans["cost-model"], plans["learned"]):
            same = p0.info()["order"][:2] == p1.info()["order"][:2] if sv_mode == -2 else \
                p0.info()["order"][0] == p1.info()["order"][0]
            if same:
                got, want = a1[name]["keys"], a0[name]["keys"]
            else:
                if sv_mode == -2:
                    continue  # an edge slice is defined by each plan's own first two vertices
                r = huge.count(G, p1, work_limit=int(4e10), **kw,
                               **dict(batch_kw(p0, 0), slice_vertex=p0.info()["order"][0]))
                if r["stopped"]:
                    continue
                got, want = [(r["count"], r["hash_sum"], r["hash_xor"])], a0[name]["keys"][:1]
            if got != want:
                raise SystemExit("learned and cost-model plans disagree on %s: %s vs %s" % (name, got, want))
            checked += 1

    main_mode = modes[-1]
    acc, elapsed = results[main_mode]
    total = sum(v["count"] for k_, v in acc.items() if not k_.startswith("_"))
    kms, kl, kb = acc["_kms"], acc["_kl"], acc["_kb"]
    dom = max(range(4), key=lambda c: kms[c])
    avg_ms = kms[dom] / max(1, kl[dom])
    bytes_per_launch = kb[dom] / max(1, kl[dom])
    achieved = (bytes_per_launch / (avg_ms * 1e-3)) / 1e9 if avg_ms > 0 else 0.0
    traffic = recorded_traffic(args.workload, bytes_per_launch) if (args.tune and args.strategy < 0 and not args.batched
                                                  and dom == 3 and main_mode == "cost-model") else None
    if args.engine == "graph":  # no per-launch timing inside replays
        achieved = None
    roof = {"bound": "hbm", "achieved": round(achieved, 2) if achieved is not None else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved is not None else None, "traffic": traffic,
            "traffic_gbs": round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic and avg_ms > 0 else None,
            "kernel": ("last-level intersection + counting SINK: k_extend*<W,COUNT> launches, one per probe-length "
                       "bucket with its tuned strategy") if (dom == 3 and args.tune)
                      else KC_KERNELS[dom].replace("k_extend*", STRAT_KERNEL.get(args.strategy, "k_extend")),
            "avg_launch_ms": round(avg_ms, 4),
            "alg_bytes_per_launch": bytes_per_launch, "launches": kl[dom],
            "kernel_ms_by_class": {KC_NAMES[c]: round(kms[c], 3) for c in range(4)}}
    cfg = {"workload": W["desc"], "plan": main_mode,
           "batches": "%d root batches, batch i timed at step i" % nb if nb > 1 else "whole graph per step",
           "engine": args.engine if not args.batched else "batch", "strategy": args.strategy,
           "hash": not args.no_hash, "frontier_cap_bytes": cap, "peak_frontier_bytes": acc.get("_peak", 0),
           "graph_load_ms": info["load_ms"],
           "n": g.n, "m": g.m, "queries": len(queries)}
    if len(queries) <= 4:
        cfg["counts"] = {k_: [x[0] for x in v["keys"]] for k_, v in acc.items() if not k_.startswith("_")}
        cfg["query_ms_median"] = {k_: sorted(v["ms"])[len(v["ms"]) // 2] for k_, v in acc.items()
                                  if not k_.startswith("_")}
    if tune_info:
        cfg["autotune"] = tune_info
    if args.compare:
        e0, e1 = results["cost-model"][1], results["learned"][1]
        a0 = results["cost-model"][0]
        ratios = []
        per = {}
        for (name, k, p0, _), (_, _, p1, _) in zip(plans["cost-model"], plans["learned"]):
            t0_ = sum(a0[name]["ms"])
            t1_ = sum(acc[name]["ms"])
            ratios.append(t0_ / max(t1_, 1e-9))
            per[name] = {"order_cost_model": p0.info()["order"], "order_learned": p1.info()["order"],
                         "ms_cost_model": round(t0_, 2), "ms_learned": round(t1_, 2)}
        import math
        cfg["compare"] = {"cost_model_s": round(e0, 3), "learned_s": round(e1, 3),
                          "speedup_total": round(e0 / max(e1, 1e-9), 4),
                          "speedup_geomean": round(math.exp(sum(math.log(r) for r in ratios) / len(ratios)), 4),
                          "orders_changed": sum(1 for v in per.values() if v["order_cost_model"] != v["order_learned"]),
                          "exactness_checked": "%d of %d queries: learned plan vs cost-model plan, "
                                               "equal count and hashes (same batches, or the cost-model "
                                               "plan's batch 0 within 4e10 candidates)" % (checked, len(queries)),
                          "plan_ms_learned": round(sum(x[3] for x in plans["learned"]), 1),
                          "per_query": per if len(per) <= 64 else None}
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
        "config": cfg,
        "roofline": roof,
    }
    gbs, _ = copy_bandwidth(torch)
    out["roofline"]["copy_gbs"] = round(gbs, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / gbs, 4) if gbs > 0 and achieved is not None else None
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        log("cpu baseline: oracle on root slices, %d threads, budget %.0f s" % (threads, args.cpu_budget))
        out["cpu_baseline"] = cpu_baseline(g, queries, args.cpu_budget, threads)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
