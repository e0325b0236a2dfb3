"""Benchmark: subgraph enumeration throughput on one MI355X.

Default workload (the learned-plan configuration): R-MAT scale 26, edge
factor 16, (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), symmetrised and
deduplicated, seed 5 (67.1M vertices, ~1.05B undirected edges, int32 CSR with
int64 offsets), and 32 random connected 4-6-vertex query patterns (seed 5,
one per isomorphism class) that the learned model never saw: labelled
patterns of its training set are skipped, which leaves 5- and 6-vertex ones.
Whole-graph counts of these patterns run to 10^12..10^20, so every query is
timed on samples: root slice s of S_q, the matches whose first matched vertex
has degree rank r with r mod S_q == s (every S_q-th vertex in degree order, so
every slice holds the same share of each degree class; the engines gather
only the slice's edge-array entries).  It is an unbiased 1/S_q sample of that
plan's work.  S_q is fixed per query: the smallest power of 4 from 2^10 at
which every root slice the run uses (timed and warmup), under the cost-model
plan and under the learned plan, examines at most 1e9 candidates; so every
mode processes the same fraction of each query, and no step meets a root
whose work has no bound.  Patterns are drawn in seed order and kept when such
an S_q <= 2^24 exists (at least 4 roots per slice); the JSON line says how
many were skipped.
(Edge slices, every S-th entry of the CSR, sample hub lists in proportion to
their degree, but here a single hub entry of most 5-6-vertex patterns holds
more than 1e9 candidates: no edge sample of them fits any budget.)
One step = one slice of every query.

Modes, timed on the same steps:
  cost-model          the plain cost-model plans (Algorithm 1's estimator),
                      one huge_count per query (level engine);
  cost-model-batched  the same plans in one huge_count_batch per step
                      (batched rounds: device scheduler, one replayed graph);
  learned             the learned plans (the MLP picks the order among all
                      connected ones, its two best measured against the cost
                      model's on a small sample), one huge_count per query;
  learned-batched     the learned plans batched: the headline.
Query time includes planning, paid once per query while the timed slices are
a fraction K/S_q of it.  So each query's sample is scaled to the whole query:
count S_q * (sampled count) / K, run time S_q * (sampled seconds) / K (per
batch of equal S_q in the batched modes); a mode's query time = planning +
those run times; value = the workload's scaled embeddings (pooled over the
distinct plans' samples) / the headline mode's query time.  Equivalently, the
sampled rate with planning charged in proportion to the sampled fraction.
The timed steps are slices 0..K-1, the lowest position in every degree
stratum (warmup: the next ones), so the scaled figures describe those strata,
not the hubs' own slices.  The raw sampled rates are in
config.modes[*].sampled.

Exactness: for every query both plans run one shared sample (the double slice:
root slice 1 of S_q of the learned plan's first vertex AND root slice 0 of S_q
of the cost-model plan's first vertex, each plan reading only its own slice's
entries) and must return the same count and both set-hashes.

Roofline: the dominant kernel class of a profiled pass of the cost-model mode
on the same steps (HIP events around every launch, on the exec stream):
algorithmic bytes per launch / average launch time, against 8 TB/s.  The
timed modes run without events.  cpu_baseline: the oracle on the same slices
(cost-model order, same root slice), on the host's cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KC_NAMES = ["prepare", "scan", "extend", "extend_sink"]
KC_KERNELS = ["k_prepare<W,LAST>", "k_tile_scan/k_tile_reduce", "k_extend*<W,EMIT>",
              "k_extend*<W,COUNT> (last-level intersection + counting SINK)"]

WORKLOADS = {
    "c5": {
        "desc": "R-MAT scale 26, edge factor 16, (0.57,0.19,0.19,0.05), seed 5: 32 held-out random 4-6 vertex "
                "patterns (seed 5, the first 32 drawn whose root slices fit 1e9 candidates at some S <= 2^24); "
                "learned/batched vs cost-model plans",
        "graph": ("rmat", dict(scale=26, edge_factor=16, seed=5)),
        "queries": ("heldout", dict(count=32, draw=400, seed=5, kmin=4, kmax=6)),
        "cap": 16 << 30,
        "budget": 1e9,
        "modes": ["cost-model", "cost-model-batched", "learned", "learned-batched"],
    },
    "c4": {
        "desc": "R-MAT scale 24, edge factor 16, (0.57,0.19,0.19,0.05), seed 4: 64 random connected 3-6 vertex "
                "patterns (seed 4, the first 64 drawn whose root slices fit 5e7 candidates at some S <= 2^24); batched vs "
                "one query at a time",
        "graph": ("rmat", dict(scale=24, edge_factor=16, seed=4)),
        "queries": ("random", dict(count=64, draw=600, seed=4, kmin=3, kmax=6)),
        "cap": 16 << 30,
        "budget": 5e7,
        "modes": ["cost-model", "cost-model-batched"],
    },
    "c2": {
        "desc": "R-MAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), seed 2: 4-clique, diamond, 4-cycle",
        "graph": ("rmat", dict(scale=22, edge_factor=16, seed=2)),
        "queries": ["4-clique", "diamond", "4-cycle"],
        "cap": 4 << 30,
        "slices": 64,
        "modes": ["cost-model"],
    },
    "c3": {
        "desc": "Chung-Lu n=3072441, mean degree 76, gamma 2.2, seed 3: 5-clique, house, frontier cap 32 GiB",
        "graph": ("chung_lu", dict(n=3072441, dbar=76, gamma=2.2, seed=3)),
        "queries": ["5-clique", "house"],
        "cap": 32 << 30,
        "slices": 1 << 14,
        "modes": ["cost-model"],
    },
    "c1": {
        "desc": "Chung-Lu n=16384, mean degree 16, gamma 2.5, exact, seed 1: triangle, 4-cycle",
        "graph": ("chung_lu", dict(n=16384, dbar=16, gamma=2.5, seed=1, exact=True)),
        "queries": ["triangle", "4-cycle"],
        "cap": 4 << 30,
        "slices": 1,
        "modes": ["cost-model"],
    },
}
MODEL_PATH = os.path.join(ROOT, "paper_2103_14294_amd", "mlp_work.npz")

# HBM traffic of the dominant kernel class per workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) of this benchmark's
# profiled pass, scaled by what the same counters read for the benchmark's own
# 4 GiB device copy, recorded per algorithmic byte (a run's traffic per launch is
# that ratio times its own algorithmic bytes per launch).  Valid only for the
# kernel sources whose digest is given; null for any other sources or workload.
TRAFFIC = {
    # R-MAT 26 held-out patterns (the default run's queries and slices, 20 steps, 5 warmup, the cost-model
    # mode timed): the 153 sink-class dispatches of the profiled pass, FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0
    # (factors from the 4 GiB copy), 146.3 MB per launch against 140.2 MB of algorithmic bytes
    "c5": {"per_alg_byte": 1.0436, "sources_sha256_16": "132c0462edc1778f"},
}
KERNEL_SOURCES = ["paper_2103_14294_amd/csrc/" + f for f in
                  ("extend.hip", "tiles.h", "devfuncs.h", "internal.h", "round_sched.h", "graph.hip", "mround.hip",
                   "scan_tiles.h", "prims.hip", "prims.h", "engine.cpp", "mbatch.cpp")] + ["include/huge.h"]


def sources_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, alg_bytes_per_launch):
    rec = TRAFFIC.get(workload)
    if rec is None or rec["sources_sha256_16"] != sources_digest():
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


def training_patterns():
    """Labelled edge sets the learned model was trained on: every labelled connected
    4-vertex pattern and the random 5-6-vertex ones of the training run's seed."""
    from graphgen import patterns as P
    from paper_2103_14294_amd import learn

    seen = {(4, tuple(sorted(p["edges"]))) for p in learn.labelled_connected(4)}
    for p in P.random_patterns(2100, seed=1, kmin=5, kmax=6, distinct="labelled"):
        seen.add((p["k"], tuple(sorted(p["edges"]))))
    return seen


SLICE = dict(slice_vertex=-1)  # root slices of each plan's first matched vertex, strided by degree rank


def slice_of(step, S):
    """The slice that step `step` runs: slice `step` (mod S).  Slice s holds the
    ranks s, s + S, s + 2S, ...: the timed steps take the lowest position in
    every degree stratum.  (A spread-out permutation of the slices was tried:
    about one slice in a few hundred then holds a high-degree root whose 6-vertex
    matches alone take minutes, which no bounded step can time.)"""
    return step % S if S > 1 else 0
S_MIN, S_MAX = 1 << 10, 1 << 24


def pilot(huge, G, plans, budget, ws, cap, nslices):
    """The smallest power-of-4 slice count S in [S_MIN, S_MAX] at which every plan
    of the query examines at most `budget` candidates in each root slice the run
    will use (slices 0..nslices-1), or None.  The descent tests the first two
    slices; the chosen S is then checked on all of them (and raised by 4 while
    some slice holds a heavier root)."""
    def fits(S, ids):
        for p in plans:
            for s in ids:
                r = huge.count(G, p, slice_count=S, slice_id=slice_of(s, S), slice_mode=huge.SLICE_STRIDE,
                               work_limit=int(budget), hash=False, workspace=ws, cap=cap, **SLICE)
                if r["stopped"]:
                    return False
        return True

    if not fits(S_MAX, (0, 1)):
        return None
    S = S_MAX
    while S > S_MIN and fits(S // 4, (0, 1)):
        S //= 4
    while not fits(S, range(nslices)):
        if S >= S_MAX:
            return None
        S *= 4
    return S


def candidate_patterns(W):
    """The random workloads' patterns in draw order, [(name, k, edges)]: seeded, one
    per isomorphism class, held-out ones outside the learned model's training set."""
    from graphgen import patterns as P

    kind, kw = W["queries"]
    seen = training_patterns() if kind == "heldout" else set()
    pats = P.random_patterns(kw["draw"], seed=kw["seed"], kmin=kw["kmin"], kmax=kw["kmax"],
                             accept=lambda k, e: (k, tuple(sorted(e))) not in seen)
    return [("%s-k%d-%d" % (p["family"], p["k"], i), p["k"], p["edges"]) for i, p in enumerate(pats)]


def build_queries(huge, G, W, ws, cap, nslices, learned_plan=None):
    """[(name, k, edges)], their cost-model plans, learned plans (or None), planning
    seconds of the kept learned plans, slice counts and the number of rejected
    patterns.  Named queries take the workload's fixed slice count; random ones are
    drawn in seed order (held-out ones skip the learned model's training patterns)
    and kept when the pilot finds a slice count for all their plans, until the
    workload's count is reached.  learned_plan(k, edges) -> (plan, seconds)."""
    from graphgen import patterns as P

    q = W["queries"]
    if isinstance(q, list):
        qs = [(n,) + tuple(P.NAMED[n]) for n in q]
        lp = [learned_plan(k, e) for _, k, e in qs] if learned_plan else None
        return (qs, [huge.plan(G, k, e) for _, k, e in qs], [x[0] for x in lp] if lp else None,
                sum(x[1] for x in lp) if lp else 0.0, [W["slices"]] * len(qs), 0)
    qs, cms, lps, lsec, slices, rejected = [], [], [], 0.0, [], 0
    for name, k, e in candidate_patterns(W):
        pl = huge.plan(G, k, e)
        lp, ls = learned_plan(k, e) if learned_plan else (None, 0.0)
        S = pilot(huge, G, [pl] + ([lp] if lp else []), W["budget"], ws, cap, nslices)
        log("pilot %s: %s" % (name, "S=2^%d" % (S.bit_length() - 1) if S else "rejected"))
        if S is None:
            rejected += 1
            continue
        qs.append((name, k, e))
        cms.append(pl)
        lps.append(lp)
        lsec += ls
        slices.append(S)
        if len(qs) == q[1]["count"]:
            break
    if len(qs) < q[1]["count"]:
        raise SystemExit("only %d of %d patterns fit the sampling budget" % (len(qs), q[1]["count"]))
    return qs, cms, (lps if learned_plan else None), lsec, slices, rejected


BUSHY = {
    "desc": "Chung-Lu n=16384, mean degree 16, gamma 2.5, exact, seed 1 (the C1 graph): path- and cycle-like "
            "queries, whole; bushy plans of Algorithm 1 (machines 1, and 1e9 so that parts are pushed) vs the "
            "left-deep cost-model plan",
    "graph": ("chung_lu", dict(n=16384, dbar=16, gamma=2.5, seed=1, exact=True)),
    "queries": ["4-path", "tailed-triangle", "diamond", "5-cycle", "house", "6-cycle"],
    "modes": {"cost-model": None, "bushy": 1.0, "bushy-push": 1e9},
}


def bench_bushy(args, huge, torch):
    """The bushy-plan line: every query whole, per mode, timed over the steps;
    all modes must give the oracle's count and hashes."""
    import oracle
    from graphgen import patterns as P

    g = make_graph(BUSHY["graph"])
    G = huge.load(g.row_ptr, g.col)
    qs = [(n,) + tuple(P.NAMED[n]) for n in BUSHY["queries"]]
    plans, trees = {}, {}
    for m, machines in BUSHY["modes"].items():
        if machines is None:
            plans[m] = [huge.plan(G, k, e) for _, k, e in qs]
        else:
            plans[m] = [huge.plan_bushy(G, k, e, machines=machines) for _, k, e in qs]
            trees[m] = {q[0]: [nd["kind"] for nd in p.bushy_nodes()] for q, p in zip(qs, plans[m])}
    # the oracle on the three cheapest queries (the baseline, and a parity check of the first mode there)
    threads = min(16, os.cpu_count() or 1)
    t_o = time.perf_counter()
    oref = {n: oracle.enumerate_query(g.row_ptr, g.col, k, e, threads=threads) for n, k, e in qs[:3]}
    t_o = time.perf_counter() - t_o
    ref = [None] * len(qs)
    res = {}
    for m in BUSHY["modes"]:
        for _ in range(args.warmup):
            for p in plans[m]:
                huge.count(G, p)
        per = [0.0] * len(qs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for i, p in enumerate(plans[m]):
                t1 = time.perf_counter()
                r = huge.count(G, p)
                per[i] += time.perf_counter() - t1
                key = (r["count"], r["hash_sum"], r["hash_xor"])
                if ref[i] is None:
                    ref[i] = key
                    o = oref.get(qs[i][0])
                    if o is not None and key != (o["count"], o["hash_sum"], o["hash_xor"]):
                        raise SystemExit("%s disagrees with the oracle on %s" % (m, qs[i][0]))
                if key != ref[i]:
                    raise SystemExit("%s disagrees with %s on %s" % (m, list(BUSHY["modes"])[0], qs[i][0]))
        torch.cuda.synchronize()
        res[m] = (time.perf_counter() - t0, per)
        log("[%s] %.3f s" % (m, res[m][0]))
    total = sum(r[0] for r in ref)
    main = "bushy"
    el = res[main][0]
    out = {
        "metric": "embeddings/sec, bushy plans (Algorithm 1) vs the left-deep cost-model plan, 1 GPU",
        "value": total * args.steps / el,
        "unit": "embeddings/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": BUSHY["desc"], "mode": main, "n": g.n, "m": g.m, "embeddings_per_step": total,
                   "trees": trees,
                   "modes": {m: {"s": round(res[m][0], 4), "embeddings_per_s": total * args.steps / res[m][0],
                                 "per_query_ms": {q[0]: round(t * 1e3 / args.steps, 3)
                                                  for q, t in zip(qs, res[m][1])}} for m in res},
                   "exactness": "every mode, every step: count, hash_sum and hash_xor equal to the first mode's; "
                                "the first mode's equal to the oracle's on %s" % ", ".join(oref)},
        "roofline": None,
        "cpu_baseline": {"value": sum(o["count"] for o in oref.values()) / t_o, "unit": "embeddings/s",
                         "cores": threads, "kind": "oracle",
                         "sample": "%s, whole, once (%.1f s)" % (", ".join(oref), t_o)},
    }
    print(json.dumps(out), flush=True)


VARIANTS = {
    "desc": "Chung-Lu n=131072, mean degree 12, gamma 2.6, seed 8, whole: motif counts (every connected 3- and "
            "4-vertex pattern, non-induced and induced), labelled queries (4 labels, numpy Philox seed 8), induced "
            "queries, directed queries (the graph oriented, 20% of pairs both ways, seed 8) and hop-constrained "
            "s-t path counts (up to 5 hops)",
    "graph": ("chung_lu", dict(n=131072, dbar=12, gamma=2.6, seed=8)),
    "labels": 4,
    "motif_k": [3, 4],
    "labelled": [("triangle", [0, 1, 2]), ("4-cycle", [0, 1, 0, 1]), ("diamond", [0, 1, 2, 1]),
                 ("house", [0, 1, 2, 3, -1])],
    "induced": ["4-cycle", "4-path", "diamond", "house"],
    "directed": {"cycle3": (3, [(0, 1), (1, 2), (2, 0)]), "transitive3": (3, [(0, 1), (1, 2), (0, 2)]),
                 "bifan": (4, [(0, 2), (0, 3), (1, 2), (1, 3)]), "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
                 "ffl-diamond": (4, [(0, 1), (0, 2), (1, 3), (2, 3), (1, 2)])},
    "path_hops": 5,
    "path_pairs": 3,
    # the oracle on the items it finishes in seconds (the CPU baseline, and the exactness check there)
    "oracle_motifs": ["triangle", "4-clique", "diamond", "4-cycle", "tailed-triangle"],
}


def bench_variants(args, huge, torch):
    """The line of the paper's variants on the same kernels: every item whole,
    timed over the steps, each step's results equal to the first step's; the
    oracle checks the items it finishes in seconds (and is their CPU baseline);
    the roofline is the dominant kernel class of a profiled pass over the
    level-engine items (labelled, induced and directed queries)."""
    import numpy as np

    import graphgen as gg
    import oracle
    from graphgen import patterns as P

    V = VARIANTS
    g = make_graph(V["graph"])
    rng = np.random.Generator(np.random.Philox(V["graph"][1]["seed"]))
    labels = rng.integers(0, V["labels"], g.n).astype(np.int32)
    d = gg.orient(g, 0.2, seed=V["graph"][1]["seed"])
    G = huge.load(g.row_ptr, g.col)
    GL = huge.load(g.row_ptr, g.col, labels=labels)
    GD = huge.load_directed(d.out_rp, d.out_col)
    deg = np.diff(g.row_ptr)
    # s-t pairs: vertices of middle degree, seeded
    mid = np.flatnonzero((deg >= 8) & (deg <= 16))
    pairs = [tuple(int(x) for x in rng.choice(mid, 2, replace=False)) for _ in range(V["path_pairs"])]

    items = []  # (name, kind, run() -> (embeddings, key), oracle() -> key or None)
    for k in V["motif_k"]:
        def run_m(k=k):
            out = huge.motif_count(G, k)
            return sum(m["noninduced"] for m in out), tuple((m["noninduced"], m["induced"], m["hash_sum"],
                                                             m["hash_xor"]) for m in out)
        items.append(("motifs-k%d" % k, "motif", run_m))
    lvl = []
    for name, ql in V["labelled"]:
        k, e = P.NAMED[name]
        lvl.append(("labelled-" + name, GL, huge.plan(GL, k, e, labels=ql),
                    dict(vlabels=labels, qlabels=np.asarray(ql, dtype=np.int32)), k, e, False))
    for name in V["induced"]:
        k, e = P.NAMED[name]
        lvl.append(("induced-" + name, G, huge.plan(G, k, e, induced=True), dict(induced=True), k, e, False))
    for name, (k, e) in V["directed"].items():
        lvl.append(("directed-" + name, GD, huge.plan_directed(GD, k, e), None, k, e, True))
    for name, GG, pl, okw, k, e, directed in lvl:
        def run_q(GG=GG, pl=pl):
            r = huge.count(GG, pl)
            return r["count"], (r["count"], r["hash_sum"], r["hash_xor"])
        items.append((name, "query", run_q))
    for s_, t_ in pairs:
        def run_p(s_=s_, t_=t_):
            c = huge.count_paths(G, s_, t_, V["path_hops"])
            return sum(c), tuple(c)
        items.append(("paths-%d-%d" % (s_, t_), "paths", run_p))

    ref, per = {}, {}
    for _ in range(args.warmup):
        for name, _, run in items:
            run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    emb = 0
    for _ in range(args.steps):
        for name, _, run in items:
            t1 = time.perf_counter()
            n, key = run()
            per[name] = per.get(name, 0.0) + time.perf_counter() - t1
            emb += n
            if ref.setdefault(name, key) != key:
                raise SystemExit("%s changed between steps" % name)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log("[variants] %.3f s for %d steps" % (el, args.steps))

    # the oracle: the cheap motif patterns (non-induced, whole), every labelled and directed query, the
    # induced 4-cycle and diamond, and the path counts (each length a pinned all-maps path query)
    threads = min(16, os.cpu_count() or 1)
    checked, o_emb, t_o = [], 0, time.perf_counter()
    motifs = {k: huge.motif_count(G, k) for k in V["motif_k"]}
    for name in V["oracle_motifs"]:
        k, e = P.NAMED[name]
        r = oracle.enumerate_query(g.row_ptr, g.col, k, e, threads=threads)
        key = oracle.iso_key(k, e)
        hit = [m for m in motifs[k] if oracle.iso_key(k, m["edges"]) == key]
        if len(hit) != 1 or (hit[0]["noninduced"], hit[0]["hash_sum"], hit[0]["hash_xor"]) != \
                (r["count"], r["hash_sum"], r["hash_xor"]):
            raise SystemExit("motif %s disagrees with the oracle" % name)
        checked.append("motif " + name)
        o_emb += r["count"]
    for name, GG, pl, okw, k, e, directed in lvl:
        if name.startswith("induced-") and name not in ("induced-4-cycle", "induced-diamond"):
            continue
        if directed:
            r = oracle.enumerate_directed(d.row_ptr, d.col, d.out_rp, d.out_col, k, e, threads=threads)
        else:
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, threads=threads, **okw)
        if ref[name] != (r["count"], r["hash_sum"], r["hash_xor"]):
            raise SystemExit("%s disagrees with the oracle: %s vs %s" % (name, ref[name], r["count"]))
        checked.append(name)
        o_emb += r["count"]
    rk = oracle.ranks(g.row_ptr)
    for s_, t_ in pairs:
        want = [0]
        for L in range(1, V["path_hops"] + 1):
            e = [(i, i + 1) for i in range(L)]
            r = oracle.enumerate_query(g.row_ptr, g.col, L + 1, e, mode=oracle.MODE_ALL, order=list(range(L + 1)),
                                       slice_count=g.n, slice_id=int(rk[s_]), slice_vertex=0, slice_mode=1,
                                       slice2=(L, g.n, int(rk[t_])), ranks=rk, threads=threads)
            want.append(r["count"])
        if tuple(want) != ref["paths-%d-%d" % (s_, t_)]:
            raise SystemExit("paths %d-%d disagree with the oracle: %s vs %s" % (s_, t_, ref["paths-%d-%d" % (s_, t_)], want))
        checked.append("paths-%d-%d" % (s_, t_))
        o_emb += sum(want)
    t_o = time.perf_counter() - t_o

    # profiled pass over the level-engine items: the dominant kernel class against the HBM roof
    kms, kl, kb = [0.0] * 4, [0] * 4, [0.0] * 4
    for name, GG, pl, okw, k, e, directed in lvl:
        r = huge.count(GG, pl, profile=True)
        for c in range(4):
            kms[c] += r["kernel_ms"][c]
            kl[c] += r["kernel_launches"][c]
            kb[c] += r["alg_bytes"][c]
    dom = max(range(4), key=lambda c: kms[c])
    avg_ms = kms[dom] / max(1, kl[dom])
    bpl = kb[dom] / max(1, kl[dom])
    ach = (bpl / (avg_ms * 1e-3)) / 1e9 if avg_ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": KC_KERNELS[dom] + ", level engine; profiled pass over the labelled, induced and directed "
                      "queries", "avg_launch_ms": round(avg_ms, 4), "alg_bytes_per_launch": bpl, "launches": kl[dom],
            "kernel_ms_by_class": {KC_NAMES[c]: round(kms[c], 3) for c in range(4)},
            "launches_by_class": {KC_NAMES[c]: kl[c] for c in range(4)}}
    out = {
        "metric": "embeddings/sec, the paper's variants (motifs, labelled, induced, directed, s-t paths), 1 GPU",
        "value": emb / el,
        "unit": "embeddings/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": V["desc"], "n": g.n, "m": g.m, "arcs": int(d.out_rp[-1]), "path_pairs": pairs,
                   "embeddings_per_step": emb // args.steps,
                   "per_item_ms": {name: round(per[name] * 1e3 / args.steps, 3) for name, _, _ in items},
                   "per_item_embeddings": {name: (ref[name][0] if kind == "query" else
                                                  sum(ref[name]) if kind == "paths" else
                                                  sum(x[0] for x in ref[name])) for name, kind, _ in items},
                   "motifs": {"k%d" % k: [{"edges": m["edges"], "noninduced": m["noninduced"],
                                           "induced": m["induced"]} for m in motifs[k]] for k in motifs},
                   "path_counts": {"%d-%d" % pq: list(ref["paths-%d-%d" % pq]) for pq in pairs},
                   "exactness": "every item, every step: equal to the first step; equal to the oracle on " +
                                ", ".join(checked)},
        "roofline": roof,
        "cpu_baseline": {"value": o_emb / t_o if t_o > 0 else 0.0, "unit": "embeddings/s", "cores": threads,
                         "kind": "oracle", "sample": "the checked items above, whole, once (%.1f s)" % t_o},
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(g, queries, orders, slices, steps, budget_s, threads):
    """The oracle, as it stands, on the slices the GPU times (each query's cost-model
    order and strided slice s of S_q, s = 0, 1, ...), until the time budget."""
    import oracle

    t_rank = time.perf_counter()
    ranks = oracle.ranks(g.row_ptr)
    t_rank = time.perf_counter() - t_rank
    tot_cnt, tot_t, runs = 0, 0.0, 0
    s = 0
    t_end = time.perf_counter() + budget_s
    while time.perf_counter() < t_end and s < max(1, steps):
        for (name, k, e), o, S in zip(queries, orders, slices):
            if time.perf_counter() >= t_end:
                break
            t0 = time.perf_counter()
            kw = {} if S <= 1 else dict(slice_count=S, slice_id=s % S, slice_vertex=o[0], slice_mode=1)
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, order=o, threads=threads, ranks=ranks, **kw)
            tot_t += time.perf_counter() - t0
            tot_cnt += r["count"]
            runs += 1
        s += 1
    return {
        "value": tot_cnt / tot_t if tot_t > 0 else 0.0,
        "unit": "embeddings/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "the GPU's timed slices in step order (each query's cost-model order, root slice s of its "
                  "S_q): %d oracle runs over steps 0..%d, %d embeddings in %.1f s (degree ranks computed once, "
                  "%.1f s, not counted)" % (runs, s - 1, tot_cnt, tot_t, t_rank),
    }


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
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS) + ["bushy", "variants"])
    ap.add_argument("--modes", default=None, help="comma-separated subset of the workload's modes")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--model", default=MODEL_PATH, help="learned cost model (.npz)")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="skip autotuning the per-bucket dispatch before timing (library default kernels)")
    ap.add_argument("--profile-steps", type=int, default=2, help="steps of the profiled pass (roofline)")
    ap.add_argument("--cap", type=float, default=None, help="frontier cap in bytes (default: the workload's)")
    ap.add_argument("--budget", type=float, default=None,
                    help="candidates a sampled slice may examine (default: the workload's)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the 4 GiB device copy (counter calibration) and print its bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (see the sharding design); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2103_14294_amd as huge

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    if args.copy_only:
        gbs, moved = copy_bandwidth(torch)
        print(json.dumps({"copy_gbs": round(gbs, 1), "bytes_per_copy": moved, "copies": 6}), flush=True)
        return
    if args.workload == "bushy":
        bench_bushy(args, huge, torch)
        return
    if args.workload == "variants":
        bench_variants(args, huge, torch)
        return
    W = dict(WORKLOADS[args.workload])
    if args.budget is not None:
        W["budget"] = args.budget
    modes = args.modes.split(",") if args.modes else list(W["modes"])
    t0 = time.perf_counter()
    g = make_graph(W["graph"])
    log("graph %s: n=%d m=%d (%.1f s to generate)" % (args.workload, g.n, g.m, time.perf_counter() - t0))
    G = huge.load(g.row_ptr, g.col)
    info = G.info()
    log("loaded on GPU in %.1f ms (max degree %d)" % (info["load_ms"], info["max_degree"]))
    ws = huge.Workspace()
    cap = int(args.cap) if args.cap is not None else W["cap"]
    # the query selection checks every plan the workload compares, whichever modes this run times, so
    # a run of a subset of the modes (a profiling pass) times the same queries on the same slices
    model = huge.Model.load(args.model) if any(m.startswith("learned") for m in list(W["modes"]) + modes) \
        else None

    def learned_plan(k, e):
        torch.cuda.synchronize()
        t_p = time.perf_counter()
        p = huge.plan(G, k, e, learned=model, verify=True)
        torch.cuda.synchronize()
        return p, time.perf_counter() - t_p

    t_q = time.perf_counter()
    nslices = args.steps + args.warmup
    pc = os.environ.get("HUGE_PILOT_CACHE")  # reuse a previous run's query selection (profiling passes)
    pkey = "%s|%d|%s|%g" % (args.workload, nslices, ",".join(W["modes"]), W.get("budget", 0))
    pcd = json.load(open(pc)) if pc and os.path.exists(pc) else {}
    if pkey in pcd:
        d = pcd[pkey]
        queries = [(n, k, [tuple(x) for x in e]) for n, k, e in d["queries"]]
        cm_plans = [huge.plan(G, k, e) for _, k, e in queries]
        lp = [learned_plan(k, e) for _, k, e in queries] if model is not None else None
        l_plans, l_sec = ([x[0] for x in lp], sum(x[1] for x in lp)) if lp else (None, 0.0)
        slices, rejected = d["slices"], d["rejected"]
    else:
        queries, cm_plans, l_plans, l_sec, slices, rejected = build_queries(
            huge, G, W, ws, cap, nslices, learned_plan if model is not None else None)
        if pc:
            pcd[pkey] = {"queries": queries, "slices": slices, "rejected": rejected}
            with open(pc, "w") as f:
                json.dump(pcd, f)
    log("%d queries (%d drawn patterns rejected: no slice count up to 2^24 fits the budget), %.1f s; "
        "slices per query: %s" % (len(queries), rejected, time.perf_counter() - t_q, slices))

    tune_info, table = None, None
    if args.tune:
        t_t = time.perf_counter()
        # sample: root slice 1 of the largest S_q, for the first 8 queries
        table = huge.autotune(G, cm_plans[:8], cache=os.environ.get("HUGE_TUNE_CACHE"),
                              slice_count=max(slices), slice_id=1, slice_mode=huge.SLICE_STRIDE, cap=cap, **SLICE)
        tune_info = {"tune_s": round(time.perf_counter() - t_t, 2),
                     "strategy": {str(j): table.to_dict()["strategy"][j] for j in range(huge.KMAX + 1)
                                  if any(table.items[j][c] for c in range(huge.TUNE_BUCKETS))},
                     "chunk_rows": {str(j): table.chunk_rows[j] for j in range(huge.KMAX + 1) if table.chunk_rows[j]}}
        log("autotuned in %.1f s: %s" % (tune_info["tune_s"], json.dumps(tune_info)))

    plans = {"cost-model": cm_plans}
    plan_s = {"cost-model": 0.0}
    if model is not None:
        plans["learned"] = l_plans
        plan_s["learned"] = l_sec
        log("learned planning: %.2f s for %d queries" % (plan_s["learned"], len(queries)))

    kw = dict(cap=cap, tune=table, hash=True)

    groups = {}  # queries with equal S_q: one batched call per step
    for i, S in enumerate(slices):
        groups.setdefault(S, []).append(i)

    def run_step(mode, step, acc, profile=False):
        base = mode.replace("-batched", "")
        pl = plans[base]
        rs = [None] * len(pl)
        unit_s = acc.setdefault("_unit_s", {})  # seconds per timing unit (a query, or a batch of equal S_q)
        if mode.endswith("-batched"):
            for S, idx in groups.items():
                t0 = time.perf_counter()
                out = huge.count_batch(G, [pl[i] for i in idx], engine=huge.ENGINE_GRAPH, workspace=ws,
                                       slice_count=S, slice_id=slice_of(step, S), slice_mode=huge.SLICE_STRIDE,
                                       **SLICE, **kw)
                unit_s[("g", S)] = unit_s.get(("g", S), 0.0) + time.perf_counter() - t0
                for i, r in zip(idx, out):
                    rs[i] = r
        else:
            for i, (p, S) in enumerate(zip(pl, slices)):
                t0 = time.perf_counter()
                rs[i] = huge.count(G, p, workspace=ws, profile=profile, slice_count=S, slice_id=slice_of(step, S),
                                   slice_mode=huge.SLICE_STRIDE, **SLICE, **kw)
                unit_s[("q", i)] = unit_s.get(("q", i), 0.0) + time.perf_counter() - t0
        for i, r in enumerate(rs):
            a = acc.setdefault(i, {"count": 0, "ms": 0.0, "keys": []})
            a["count"] += r["count"]
            a["ms"] += r["query_ms"]
            a["keys"].append((r["count"], r["hash_sum"], r["hash_xor"]))
            acc["_peak"] = max(acc.get("_peak", 0), r["peak_frontier_bytes"])
            if profile:
                for c in range(4):
                    acc["_kms"][c] += r["kernel_ms"][c]
                    acc["_kl"][c] += r["kernel_launches"][c]
                    acc["_kb"][c] += r["alg_bytes"][c]

    results = {}
    for m in modes:
        for i in range(args.warmup):  # warmup on the slices after the timed ones: none is seen twice
            run_step(m, args.steps + i, {})
            log("warmup [%s] %d done" % (m, i))
        acc = {}
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            run_step(m, s_, acc)
            log("step %d [%s] done" % (s_, m))
        torch.cuda.synchronize()
        results[m] = (acc, time.perf_counter() - t_start)
        log("[%s] %.3f s, %d embeddings" % (m, results[m][1], sum(acc[i]["count"] for i in range(len(queries)))))

    # the same slices give the same matches in every mode of one plan
    for m in modes:
        base = m.replace("-batched", "")
        other = base if m.endswith("-batched") else base + "-batched"
        if other in results:
            for i in range(len(queries)):
                if results[m][0][i]["keys"] != results[other][0][i]["keys"]:
                    raise SystemExit("modes %s and %s disagree on %s" % (m, other, queries[i][0]))

    # exactness of the learned plans: a shared double slice per query
    exact = None
    if "learned" in plans:
        ok = nonzero = 0
        for i, ((name, k, e), pc, pl_) in enumerate(zip(queries, plans["cost-model"], plans["learned"])):
            oc, ol = pc.info()["order"], pl_.info()["order"]
            S = slices[i]
            if oc[0] == ol[0]:
                a = huge.count(G, pc, workspace=ws, slice_count=S, slice_id=0, slice_mode=huge.SLICE_STRIDE,
                               cap=cap, **SLICE)
                b = huge.count(G, pl_, workspace=ws, slice_count=S, slice_id=0, slice_mode=huge.SLICE_STRIDE,
                               cap=cap, **SLICE)
            else:
                a = huge.count(G, pc, workspace=ws, slice_count=S, slice_id=0, slice_mode=huge.SLICE_STRIDE,
                               slice2=(ol[0], S, 1), cap=cap, **SLICE)
                b = huge.count(G, pl_, workspace=ws, slice_count=S, slice_id=1, slice_mode=huge.SLICE_STRIDE,
                               slice2=(oc[0], S, 0), cap=cap, **SLICE)
            ka, kb = (a["count"], a["hash_sum"], a["hash_xor"]), (b["count"], b["hash_sum"], b["hash_xor"])
            if ka != kb:
                raise SystemExit("learned and cost-model plans disagree on %s: %s vs %s" % (name, ka, kb))
            ok += 1
            nonzero += ka[0] > 0
        exact = "%d of %d queries (%d with matches in the sample): equal count, hash_sum and hash_xor on a " \
                "shared sample, root slice 0 of S_q of the cost-model plan's first vertex and root slice 1 of " \
                "S_q of the learned plan's (slice 0 of both when they start at the same vertex), each plan " \
                "reading only its own slice's entries" % (ok, len(queries), nonzero)

    # profiled pass (roofline): the cost-model mode's kernels with HIP events, same slices
    prof = {"_kms": [0.0] * 4, "_kl": [0] * 4, "_kb": [0.0] * 4}
    for s_ in range(min(args.profile_steps, args.steps)):
        run_step("cost-model", s_, prof, profile=True)
    kms, kl, kb = prof["_kms"], prof["_kl"], prof["_kb"]
    dom = max(range(4), key=lambda c: kms[c])
    avg_ms = kms[dom] / max(1, kl[dom])
    bytes_per_launch = kb[dom] / max(1, kl[dom])
    achieved = (bytes_per_launch / (avg_ms * 1e-3)) / 1e9 if avg_ms > 0 else 0.0
    traffic = recorded_traffic(args.workload, bytes_per_launch) if table is not None else None
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_gbs": round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic and avg_ms > 0 else None,
            "traffic_frac": round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic and avg_ms > 0
            else None,
            "achieved_is": "algorithmic bytes (merge intersection over symmetry-breaking-trimmed lists) per launch / "
                           "average launch time; traffic is measured HBM bytes per launch",
            "kernel": KC_KERNELS[dom] + ", level engine, tuned per-bucket dispatch; profiled pass of the "
                      "cost-model mode over the same slices",
            "avg_launch_ms": round(avg_ms, 4), "alg_bytes_per_launch": bytes_per_launch, "launches": kl[dom],
            "sources_sha256_16": sources_digest(),
            "kernel_ms_by_class": {KC_NAMES[c]: round(kms[c], 3) for c in range(4)},
            "launches_by_class": {KC_NAMES[c]: kl[c] for c in range(4)},
            "alg_bytes_by_class": {KC_NAMES[c]: kb[c] for c in range(4)}}

    # Whole-query estimates.  Slice s of S_q is an unbiased 1/S_q sample of a
    # query's matches and of its plan's work, so over K sampled slices a query's
    # whole count is S_q * (sampled count) / K and its whole run time S_q *
    # (sampled seconds) / K; planning is paid once per query.  A mode's query
    # time is its planning plus those run times (per batch of equal S_q for the
    # batched modes); the workload's embeddings are pooled over the distinct
    # plans' samples (each estimates the same matches).
    K = args.steps
    nq = len(queries)
    est_emb = {}
    for m in modes:
        b_ = m.replace("-batched", "")
        est_emb[b_] = sum(slices[i] * results[m][0][i]["count"] for i in range(nq)) / K
    pooled = sum(est_emb.values()) / len(est_emb)
    est_time = {}
    for m in modes:
        us = results[m][0].get("_unit_s", {})
        run_s = sum((u[1] if u[0] == "g" else slices[u[1]]) * t for u, t in us.items()) / K
        est_time[m] = plan_s.get(m.replace("-batched", ""), 0.0) + run_s
    main_mode = modes[-1]
    acc, elapsed = results[main_mode]
    cfg = {"workload": W["desc"], "mode": main_mode, "n": g.n, "m": g.m, "queries": nq,
           "slices": "per query: root slice `step` of S_q (first matched vertex of degree rank r with "
                     "r mod S_q == step); S_q = %s"
                     % json.dumps(dict(zip([q[0] for q in queries], slices))) if nq <= 64
           else "per query", "frontier_cap_bytes": cap, "peak_frontier_bytes": acc.get("_peak", 0),
           "graph_load_ms": info["load_ms"], "patterns_rejected_by_pilot": rejected,
           "value_is": "scaled embeddings (S_q x sampled count / steps per query, pooled over the distinct "
                       "plans' samples) / scaled query time of the mode (planning once per query + S_q x sampled "
                       "seconds / steps): the sampled rate with planning charged in proportion to the sampled "
                       "fraction",
           "estimated_embeddings": pooled,
           "estimated_embeddings_by_plan": est_emb}
    if tune_info:
        cfg["autotune"] = tune_info
    mstat = {}
    for m in modes:
        a, el = results[m]
        pt = plan_s.get(m.replace("-batched", ""), 0.0)
        cnt = sum(a[i]["count"] for i in range(nq))
        mstat[m] = {"estimated_query_time_s": round(est_time[m], 3), "planning_s": round(pt, 4),
                    "embeddings_per_s": pooled / est_time[m] if est_time[m] > 0 else 0.0,
                    "sampled": {"timed_s": round(el, 4), "embeddings": cnt,
                                "embeddings_per_s": cnt / el if el > 0 else 0.0,
                                "ms_per_step": round(el * 1e3 / K, 3)}}
    cfg["modes"] = mstat
    if len(modes) > 1:
        cmpd = {"query_time_ratio_vs_" + modes[0]: {m: round(est_time[modes[0]] / max(1e-12, est_time[m]), 4)
                                                     for m in modes[1:]}}
        if "learned" in results:
            ratios, per, changed = [], {}, 0
            for i, (name, k, e) in enumerate(queries):
                t_c = slices[i] * results["cost-model"][0]["_unit_s"][("q", i)] / K
                t_l = slices[i] * results["learned"][0]["_unit_s"][("q", i)] / K
                ratios.append(t_c / max(t_l, 1e-12))
                oc, ol = plans["cost-model"][i].info()["order"], plans["learned"][i].info()["order"]
                changed += oc != ol
                per[name] = {"order_cost_model": oc, "order_learned": ol, "S": slices[i],
                             "est_s_cost_model": round(t_c, 2), "est_s_learned": round(t_l, 2),
                             "segment_rows_learned": huge.segment_rows(G, plans["learned"][i], cap=cap, tune=table)[2:k]}
            cmpd["learned_vs_cost_model_per_query_geomean"] = round(math.exp(sum(math.log(r) for r in ratios) /
                                                                             len(ratios)), 4)
            cmpd["orders_changed"] = changed
            cmpd["exactness"] = exact
            cmpd["per_query"] = per
        cfg["compare"] = cmpd
    out = {
        "metric": "embeddings/sec + query time, learned/batched vs cost-model plan, 1 GPU",
        "value": pooled / est_time[main_mode] if est_time[main_mode] > 0 else 0.0,
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
    out["roofline"]["frac_of_copy"] = round(achieved / gbs, 4) if gbs > 0 else None
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        log("cpu baseline: oracle on the timed slices, %d threads, budget %.0f s" % (threads, args.cpu_budget))
        out["cpu_baseline"] = cpu_baseline(g, queries, [p.info()["order"] for p in plans["cost-model"]], slices,
                                           args.steps, args.cpu_budget, threads)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
