"""Motif counting (every connected k-vertex pattern, non-induced and induced)
against the definitions: brute force over every k-vertex set of small graphs,
the oracle's per-pattern counts and hashes, and closed forms (in K_n only the
k-clique occurs induced, C(n, k) times; in a cycle C_n only the k-path, n times)."""
import math

import pytest

import graphgen as gg
import oracle
from tests.gpu_common import need_gpu

pytestmark = pytest.mark.gpu

N_CLASSES = {2: 1, 3: 2, 4: 6, 5: 21, 6: 112}


@pytest.fixture(scope="module")
def H():
    return need_gpu()


def _by_key(res, k):
    return {oracle._iso_key(k, m["edges"]): m for m in res}


@pytest.mark.parametrize("k", [3, 4, 5])
@pytest.mark.parametrize("engine", ["levels", "graph"])
def test_motifs_match_brute_force(H, k, engine):
    for seed, n, p in [(3, 11, 0.45), (4, 12, 0.3)]:
        g = gg.gnp(n, p, seed=seed)
        G = H.load(g.row_ptr, g.col)
        res = H.motif_count(G, k, engine=H.ENGINE_GRAPH if engine == "graph" else H.ENGINE_LEVELS)
        assert len(res) == N_CLASSES[k]
        want = oracle.motif_counts(g.row_ptr, g.col, k)
        got = _by_key(res, k)
        for key, m in got.items():
            assert (m["noninduced"], m["induced"]) == want.get(key, (0, 0)), (seed, key)


def test_motifs_match_the_oracle_per_pattern(H):
    g = gg.chung_lu(1500, 8, 2.4, seed=71)
    G = H.load(g.row_ptr, g.col)
    res = H.motif_count(G, 5, engine=H.ENGINE_GRAPH)
    for m in res:
        ref = oracle.enumerate_query(g.row_ptr, g.col, 5, m["edges"])
        assert (m["noninduced"], m["hash_sum"], m["hash_xor"]) == (ref["count"], ref["hash_sum"], ref["hash_xor"])
        ind = oracle.enumerate_query(g.row_ptr, g.col, 5, m["edges"], induced=True)
        assert m["induced"] == ind["count"], m["edges"]


def test_motif_closed_forms(H):
    K = gg.complete(9)
    G = H.load(K.row_ptr, K.col)
    for k in (3, 4, 5, 6):
        res = H.motif_count(G, k)
        for m in res:
            clique = m["n_edges"] if "n_edges" in m else len(m["edges"])
            full = len(m["edges"]) == k * (k - 1) // 2
            assert m["induced"] == (math.comb(9, k) if full else 0), (k, m["edges"])
    C = gg.cycle(10)
    Gc = H.load(C.row_ptr, C.col)
    for k in (3, 4, 5, 6):
        res = H.motif_count(Gc, k)
        for m in res:
            is_path = len(m["edges"]) == k - 1 and max(sum(1 for e in m["edges"] if v in e) for v in range(k)) <= 2
            assert m["induced"] == (10 if is_path else 0), (k, m["edges"])
            assert m["noninduced"] == (10 if is_path else 0), (k, m["edges"])


def test_motif_errors(H):
    g = gg.gnp(10, 0.4, seed=5)
    G = H.load(g.row_ptr, g.col)
    for bad in [dict(k=7), dict(k=1), dict(k=4, slice_count=2, slice_id=1)]:
        k = bad.pop("k")
        with pytest.raises(H.HugeError):
            H.motif_count(G, k, **bad)
