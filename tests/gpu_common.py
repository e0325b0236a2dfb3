"""Helpers shared by the GPU test modules."""
import numpy as np
import pytest

import oracle


def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_14294_amd as H

    H.load_library()
    return H


def cmp_key(r, k):
    return (r["count"], r["hash_sum"], r["hash_xor"])


def oracle_run(g, k, e, order=None, **kw):
    return oracle.enumerate_query(g.row_ptr, g.col, k, e, order=order, **kw)


def assert_parity(H, G, g, k, e, order=None, levels=True, **kw):
    """GPU count/hash (and level counts for the plan's order) equal the oracle's."""
    p = H.plan(G, k, e, order=order)
    used = p.info()["order"]
    r = H.count(G, p, **kw)
    okw = {}
    if kw.get("slice_count", 1) > 1:
        okw = {"slice_count": kw["slice_count"], "slice_id": kw.get("slice_id", 0),
               "slice_vertex": kw.get("slice_vertex", 0)}
    ref = oracle_run(g, k, e, order=used, **okw)
    assert cmp_key(r, k) == cmp_key(ref, k), (k, e, used, r, ref)
    if levels:
        assert r["level_counts"][:k] == ref["level_counts"][:k], (k, e, used, r["level_counts"], ref["level_counts"])
    return r, ref
