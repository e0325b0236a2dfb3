"""huge_count_noalloc through the C ABI: the entry point that runs inside the
library's own file-scope device array gives huge_count's results bit for bit,
on two calls in a row where the second has a smaller input (the array keeps
the first call's contents), and rejects options it cannot hold."""
import ctypes

import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    return need_gpu()


def _noalloc(H, G, p, **kw):
    """Direct C-ABI call (ctypes), no workspace."""
    lib = H.load_library()
    o = H.exec_opts(**kw)
    r = H.Result()
    st = lib.huge_count_noalloc(G.handle, p.handle, ctypes.byref(o), ctypes.byref(r))
    if st not in (0, 1):
        raise H.HugeError(st, lib.huge_last_error().decode())
    return r.to_dict()


def test_noalloc_matches_huge_count_on_two_calls(H):
    big = gg.rmat(15, 16, seed=61)
    small = gg.chung_lu(3000, 8, 2.4, seed=62)
    Gb, Gs = H.load(big.row_ptr, big.col), H.load(small.row_ptr, small.col)
    kw = dict(cap=64 << 20, chunk_rows=1 << 18)
    cases = [(Gb, "house", {}), (Gs, "diamond", {}),  # second call: smaller graph and query
             (Gb, "5-clique", dict(slice_count=16, slice_id=5, slice_vertex=-1, slice_mode=H.SLICE_STRIDE)),
             (Gs, "triangle", dict(slice_count=3, slice_id=1, slice_vertex=-1))]
    for G, name, sl in cases:
        p = H.plan(G, *P.NAMED[name])
        k = P.NAMED[name][0]
        print("noalloc %s %s" % (name, sl), flush=True)
        got = _noalloc(H, G, p, **kw, **sl)
        want = H.count(G, p, **kw, **sl)
        assert cmp_key(got, k) == cmp_key(want, k), name
        assert got["level_counts"][:k] == want["level_counts"][:k], name
        assert got["peak_frontier_bytes"] <= 64 << 20
    # the same call again after a larger one gives the same result
    p = H.plan(Gs, *P.NAMED["diamond"])
    assert cmp_key(_noalloc(H, Gs, p, **kw), 4) == cmp_key(H.count(Gs, p, **kw), 4)


def test_noalloc_tuned_table(H):
    g = gg.rmat(13, 16, seed=63)
    G = H.load(g.row_ptr, g.col)
    plans = [H.plan(G, *P.NAMED[n]) for n in ["diamond", "4-clique"]]
    t = H.autotune(G, plans, slice_count=4, slice_id=3, slice_vertex=-1)
    for p in plans:
        got = _noalloc(H, G, p, cap=32 << 20, chunk_rows=1 << 16, tune=t)
        want = H.count(G, p, cap=32 << 20, chunk_rows=1 << 16, tune=t)
        assert cmp_key(got, p.k) == cmp_key(want, p.k)


def test_noalloc_rejects_what_it_cannot_hold(H):
    g = gg.chung_lu(2000, 8, 2.4, seed=64)
    G = H.load(g.row_ptr, g.col)
    p = H.plan(G, *P.NAMED["house"])
    assert H.noalloc_capacity() == 256 << 20
    with pytest.raises(H.HugeError) as e:
        _noalloc(H, G, p, cap=1 << 30)
    assert e.value.name == "HUGE_ENOMEM"
    for bad in [dict(profile=True), dict(engine=H.ENGINE_GRAPH), dict(cap=float("inf"))]:
        with pytest.raises(H.HugeError) as e:
            _noalloc(H, G, p, **bad)
        assert e.value.name == "HUGE_EINVAL", bad
    ws = H.Workspace()
    import torch
    buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    o = H.exec_opts(cap=1 << 20)
    o.workspace, o.workspace_bytes = buf.data_ptr(), buf.numel()
    r = H.Result()
    assert H.load_library().huge_count_noalloc(G.handle, p.handle, ctypes.byref(o), ctypes.byref(r)) == -1
