"""Whole-graph pattern counts from adjacency-matrix identities (scipy.sparse).

These are independent of any enumerator: they come from walk counting.
* triangles  = trace(A^3) / 6
* 4-cycles   = (trace(A^4) - 2 * sum_i d_i^2 + sum_i d_i) / 8
  (closed 4-walks: d_i^2 back-and-forth walks from i over two neighbours,
  sum_{j in N(i)} (d_j - 1) walks i-j-k-j-i, and 8 per 4-cycle)
* diamonds   = sum over undirected edges (u,v) of C(t_uv, 2), t_uv = (A^2)_uv
  (a diamond is fixed by its chord and the two common neighbours of the chord)
"""
import numpy as np
import scipy.sparse as sp


def adjacency(csr):
    n = csr.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(csr.row_ptr))
    data = np.ones(csr.nnz, dtype=np.int64)
    return sp.csr_matrix((data, (rows, csr.col.astype(np.int64))), shape=(n, n))


def triangles(csr):
    A = adjacency(csr)
    A2 = A @ A
    return int(A2.multiply(A).sum()) // 6


def four_cycles(csr):
    A = adjacency(csr)
    A2 = A @ A
    tr4 = int(A2.multiply(A2).sum())
    d = np.diff(csr.row_ptr).astype(np.int64)
    v = tr4 - 2 * int((d * d).sum()) + int(d.sum())
    assert v % 8 == 0
    return v // 8


def diamonds(csr):
    A = adjacency(csr)
    A2 = A @ A
    t = A2.multiply(A).tocoo()
    vals = t.data.astype(np.int64)
    # each undirected edge appears twice
    return int((vals * (vals - 1) // 2).sum()) // 2
