"""Query patterns: the named ones and a seeded random generator.

Patterns are (k, edges) with query vertices 0..k-1.  The random generator
draws from the families used for the batched and learned-plan workloads:
paths, cycles, cliques, chorded cycles and random connected graphs, with k
uniform in [kmin, kmax], relabels vertices by a seeded permutation and drops
isomorphic duplicates (brute-force canonical form).  Uses Python's own
Mersenne-Twister ``random.Random(seed)``; contains no part of the
enumeration method.
"""
from __future__ import annotations

import itertools
import random

NAMED = {
    "edge": (2, [(0, 1)]),
    "wedge": (3, [(0, 1), (1, 2)]),
    "triangle": (3, [(0, 1), (1, 2), (0, 2)]),
    "4-path": (4, [(0, 1), (1, 2), (2, 3)]),
    "3-star": (4, [(0, 1), (0, 2), (0, 3)]),
    "4-cycle": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "tailed-triangle": (4, [(0, 1), (1, 2), (0, 2), (2, 3)]),
    "diamond": (4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]),
    "4-clique": (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]),
    "5-cycle": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]),
    "house": (5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4)]),
    "5-clique": (5, [(a, b) for a in range(5) for b in range(a + 1, 5)]),
    "6-cycle": (6, [(i, (i + 1) % 6) for i in range(6)]),
    "6-clique": (6, [(a, b) for a in range(6) for b in range(a + 1, 6)]),
}


def canonical_form(k, edges):
    """Lexicographically smallest sorted edge tuple over all relabellings."""
    best = None
    for p in itertools.permutations(range(k)):
        t = tuple(sorted((min(p[a], p[b]), max(p[a], p[b])) for a, b in edges))
        if best is None or t < best:
            best = t
    return best


def is_connected(k, edges):
    adj = {v: set() for v in range(k)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    seen = {0}
    stack = [0]
    while stack:
        a = stack.pop()
        for b in adj[a]:
            if b not in seen:
                seen.add(b)
                stack.append(b)
    return len(seen) == k


def _family(rng, k):
    fam = rng.choice(["path", "cycle", "clique", "chorded", "random"])
    if fam == "cycle" and k < 3:
        fam = "path"
    if fam == "chorded" and k < 4:
        fam = "cycle"
    if fam == "path":
        e = [(i, i + 1) for i in range(k - 1)]
    elif fam == "cycle":
        e = [(i, (i + 1) % k) for i in range(k)]
    elif fam == "clique":
        e = [(a, b) for a in range(k) for b in range(a + 1, k)]
    elif fam == "chorded":
        e = [(i, (i + 1) % k) for i in range(k)]
        chords = [(a, b) for a in range(k) for b in range(a + 2, k) if not (a == 0 and b == k - 1)]
        c = rng.randint(1, max(1, k - 3))
        rng.shuffle(chords)
        e += chords[:c]
    else:
        e = [(rng.randrange(i), i) for i in range(1, k)]
        have = set(e)
        for a in range(k):
            for b in range(a + 1, k):
                if (a, b) not in have and rng.random() < 0.35:
                    e.append((a, b))
    return fam, e


def random_patterns(count, seed, kmin=3, kmax=6, accept=None, max_tries=100000, distinct="iso"):
    """``count`` distinct random connected patterns.

    ``distinct="iso"`` keeps one pattern per isomorphism class (there are only
    139 connected graphs of 4..6 vertices); ``distinct="labelled"`` keeps
    distinct labelled edge sets, so isomorphic patterns with different vertex
    numbering (hence different symmetry-breaking constraints and prefixes)
    count separately.  ``accept(k, edges) -> bool`` lets the caller reject
    patterns (for example by an estimated result budget).  Returns a list of
    dicts {"k", "edges", "family"} with vertices relabelled by a seeded
    permutation.
    """
    if distinct not in ("iso", "labelled"):
        raise ValueError("distinct must be 'iso' or 'labelled'")
    rng = random.Random(seed)
    out, seen = [], set()
    tries = 0
    while len(out) < count and tries < max_tries:
        tries += 1
        k = rng.randint(kmin, kmax)
        fam, e = _family(rng, k)
        perm = list(range(k))
        rng.shuffle(perm)
        e = sorted({(min(perm[a], perm[b]), max(perm[a], perm[b])) for a, b in e})
        if not is_connected(k, e):
            continue
        cf = (k, canonical_form(k, e)) if distinct == "iso" else (k, tuple(e))
        if cf in seen:
            continue
        if accept is not None and not accept(k, e):
            continue
        seen.add(cf)
        out.append({"k": k, "edges": e, "family": fam})
    return out


def all_connected(k):
    """Every connected graph on k vertices, one per isomorphism class (k <= 5)."""
    pairs = [(a, b) for a in range(k) for b in range(a + 1, k)]
    seen, out = set(), []
    for mask in range(1, 1 << len(pairs)):
        e = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        if len(e) < k - 1 or not is_connected(k, e):
            continue
        cf = canonical_form(k, e)
        if cf in seen:
            continue
        seen.add(cf)
        out.append(list(cf))
    return out
