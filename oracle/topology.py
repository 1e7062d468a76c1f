"""Access-matrix oracle (CPU, exact integers).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Section IV (effects of graph topology, Fig. 5): in one pull sweep, each
in-edge u -> v is a read, by the thread (worker) that owns v, of data owned
by the worker that owns u.  Counting reads per (reader, owner) pair under the
static blocked partition gives a coarsened adjacency matrix; the paper
compares how much of it lies on the diagonal.

Workers own contiguous vertex blocks [first[w], first[w+1]).  They are
coarsened into B groups of consecutive workers: group(w) = floor(w * B / P).
"""
from __future__ import annotations

import numpy as np


def owners(first, n):
    """Worker of every vertex 0..n-1 given block starts first[0..P]."""
    first = np.asarray(first, dtype=np.int64)
    return np.searchsorted(first, np.arange(n), side="right") - 1


def access_matrix(g, first, groups):
    """(counts [groups, groups] int64, same_worker) for the CSR graph g."""
    first = np.asarray(first, dtype=np.int64)
    P = first.shape[0] - 1
    own = owners(first, g.n)
    deg = np.diff(g.ptr.astype(np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = g.idx.astype(np.int64)
    rw, ow = own[dst], own[src]
    rg, og = rw * groups // P, ow * groups // P
    counts = np.bincount(rg * groups + og, minlength=groups * groups).reshape(groups, groups).astype(np.int64)
    return counts, int((rw == ow).sum())


def access_matrix_loops(g, first, groups):
    """The same by plain loops over every edge (tiny graphs)."""
    P = len(first) - 1

    def owner(v):
        for w in range(P):
            if first[w] <= v < first[w + 1]:
                return w
        raise ValueError(v)

    counts = [[0] * groups for _ in range(groups)]
    same = 0
    for u in range(g.n):
        for e in range(int(g.ptr[u]), int(g.ptr[u + 1])):
            v = int(g.idx[e])
            r, o = owner(v), owner(u)
            counts[r * groups // P][o * groups // P] += 1
            same += r == o
    return np.array(counts, dtype=np.int64), same


def shares(counts):
    """(diagonal share, diagonal share expected if reads ignored the reader)."""
    c = np.asarray(counts, dtype=np.float64)
    tot = c.sum()
    if tot == 0:
        return 0.0, 0.0
    return float(np.trace(c) / tot), float((c.sum(1) * c.sum(0)).sum() / tot ** 2)
