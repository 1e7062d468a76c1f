"""Small hand-made and random graphs for the test suite (inputs only)."""
from __future__ import annotations

import numpy as np

import graphgen as gg


def random_graph(n, m, seed, self_loops=True, dedup=True, weights=None):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    w = None if weights is None else rng.integers(weights[0], weights[1] + 1, size=src.size)
    return gg.from_edges(n, src, dst, w=w, weight_seed=seed, dedup=dedup, name=f"rand{n}_{m}_{seed}")


def dangling_heavy(n, seed):
    """Only a third of the vertices have out-edges."""
    rng = np.random.default_rng(seed)
    k = max(1, n // 3)
    src = rng.integers(0, k, size=3 * n)
    dst = rng.integers(0, n, size=3 * n)
    return gg.from_edges(n, src, dst, weight_seed=seed, name=f"dangling{n}")


def cycle(n):
    s = np.arange(n)
    return gg.from_edges(n, s, (s + 1) % n, w=np.full(n, 3), name=f"cycle{n}")


def complete(n):
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s != d
    return gg.from_edges(n, s[keep], d[keep], weight_seed=1, name=f"complete{n}")


def in_star(n):
    """Leaves 1..n-1 point to hub 0; the hub is dangling."""
    leaves = np.arange(1, n)
    return gg.from_edges(n, leaves, np.zeros(n - 1, dtype=np.int64), weight_seed=2, name=f"instar{n}")


def hubs_at_run_limit(seed, n=40_000, m=160_000):
    """Random edges plus hubs around the batched calls' run limit of 4096
    in-edges: vertex 1000 has exactly 4096 in-edges, 1001 has 4097, 1002 one,
    1003 6000 and 25000 4096 (each from distinct sources).  The cut of the
    batched tiles then makes 1000, 1001, 1002 and 1003 single-vertex runs,
    1002 a low-degree one stranded between two hubs."""
    rng = np.random.default_rng(seed)
    hubs = {1000: 4096, 1001: 4097, 1002: 1, 1003: 6000, 25000: 4096}
    dst = rng.integers(0, n, size=m)
    dst = dst[~np.isin(dst, list(hubs))]
    src = rng.integers(0, n, size=dst.size)
    srcs, dsts = [src], [dst]
    for h, deg in hubs.items():
        srcs.append(rng.choice(n, size=deg, replace=False))
        dsts.append(np.full(deg, h))
    return gg.from_edges(n, np.concatenate(srcs), np.concatenate(dsts), weight_seed=seed, dedup=True,
                         name=f"runlimit{n}")


def out_star(n):
    """Hub 0 points to leaves 1..n-1; every leaf is dangling."""
    leaves = np.arange(1, n)
    return gg.from_edges(n, np.zeros(n - 1, dtype=np.int64), leaves, weight_seed=3, name=f"outstar{n}")


def empty(n):
    return gg.from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64), name=f"empty{n}")


def two_scc(n, seed):
    """Two random strongly connected halves joined by one edge 0 -> n/2."""
    h = n // 2
    rng = np.random.default_rng(seed)
    s1 = np.concatenate([np.arange(h), rng.integers(0, h, 2 * h)])
    d1 = np.concatenate([(np.arange(h) + 1) % h, rng.integers(0, h, 2 * h)])
    s2 = s1 + h
    d2 = d1 + h
    src = np.concatenate([s1, s2, [0]])
    dst = np.concatenate([d1, d2, [h]])
    return gg.from_edges(2 * h, src, dst, weight_seed=seed, name=f"twoscc{n}")
