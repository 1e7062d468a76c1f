"""Single-source shortest paths oracle (exact integers, CPU).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

The paper evaluates pull-based Bellman-Ford with 32-bit unsigned path lengths
and stops when an iteration produces no update (section IV, evaluation
setup).  Readings used here:

* initial values: 0 at the source, "infinity" elsewhere;
* a pull sweep sets d'(v) = min(d(v), min over in-edges (u, v) of d(u) + w(u, v));
* an "update" is a strict decrease of some d(v);
* results are returned as uint32 with 0xFFFFFFFF for unreachable vertices.

Arithmetic is exact int64 (no overflow for weights <= 255 and n < 2**24), so
these functions give true distances; the 32-bit saturation of the product
never triggers on graphs whose longest path fits in 32 bits.
"""
from __future__ import annotations

import heapq

import numpy as np

INF32 = 0xFFFFFFFF
_BIG = np.int64(1) << np.int64(62)


def edge_list(g):
    deg = np.diff(g.ptr.astype(np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    return src, g.idx.astype(np.int64), g.w.astype(np.int64)


def _to_u32(d):
    out = np.where(d >= INF32, INF32, d)
    return out.astype(np.uint32)


def bellman_ford_sync(g, source, max_sweeps=None, keep_iterates=False):
    """Synchronous (Jacobi) Bellman-Ford.  Each sweep reads only the previous
    sweep's distances.  Stops after the first sweep with no strict decrease;
    that confirming sweep is counted.

    Returns (dist_u32, sweeps, iterates) with iterates[k] the uint32 vector
    after sweep k+1 when ``keep_iterates``.
    """
    n = g.n
    if not 0 <= source < n:
        raise ValueError("source out of range")
    src, dst, w = edge_list(g)
    d = np.full(n, _BIG, dtype=np.int64)
    d[source] = 0
    sweeps, iterates = 0, []
    limit = n + 1 if max_sweeps is None else max_sweeps
    while sweeps < limit:
        cand = d[src] + w
        cand[d[src] >= _BIG] = _BIG
        dn = d.copy()
        np.minimum.at(dn, dst, cand)
        sweeps += 1
        changed = bool((dn < d).any())
        d = dn
        if keep_iterates:
            iterates.append(_to_u32(d))
        if not changed:
            break
    return _to_u32(d), sweeps, iterates


def dijkstra(g, source):
    """Textbook Dijkstra with a binary heap (lazy deletion)."""
    n = g.n
    ptr = g.ptr.astype(np.int64)
    idx = g.idx
    w = g.w
    dist = [None] * n
    best = {source: 0}
    heap = [(0, source)]
    while heap:
        du, u = heapq.heappop(heap)
        if dist[u] is not None:
            continue
        dist[u] = du
        for e in range(ptr[u], ptr[u + 1]):
            v = int(idx[e])
            nd = du + int(w[e])
            if dist[v] is None and nd < best.get(v, 1 << 62):
                best[v] = nd
                heapq.heappush(heap, (nd, v))
    return np.array([INF32 if x is None or x >= INF32 else x for x in dist], dtype=np.uint32)


def floyd_warshall(g):
    """All-pairs shortest paths, O(n^3); tiny graphs only."""
    n = g.n
    big = 1 << 60
    D = np.full((n, n), big, dtype=np.int64)
    np.fill_diagonal(D, 0)
    src, dst, w = edge_list(g)
    for u, v, ww in zip(src.tolist(), dst.tolist(), w.tolist()):
        D[u, v] = min(D[u, v], ww)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return np.where(D >= big, INF32, D).astype(np.uint64)


def bounded_hop_distances(g, source, hops):
    """Shortest length over paths with at most ``hops`` edges, by brute-force
    dynamic programming over path length (tiny graphs)."""
    n = g.n
    big = 1 << 60
    src, dst, w = edge_list(g)
    best = np.full(n, big, dtype=np.int64)
    best[source] = 0
    layer = best.copy()  # shortest with exactly k edges, k = 0
    for _ in range(hops):
        nxt = np.full(n, big, dtype=np.int64)
        for u, v, ww in zip(src.tolist(), dst.tolist(), w.tolist()):
            if layer[u] < big and layer[u] + ww < nxt[v]:
                nxt[v] = layer[u] + ww
        layer = nxt
        best = np.minimum(best, layer)
    return np.where(best >= big, INF32, best).astype(np.uint32)


def certificate(g, source, dist):
    """Check that ``dist`` (uint32, 0xFFFFFFFF = unreachable) are the exact
    shortest-path distances from ``source`` with positive weights, in O(m):

    1. dist[source] == 0;
    2. every edge (u, v) with finite dist[u] satisfies dist[v] <= dist[u] + w;
    3. every finite v != source has a tight in-edge: dist[v] == dist[u] + w
       for some u with finite dist[u];
    4. infinite vertices have no finite in-neighbour (implied by 2).

    With w >= 1, following tight edges strictly decreases dist, so every
    tight chain ends at the source; together with 2 this forces dist to be
    the true distances.  Returns (ok, message).
    """
    d = np.asarray(dist).astype(np.int64)
    src, dst, w = edge_list(g)
    if (w < 1).any():
        return False, "certificate needs weights >= 1"
    if d[source] != 0:
        return False, "dist[source] != 0"
    fin_u = d[src] != INF32
    lhs = d[dst[fin_u]]
    rhs = d[src[fin_u]] + w[fin_u]
    bad = lhs > rhs
    if bad.any():
        k = int(np.flatnonzero(bad)[0])
        return False, f"edge {int(src[fin_u][k])}->{int(dst[fin_u][k])} violates d[v] <= d[u] + w"
    tight = np.zeros(g.n, dtype=bool)
    tight[dst[fin_u][lhs == rhs]] = True
    need = (d != INF32)
    need[source] = False
    missing = need & ~tight
    if missing.any():
        return False, f"vertex {int(np.flatnonzero(missing)[0])} has no tight in-edge"
    return True, "ok"
