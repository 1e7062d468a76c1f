"""Seeded synthetic graph inputs shared by the CPU oracle and the GPU path.

This module only *makes inputs*: edge lists, weights and source vertices.  It
holds none of the arithmetic of the method under study (no PageRank, no
relaxation, no transposition into in-edge form), so that the oracle and the
HIP library stay independent of each other while reading identical inputs.

Every graph is returned in out-edge CSR form, the form a user hands to the
library: ``ptr`` (uint64, n+1), ``idx`` (uint32 destinations, sorted within
each source), ``w`` (uint32 weights in [1, 255]).  Duplicate edges are removed;
self-loops are kept unless a generator says otherwise.

Random numbers come from numpy's PCG64 bit generator, one independent stream
per purpose (``edges``, ``perm``, ``weights``, ``sources``) derived from the
graph's master seed, so the same seed always yields the same graph.

Workload shapes follow the paper's evaluation section, which measures on the
GAP suite (Kron, Urand, Road, Twitter, Web).  Those datasets are not available
here; the synthetic stand-ins are:

* R-MAT (Chakrabarti, Zhan, Faloutsos 2004) for Kron: skewed degrees and
  long-range edges, ids randomly permuted;
* Erdos-Renyi G(n, m) for Urand;
* a diagonal-banded graph for Web's clustering along the main diagonal, which
  the paper's topology subsection identifies as the case where delaying
  updates does not help.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = [
    "CSRGraph",
    "rmat",
    "erdos_renyi",
    "banded",
    "from_edges",
    "path_graph",
    "pick_sources",
    "stream",
]

_STREAM_IDS = {"edges": 1, "perm": 2, "weights": 3, "sources": 4, "extra": 5}


def stream(seed: int, name: str) -> np.random.Generator:
    """Independent PCG64 stream ``name`` of master seed ``seed``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), _STREAM_IDS[name]])))


@dataclasses.dataclass
class CSRGraph:
    """Directed graph in out-edge CSR form (the library's input form)."""

    n: int
    ptr: np.ndarray  # uint64 [n+1]
    idx: np.ndarray  # uint32 [m], destination of each out-edge
    w: np.ndarray    # uint32 [m], edge weight in [1, 255]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.idx.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.uint64(self.n).tobytes())
        for a in (self.ptr, self.idx, self.w):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def from_edges(n: int, src, dst, w=None, *, weight_seed: int = 0, dedup: bool = True, name: str = "") -> CSRGraph:
    """Build CSR from an edge list.

    Edges are sorted by (src, dst).  With ``dedup`` repeated (src, dst) pairs
    collapse to one edge.  When ``w`` is None each remaining edge draws a weight
    uniform in [1, 255] from the ``weights`` stream of ``weight_seed``, in
    (src, dst)-sorted order.
    """
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    if n < 0 or (src.size and (int(src.max()) >= n or int(dst.max()) >= n)):
        raise ValueError("vertex id out of range")
    key = (src << np.uint64(32)) | dst
    if w is None:
        key = np.unique(key) if dedup else np.sort(key, kind="stable")
        ww = None
    else:
        ww = np.asarray(w, dtype=np.uint32)
        order = np.argsort(key, kind="stable")
        key = key[order]
        ww = ww[order]
        if dedup:
            keep = np.ones(key.shape, dtype=bool)
            keep[1:] = key[1:] != key[:-1]
            key = key[keep]
            ww = ww[keep]
    s = (key >> np.uint64(32)).astype(np.uint32)
    d = (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    counts = np.bincount(s, minlength=n).astype(np.uint64) if n else np.zeros(0, np.uint64)
    ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=ptr[1:])
    if ww is None:
        ww = stream(weight_seed, "weights").integers(1, 256, size=d.shape[0], dtype=np.uint32)
    return CSRGraph(n=n, ptr=ptr, idx=d, w=ww, name=name)


def rmat(scale: int, edge_factor: int = 16, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 0,
         permute: bool = True) -> CSRGraph:
    """R-MAT graph: ``edge_factor * 2**scale`` samples of recursive quadrant
    choice with probabilities a/b/c/d (a: src bit 0, dst bit 0; b: src 0, dst 1;
    c: src 1, dst 0; d: src 1, dst 1), no per-level noise, directed, ids
    permuted by a random permutation of the ``perm`` stream, duplicates
    removed, self-loops kept."""
    a, b, c, d = abcd
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("a+b+c+d must be 1")
    n = 1 << scale
    m = edge_factor * n
    rng = stream(seed, "edges")
    src = np.zeros(m, dtype=np.uint32)
    dst = np.zeros(m, dtype=np.uint32)
    t1, t2, t3 = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    for level in range(scale):
        r = rng.random(m, dtype=np.float32)
        sbit = (r >= t2).astype(np.uint32)
        dbit = (((r >= t1) & (r < t2)) | (r >= t3)).astype(np.uint32)
        src |= sbit << np.uint32(level)
        dst |= dbit << np.uint32(level)
        del r, sbit, dbit
    if permute:
        perm = stream(seed, "perm").permutation(n).astype(np.uint32)
        src = perm[src]
        dst = perm[dst]
    return from_edges(n, src, dst, weight_seed=seed, name=f"rmat{scale}")


def erdos_renyi(n: int, avg_degree: float, seed: int = 0) -> CSRGraph:
    """G(n, m) with m = round(avg_degree * n) uniform samples, self-loops
    dropped, duplicates removed (so the final edge count can be slightly
    below m)."""
    m = int(round(avg_degree * n))
    rng = stream(seed, "edges")
    src = rng.integers(0, n, size=m, dtype=np.uint32)
    dst = rng.integers(0, n, size=m, dtype=np.uint32)
    keep = src != dst
    return from_edges(n, src[keep], dst[keep], weight_seed=seed, name=f"er{n}")


def banded(n: int, out_degree: int = 16, half_width: int = 4096, p_long: float = 0.01,
           seed: int = 0) -> CSRGraph:
    """Diagonal-banded graph: every vertex v draws ``out_degree`` targets.  Each
    is long-range with probability ``p_long`` (uniform over all vertices other
    than v), otherwise v+o with o uniform in [-half_width, half_width] minus
    {0}, redrawn while v+o falls outside [0, n).  Duplicates removed."""
    if n < 2:
        raise ValueError("banded graph needs n >= 2")
    rng = stream(seed, "edges")
    m = n * out_degree
    src = np.repeat(np.arange(n, dtype=np.int64), out_degree)
    is_long = rng.random(m, dtype=np.float32) < np.float32(p_long)
    dst = np.empty(m, dtype=np.int64)
    nl = int(is_long.sum())
    t = rng.integers(0, n - 1, size=nl, dtype=np.int64)
    sl = src[is_long]
    t += (t >= sl)
    dst[is_long] = t
    todo = np.flatnonzero(~is_long)
    hw = min(half_width, n - 1)
    while todo.size:
        mag = rng.integers(1, hw + 1, size=todo.size, dtype=np.int64)
        sign = rng.integers(0, 2, size=todo.size, dtype=np.int64) * 2 - 1
        cand = src[todo] + sign * mag
        ok = (cand >= 0) & (cand < n)
        dst[todo[ok]] = cand[ok]
        todo = todo[~ok]
    return from_edges(n, src.astype(np.uint32), dst.astype(np.uint32), weight_seed=seed,
                      name=f"banded{n}")


def path_graph(n: int, weight: int = 1) -> CSRGraph:
    """Directed path 0 -> 1 -> ... -> n-1 with constant weight."""
    src = np.arange(max(n - 1, 0), dtype=np.uint32)
    return from_edges(n, src, src + 1, w=np.full(src.shape, weight, np.uint32), name=f"path{n}")


def pick_sources(g: CSRGraph, k: int, seed: int) -> np.ndarray:
    """``k`` distinct SSSP sources, uniform among vertices with out-degree >= 1,
    drawn from the ``sources`` stream."""
    deg = np.diff(g.ptr.astype(np.int64))
    cand = np.flatnonzero(deg > 0)
    if cand.size == 0:
        return np.zeros(0, dtype=np.uint32)
    k = min(k, cand.size)
    pick = stream(seed, "sources").choice(cand.size, size=k, replace=False)
    return cand[pick].astype(np.uint32)
