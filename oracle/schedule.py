"""Sequential emulation of the paper's three commit policies (tiny graphs).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

Follows section III of the paper ("Delayed Asynchronous Graph Algorithms"):

* work is split into contiguous vertex blocks, one per thread, balanced by the
  number of in-neighbours (design decisions, blocked partitioning);
* a thread walks its block in vertex order and, for each vertex, pulls its
  in-neighbours' values from the *global* array (the global-read variant of
  the subsection on local vs global reads);
* the new value goes into a thread-local buffer; the buffer is copied to the
  global array when it holds ``delta`` values or when the thread has finished
  its block; ``delta = 0`` means no buffer (every value is written to the
  global array at once: the asynchronous algorithm);
* in synchronous mode outputs go to a separate array that replaces the input
  array only after every thread is done (one barrier per iteration).

Threads are interleaved round-robin one vertex at a time; the real machine's
interleaving is arbitrary, so this emulator is used for invariants that hold
for every interleaving, never for exact sweep counts of a GPU run.

PageRank publishes the contribution c_v = x_v / outdeg(v) (0 if dangling);
the score x_v is private to its owner.  The mass a sweep spreads uniformly is
measured in the previous sweep, either as the dangling mass itself
(``spread="dangling"``) or as one minus the non-dangling mass
(``spread="deficit"``, the form the GPU library uses); both equal the
dangling mass whenever the scores sum to 1, so they give the same fixed
point.  The residual of a vertex is its new score minus its previous score.
"""
from __future__ import annotations

import numpy as np

SYNC, ASYNC, DELAYED = "sync", "async", "delayed"
_BIG = 1 << 62


def blocks_by_in_edges(g, P):
    """P contiguous blocks with about m/P in-edges each: block t starts at the
    first vertex whose cumulative in-degree reaches t*m/P."""
    indeg = np.bincount(g.idx.astype(np.int64), minlength=g.n)
    cum = np.concatenate([[0], np.cumsum(indeg)])
    m = cum[-1]
    bounds = [0]
    for t in range(1, P):
        b = int(np.searchsorted(cum, t * m / P, side="left"))
        bounds.append(min(max(b, bounds[-1]), g.n))
    bounds.append(g.n)
    return bounds


def _in_lists(g):
    deg = np.diff(g.ptr.astype(np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    ins = [[] for _ in range(g.n)]
    for u, v, w in zip(src.tolist(), g.idx.tolist(), g.w.tolist()):
        ins[v].append((u, w))
    return ins, deg


def _run(g, mode, delta, bounds, n_sweeps_max, update, publish_init, stop):
    """Generic driver.  ``update(v, read)`` returns (published, private_info)."""
    G = publish_init
    P = len(bounds) - 1
    history = []
    for sweep in range(n_sweeps_max):
        out = G.copy() if mode == SYNC else None
        cursors = [bounds[t] for t in range(P)]
        bufs = [[] for _ in range(P)]
        buf_start = [bounds[t] for t in range(P)]
        info = []
        active = True
        while active:
            active = False
            for t in range(P):
                v = cursors[t]
                if v >= bounds[t + 1]:
                    continue
                active = True
                val, inf = update(v, G)
                info.append((v, inf))
                if mode == SYNC:
                    out[v] = val
                elif mode == ASYNC or delta == 0:
                    G[v] = val
                else:
                    bufs[t].append(val)
                    if len(bufs[t]) == delta:
                        s = buf_start[t]
                        G[s:s + len(bufs[t])] = bufs[t]
                        buf_start[t] = s + len(bufs[t])
                        bufs[t] = []
                cursors[t] = v + 1
                if cursors[t] == bounds[t + 1] and mode == DELAYED and bufs[t]:
                    s = buf_start[t]
                    G[s:s + len(bufs[t])] = bufs[t]
                    buf_start[t] = s + len(bufs[t])
                    bufs[t] = []
        if mode == SYNC:
            G = out
        history.append(info)
        if stop(info):
            break
    return G, history


def sssp(g, source, mode=SYNC, delta=0, P=1, bounds=None, max_sweeps=None):
    """Bellman-Ford under the emulated schedule.  Returns (dist_u32, sweeps,
    per-sweep distance snapshots)."""
    n = g.n
    bounds = bounds if bounds is not None else blocks_by_in_edges(g, P)
    ins, _ = _in_lists(g)
    G = np.full(n, _BIG, dtype=object)
    G[source] = 0
    snaps = []

    def update(v, read):
        old = read[v]
        best = old
        for u, w in ins[v]:
            du = read[u]
            if du < _BIG and du + w < best:
                best = du + w
        return best, best < old

    def stop(info):
        return not any(ch for _, ch in info)

    limit = n + 2 if max_sweeps is None else max_sweeps
    sweeps = 0
    Gcur = G
    # drive one sweep at a time to keep snapshots
    while sweeps < limit:
        Gcur, hist = _run(g, mode, delta, bounds, 1, update, Gcur, stop)
        sweeps += 1
        snaps.append(np.array([min(int(x), 0xFFFFFFFF) for x in Gcur], dtype=np.uint32))
        if stop(hist[0]):
            break
    return snaps[-1], sweeps, snaps


def pagerank(g, mode=SYNC, delta=0, P=1, bounds=None, alpha=0.85, tol=1e-10, max_sweeps=10_000,
             spread="dangling"):
    """PageRank under the emulated schedule.  Returns (x, sweeps, residuals)."""
    if spread not in ("dangling", "deficit"):
        raise ValueError("spread must be 'dangling' or 'deficit'")
    n = g.n
    bounds = bounds if bounds is not None else blocks_by_in_edges(g, P)
    ins, deg = _in_lists(g)
    x = np.full(n, 1.0 / n)
    c = np.where(deg > 0, x / np.maximum(deg, 1), 0.0)
    state = {"D": float(x[deg == 0].sum())}
    residuals = []

    def update(v, read):
        s = 0.0
        for u, _ in ins[v]:
            s += read[u]
        xn = (1.0 - alpha) / n + alpha * (s + state["D"] / n)
        cn = xn / deg[v] if deg[v] > 0 else 0.0
        return cn, xn

    def stop(info):
        return False

    sweeps = 0
    while sweeps < max_sweeps:
        c, hist = _run(g, mode, delta, bounds, 1, update, c, stop)
        sweeps += 1
        r = 0.0
        D = 0.0
        S = 0.0
        for v, xn in hist[0]:
            r += abs(xn - x[v])
            x[v] = xn
            if deg[v] == 0:
                D += xn
            else:
                S += xn
        state["D"] = D if spread == "dangling" else 1.0 - S
        residuals.append(r)
        if r < tol:
            break
    return x, sweeps, residuals
