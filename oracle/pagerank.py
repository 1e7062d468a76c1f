"""PageRank oracle (float64, CPU, plain numpy).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

The paper evaluates pull-based PageRank with floating-point scores and stops
when the total absolute score change between the last two iterations falls
below a threshold (section IV, evaluation setup).  It gives no formula, so the
oracle uses the standard damped form (reading R1 of the design notes):

    T(x)_v = (1 - alpha)/N + alpha * ( sum_{u -> v} x_u / outdeg(u) + D(x)/N )
    D(x)   = sum_{u : outdeg(u) = 0} x_u          (dangling mass, spread evenly)

Edges are counted with multiplicity and self-loops count in outdeg.  The
linear part alpha*(A + (1/N) 1 delta^T) is alpha times a column-stochastic
matrix, so T is an alpha-contraction in the L1 norm with a unique fixed point
x* whose entries sum to 1.

Every function takes the out-edge CSR graph produced by ``graphgen`` and
expands it to an edge list itself.
"""
from __future__ import annotations

import numpy as np

ALPHA = 0.85


def edge_list(g):
    """(src, dst) int64 arrays of every edge u -> v of the CSR graph."""
    deg = np.diff(g.ptr.astype(np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = g.idx.astype(np.int64)
    return src, dst


def out_degree(g):
    return np.diff(g.ptr.astype(np.int64))


def apply_T(x, src, dst, deg, alpha=ALPHA):
    """One synchronous (Jacobi) sweep: every vertex pulls from its in-neighbours'
    previous values (introduction: values computed in one iteration become
    visible only at the start of the next)."""
    n = x.shape[0]
    x = np.asarray(x, dtype=np.float64)
    contrib = np.zeros(n, dtype=np.float64)
    nz = deg > 0
    contrib[nz] = x[nz] / deg[nz]
    pulled = np.bincount(dst, weights=contrib[src], minlength=n)
    dangling = float(x[~nz].sum())
    return (1.0 - alpha) / n + alpha * (pulled + dangling / n)


def pagerank_jacobi(g, alpha=ALPHA, tol=1e-6, max_sweeps=10_000, x0=None, keep_iterates=False):
    """Synchronous PageRank from x0 = 1/N until the L1 change of a sweep drops
    below ``tol`` (strictly).  The confirming sweep is counted.

    Returns (x, sweeps, residuals, iterates) where residuals[k] is the L1
    change of sweep k+1 and iterates[k] the vector after sweep k+1 (only when
    ``keep_iterates``).
    """
    n = g.n
    src, dst = edge_list(g)
    deg = out_degree(g)
    x = np.full(n, 1.0 / n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    residuals, iterates = [], []
    sweeps = 0
    while sweeps < max_sweeps:
        xn = apply_T(x, src, dst, deg, alpha)
        r = float(np.abs(xn - x).sum())
        x = xn
        sweeps += 1
        residuals.append(r)
        if keep_iterates:
            iterates.append(x.copy())
        if r < tol:
            break
    return x, sweeps, residuals, iterates


def union_jacobi_sweep(graphs, xs, alpha=ALPHA, per_graph=True):
    """One synchronous sweep of a set of graphs stored as one union of
    N = sum n_i vertices (the paper treats one graph; sets are an extension,
    reading R28 of the design notes).  ``xs[i]`` is graph i's part of the
    union vector.  Teleport is (1 - alpha)/N everywhere.  The dangling mass
    is spread either over the graph's own vertices (per_graph: D_i / n_i,
    so graph i keeps the mass n_i/N it starts with) or, as in a single graph
    of N vertices, over the whole union (D / N with D = sum_i D_i)."""
    N = sum(g.n for g in graphs)
    parts, dang = [], []
    for g, x in zip(graphs, xs):
        src, dst = edge_list(g)
        deg = out_degree(g)
        x = np.asarray(x, dtype=np.float64)
        contrib = np.zeros(g.n, dtype=np.float64)
        nz = deg > 0
        contrib[nz] = x[nz] / deg[nz]
        parts.append(np.bincount(dst, weights=contrib[src], minlength=g.n))
        dang.append(float(x[~nz].sum()))
    D = sum(dang)
    out = []
    for g, pulled, d_i in zip(graphs, parts, dang):
        spread = d_i / g.n if per_graph else D / N
        out.append((1.0 - alpha) / N + alpha * (pulled + spread))
    return out


def pagerank_fixed_point(g, alpha=ALPHA, tol=1e-12, max_sweeps=100_000):
    """x* to within the float64 noise floor: Jacobi iteration until the L1
    change is below ``tol`` (1e-12 by default), then one normalisation."""
    x, _, _, _ = pagerank_jacobi(g, alpha, tol, max_sweeps)
    return x / x.sum()


def certificate(g, x, alpha=ALPHA):
    """Upper bound on ||x - x*||_1 valid for any vector x:
    ||x - x*|| <= ||T(x) - x|| / (1 - alpha), because T is an
    alpha-contraction in L1."""
    src, dst = edge_list(g)
    deg = out_degree(g)
    x = np.asarray(x, dtype=np.float64)
    return float(np.abs(apply_T(x, src, dst, deg, alpha) - x).sum()) / (1.0 - alpha)


def transition_matrix(g):
    """Dense column-stochastic M with M[v, u] = (#edges u->v)/outdeg(u) and a
    uniform column 1/N for every dangling u (tiny graphs only)."""
    n = g.n
    src, dst = edge_list(g)
    deg = out_degree(g)
    M = np.zeros((n, n), dtype=np.float64)
    for u, v in zip(src.tolist(), dst.tolist()):
        M[v, u] += 1.0 / deg[u]
    for u in range(n):
        if deg[u] == 0:
            M[:, u] = 1.0 / n
    return M


def pagerank_dense(g, alpha=ALPHA):
    """Fixed point by direct solve of (I - alpha M) x = (1 - alpha)/N 1."""
    n = g.n
    M = transition_matrix(g)
    return np.linalg.solve(np.eye(n) - alpha * M, np.full(n, (1.0 - alpha) / n))


# ------------------------------------------------- personalised PageRank --
#
# Personalised PageRank with a one-hot restart vector e_s (batched queries of
# the sweep library): teleport and dangling mass both go to the restart vertex
# s, so the linear part stays alpha times a column-stochastic matrix:
#
#     P_s(x)_v = (1 - alpha) [v = s] + alpha ( sum_{u -> v} x_u / outdeg(u) + D(x) [v = s] )


def apply_ppr(x, src, dst, deg, s, alpha=ALPHA):
    """One synchronous personalised-PageRank sweep with restart vertex s."""
    n = x.shape[0]
    x = np.asarray(x, dtype=np.float64)
    contrib = np.zeros(n, dtype=np.float64)
    nz = deg > 0
    contrib[nz] = x[nz] / deg[nz]
    out = alpha * np.bincount(dst, weights=contrib[src], minlength=n)
    out[s] += (1.0 - alpha) + alpha * float(x[~nz].sum())
    return out


def ppr_jacobi(g, s, alpha=ALPHA, tol=1e-12, max_sweeps=100_000):
    """Synchronous personalised PageRank from x0 = e_s until the L1 change of
    a sweep drops below tol.  Returns (x, sweeps)."""
    src, dst = edge_list(g)
    deg = out_degree(g)
    x = np.zeros(g.n)
    x[s] = 1.0
    sweeps = 0
    while sweeps < max_sweeps:
        xn = apply_ppr(x, src, dst, deg, s, alpha)
        r = float(np.abs(xn - x).sum())
        x = xn
        sweeps += 1
        if r < tol:
            break
    return x, sweeps


def ppr_fixed_point(g, s, alpha=ALPHA, tol=1e-12):
    x, _ = ppr_jacobi(g, s, alpha, tol)
    return x / x.sum()


def ppr_dense(g, s, alpha=ALPHA):
    """Direct solve of (I - alpha M_s) x = (1 - alpha) e_s, where M_s has the
    column of each dangling vertex equal to e_s (tiny graphs)."""
    n = g.n
    src, dst = edge_list(g)
    deg = out_degree(g)
    M = np.zeros((n, n))
    for u, v in zip(src.tolist(), dst.tolist()):
        M[v, u] += 1.0 / deg[u]
    for u in range(n):
        if deg[u] == 0:
            M[s, u] = 1.0
    rhs = np.zeros(n)
    rhs[s] = 1.0 - alpha
    return np.linalg.solve(np.eye(n) - alpha * M, rhs)


def ppr_certificate(g, x, s, alpha=ALPHA):
    """Upper bound on ||x - x*_s||_1: ||P_s(x) - x||_1 / (1 - alpha)."""
    src, dst = edge_list(g)
    deg = out_degree(g)
    x = np.asarray(x, dtype=np.float64)
    return float(np.abs(apply_ppr(x, src, dst, deg, s, alpha) - x).sum()) / (1.0 - alpha)
