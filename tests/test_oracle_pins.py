"""Pins of the CPU oracle against facts outside itself (no GPU).

Each test compares the oracle with something it does not share code with:
closed forms derived by hand from the fixed-point equation, an independent
library (networkx, scipy), brute force on tiny inputs, or an invariant fixed by
the mathematics (contraction, mass conservation, optimality certificates).
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import schedule as osch
from oracle import sssp as osp
from tests import graphs as tg

ALPHA = 0.85


# ---------------------------------------------------------------- PageRank --

@pytest.mark.parametrize("n", [1, 2, 7, 33])
def test_pr_uniform_closed_forms(n):
    """Directed cycle, complete digraph and the edgeless graph (all dangling)
    have the uniform vector 1/N as fixed point."""
    for g in (tg.cycle(n), tg.empty(n)) + ((tg.complete(n),) if n > 1 else ()):
        x = opr.pagerank_fixed_point(g)
        np.testing.assert_allclose(x, np.full(n, 1.0 / n), rtol=0, atol=1e-11)


@pytest.mark.parametrize("n", [2, 5, 17, 200])
def test_pr_in_star_closed_form(n):
    """Leaves -> dangling hub.  Solving x_leaf = (1-a)/N + a x_hub/N,
    x_hub = (1-a)/N + a((N-1) x_leaf + x_hub/N) with sum 1 gives
    x_hub = (1 + (N-1)a) / (N + (N-1)a), x_leaf = (1 - x_hub)/(N-1)."""
    g = tg.in_star(n)
    x = opr.pagerank_fixed_point(g)
    hub = (1 + (n - 1) * ALPHA) / (n + (n - 1) * ALPHA)
    leaf = (1 - hub) / (n - 1)
    assert abs(x[0] - hub) < 1e-11
    np.testing.assert_allclose(x[1:], leaf, rtol=0, atol=1e-11)


def test_pr_in_star_n5_values():
    """Numerical values for N = 5 kept as a golden fixture."""
    g = tg.in_star(5)
    x = opr.pagerank_fixed_point(g)
    vals = _golden("pagerank_closed_forms.txt")
    assert abs(x[0] - vals["instar5_hub"]) < 5e-8
    assert abs(x[1] - vals["instar5_leaf"]) < 5e-8


@pytest.mark.parametrize("n", [2, 5, 64])
def test_pr_out_star_closed_form(n):
    """Hub -> dangling leaves.  The hub has no in-edges, so
    x_hub = (1-a)/N + a D/N with D = 1 - x_hub, i.e. x_hub = 1/(N + a).
    This pins the direction of the pull (in-edges, not out-edges)."""
    g = tg.out_star(n)
    x = opr.pagerank_fixed_point(g)
    hub = 1.0 / (n + ALPHA)
    assert abs(x[0] - hub) < 1e-11
    np.testing.assert_allclose(x[1:], (1 - hub) / (n - 1), rtol=0, atol=1e-11)


def test_pr_two_vertex_closed_form():
    """0 -> 1 with 1 dangling: x0 = 1/(2 + a), x1 = (1 + a)/(2 + a)."""
    g = gg.from_edges(2, [0], [1])
    x = opr.pagerank_fixed_point(g)
    assert abs(x[0] - 1 / (2 + ALPHA)) < 1e-11
    assert abs(x[1] - (1 + ALPHA) / (2 + ALPHA)) < 1e-11


@pytest.mark.parametrize("seed", range(6))
def test_pr_dense_solve(seed):
    """Jacobi fixed point equals the direct linear solve on tiny random
    graphs, including self-loops, dangling-heavy and multigraph inputs."""
    n = 5 + 9 * seed
    graphs = [tg.random_graph(n, 3 * n, seed), tg.dangling_heavy(n, seed),
              tg.random_graph(n, 4 * n, seed + 100, dedup=False)]
    for g in graphs:
        x = opr.pagerank_fixed_point(g)
        xd = opr.pagerank_dense(g)
        assert np.abs(x - xd).sum() < 1e-11
        assert abs(xd.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_pr_networkx(seed):
    """Independent implementation: networkx.pagerank (uniform teleport and
    uniform redistribution of dangling mass by default)."""
    nx = pytest.importorskip("networkx")
    g = tg.random_graph(600, 2400, seed) if seed == 0 else tg.dangling_heavy(900, seed)
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    src, dst = opr.edge_list(g)
    G.add_edges_from(zip(src.tolist(), dst.tolist()))
    ref = nx.pagerank(G, alpha=ALPHA, tol=1e-15, max_iter=100000)
    ref = np.array([ref[i] for i in range(g.n)])
    x = opr.pagerank_fixed_point(g)
    assert np.abs(x - ref).sum() < 1e-11


@pytest.mark.parametrize("seed", range(3))
def test_pr_mass_and_contraction(seed):
    """Every Jacobi iterate keeps total mass 1; T is an alpha-contraction in
    L1; the change per sweep shrinks by at least alpha."""
    g = tg.dangling_heavy(120, seed)
    x, sweeps, res, its = opr.pagerank_jacobi(g, tol=1e-12, keep_iterates=True)
    for it in its:
        assert abs(it.sum() - 1.0) < 1e-13
    for a, b in zip(res, res[1:]):
        assert b <= ALPHA * a * (1 + 1e-9) + 1e-16
    rng = np.random.default_rng(seed)
    src, dst = opr.edge_list(g)
    deg = opr.out_degree(g)
    for _ in range(5):
        u, v = rng.random(g.n), rng.random(g.n)
        lhs = np.abs(opr.apply_T(u, src, dst, deg) - opr.apply_T(v, src, dst, deg)).sum()
        assert lhs <= ALPHA * np.abs(u - v).sum() * (1 + 1e-12)


def test_pr_certificate_bounds_error():
    """||T(x) - x||/(1 - a) bounds ||x - x*|| for arbitrary perturbations."""
    g = tg.random_graph(300, 1500, 7)
    xs = opr.pagerank_dense(g)
    rng = np.random.default_rng(3)
    assert opr.certificate(g, xs) < 1e-13
    for scale in (1e-3, 1e-6, 1e-9):
        x = xs + scale * rng.standard_normal(g.n) / g.n
        err = np.abs(x - xs).sum()
        cert = opr.certificate(g, x)
        assert err <= cert * (1 + 1e-9) + 1e-15
        assert cert <= err * (1 + ALPHA) / (1 - ALPHA) * (1 + 1e-9) + 1e-15


def _perturbations(xs, rng):
    """Vectors around a fixed point x*: random signed noise at three scales,
    a uniform rescale of x* (the direction in which the certificate is
    tight) and mass moved between two vertices."""
    n = xs.size
    out = [xs + sc * rng.standard_normal(n) / n for sc in (1e-3, 1e-6, 1e-9)]
    out += [xs * (1 + t) for t in (1e-4, -3e-7)]
    y = xs.copy()
    y[0] += 1e-5
    y[n - 1] -= 1e-5
    out.append(y)
    return out


@pytest.mark.parametrize("gname", ["random", "dangling"])
def test_ppr_certificate_bounds_error(gname):
    """||P_s(x) - x||/(1 - a) bounds ||x - x*_s|| from above, and by
    contraction it is at most (1 + a)/(1 - a) times that error, for any x.
    x*_s comes from the dense direct solve, not from the certificate's own
    sweep.  On x = (1 + t) x*_s the bound is exact (P_s is affine and maps
    (1 + t) x* to (1 + t) x* - t (1 - a) e_s), so a certificate that drops its
    1/(1 - a) factor falls below the true error there."""
    g = tg.random_graph(120, 500, 11) if gname == "random" else tg.dangling_heavy(90, 5)
    s = int(gg.pick_sources(g, 1, seed=2)[0])
    xs = opr.ppr_dense(g, s)
    assert opr.ppr_certificate(g, xs, s) < 1e-13
    rng = np.random.default_rng(9)
    for x in _perturbations(xs, rng):
        err = np.abs(x - xs).sum()
        cert = opr.ppr_certificate(g, x, s)
        assert err <= cert * (1 + 1e-9) + 1e-15
        assert cert <= err * (1 + ALPHA) / (1 - ALPHA) * (1 + 1e-9) + 1e-15
    for t in (1e-4, -3e-7):
        assert abs(opr.ppr_certificate(g, xs * (1 + t), s) - abs(t)) < 1e-6 * abs(t) + 1e-14


def test_pr_stopping_rule():
    """Stops at the first sweep whose L1 change is strictly below tol, and the
    returned count includes that sweep."""
    g = tg.random_graph(200, 900, 4)
    x, sweeps, res, _ = opr.pagerank_jacobi(g, tol=1e-6)
    assert res[-1] < 1e-6 and all(r >= 1e-6 for r in res[:-1])
    assert len(res) == sweeps


def test_pr_union_per_graph_mass_is_each_graph_alone():
    """Reading R28 (graph sets).  With each graph's dangling mass spread over
    its own vertices, the union's synchronous iterates restricted to graph i
    are graph i's own Jacobi iterates times n_i/N, for every sweep; spreading
    one dangling mass over the whole union instead moves mass between the
    graphs (their shares drift from n_i/N), although after normalising each
    graph both forms reach the same fixed points."""
    graphs = [tg.dangling_heavy(40, 2), gg.rmat(6, seed=3), tg.in_star(30), tg.complete(7)]
    N = sum(g.n for g in graphs)
    alone = [opr.pagerank_jacobi(g, tol=0.0, max_sweeps=12, keep_iterates=True)[3] for g in graphs]
    xs = [np.full(g.n, 1.0 / N) for g in graphs]
    ys = [x.copy() for x in xs]
    drift = 0.0
    for k in range(12):
        xs = opr.union_jacobi_sweep(graphs, xs, per_graph=True)
        ys = opr.union_jacobi_sweep(graphs, ys, per_graph=False)
        for g, x, y, it in zip(graphs, xs, ys, alone):
            np.testing.assert_allclose(x, it[k] * g.n / N, rtol=1e-12, atol=0.0)
            drift = max(drift, abs(y.sum() - g.n / N))
    assert drift > 1e-3  # the global spread does move mass between graphs
    for _ in range(400):
        ys = opr.union_jacobi_sweep(graphs, ys, per_graph=False)
    for g, y in zip(graphs, ys):
        np.testing.assert_allclose(y / y.sum(), opr.pagerank_fixed_point(g), rtol=0.0, atol=1e-10)


# -------------------------------------------------------------------- SSSP --

@pytest.mark.parametrize("seed", range(5))
def test_sssp_bf_matches_dijkstra_scipy_fw(seed):
    """Synchronous Bellman-Ford == heap Dijkstra == scipy Dijkstra ==
    Floyd-Warshall row, with unreachable vertices."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    n = 20 + 20 * seed
    g = tg.random_graph(n, int(1.5 * n), seed)
    src, dst, w = osp.edge_list(g)
    mat = csr_matrix((w.astype(np.float64), (src, dst)), shape=(n, n))
    fw = osp.floyd_warshall(g) if n <= 64 else None
    for s in range(0, n, max(1, n // 5)):
        bf, _, _ = osp.bellman_ford_sync(g, s)
        dj = osp.dijkstra(g, s)
        ref = sp_dijkstra(mat, directed=True, indices=s)
        ref = np.where(np.isinf(ref), osp.INF32, ref).astype(np.uint32)
        np.testing.assert_array_equal(bf, dj)
        np.testing.assert_array_equal(bf, ref)
        if fw is not None:
            np.testing.assert_array_equal(bf, fw[s].astype(np.uint32))


def test_sssp_certificate_accepts_and_rejects():
    g = tg.random_graph(80, 300, 11)
    d, _, _ = osp.bellman_ford_sync(g, 0)
    ok, msg = osp.certificate(g, 0, d)
    assert ok, msg
    reach = np.flatnonzero((d != osp.INF32) & (np.arange(g.n) != 0))
    unreach = np.flatnonzero(d == osp.INF32)
    assert reach.size and unreach.size
    for mutate in ("plus", "minus", "inf", "finite"):
        e = d.astype(np.int64).copy()
        if mutate == "plus":
            e[reach[0]] += 1
        elif mutate == "minus":
            e[reach[-1]] -= 1
        elif mutate == "inf":
            e[reach[1]] = osp.INF32
        else:
            e[unreach[0]] = 5
        ok, _ = osp.certificate(g, 0, e.astype(np.uint32))
        assert not ok, mutate


@pytest.mark.parametrize("seed", range(4))
def test_sssp_sync_hop_invariant(seed):
    """After k synchronous sweeps, d = shortest length over paths of at most k
    edges (brute force), and the sweep count is 1 + max hop count h(v), h(v)
    the fewest edges on a shortest path to v."""
    g = tg.random_graph(30, 70, seed, weights=(1, 9))
    d, sweeps, its = osp.bellman_ford_sync(g, 0, keep_iterates=True)
    for k, it in enumerate(its, start=1):
        np.testing.assert_array_equal(it, osp.bounded_hop_distances(g, 0, k))
    h = np.zeros(g.n, dtype=np.int64)
    for v in range(g.n):
        if d[v] == osp.INF32:
            continue
        k = 0
        while osp.bounded_hop_distances(g, 0, k)[v] != d[v]:
            k += 1
        h[v] = k
    assert sweeps == 1 + h.max()


@pytest.mark.parametrize("n", [1, 2, 10, 50])
def test_sssp_path_graph(n):
    """Path 0 -> ... -> n-1 with unit weights: distances 0..n-1; synchronous
    Bellman-Ford needs exactly n sweeps (n-1 with changes plus the confirming
    one); a single in-order asynchronous worker needs 2."""
    g = gg.path_graph(n)
    d, sweeps, _ = osp.bellman_ford_sync(g, 0)
    np.testing.assert_array_equal(d, np.arange(n, dtype=np.uint32))
    assert sweeps == n
    da, sa, _ = osch.sssp(g, 0, mode=osch.ASYNC, P=1)
    np.testing.assert_array_equal(da, d)
    assert sa == (2 if n > 1 else 1)


# --------------------------------------------------- emulated commit modes --

@pytest.mark.parametrize("seed", range(3))
def test_schedule_modes_same_fixed_point(seed):
    """Every commit mode reaches the same answer (chaotic relaxation): SSSP
    bit-exact, PageRank within 1e-9 of the dense solve."""
    g = tg.random_graph(60, 240, seed)
    xs = opr.pagerank_dense(g)
    d0, _, _ = osp.bellman_ford_sync(g, 0)
    for mode, delta, P in [(osch.SYNC, 0, 4), (osch.ASYNC, 0, 4), (osch.DELAYED, 4, 4),
                           (osch.DELAYED, 1, 3), (osch.DELAYED, 1000, 5)]:
        x, _, _ = osch.pagerank(g, mode, delta, P, tol=1e-12)
        assert np.abs(x / x.sum() - xs).sum() < 1e-9
        d, _, _ = osch.sssp(g, 0, mode, delta, P)
        np.testing.assert_array_equal(d, d0)


def test_schedule_sync_equals_jacobi():
    """The emulated synchronous schedule is exactly the Jacobi oracle."""
    g = tg.dangling_heavy(50, 2)
    _, s1, r1 = osch.pagerank(g, osch.SYNC, 0, P=3, tol=1e-9)
    _, s2, r2, _ = opr.pagerank_jacobi(g, tol=1e-9)
    assert s1 == s2
    np.testing.assert_allclose(r1, r2, rtol=1e-10, atol=1e-15)
    d1, t1, snaps1 = osch.sssp(g, 0, osch.SYNC, 0, P=3)
    d2, t2, its2 = osp.bellman_ford_sync(g, 0, keep_iterates=True)
    assert t1 == t2
    for a, b in zip(snaps1, its2):
        np.testing.assert_array_equal(a, b)


def test_schedule_delta_whole_block_is_sync():
    """Equal blocks, lock-step threads and delta = block size: nobody flushes
    before the sweep ends, so delayed == synchronous sweep by sweep (the
    paper's statement that delta equal to the per-thread output count gives
    the synchronous algorithm)."""
    g = tg.random_graph(48, 200, 5)
    bounds = [0, 12, 24, 36, 48]
    _, s1, snaps1 = osch.sssp(g, 0, osch.DELAYED, 12, bounds=bounds)
    _, s2, its2 = osp.bellman_ford_sync(g, 0, keep_iterates=True)
    assert s1 == s2
    for a, b in zip(snaps1, its2):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("seed", range(3))
def test_schedule_sssp_monotone(seed):
    """P-9: in any commit mode, reads are never staler than the previous
    sweep, so the distances after sweep k are <= the synchronous ones and the
    asynchronous/delayed sweep count never exceeds the synchronous one."""
    g = tg.random_graph(80, 260, seed + 20)
    _, ss, its = osp.bellman_ford_sync(g, 0, keep_iterates=True)
    for mode, delta, P in [(osch.ASYNC, 0, 4), (osch.DELAYED, 3, 4), (osch.DELAYED, 64, 2)]:
        _, sm, snaps = osch.sssp(g, 0, mode, delta, P)
        assert sm <= ss
        for k, s in enumerate(snaps):
            ref = its[min(k, len(its) - 1)]
            assert (s.astype(np.int64) <= ref.astype(np.int64)).all()


# ---------------------------------------------------------------- helpers --

def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()[:2]
            vals[k] = float(v)
    return vals


def test_schedule_deficit_spread():
    """Spreading 1 - (non-dangling mass) instead of the dangling mass: the
    synchronous schedule is unchanged sweep by sweep (scores always sum to 1
    there), every mode reaches the same fixed point."""
    g = tg.dangling_heavy(90, 4)
    xs = opr.pagerank_dense(g)
    _, s1, r1 = osch.pagerank(g, osch.SYNC, 0, P=3, tol=1e-10, spread="deficit")
    _, s2, r2, _ = opr.pagerank_jacobi(g, tol=1e-10)
    assert s1 == s2
    np.testing.assert_allclose(r1, r2, rtol=1e-9, atol=1e-15)
    for mode, delta in [(osch.ASYNC, 0), (osch.DELAYED, 5)]:
        x, _, _ = osch.pagerank(g, mode, delta, P=4, tol=1e-12, spread="deficit")
        assert np.abs(x / x.sum() - xs).sum() < 1e-9


# ------------------------------------------------ personalised PageRank ----

@pytest.mark.parametrize("n", [3, 8, 21])
def test_ppr_cycle_closed_form(n):
    """Directed cycle, restart at s: mass decays by alpha per hop, so
    x_{s+k} = (1 - a) a^k / (1 - a^n)."""
    g = tg.cycle(n)
    for s in (0, n // 2):
        x = opr.ppr_fixed_point(g, s)
        k = (np.arange(n) - s) % n
        ref = (1 - ALPHA) * ALPHA ** k / (1 - ALPHA ** n)
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-11)


def test_ppr_out_star_closed_form():
    """Hub 0 -> dangling leaves, restart at the hub: dangling mass returns to
    the hub, x_hub = (1 - a) + a (1 - x_hub) -> x_hub = 1/(1 + a), and the
    leaves share the rest equally."""
    n = 9
    g = tg.out_star(n)
    x = opr.ppr_fixed_point(g, 0)
    assert abs(x[0] - 1 / (1 + ALPHA)) < 1e-11
    np.testing.assert_allclose(x[1:], (1 - 1 / (1 + ALPHA)) / (n - 1), rtol=0, atol=1e-11)


@pytest.mark.parametrize("seed", range(4))
def test_ppr_dense_and_networkx(seed):
    """Jacobi fixed point == direct solve == networkx with personalization
    and dangling distribution both e_s (an independent implementation)."""
    nx = pytest.importorskip("networkx")
    g = tg.dangling_heavy(40 + 10 * seed, seed) if seed % 2 else tg.random_graph(50, 160, seed)
    s = int(gg.pick_sources(g, 1, seed=seed)[0])
    x = opr.ppr_fixed_point(g, s)
    assert np.abs(x - opr.ppr_dense(g, s)).sum() < 1e-10
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    src, dst = opr.edge_list(g)
    G.add_edges_from(zip(src.tolist(), dst.tolist()))
    e = {v: (1.0 if v == s else 0.0) for v in range(g.n)}
    ref = nx.pagerank(G, alpha=ALPHA, personalization=e, dangling=e, tol=1e-15, max_iter=100000)
    ref = np.array([ref[i] for i in range(g.n)])
    assert np.abs(x - ref).sum() < 1e-10
    assert opr.ppr_certificate(g, x, s) < 1e-9


# ------------------------------------------------------------ access matrix --

def test_access_matrix_matches_loops_and_invariants():
    from oracle import topology as otop
    g = gg.rmat(7, seed=3)
    first = [0, 10, 40, 41, 90, g.n]  # uneven blocks, one of a single vertex
    for groups in (1, 2, 5):
        a, sa = otop.access_matrix(g, first, groups)
        b, sb = otop.access_matrix_loops(g, first, groups)
        np.testing.assert_array_equal(a, b)
        assert sa == sb
        assert a.sum() == g.m  # every edge is one read
    one, _ = otop.access_matrix(g, first, 1)
    assert one[0, 0] == g.m


def test_access_matrix_special_cases():
    from oracle import topology as otop
    n = 12
    # only self-loops: every read is the reader's own value
    g = gg.from_edges(n, np.arange(n), np.arange(n), name="loops")
    c, same = otop.access_matrix(g, [0, 4, 8, 12], 3)
    assert same == n and np.trace(c) == n
    # edges only from block 0 into block 2: all reads by worker 2 of worker 0's values
    g = gg.from_edges(n, np.array([0, 1, 2, 3]), np.array([8, 9, 10, 11]), name="cross")
    c, same = otop.access_matrix(g, [0, 4, 8, 12], 3)
    assert same == 0 and c[2, 0] == 4 and c.sum() == 4
    d, u = otop.shares(c)
    assert d == 0.0 and u == 0.0  # row 2 and column 0 never meet on the diagonal
    # complete graph without self-loops, blocks of 4: 4*3 reads inside a block,
    # 4*4 from each other block; the uniform expectation is 1/3
    g = tg.complete(12)
    c, _ = otop.access_matrix(g, [0, 4, 8, 12], 3)
    np.testing.assert_array_equal(c, np.full((3, 3), 16) - 4 * np.eye(3, dtype=np.int64))
    d, u = otop.shares(c)
    assert abs(d - 36 / 132) < 1e-15 and abs(u - 1 / 3) < 1e-15
