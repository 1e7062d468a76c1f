"""Pins of the C PageRank oracle (CPU only).  It must reproduce what the
mathematics and the independently pinned numpy oracle fix:

* the closed forms (cycle, edgeless, in-star hub, out-star hub, two-vertex
  chain) and a dense direct solve on small graphs with dangling vertices,
  self-loops and duplicate edges;
* the numpy oracle's Jacobi iterates sweep by sweep (the same per-vertex
  summation order) to 1e-15 relative L1, and the same sweep count at a tol;
* mass 1 of every iterate (the Jacobi map conserves mass);
* the same result for any thread count;
* for personalised PageRank: the dense solve, the out-star closed form, the
  dangling restart vertex (x* = e_s), and the numpy oracle's iterates.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen as gg
from oracle import cpr
from oracle import pagerank as opr
from tests import graphs as tg

A = 0.85


def test_closed_forms():
    n = 5
    x = cpr.pagerank_fixed_point(tg.in_star(n))
    assert abs(x[0] - (1 + (n - 1) * A) / (n + (n - 1) * A)) < 1e-12
    assert np.abs(x[1:] - ((1 - A) / n + A * x[0] / n)).max() < 1e-12
    x = cpr.pagerank_fixed_point(tg.out_star(n))
    assert abs(x[0] - 1 / (n + A)) < 1e-12
    for g in (tg.cycle(7), tg.complete(6), tg.empty(9)):
        x = cpr.pagerank_fixed_point(g)
        assert np.abs(x - 1 / g.n).max() < 1e-12
    x = cpr.pagerank_fixed_point(gg.from_edges(2, [0], [1]))
    assert abs(x[0] - 1 / (2 + A)) < 1e-12


@pytest.mark.parametrize("g", [tg.random_graph(60, 200, 1), tg.dangling_heavy(50, 2),
                               tg.random_graph(40, 300, 3, dedup=False)], ids=["random", "dangling", "multi"])
def test_dense_solve(g):
    assert np.abs(cpr.pagerank_fixed_point(g) - opr.pagerank_dense(g)).sum() < 1e-12


@pytest.mark.parametrize("g", [gg.rmat(12, seed=4), tg.dangling_heavy(3000, 7), gg.banded(20_000, 16, 300, 0.01,
                                                                                          seed=2)],
                         ids=["rmat12", "dangling", "banded"])
def test_iterates_match_numpy_oracle(g):
    for k in (1, 2, 5):
        xc, sc, rc = cpr.pagerank_jacobi(g, tol=0.0, max_sweeps=k)
        xp, sp, rp, _ = opr.pagerank_jacobi(g, tol=0.0, max_sweeps=k)
        assert sc == sp == k
        assert np.abs(xc - xp).sum() <= 1e-15 * np.abs(xp).sum() + 1e-18
        assert abs(rc - rp[-1]) <= 1e-12 * rp[-1]
        assert abs(xc.sum() - 1.0) < 1e-12
    xc, sc, _ = cpr.pagerank_jacobi(g, tol=1e-9)
    _, sp, _, _ = opr.pagerank_jacobi(g, tol=1e-9)
    assert sc == sp


def test_thread_count_does_not_change_the_result(tmp_path):
    code = ("import sys, numpy as np; sys.path.insert(0, %r); import graphgen as gg; from oracle import cpr; "
            "x, s, r = cpr.pagerank_jacobi(gg.rmat(11, seed=3), tol=1e-10); np.save(sys.argv[1], x)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for threads in (1, 3):
        f = str(tmp_path / f"x{threads}.npy")
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        subprocess.run([sys.executable, "-c", code % root, f], check=True, env=env, timeout=300)
        outs.append(np.load(f))
    assert np.array_equal(outs[0], outs[1])


def test_malformed_input_refused():
    g = tg.random_graph(10, 30, 1)
    bad = gg.CSRGraph(g.n, g.ptr, np.where(g.idx == 0, 10, g.idx).astype(np.uint32), g.w, "bad")
    with pytest.raises(ValueError):
        cpr.pagerank_jacobi(bad)


def test_ppr_pins():
    for g, s in [(tg.random_graph(60, 200, 1), 5), (tg.dangling_heavy(50, 2), 3)]:
        assert np.abs(cpr.ppr_fixed_point(g, s) - opr.ppr_dense(g, s)).sum() < 1e-12
    n = 9
    x = cpr.ppr_fixed_point(tg.out_star(n), 0)
    assert abs(x[0] - 1 / (1 + A)) < 1e-12
    assert np.abs(x[1:] - (1 - 1 / (1 + A)) / (n - 1)).max() < 1e-12
    g = tg.dangling_heavy(40, 4)
    s = int(np.flatnonzero(np.diff(g.ptr.astype(np.int64)) == 0)[0])
    x = cpr.ppr_fixed_point(g, s)
    assert abs(x[s] - 1.0) < 1e-12 and abs(x.sum() - 1.0) < 1e-12


def test_ppr_iterates_match_numpy_oracle():
    g = gg.rmat(12, seed=4)
    s = int(gg.pick_sources(g, 1, seed=1)[0])
    for k in (1, 3):
        xc, sc, _ = cpr.pagerank_jacobi(g, tol=0.0, max_sweeps=k, restart=s)
        xp, sp = opr.ppr_jacobi(g, s, tol=0.0, max_sweeps=k)
        assert sc == sp == k
        assert np.abs(xc - xp).sum() <= 1e-15
    with pytest.raises(ValueError):
        cpr.pagerank_jacobi(g, restart=g.n)
