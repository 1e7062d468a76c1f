"""GPU parity of graph sets stored as one union graph (many uneven graphs
swept together, one launch per sweep).

* dg_set_sssp: each graph's distances bit-exact against the oracle's
  Bellman-Ford from that graph's source, in every mode, and each graph's
  own sweep count (equal to the oracle's in synchronous mode).
* dg_set_pagerank: each graph's scores (renormalised on its own) within L1
  1e-6 of the oracle's fixed point for that graph alone, float64 storage,
  every mode; synchronous sweeps reproduce each graph's own Jacobi sweeps.  The set stops when every graph's own normalised change is
  below tol, and reports for each graph the first sweep that took it there.
  Float32 is refused below its floor (tol < 1e-7) and accepted above it.
* 64 uneven graphs (R-MAT and G(n, m)) in one set.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp
from tests import graphs as tg
from tests.test_gpu_set import uneven_graphs

pytestmark = pytest.mark.gpu

MODES = [("sync", 1), ("async", 1), ("delayed", 1), ("delayed", 64), ("delayed", 1024), ("delayed", 0xFFFFFFFF)]


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


@pytest.fixture(scope="module")
def graphs():
    return uneven_graphs()


@pytest.fixture(scope="module")
def uset(dg, graphs):
    S = dg.GraphSet(graphs)
    yield S
    S.close()


def test_union_sssp_all_modes(dg, uset, graphs):
    rng = np.random.default_rng(11)
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    refs = [osp.bellman_ford_sync(g, int(s))[:2] for g, s in zip(graphs, sources)]
    ref_sweeps = np.array([r[1] for r in refs])
    for mode, d in MODES:
        out, sw, st = uset.sssp(sources, mode=mode, d=d)
        parts = uset.split(out.cpu().numpy())
        for g, part, (ref, _) in zip(graphs, parts, refs):
            np.testing.assert_array_equal(part, ref, err_msg=f"{g.name} {mode} d={d}")
        # each graph's own count: the first sweep in which it changed nothing
        assert st.converged and sw.max() == st.sweeps and (sw >= 1).all()
        if mode == "sync":
            np.testing.assert_array_equal(sw, ref_sweeps)  # Jacobi sweeps, graph by graph
        else:
            assert (sw <= ref_sweeps).all(), (mode, d, sw, ref_sweeps)
        print(f"union sssp {mode} d={d}: sweeps {st.sweeps} t={st.seconds * 1e3:.2f} ms", flush=True)


def test_union_pagerank_all_modes_f64(dg, uset, graphs):
    refs = [opr.pagerank_fixed_point(g) for g in graphs]
    for mode, d in MODES:
        out, sw, st = uset.pagerank(tol=1e-8, mode=mode, d=d, dtype="f64", max_sweeps=20_000)
        parts = uset.split(out.cpu().numpy())
        errs = [float(np.abs(p - r).sum()) for p, r in zip(parts, refs)]
        worst = int(np.argmax(errs))
        print(f"union pagerank f64 {mode} d={d}: sweeps {st.sweeps} max L1 err {errs[worst]:.2e} "
              f"({graphs[worst].name})", flush=True)
        assert errs[worst] <= 1e-6, (mode, d, graphs[worst].name, errs[worst])
        for p in parts:
            assert abs(p.sum() - 1.0) < 1e-12
        assert st.converged
        # per-graph stop: every graph met the rule, the last one at the set's final sweep
        assert (sw >= 1).all() and (sw <= st.sweeps).all() and sw.max() == st.sweeps, sw


def test_union_pagerank_sync_is_each_graph_alone(dg, uset, graphs):
    """Each graph keeps its own mass in the set (its dangling deficit is
    spread over its own vertices), so synchronous set sweeps are each graph's
    own Jacobi iterates, scaled: per-graph sweep counts equal the oracle's
    for the graph alone, within one for rounding at the threshold."""
    tol = 1e-8
    out, sw, st = uset.pagerank(tol=tol, mode="sync", dtype="f64", max_sweeps=20_000)
    assert st.converged
    for g, s_g, part in zip(graphs, sw.tolist(), uset.split(out.cpu().numpy())):
        x_ref, ref_sweeps, _, _ = opr.pagerank_jacobi(g, tol=tol)
        assert abs(s_g - ref_sweeps) <= 1, (g.name, s_g, ref_sweeps)
        assert float(np.abs(part - x_ref / x_ref.sum()).sum()) <= 1e-9, g.name


def test_union_pagerank_f32(dg, graphs):
    """Float32 storage: refused below its rounding floor, and above it each
    graph (1 vertex next to 20000 included) within the stopping rule's
    bound alpha / (1 - alpha) * tol plus float32 rounding of its scores."""
    S = dg.GraphSet(graphs)
    with pytest.raises(dg.DGError) as e:
        S.pagerank(tol=5e-8, dtype="f32")
    assert e.value.status == dg.DG_ERR_UNSUPPORTED
    for mode, d in (("sync", 1), ("async", 1), ("delayed", 64)):
        out, sw, st = S.pagerank(tol=1e-6, mode=mode, d=d, dtype="f32")
        for p, g in zip(S.split(out.cpu().numpy()), graphs):
            err = float(np.abs(p - opr.pagerank_fixed_point(g)).sum())
            assert err <= 1.1 * 0.85 / 0.15 * 1e-6 + 3e-7, (mode, g.name, err)
        assert (sw >= 1).all() and sw.max() == st.sweeps
    S.close()


def test_union_64_uneven_graphs(dg):
    """64 graphs: R-MAT scales 8-13 mixed with G(n, m) of average degree
    8-32, one launch per sweep for all of them."""
    rng = np.random.default_rng(64)
    graphs = []
    for i in range(64):
        if i % 2 == 0:
            graphs.append(gg.rmat(int(rng.integers(8, 14)), seed=200 + i))
        else:
            graphs.append(gg.erdos_renyi(int(rng.integers(500, 5000)), float(rng.integers(8, 33)), seed=200 + i))
    S = dg.GraphSet(graphs)
    assert S.info().graphs == 64
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    out, sw, st = S.sssp(sources, mode="async")
    print(f"64-graph union sssp async: sweeps {st.sweeps} t={st.seconds * 1e3:.2f} ms", flush=True)
    for part, g, s in zip(S.split(out.cpu().numpy()), graphs, sources.tolist()):
        np.testing.assert_array_equal(part, osp.bellman_ford_sync(g, s)[0], err_msg=g.name)
    out, sw, st = S.pagerank(tol=1e-8, mode="delayed", d=64, dtype="f64")
    print(f"64-graph union pagerank f64 delayed: sweeps {st.sweeps} t={st.seconds * 1e3:.2f} ms, "
          f"per-graph sweeps {sw.min()}..{sw.max()}", flush=True)
    assert (sw >= 1).all() and sw.max() == st.sweeps
    for part, g in zip(S.split(out.cpu().numpy()), graphs):
        assert float(np.abs(part - opr.pagerank_fixed_point(g)).sum()) <= 1e-6, g.name
    S.close()


def test_union_validation(dg, graphs):
    S = dg.GraphSet(graphs[:3])
    with pytest.raises(dg.DGError):
        S.sssp(np.array([0, 0, graphs[2].n], np.uint32))  # source outside its graph
    with pytest.raises(dg.DGError):
        S.pagerank(damping=1.0)
    S.close()


def test_union_more_graphs_than_workers(dg):
    """2000 tiny graphs (1 to 6 vertices, some edgeless): more graphs than the
    default 1280 workers, so every graph still gets a worker of its own.
    SSSP bit-exact with the oracle's per-graph sweep counts in synchronous
    mode; PageRank within the stopping rule's bound for every graph."""
    rng = np.random.default_rng(2000)
    graphs = []
    for i in range(2000):
        n = int(rng.integers(1, 7))
        m = int(rng.integers(0, 3 * n + 1))
        graphs.append(tg.random_graph(n, m, 3000 + i, dedup=False))
    S = dg.GraphSet(graphs)
    info = S.info()
    assert info.graphs == 2000 and info.workers >= 2000
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    refs = [osp.bellman_ford_sync(g, int(s))[:2] for g, s in zip(graphs, sources)]
    for mode, d in (("sync", 1), ("async", 1), ("delayed", 64)):
        out, sw, st = S.sssp(sources, mode=mode, d=d)
        for part, (ref, _) in zip(S.split(out.cpu().numpy()), refs):
            np.testing.assert_array_equal(part, ref)
        if mode == "sync":
            np.testing.assert_array_equal(sw, [r[1] for r in refs])
    out, sw, st = S.pagerank(tol=1e-9, mode="delayed", d=64, dtype="f64")
    for part, g in zip(S.split(out.cpu().numpy()), graphs):
        assert float(np.abs(part - opr.pagerank_fixed_point(g)).sum()) <= 1e-8, g.name
    assert (sw >= 1).all() and sw.max() == st.sweeps
    S.close()
