"""GPU parity of graph sets (many uneven graphs swept in one launch per sweep).

Each graph of the set is checked against the oracle on its own:

* dg_set_sssp: distances bit-exact against the oracle's Bellman-Ford from the
  graph's source, in every mode, and the per-graph sweep counts are
  plausible (synchronous mode: exactly the oracle's count).
* dg_set_pagerank: each graph's scores within L1 1e-8 (float64 storage,
  tol 1e-9) or 1e-6 (float32, tol 1e-7) of the oracle's fixed point for that
  graph alone, in every mode.
* Captured (HIP graph) and eager launches give the same bits in synchronous
  mode, and a cached capture replays correctly for a second call with other
  sources.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp
from tests import graphs as tg

pytestmark = pytest.mark.gpu

# These tests ran the first implementation of set sweeps (a global tile work
# list with per-graph fold kernels, chunks of sweeps captured into a HIP
# graph).  Its first GPU run, test_set_sssp_all_modes with a captured
# synchronous chunk, stopped making progress and no cause was identified; that
# implementation was removed.  Sets now run as one union graph on the
# single-graph kernels and are tested in test_gpu_set_union.py.  These tests
# stay, skipped.
SWEEPS_OFF = pytest.mark.skip(reason="ran the removed captured-chunk set implementation, whose first GPU run "
                                     "stalled with no cause identified; see test_gpu_set_union.py")

MODES = [("sync", 1), ("async", 1), ("delayed", 1), ("delayed", 64), ("delayed", 1024), ("delayed", 0xFFFFFFFF)]


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


def uneven_graphs():
    """Sizes from 1 to 20000 vertices, a hub beyond one tile, dangling-heavy,
    edgeless, long paths (many sweeps) and dense ones (few)."""
    return [
        gg.rmat(10, seed=1), gg.rmat(12, seed=2), gg.erdos_renyi(3000, 8, seed=3), tg.in_star(20_000),
        tg.dangling_heavy(2000, 4), gg.path_graph(300, weight=7), tg.cycle(50), tg.complete(20), tg.empty(7),
        tg.two_scc(400, 5), gg.banded(20_000, 8, 256, 0.01, seed=5), gg.rmat(8, seed=9),
        gg.from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64), weight_seed=1, name="single"),
        tg.out_star(300),
    ]


@pytest.fixture(scope="module")
def graphs():
    return uneven_graphs()


@pytest.fixture(scope="module")
def gset(dg, graphs):
    S = dg.GraphSet(graphs)
    yield S
    S.close()


def test_set_info(gset, graphs):
    info = gset.info()
    assert info.graphs == len(graphs)
    assert info.n == sum(g.n for g in graphs)
    assert info.m == sum(g.m for g in graphs)
    assert info.has_weights == 1


@SWEEPS_OFF
def test_set_sssp_all_modes(dg, gset, graphs):
    rng = np.random.default_rng(11)
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    refs = [osp.bellman_ford_sync(g, int(s))[:2] for g, s in zip(graphs, sources)]
    for mode, d in MODES:
        for eager in (False, True):
            out, sw, st = gset.sssp(sources, mode=mode, d=d, eager=eager)
            parts = gset.split(out.cpu().numpy())
            for i, (g, (ref, ref_sweeps)) in enumerate(zip(graphs, refs)):
                np.testing.assert_array_equal(parts[i], ref, err_msg=f"{g.name} {mode} d={d} eager={eager}")
                assert sw[i] >= 1
                if mode == "sync":
                    assert sw[i] == ref_sweeps, (g.name, sw[i], ref_sweeps)
            assert st.converged and st.sweeps == sw.max()
        print(f"set sssp {mode} d={d}: sweeps max {sw.max()} t={st.seconds * 1e3:.2f} ms", flush=True)


@pytest.mark.parametrize("dtype,tol,bound", [("f64", 1e-9, 1e-8), ("f32", 1e-7, 1e-6)])
@SWEEPS_OFF
def test_set_pagerank_all_modes(dg, gset, graphs, dtype, tol, bound):
    refs = [opr.pagerank_fixed_point(g) for g in graphs]
    for mode, d in MODES:
        out, sw, st = gset.pagerank(tol=tol, mode=mode, d=d, dtype=dtype, max_sweeps=5000)
        parts = gset.split(out.cpu().numpy())
        errs = [float(np.abs(p - r).sum()) for p, r in zip(parts, refs)]
        worst = int(np.argmax(errs))
        print(f"set pagerank {dtype} {mode} d={d}: sweeps {sw.tolist()} max L1 err {errs[worst]:.2e} "
              f"({graphs[worst].name}) t={st.seconds * 1e3:.2f} ms", flush=True)
        assert errs[worst] <= bound, (mode, d, graphs[worst].name, errs[worst])
        for p in parts:
            assert abs(p.sum() - 1.0) < 1e-9
        assert st.converged and (sw >= 1).all()


@SWEEPS_OFF
def test_set_pagerank_sync_sweeps_match_oracle(dg, gset, graphs):
    """Synchronous sweeps of each graph follow the oracle's Jacobi iteration,
    so each graph stops after the oracle's number of sweeps (float64)."""
    _, sw, _ = gset.pagerank(tol=1e-8, mode="sync", dtype="f64", max_sweeps=5000)
    for i, g in enumerate(graphs):
        _, ref_sweeps, res, _ = opr.pagerank_jacobi(g, tol=1e-8)
        # a residual within rounding of the tolerance may stop one sweep apart
        near = any(abs(r - 1e-8) < 1e-12 for r in res)
        assert sw[i] == ref_sweeps or (near and abs(int(sw[i]) - ref_sweeps) <= 1), (g.name, sw[i], ref_sweeps)


@SWEEPS_OFF
def test_set_capture_matches_eager_and_replays(dg, gset, graphs):
    a, _, _ = gset.pagerank(tol=1e-9, mode="sync", dtype="f64", eager=True)
    for _ in range(3):  # the captured chunk is cached and replayed across calls
        b, _, _ = gset.pagerank(tol=1e-9, mode="sync", dtype="f64")
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    rng = np.random.default_rng(3)
    for rep in range(3):
        sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
        e, _, _ = gset.sssp(sources, mode="sync", eager=True)
        c, _, _ = gset.sssp(sources, mode="sync")
        np.testing.assert_array_equal(e.cpu().numpy(), c.cpu().numpy())
        parts = gset.split(c.cpu().numpy())
        for i in (0, 5, 10):
            np.testing.assert_array_equal(parts[i], osp.bellman_ford_sync(graphs[i], int(sources[i]))[0])


@SWEEPS_OFF
def test_set_of_many_small_graphs(dg):
    """64 uneven graphs (R-MAT scales 6-11 mixed with G(n, m) of average degree
    8-32), one launch per sweep for all of them."""
    rng = np.random.default_rng(64)
    graphs = []
    for i in range(64):
        if i % 2 == 0:
            graphs.append(gg.rmat(int(rng.integers(6, 12)), seed=100 + i))
        else:
            graphs.append(gg.erdos_renyi(int(rng.integers(100, 3000)), float(rng.integers(8, 33)), seed=100 + i))
    S = dg.GraphSet(graphs)
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    out, sw, st = S.sssp(sources, mode="async")
    parts = S.split(out.cpu().numpy())
    for i, g in enumerate(graphs):
        np.testing.assert_array_equal(parts[i], osp.bellman_ford_sync(g, int(sources[i]))[0], err_msg=g.name)
    out, sw, st = S.pagerank(tol=1e-7, mode="delayed", d=64)
    parts = S.split(out.cpu().numpy())
    for i, g in enumerate(graphs):
        assert np.abs(parts[i] - opr.pagerank_fixed_point(g)).sum() <= 1e-6, g.name
    S.close()
