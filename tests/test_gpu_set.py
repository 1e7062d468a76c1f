"""GPU parity of graph sets run as recorded chunks of sweeps (captured
launches of the union graph, dg_set_set_capture), against the oracle and
against one launch per sweep.

Each graph of the set is checked against the oracle on its own:

* dg_set_sssp: distances bit-exact against the oracle's Bellman-Ford from the
  graph's source, in every mode, captured and eager, and the per-graph sweep
  counts (synchronous mode: exactly the oracle's count).
* dg_set_pagerank: each graph's scores within L1 1e-8 (float64 storage,
  tol 1e-9) or the stopping rule's bound (float32, tol 1e-6) of the oracle's
  fixed point for that graph alone, in every mode; synchronous sweeps agree
  captured and eager to rounding (L1 1e-13: the in-edge sums use LDS
  atomics, whose order varies between any two runs).
* The recorded chunks are replayed across calls (with eager device work and
  synchronisations between the replays), for other sources too.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp
from tests import graphs as tg

pytestmark = pytest.mark.gpu

CHUNK = 8  # sweeps per recorded chunk

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


def test_set_sssp_all_modes(dg, gset, graphs):
    rng = np.random.default_rng(11)
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    refs = [osp.bellman_ford_sync(g, int(s))[:2] for g, s in zip(graphs, sources)]
    for mode, d in MODES:
        for chunk in (CHUNK, 0):
            print(f"set sssp {mode} d={d} chunk={chunk}", flush=True)
            gset.set_capture(chunk)
            out, sw, st = gset.sssp(sources, mode=mode, d=d)
            parts = gset.split(out.cpu().numpy())
            for i, (g, (ref, ref_sweeps)) in enumerate(zip(graphs, refs)):
                np.testing.assert_array_equal(parts[i], ref, err_msg=f"{g.name} {mode} d={d} chunk={chunk}")
                assert sw[i] >= 1
                if mode == "sync":
                    assert sw[i] == ref_sweeps, (g.name, sw[i], ref_sweeps)
            assert st.converged and st.sweeps == sw.max()
        print(f"set sssp {mode} d={d}: sweeps max {sw.max()} t={st.seconds * 1e3:.2f} ms", flush=True)
    gset.set_capture(0)


@pytest.mark.parametrize("dtype,tol,bound", [("f64", 1e-9, 1e-8), ("f32", 1e-6, 1.1 * 0.85 / 0.15 * 1e-6 + 3e-7)])
def test_set_pagerank_all_modes(dg, gset, graphs, dtype, tol, bound):
    refs = [opr.pagerank_fixed_point(g) for g in graphs]
    gset.set_capture(CHUNK)
    for mode, d in MODES:
        print(f"set pagerank {dtype} {mode} d={d}", flush=True)
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
    gset.set_capture(0)


def test_set_pagerank_sync_sweeps_match_oracle(dg, gset, graphs):
    """Synchronous sweeps of each graph follow the oracle's Jacobi iteration,
    so each graph stops after the oracle's number of sweeps (float64),
    captured launches."""
    gset.set_capture(CHUNK)
    _, sw, _ = gset.pagerank(tol=1e-8, mode="sync", dtype="f64", max_sweeps=5000)
    gset.set_capture(0)
    for i, g in enumerate(graphs):
        _, ref_sweeps, res, _ = opr.pagerank_jacobi(g, tol=1e-8)
        # a residual within rounding of the tolerance may stop one sweep apart
        near = any(abs(r - 1e-8) < 1e-12 for r in res)
        assert sw[i] == ref_sweeps or (near and abs(int(sw[i]) - ref_sweeps) <= 1), (g.name, sw[i], ref_sweeps)


def test_set_capture_matches_eager_and_replays(dg, gset, graphs):
    import torch
    gset.set_capture(0)
    a, _, sa = gset.pagerank(tol=1e-9, mode="sync", dtype="f64")
    rng = np.random.default_rng(3)
    srcs = [np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32) for _ in range(3)]
    eager = [gset.sssp(s_, mode="sync")[0].cpu().numpy() for s_ in srcs]
    gset.set_capture(CHUNK)
    for rep in range(3):  # the recorded chunks are kept and replayed across calls
        print(f"set capture replay {rep}", flush=True)
        b, _, sb = gset.pagerank(tol=1e-9, mode="sync", dtype="f64")
        # in-edge sums in LDS atomics: runs differ in the last bits only
        assert float(np.abs(a.cpu().numpy() - b.cpu().numpy()).sum()) <= 1e-13
        assert abs(sb.sweeps - sa.sweeps) <= 1
        x = torch.ones(1 << 20, device="cuda").cumsum(0)  # eager device work between replays
        torch.cuda.synchronize()
        assert float(x[-1]) == float(1 << 20)
    for rep, (s_, e) in enumerate(zip(srcs, eager)):
        c, _, _ = gset.sssp(s_, mode="sync")
        np.testing.assert_array_equal(e, c.cpu().numpy(), err_msg=f"sources {rep}")
        parts = gset.split(c.cpu().numpy())
        for i in (0, 5, 10):
            np.testing.assert_array_equal(parts[i], osp.bellman_ford_sync(graphs[i], int(s_[i]))[0])
    gset.set_capture(0)


def test_set_of_many_small_graphs(dg):
    """64 uneven graphs (R-MAT scales 6-11 mixed with G(n, m) of average degree
    8-32), swept together as recorded chunks."""
    rng = np.random.default_rng(64)
    graphs = []
    for i in range(64):
        if i % 2 == 0:
            graphs.append(gg.rmat(int(rng.integers(6, 12)), seed=100 + i))
        else:
            graphs.append(gg.erdos_renyi(int(rng.integers(100, 3000)), float(rng.integers(8, 33)), seed=100 + i))
    S = dg.GraphSet(graphs)
    S.set_capture(CHUNK)
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    print("64-graph set, captured", flush=True)
    out, sw, st = S.sssp(sources, mode="async")
    parts = S.split(out.cpu().numpy())
    for i, g in enumerate(graphs):
        np.testing.assert_array_equal(parts[i], osp.bellman_ford_sync(g, int(sources[i]))[0], err_msg=g.name)
    out, sw, st = S.pagerank(tol=1e-8, mode="delayed", d=64, dtype="f64")
    parts = S.split(out.cpu().numpy())
    for i, g in enumerate(graphs):
        assert np.abs(parts[i] - opr.pagerank_fixed_point(g)).sum() <= 1e-6, g.name
    S.close()
