"""GPU parity of the HIP sweeps against the CPU oracle (needs an MI355X).

Tolerances:
* SSSP: bit-exact in every mode (integers).
* PageRank: L1 distance to the oracle's float64 fixed point <= 1e-6 in every
  mode and precision.  The stopping rule bounds the change of the last sweep,
  not the error, so parity runs stop at tol = 1e-8 (f64) / 1e-7 (f32), where
  the synchronous error bound alpha/(1-alpha)*tol stays below 1e-6.
* Synchronous per-sweep iterates agree with the oracle's Jacobi iterates to
  1e-13 relative L1 (float64; only the summation order differs).
"""
import ctypes as C
import json
import os

import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp
from tests import graphs as tg

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
MODES = [("sync", 0), ("async", 0), ("delayed", 1), ("delayed", 64), ("delayed", 1024), ("delayed", 0xFFFFFFFF),
         ("delayed_local", 64), ("delayed_local", 0xFFFFFFFF)]
PR_TOL = {"f64": 1e-8, "f32": 1e-7}


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


def _np(t):
    return t.cpu().numpy()


_cache = {}


def _graph(name):
    if name not in _cache:
        if name == "rmat10":
            g = gg.rmat(10, seed=10)
        elif name == "rmat14":
            g = gg.rmat(14, seed=14)
        elif name == "rmat16":
            g = gg.rmat(16, seed=16)
        elif name == "banded":
            g = gg.banded(60_000, 16, 4096, 0.01, seed=3)
        elif name == "er":
            g = gg.erdos_renyi(30_001, 12, seed=5)
        elif name == "instar":
            g = tg.in_star(20_000)
        elif name == "multi":
            g = tg.random_graph(3001, 20_000, 7, dedup=False)
        else:
            raise KeyError(name)
        _cache[name] = (g, opr.pagerank_fixed_point(g))
    return _cache[name]


def _sources(g, k=2):
    return gg.pick_sources(g, k, seed=1).tolist()


def test_rmat10_golden_sync(dg):
    """Small R-MAT against the stored oracle values: synchronous PageRank
    float64 within 1e-6 (and sweep count within one of the oracle's, the only
    difference being summation order at the threshold), synchronous
    Bellman-Ford bit-exact with the exact sweep count."""
    with open(os.path.join(HERE, "golden", "rmat10_seed10.json")) as f:
        gold = json.load(f)
    g = gg.rmat(10, seed=10)
    assert g.sha256() == gold["sha256"]
    G = dg.Graph.from_csr(g)
    x, st = G.pagerank(tol=1e-7, mode="sync", dtype="f64")
    assert np.abs(_np(x) - np.array(gold["pagerank_fixed_point"])).sum() <= 1e-6
    assert abs(st.sweeps - gold["pagerank_sync_sweeps_tol1e-7"]) <= 1
    d, st = G.sssp(0, mode="sync")
    np.testing.assert_array_equal(_np(d), np.array(gold["sssp_dist"], dtype=np.uint32))
    assert st.sweeps == gold["sssp_sync_sweeps"]
    G.close()


@pytest.mark.parametrize("name", ["rmat10", "rmat14", "banded", "er", "instar", "multi"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pagerank_all_modes(dg, name, dtype):
    g, xs = _graph(name)
    G = dg.Graph.from_csr(g)
    for mode, d in MODES:
        x, st = G.pagerank(tol=PR_TOL[dtype], mode=mode, d=max(d, 1), dtype=dtype, max_sweeps=2000)
        xv = _np(x)
        err = np.abs(xv - xs).sum()
        assert err <= 1e-6, (name, dtype, mode, d, err, st)
        assert abs(xv.sum() - 1.0) < 1e-12
        assert st.converged and st.sweeps >= 1
        print(f"{name} {dtype} {mode:7s} d={d:<10d} sweeps={st.sweeps:3d} err={err:.2e}")
    G.close()


@pytest.mark.parametrize("name", ["rmat10", "rmat14", "banded", "er", "instar", "multi"])
def test_sssp_all_modes_bit_exact(dg, name):
    g, _ = _graph(name)
    G = dg.Graph.from_csr(g)
    for src in _sources(g):
        ref, ref_sweeps, _ = osp.bellman_ford_sync(g, src)
        for mode, d in MODES:
            dist, st = G.sssp(src, mode=mode, d=max(d, 1))
            np.testing.assert_array_equal(_np(dist), ref, err_msg=f"{name} src={src} {mode} d={d}")
            assert st.converged
            if mode == "sync":
                assert st.sweeps == ref_sweeps
            else:
                assert st.sweeps <= ref_sweeps  # never staler than synchronous
    G.close()


@pytest.mark.parametrize("variant", ["wide", "wide_inflight", "narrow"])
@pytest.mark.parametrize("name", ["rmat14", "banded", "instar"])
def test_sweep_variants(dg, name, variant):
    """Every sweep variant, forced on graphs with a resident table (rmat14),
    without one (banded) and with a hub tile (instar): PageRank within 1e-6
    of the oracle in every mode and precision, SSSP bit-exact in every mode
    with the oracle's synchronous sweep count."""
    g, xs = _graph(name)
    G = dg.Graph.from_csr(g, sweep_variant=variant)
    assert G.info().sweep_variant == dg.SWEEP_VARIANTS[variant]
    for dtype in ("f64", "f32"):
        for mode, d in MODES:
            x, st = G.pagerank(tol=PR_TOL[dtype], mode=mode, d=max(d, 1), dtype=dtype, max_sweeps=2000)
            err = np.abs(_np(x) - xs).sum()
            assert err <= 1e-6 and st.converged, (name, variant, dtype, mode, d, err, st)
    src = _sources(g, 1)[0]
    ref, ref_sweeps, _ = osp.bellman_ford_sync(g, src)
    for mode, d in MODES:
        dist, st = G.sssp(src, mode=mode, d=max(d, 1))
        np.testing.assert_array_equal(_np(dist), ref, err_msg=f"{name} {variant} {mode} d={d}")
        assert st.converged and (st.sweeps == ref_sweeps if mode == "sync" else st.sweeps <= ref_sweeps)
    G.close()


def test_sync_per_sweep_iterates(dg):
    """Synchronous sweeps reproduce the oracle's Jacobi iterates one by one
    (PageRank float64 to 1e-13 relative L1, Bellman-Ford bit-exact)."""
    g, _ = _graph("rmat14")
    G = dg.Graph.from_csr(g)
    _, _, _, its = opr.pagerank_jacobi(g, tol=0.0, max_sweeps=6, keep_iterates=True)
    for k in range(1, 7):
        x, st = G.pagerank(tol=0.0, mode="sync", dtype="f64", max_sweeps=k, allow_not_converged=True)
        assert st.sweeps == k and not st.converged
        ref = its[k - 1] / its[k - 1].sum()
        assert np.abs(_np(x) - ref).sum() <= 1e-13 * np.abs(ref).sum()
    src = _sources(g, 1)[0]
    _, _, bits = osp.bellman_ford_sync(g, src, keep_iterates=True)
    for k in range(1, min(len(bits), 8) + 1):
        d, st = G.sssp(src, mode="sync", max_sweeps=k, allow_not_converged=True)
        np.testing.assert_array_equal(_np(d), bits[k - 1])
    G.close()


def test_path_graph_sync_exact(dg):
    """Path 0 -> ... -> n-1: synchronous needs exactly n sweeps (n-1 with
    changes plus the confirming one); every mode is bit-exact.  A tile's
    vertices are computed concurrently, so inside a tile even asynchronous
    sweeps advance one hop at a time."""
    n = 3000
    g = gg.path_graph(n, weight=2)
    G = dg.Graph.from_csr(g)
    ref = (2 * np.arange(n)).astype(np.uint32)
    d, st = G.sssp(0, mode="sync")
    np.testing.assert_array_equal(_np(d), ref)
    assert st.sweeps == n
    for mode, dd in [("async", 1), ("delayed", 1), ("delayed", 64), ("delayed", 0xFFFFFFFF)]:
        d, st = G.sssp(0, mode=mode, d=dd)
        np.testing.assert_array_equal(_np(d), ref)
        assert st.sweeps <= n
    G.close()


def test_commit_visibility_tile_chain(dg):
    """A chain whose consecutive vertices sit in consecutive tiles (vertex
    TILE*i -> TILE*(i+1), all other vertices isolated, so every tile holds
    TILE = 1024 vertices, the sweep workgroup's size, and one chain vertex).
    Each worker owns L/P consecutive tiles.

    * sync: the chain advances one tile per sweep: exactly L sweeps;
    * async and delayed with d <= TILE: a value committed by tile k is read
      by tile k+1 of the same worker in the same sweep, so a sweep advances
      the chain through a whole worker block: about P sweeps;
    * delayed with d = 4 tiles: commits every fourth tile, more sweeps;
    * delayed with d = whole block: nothing is visible before the block
      ends, so the chain again advances about one tile per sweep.
    """
    TILE = 1024
    L = 8192
    n = TILE * L
    src = TILE * np.arange(L - 1, dtype=np.int64)
    g = gg.from_edges(n, src, src + TILE, w=np.ones(L - 1, np.uint32))
    G = dg.Graph.from_csr(g)
    info = G.info()
    assert info.tiles == L
    P = info.workers
    ref = np.full(n, dg.DG_INF_DIST, np.uint32)
    ref[TILE * np.arange(L)] = np.arange(L)
    d, st = G.sssp(0, mode="sync")
    np.testing.assert_array_equal(_np(d), ref)
    assert st.sweeps == L and st.tile_vertices == TILE
    res = {}
    for mode, dd in [("async", 1), ("delayed", 1), ("delayed", TILE), ("delayed", 4 * TILE), ("delayed", 0xFFFFFFFF)]:
        d, st = G.sssp(0, mode=mode, d=dd)
        np.testing.assert_array_equal(_np(d), ref)
        res[(mode, dd)] = st.sweeps
        print(f"tile chain L={L} P={P} {mode} d={dd}: {st.sweeps} sweeps")
    assert res[("async", 1)] <= 2 * P + 2
    assert res[("delayed", 1)] <= 2 * P + 2
    assert res[("delayed", TILE)] <= 2 * P + 2
    assert res[("delayed", 4 * TILE)] > res[("delayed", TILE)]
    assert res[("delayed", 0xFFFFFFFF)] >= L // 4
    G.close()


def test_edge_cases(dg):
    """Single vertex, edgeless graph, self-loop only, hub beyond one chunk,
    unreachable vertices, NOT_CONVERGED, host outputs through the raw ABI."""
    # one vertex, no edge: score 1, distance 0
    G = dg.Graph(1, np.array([0, 0], np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    for mode, d in MODES:
        x, st = G.pagerank(mode=mode, d=max(d, 1), dtype="f64")
        assert abs(_np(x)[0] - 1.0) < 1e-15
        dist, _ = G.sssp(0, mode=mode, d=max(d, 1))
        assert _np(dist)[0] == 0
    G.close()
    # self-loop only
    G = dg.Graph(1, np.array([0, 1], np.uint64), np.zeros(1, np.uint32), np.array([9], np.uint32))
    x, _ = G.pagerank(dtype="f64")
    assert abs(_np(x)[0] - 1.0) < 1e-15
    G.close()
    # edgeless graph: all dangling -> uniform
    n = 777
    G = dg.Graph(n, np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    for mode, d in MODES:
        x, _ = G.pagerank(mode=mode, d=max(d, 1), dtype="f32")
        assert np.abs(_np(x) - 1.0 / n).max() < 1e-12
        dist, _ = G.sssp(5, mode=mode, d=max(d, 1))
        dv = _np(dist)
        assert dv[5] == 0 and (np.delete(dv, 5) == dg.DG_INF_DIST).all()
    G.close()
    # NOT_CONVERGED keeps the last iterate and stats
    g, xs = _graph("rmat10")
    G = dg.Graph.from_csr(g)
    with pytest.raises(dg.DGError) as ei:
        G.pagerank(tol=1e-12, max_sweeps=2)
    assert ei.value.status == dg.DG_ERR_NOT_CONVERGED
    x, st = G.pagerank(tol=1e-12, max_sweeps=2, allow_not_converged=True)
    assert st.sweeps == 2 and not st.converged
    # host output pointers through the raw C ABI
    out = np.zeros(g.n, np.float64)
    stats = dg.dg_stats()
    s = dg.dg_pagerank(G._h, 0.85, 1e-8, dg.DG_DELAYED, 64, dg.DG_F64, 1000, dg._np_ptr(out), 0,
                       C.byref(stats), None)
    assert s == dg.DG_OK and np.abs(out - xs).sum() < 1e-6
    dout = np.zeros(g.n, np.uint32)
    s = dg.dg_sssp(G._h, 0, dg.DG_ASYNC, 1, 5000, dg._np_ptr(dout), 0, C.byref(stats), None)
    assert s == dg.DG_OK
    np.testing.assert_array_equal(dout, osp.bellman_ford_sync(g, 0)[0])
    # validation on a live handle leaves outputs untouched
    s = dg.dg_sssp(G._h, g.n, dg.DG_SYNC, 1, 10, dg._np_ptr(dout), 0, None, None)
    assert s == dg.DG_ERR_INVALID_ARGUMENT
    s = dg.dg_pagerank(G._h, 1.0, 1e-6, dg.DG_SYNC, 1, dg.DG_F32, 10, dg._np_ptr(out), 0, None, None)
    assert s == dg.DG_ERR_INVALID_ARGUMENT
    s = dg.dg_pagerank(G._h, 0.85, 1e-6, dg.DG_DELAYED, 0, dg.DG_F32, 10, dg._np_ptr(out), 0, None, None)
    assert s == dg.DG_ERR_INVALID_ARGUMENT
    G.close()
    # PageRank-only graph refuses SSSP
    Gn = dg.Graph(g.n, g.ptr, g.idx, None)
    with pytest.raises(dg.DGError):
        Gn.sssp(0)
    Gn.close()


def test_csc_input_matches_csr(dg):
    """The same graph handed over as in-edges gives the same answers."""
    g, xs = _graph("rmat10")
    src = np.repeat(np.arange(g.n), np.diff(g.ptr.astype(np.int64)))
    order = np.lexsort((src, g.idx))
    cptr = np.zeros(g.n + 1, np.uint64)
    np.cumsum(np.bincount(g.idx, minlength=g.n), out=cptr[1:])
    G = dg.Graph(g.n, cptr, src[order].astype(np.uint32), g.w[order], layout="csc")
    x, _ = G.pagerank(tol=1e-8, mode="async", dtype="f64")
    assert np.abs(_np(x) - xs).sum() < 1e-6
    d, _ = G.sssp(3, mode="delayed", d=64)
    np.testing.assert_array_equal(_np(d), osp.bellman_ford_sync(g, 3)[0])
    G.close()


def test_repeatability_async(dg):
    """Asynchronous results vary run to run only within tolerance (PageRank)
    and not at all (SSSP)."""
    g, xs = _graph("rmat14")
    G = dg.Graph.from_csr(g)
    src = _sources(g, 1)[0]
    ref = osp.bellman_ford_sync(g, src)[0]
    for _ in range(5):
        x, _ = G.pagerank(tol=1e-7, mode="async", dtype="f32")
        assert np.abs(_np(x) - xs).sum() <= 1e-6
        d, _ = G.sssp(src, mode="delayed", d=1)
        np.testing.assert_array_equal(_np(d), ref)
    G.close()


@pytest.mark.parametrize("hot,workers", [(0, 0), (1000, 0), (0xFFFFFFFF, 3), (0xFFFFFFFF, 17), (50, 1)])
def test_options_hot_region_and_workers(dg, hot, workers):
    """The compact hot region and the worker count change only where values
    are stored and who computes them: results stay bit-exact (SSSP) and within
    tolerance (PageRank), in every mode."""
    g, xs = _graph("rmat14")
    G = dg.Graph.from_csr(g, hot_vertices=hot, workers=workers)
    info = G.info()
    if hot == 0:
        assert info.hot_vertices == 0 and info.hot_edges == 0
    else:
        assert 0 < info.hot_vertices <= hot
    if workers:
        assert info.workers == workers
    src = _sources(g, 1)[0]
    ref = osp.bellman_ford_sync(g, src)[0]
    for mode, d in MODES:
        x, _ = G.pagerank(tol=1e-8, mode=mode, d=max(d, 1), dtype="f64")
        assert np.abs(_np(x) - xs).sum() <= 1e-6
        dist, _ = G.sssp(src, mode=mode, d=max(d, 1))
        np.testing.assert_array_equal(_np(dist), ref)
    G.close()


def _resident_reference(g, res_opt=0xFFFFFFFF, hot_cap=524288):
    """Compact region and resident table by their definition: candidates are
    sources with out-degree above 1 and above the average, the region takes
    the largest hot_cap of them, the table the largest min(res_opt, 32768) of
    those; the automatic size (res_opt = all ones) keeps the table only if
    its sources cover at least 1/16 of the edges."""
    od = np.diff(g.ptr.astype(np.int64))
    cand = np.nonzero((od > 1) & (od > g.m / g.n))[0]
    top = cand[np.argsort(-od[cand], kind="stable")][:hot_cap]
    r = min(top.size, res_opt, 32768)
    cover = int(od[top[:r]].sum())
    if res_opt == 0xFFFFFFFF and cover * 16 < g.m:
        r, cover = 0, 0
    return top.size, int(od[top].sum()), r, cover


@pytest.mark.parametrize("name,res", [("rmat14", 0xFFFFFFFF), ("er", 0xFFFFFFFF), ("rmat14", 100),
                                      ("banded", 0xFFFFFFFF)])
def test_resident_table_sync_same_values(dg, name, res):
    """Synchronous sweeps read the resident table where they would gather the
    same values (the table is filled from the sweep's unchanging input).
    SSSP is bit-identical with and without it; PageRank agrees up to the
    order in which LDS atomics add a vertex's partial sums (which varies
    from run to run as well)."""
    g, xs = _graph(name)
    A = dg.Graph.from_csr(g, resident_vertices=res)
    B = dg.Graph.from_csr(g, resident_vertices=0)
    ia, ib = A.info(), B.info()
    K, hot_e, R, res_e = _resident_reference(g, res)
    assert (ia.hot_vertices, ia.hot_edges) == (K, hot_e) == (ib.hot_vertices, ib.hot_edges)
    assert (ia.resident_vertices, ia.resident_edges) == (R, res_e)
    assert (ib.resident_vertices, ib.resident_edges) == (0, 0)
    assert R > 0
    for dtype, tol, same in (("f32", 1e-7, 1e-6), ("f64", 1e-10, 1e-12)):
        xa, sa = A.pagerank(tol=tol, mode="sync", dtype=dtype)
        xb, sb = B.pagerank(tol=tol, mode="sync", dtype=dtype)
        assert abs(sa.sweeps - sb.sweeps) <= 1
        bound = same if sa.sweeps == sb.sweeps else 10 * tol / (1 - 0.85)  # one sweep more: within the stop rule
        assert np.abs(_np(xa) - _np(xb)).sum() <= bound, dtype
        assert np.abs(_np(xa) - xs).sum() <= 1e-6
    for src in _sources(g, 2):
        da, sa = A.sssp(src, mode="sync")
        db, sb = B.sssp(src, mode="sync")
        assert sa.sweeps == sb.sweeps
        np.testing.assert_array_equal(_np(da), _np(db))
        np.testing.assert_array_equal(_np(da), osp.bellman_ford_sync(g, src)[0])
    A.close()
    B.close()


@pytest.mark.parametrize("res", [1, 100, 8193, 0xFFFFFFFF])
def test_resident_table_async_delayed_local(dg, res):
    """Asynchronous and delayed sweeps refresh the table a segment at a time
    after every tile: table sizes below, at and across a segment boundary,
    every commit interval, and the local-read variant, all converge to the
    oracle's fixed point (PageRank) and its exact distances (SSSP)."""
    g, xs = _graph("rmat16")
    G = dg.Graph.from_csr(g, resident_vertices=res)
    assert G.info().resident_vertices == _resident_reference(g, res)[2] > 0
    src = _sources(g, 1)[0]
    ref = osp.bellman_ford_sync(g, src)[0]
    for mode, ds in (("async", (1,)), ("delayed", (1, 64, 1024, 0xFFFFFFFF)),
                     ("delayed_local", (64, 0xFFFFFFFF))):
        for d in ds:
            for dtype, tol in (("f32", 1e-7), ("f64", 1e-9)):
                x, _ = G.pagerank(tol=tol, mode=mode, d=d, dtype=dtype)
                assert np.abs(_np(x) - xs).sum() <= 1e-6, (mode, d, dtype)
            dist, _ = G.sssp(src, mode=mode, d=d)
            np.testing.assert_array_equal(_np(dist), ref, err_msg=f"{mode} d={d}")
    G.close()


@pytest.mark.parametrize("wmax,wbytes", [(255, 1), (256, 4), (1 << 24, 4)])
def test_weight_storage(dg, wmax, wbytes):
    """Weights that all fit a byte are kept as bytes, others as uint32; both
    streams give the oracle's exact distances in every mode, single-source
    and batched.  The byte case includes the largest byte value; the
    uint32 cases include a weight of 256 (the boundary) and weights up to
    2^24 (long paths that saturate nothing)."""
    import dataclasses
    g0, _ = _graph("rmat14")
    rng = np.random.default_rng(wmax)
    w = rng.integers(1, wmax + 1, size=g0.m, dtype=np.uint64).astype(np.uint32)
    w[rng.integers(0, g0.m)] = wmax  # the largest weight occurs
    g = dataclasses.replace(g0, w=w, name=f"rmat14_w{wmax}")
    G = dg.Graph.from_csr(g)
    assert G.info().weight_bytes == wbytes
    srcs = _sources(g, 3)
    refs = [osp.bellman_ford_sync(g, s)[0] for s in srcs]
    for mode, d in MODES:
        for s, ref in zip(srcs, refs):
            dist, _ = G.sssp(s, mode=mode, d=max(d, 1))
            np.testing.assert_array_equal(_np(dist), ref, err_msg=f"{mode} d={d} w<={wmax}")
        if mode != "delayed_local":
            out, _ = G.sssp_batch(srcs, mode=mode, d=max(d, 1))
            for i, ref in enumerate(refs):
                np.testing.assert_array_equal(_np(out[i]), ref, err_msg=f"batch {mode} d={d} w<={wmax}")
    G.close()
