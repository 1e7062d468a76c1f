"""GPU tests of re-partitioning and the autotuner (NEXT f2).

* After re-partitioning to any worker count, PageRank stays within L1 1e-6
  of the oracle's fixed point and SSSP stays bit-exact.
* dg_tune returns a valid choice, leaves the graph with the chosen
  partition, answers a repeated call from its cache, and the cache survives
  a save / clear / load round trip.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp

pytestmark = pytest.mark.gpu

MODES = ("sync", "async", "delayed")


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


def test_repartition_keeps_results(dg):
    g = gg.rmat(13, seed=5)
    xs = opr.pagerank_fixed_point(g)
    ref, _, _ = osp.bellman_ford_sync(g, 7)
    G = dg.Graph.from_csr(g)
    T = G.info().tiles
    for workers in (8, 40, 333, T, 0):
        G.repartition(workers)
        info = G.info()
        if workers:
            assert info.workers == min(workers, T)
        first = G.partition()
        assert first[0] == 0 and first[-1] == g.n and first.shape[0] == info.workers + 1
        for mode in MODES:
            x, st = G.pagerank(tol=1e-7, mode=mode, d=64, dtype="f32")
            assert float(np.abs(x.cpu().numpy() - xs).sum()) <= 1e-6, (workers, mode)
            dist, _ = G.sssp(7, mode=mode, d=64)
            np.testing.assert_array_equal(dist.cpu().numpy(), ref, err_msg=f"workers={workers} {mode}")
    G.close()


def test_tune_pagerank_and_cache(dg, tmp_path):
    g = gg.rmat(16, seed=16)
    G = dg.Graph.from_csr(g)
    dg.tune_cache_clear()
    t = G.tune("pagerank", dtype="f32", tol=1e-6)
    print("tuned", t, flush=True)
    assert t["mode"] in MODES and not t["from_cache"]
    assert t["workers"] == G.info().workers
    if t["mode"] == "delayed":
        assert t["d"] in (16, 64, 256, 1024, 4096, dg.DG_D_WHOLE)
    assert t["seconds"] > 0 and t["sweeps"] > 0 and t["candidates"] >= 8
    # three timed runs of the choice and of the default, with their spread
    assert t["repeats"] == 3
    assert 0 < t["seconds_min"] <= t["seconds"] <= t["seconds_max"]
    assert 0 < t["default_seconds_min"] <= t["default_seconds"] <= t["default_seconds_max"]
    assert t["sweep_variant"] in ("wide", "wide_inflight", "narrow")
    assert dg.VARIANT_NAMES[G.info().sweep_variant] == t["sweep_variant"]
    # the chosen configuration converges to the fixed point
    x, st = G.pagerank(tol=1e-7, mode=t["mode"], d=max(t["d"], 1), dtype="f32")
    assert float(np.abs(x.cpu().numpy() - opr.pagerank_fixed_point(g)).sum()) <= 1e-6
    # and is not slower than the untuned defaults by more than timing noise
    G2 = dg.Graph.from_csr(g)
    base = min(min(G2.pagerank(tol=1e-6, mode=m, d=64, dtype="f32")[1].seconds for _ in range(3)) for m in MODES)
    G2.close()
    best = min(G.pagerank(tol=1e-6, mode=t["mode"], d=max(t["d"], 1), dtype="f32")[1].seconds for _ in range(3))
    print(f"tuned {best * 1e3:.3f} ms vs best default {base * 1e3:.3f} ms", flush=True)
    assert best <= 1.25 * base
    # cache: same graph content answers at once, also through a file
    again = G.tune("pagerank", dtype="f32", tol=1e-6)
    assert again["from_cache"] and (again["mode"], again["d"], again["workers"]) == (t["mode"], t["d"], t["workers"])
    path = tmp_path / "cache.txt"
    dg.tune_cache_save(path)
    dg.tune_cache_clear()
    G3 = dg.Graph.from_csr(g)  # a new handle on the same content
    dg.tune_cache_load(path)
    third = G3.tune("pagerank", dtype="f32", tol=1e-6)
    assert third["from_cache"] and (third["mode"], third["d"]) == (t["mode"], t["d"])
    assert G3.info().workers == t["workers"]
    # the cached mapping is applied too
    assert dg.VARIANT_NAMES[G3.info().sweep_variant] == t["sweep_variant"]
    G3.close()
    G.close()


def test_tune_sssp(dg):
    g = gg.rmat(14, seed=8)
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    G = dg.Graph.from_csr(g)
    t = G.tune("sssp", src=src, keep_workers=True)
    print("tuned sssp", t, flush=True)
    assert t["mode"] in MODES and t["workers"] == G.info().workers
    dist, _ = G.sssp(src, mode=t["mode"], d=max(t["d"], 1))
    np.testing.assert_array_equal(dist.cpu().numpy(), osp.bellman_ford_sync(g, src)[0])
    G.close()


@pytest.mark.parametrize("variant", ["wide", "wide_inflight", "narrow", "auto"])
@pytest.mark.parametrize("res", [0, 1000, None])
def test_set_mapping_keeps_results(dg, variant, res):
    """Any sweep variant (re-tiled for the narrow one) and resident-table
    limit gives PageRank within 1e-6 of the oracle and exact SSSP, also in the
    batched calls, whose tiles change with the narrow variant."""
    g = gg.rmat(14, seed=5)
    xs = opr.pagerank_fixed_point(g)
    src = int(gg.pick_sources(g, 1, seed=3)[0])
    ref, _, _ = osp.bellman_ford_sync(g, src)
    G = dg.Graph.from_csr(g)
    G.set_mapping(variant, dg.DG_RESIDENT_AUTO if res is None else res)
    info = G.info()
    if variant != "auto":
        assert dg.VARIANT_NAMES[info.sweep_variant] == variant
    for mode in MODES:
        x, _ = G.pagerank(tol=1e-7, mode=mode, d=64, dtype="f32")
        assert float(np.abs(x.cpu().numpy() - xs).sum()) <= 1e-6, (variant, res, mode)
        dist, _ = G.sssp(src, mode=mode, d=64)
        np.testing.assert_array_equal(dist.cpu().numpy(), ref)
    rows, _ = G.sssp_batch(np.array([src, 0], np.uint32), mode="async")
    np.testing.assert_array_equal(rows[0].cpu().numpy(), ref)
    G.set_mapping("auto")  # back to the creation-time mapping
    assert G.info().sweep_variant == info.sweep_variant or variant != "auto"
    G.close()


@pytest.mark.parametrize("algo", ["sssp", "ppr"])
def test_tune_batch(dg, algo):
    g = gg.rmat(13, seed=9)
    G = dg.Graph.from_csr(g)
    srcs = gg.pick_sources(g, 20, seed=4)
    t = G.tune_batch(algo, srcs, dtype="f64", tol=1e-9)
    print("tuned batch", algo, t, flush=True)
    assert t["mode"] in MODES and t["candidates"] == 18 and t["repeats"] == 3
    assert 0 < t["seconds_min"] <= t["seconds"] <= t["seconds_max"] and t["seconds"] <= t["default_seconds"]
    # the graph keeps the chosen batched partition, and results stay exact
    if algo == "sssp":
        rows, st = G.sssp_batch(srcs, mode=t["mode"], d=max(t["d"], 1))
        assert st.workers == t["workers"]
        for q in (0, 19):
            np.testing.assert_array_equal(rows[q].cpu().numpy(), osp.bellman_ford_sync(g, int(srcs[q]))[0])
    else:
        rows, st = G.ppr_batch(srcs, tol=1e-9, mode=t["mode"], d=max(t["d"], 1), dtype="f64")
        assert st.workers == t["workers"]
        for q in (0, 19):
            assert float(np.abs(rows[q].cpu().numpy() - opr.ppr_fixed_point(g, int(srcs[q]))).sum()) <= 1e-8
    G.close()
