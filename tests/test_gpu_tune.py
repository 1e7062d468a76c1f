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
    base = G.info().device_bytes - 4 * (G.info().workers + 1)  # all but the worker array
    for workers in (8, 40, 333, T, 0):
        G.repartition(workers)
        info = G.info()
        if workers:
            assert info.workers == min(workers, T)
        assert info.device_bytes == base + 4 * (info.workers + 1)
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
    assert t["capture_chunk"] in (0, 16)  # stage 4: one launch per sweep or captured chunks of 16
    # the chosen configuration (launch setting included) converges to the fixed point
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
    assert third["capture_chunk"] == t["capture_chunk"]
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
    one = np.array([src], np.uint32)

    def arrays():  # entries of the tile, run and worker arrays (single-query and both batched partitions)
        i = G.info()
        wb = G.sssp_batch(one, mode="async")[1].workers + G.ppr_batch(one, tol=1e-9, mode="async", dtype="f64")[1].workers
        return i.tiles + i.batch_tiles + i.workers + wb
    b0, a0 = G.info().device_bytes, arrays()
    G.set_mapping(variant, dg.DG_RESIDENT_AUTO if res is None else res)
    info = G.info()
    # re-tiling replaces those arrays, and device_bytes follows them
    assert info.device_bytes - b0 == 4 * (arrays() - a0), variant
    if variant != "auto":
        assert dg.VARIANT_NAMES[info.sweep_variant] == variant
    # the re-tiled graph's tiles and batched tiles are the host plan's
    p = dg.plan(g.n, g.ptr, g.idx, g.w, compute_units=_cus(), sweep_variant=dg.VARIANT_NAMES[info.sweep_variant])
    assert (info.tiles, info.batch_tiles) == (p["tiles"], p["batch_tiles"]), variant
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


def _cus():
    import torch
    return torch.cuda.get_device_properties(0).multi_processor_count


@pytest.mark.parametrize("algo", ["sssp", "ppr"])
def test_tune_batch(dg, algo):
    g = gg.rmat(13, seed=9)
    G = dg.Graph.from_csr(g)
    srcs = gg.pick_sources(g, 20, seed=4)
    # one batched partition per algorithm: 8 workgroups per CU for SSSP, 5 for
    # PPR (rounded down to a multiple of 8, at most one per batched tile)
    T = G.info().batch_tiles
    assert T > G.info().tiles  # RMAT-13's tiles are split for the batched calls
    want = {a: max(1, min(_cus() * per, T)) for a, per in (("sssp", 8), ("ppr", 5))}
    want = {a: (p & ~7 if p > 8 else p) for a, p in want.items()}
    w_sssp = G.sssp_batch(srcs[:1], mode="async")[1].workers
    w_ppr = G.ppr_batch(srcs[:1], tol=1e-9, mode="async", dtype="f64")[1].workers
    assert (w_sssp, w_ppr) == (want["sssp"], want["ppr"])
    p = dg.plan(g.n, g.ptr, g.idx, g.w, compute_units=_cus())  # the host plan agrees
    assert (p["batch_tiles"], p["batch_workers_sssp"], p["batch_workers_ppr"]) == (T, w_sssp, w_ppr)
    t = G.tune_batch(algo, srcs, dtype="f64", tol=1e-9)
    print("tuned batch", algo, t, flush=True)
    assert t["mode"] in MODES and t["candidates"] == 18 and t["repeats"] == 3
    assert 0 < t["seconds_min"] <= t["seconds"] <= t["seconds_max"] and t["seconds"] <= t["default_seconds"]
    # the graph keeps the chosen batched partition for this algorithm only,
    # and results stay exact
    other = G.ppr_batch(srcs[:1], tol=1e-9, mode="async", dtype="f64")[1].workers if algo == "sssp" else \
        G.sssp_batch(srcs[:1], mode="async")[1].workers
    assert other == (w_ppr if algo == "sssp" else w_sssp)
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


def _small_set(dg, count=16, seed=64):
    rng = np.random.default_rng(seed)
    graphs = []
    for i in range(count):
        if i % 2 == 0:
            graphs.append(gg.rmat(int(rng.integers(6, 12)), seed=400 + i))
        else:
            graphs.append(gg.erdos_renyi(int(rng.integers(100, 3000)), float(rng.integers(4, 17)), seed=400 + i))
    sources = np.array([int(rng.integers(0, g.n)) for g in graphs], np.uint32)
    return graphs, sources


def test_set_repartition_keeps_results(dg):
    """A set's worker blocks rebuilt for other workgroup counts (fewer than
    the graphs: one each) keep SSSP bit-exact with each graph's oracle sweep
    counts in sync mode, and PageRank within the rule's bound."""
    graphs, sources = _small_set(dg)
    refs = [osp.bellman_ford_sync(g, int(s))[:2] for g, s in zip(graphs, sources)]
    xs = [opr.pagerank_fixed_point(g) for g in graphs]
    S = dg.GraphSet(graphs)
    for workers in (1, 16, 100, 2048, 0):
        print(f"set repartition {workers}", flush=True)
        S.repartition(workers)
        assert S.info().workers >= len(graphs)
        out, sw, _ = S.sssp(sources, mode="sync")
        for part, (ref, rs), s_g in zip(S.split(out.cpu().numpy()), refs, sw.tolist()):
            np.testing.assert_array_equal(part, ref)
            assert s_g == rs
        out, _, st = S.pagerank(tol=1e-9, mode="delayed", d=64, dtype="f64")
        assert st.converged
        for part, x in zip(S.split(out.cpu().numpy()), xs):
            assert float(np.abs(part - x).sum()) <= 1e-8
    S.close()


@pytest.mark.parametrize("algo", ["pagerank", "sssp"])
def test_set_tune(dg, algo):
    """dg_set_tune: the choice is a valid candidate, no slower than the
    default in the same measurement, the set keeps the chosen partition, and
    the chosen configuration is still exact (SSSP) or within the rule's bound
    (PageRank)."""
    graphs, sources = _small_set(dg, count=24, seed=65)
    S = dg.GraphSet(graphs)
    print(f"set tune {algo}", flush=True)
    t = S.tune(algo, sources=sources if algo == "sssp" else None, dtype="f64", tol=1e-8)
    assert t["repeats"] == 3 and t["candidates"] >= 7
    assert t["seconds"] <= t["default_seconds"] * (1 + 1e-12)
    assert t["seconds_min"] <= t["seconds"] <= t["seconds_max"]
    assert S.info().workers == t["workers"]
    mode = t["mode"]
    if algo == "sssp":
        out, _, _ = S.sssp(sources, mode=mode, d=t["d"])
        for part, g, s in zip(S.split(out.cpu().numpy()), graphs, sources.tolist()):
            np.testing.assert_array_equal(part, osp.bellman_ford_sync(g, s)[0])
    else:
        out, _, st = S.pagerank(tol=1e-8, mode=mode, d=t["d"], dtype="f64")
        assert st.converged
        for part, g in zip(S.split(out.cpu().numpy()), graphs):
            assert float(np.abs(part - opr.pagerank_fixed_point(g)).sum()) <= 1e-6
    print(f"set tune {algo}: {mode} d={t['d']} workers={t['workers']} {t['seconds'] * 1e3:.3f} ms "
          f"vs default {t['default_seconds'] * 1e3:.3f} ms", flush=True)
    S.close()


def test_repartition_batch(dg):
    """dg_graph_repartition_batch: sets one algorithm's batched partition
    (clamped to one worker per batched tile), leaves the other's alone, 0
    restores the default, an unknown algorithm is refused; results stay
    exact."""
    g = gg.rmat(14, seed=12)
    G = dg.Graph.from_csr(g)
    srcs = gg.pick_sources(g, 3, seed=5)
    T = G.info().batch_tiles
    def workers(algo):
        if algo == "sssp":
            return G.sssp_batch(srcs, mode="async")[1].workers
        return G.ppr_batch(srcs, tol=1e-9, mode="async", dtype="f64")[1].workers
    d_sssp, d_ppr = workers("sssp"), workers("ppr")
    b0 = G.info().device_bytes
    G.repartition_batch("sssp", 3)
    assert workers("sssp") == 3 and workers("ppr") == d_ppr
    assert G.info().device_bytes == b0 + 4 * (3 - d_sssp)  # the worker array is all that changed
    G.repartition_batch("ppr", 10 ** 6)
    assert workers("ppr") == T and workers("sssp") == 3
    rows, _ = G.sssp_batch(srcs, mode="delayed", d=64)
    for q, s in enumerate(srcs.tolist()):
        np.testing.assert_array_equal(rows[q].cpu().numpy(), osp.bellman_ford_sync(g, s)[0])
    p, _ = G.ppr_batch(srcs, tol=1e-9, mode="delayed", d=64, dtype="f64")
    for q, s in enumerate(srcs.tolist()):
        assert float(np.abs(p[q].cpu().numpy() - opr.ppr_fixed_point(g, s)).sum()) <= 1e-8
    G.repartition_batch("sssp", 0)
    G.repartition_batch("ppr", 0)
    assert (workers("sssp"), workers("ppr")) == (d_sssp, d_ppr)
    assert dg.dg_graph_repartition_batch(G._h, 7, 8, None) == dg.DG_ERR_INVALID_ARGUMENT
    G.close()
