"""CPU tests of the host-side layout (dg_plan_*, the construction
dg_graph_create uploads), against each part's definition written out here
with numpy:

* the in-edge form of the pull sweep (section III-A): in_ptr counts
  in-edges, and the in-edges of a vertex keep the order of their sources;
* the compact region: the K largest above-average out-degrees (ties by
  vertex id), the resident table as its first R slots in two vertex-ordered
  halves, the rest in vertex order; the automatic table only when its
  sources cover 1/16 of the edges;
* tiles: greedy runs of at most 1024 vertices and 16380 in-edges, a larger
  vertex alone; 8188 in-edges (the narrow sweep variant) when the wide
  tiles number fewer than 2 per worker; the automatic variant by tiles per
  worker (narrow < 2 <= wide with all gathers in flight <= 8 < wide);
* the blocked partition (section III-A: contiguous blocks balanced by
  in-edges): P contiguous tile ranges split at the cost quantiles;
* the tiles of the batched calls: each tile cut greedily into runs of at
  most 4096 in-edges, a larger vertex alone, never across a tile; their
  default partitions (8 and 5 workgroups per compute unit);
* byte weights exactly when every weight fits a byte;
* CSC input gives the same plan as the equivalent CSR input;
* argument validation.
"""
import dataclasses

import numpy as np
import pytest

import graphgen as gg
from tests import graphs as tg


@pytest.fixture(scope="module")
def dg():
    from paper_2110_01409_amd import dg as _dg
    return _dg


AUTO = 0xFFFFFFFF
TILE_V, TILE_E, TILE_E_NARROW = 1024, 16380, 8188
PER_CU = 1  # sweep workgroups per compute unit
WIDE, WIDE_INFLIGHT, NARROW = 1, 2, 3


def _ref_cpos(g, hot=AUTO, res=AUTO):
    n, m = g.n, g.m
    od = np.diff(g.ptr.astype(np.int64))
    cand = np.nonzero((od > 1) & (od > m / n))[0]
    top = cand[np.argsort(-od[cand], kind="stable")]
    top = top[: (524288 if hot == AUTO else hot)]
    K = top.size
    R = min(K, 32768 if res == AUTO else min(res, 32768))
    if res == AUTO and od[top[:R]].sum() * 16 < m:
        R = 0
    half = (R + 1) // 2
    order = np.concatenate([np.sort(top[:half]), np.sort(top[half:R]), np.sort(top[R:])])
    cpos = np.arange(n, dtype=np.int64)
    cpos[order] = n + np.arange(K)
    return cpos, K, int(od[top].sum()), R, int(od[top[:R]].sum())


def _greedy_tiles(in_ptr, max_e):
    deg = np.diff(in_ptr.astype(np.int64))
    tiles, nv, ne = [0], 0, 0
    for v, d in enumerate(deg):
        if nv > 0 and (nv == TILE_V or ne + d > max_e):
            tiles.append(v)
            nv, ne = 0, 0
        nv += 1
        ne += d
    if tiles[-1] != deg.size:
        tiles.append(deg.size)
    return np.array(tiles, dtype=np.int64)


def _ref_tiles(in_ptr, workers, variant=0):
    """(tile_v, sweep variant) for a partition of `workers` workers."""
    wide = _greedy_tiles(in_ptr, TILE_E)
    T = wide.size - 1
    if variant == 0:
        variant = NARROW if T < 2 * workers else WIDE_INFLIGHT if T <= 8 * workers else WIDE
    return (_greedy_tiles(in_ptr, TILE_E_NARROW) if variant == NARROW else wide), variant


def _ref_workers(tile_v, in_ptr, P):
    tv = tile_v.astype(np.int64)
    e0 = in_ptr.astype(np.int64)[tv]
    cost = 256.0 + np.diff(e0).astype(np.float64) + 4.0 * np.diff(tv).astype(np.float64)
    cum = np.concatenate([[0.0], np.cumsum(cost)])  # sequential float64 sums, as on the host
    T = tv.size - 1
    work = [0]
    for w in range(1, P):
        t = int(np.searchsorted(cum, cum[T] * w / P, side="left"))
        work.append(min(max(t, work[-1]), T))
    work.append(T)
    return np.array(work, dtype=np.int64), cost


GRAPHS = {
    "rmat12": lambda: gg.rmat(12, seed=3),
    "rmat14": lambda: gg.rmat(14, seed=14),
    "banded": lambda: gg.banded(20_000, 8, 512, 0.01, seed=22),
    "instar": lambda: tg.in_star(20_000),
    "dangling": lambda: tg.dangling_heavy(3000, 23),
    "multi": lambda: tg.random_graph(3001, 20_000, 7, dedup=False),
    "runlimit": lambda: tg.hubs_at_run_limit(5),
}


@pytest.fixture(scope="module", params=sorted(GRAPHS))
def graph(request):
    return GRAPHS[request.param]()


def test_in_edge_form_and_compact_region(dg, graph):
    g = graph
    p = dg.plan(g.n, g.ptr, g.idx, g.w)
    n, m = g.n, g.m
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.ptr.astype(np.int64)))
    dst = g.idx.astype(np.int64)
    o = np.argsort(dst, kind="stable")  # in-edges of each vertex in source order
    in_ptr = np.concatenate([[0], np.cumsum(np.bincount(dst, minlength=n))])
    cpos, K, hot_e, R, res_e = _ref_cpos(g)
    assert (p["n"], p["m"]) == (n, m)
    np.testing.assert_array_equal(p["in_ptr"], in_ptr)
    np.testing.assert_array_equal(p["cpos"], cpos)
    np.testing.assert_array_equal(p["in_src"], cpos[src[o]])
    np.testing.assert_array_equal(p["in_w"], g.w[o])
    assert (p["hot_vertices"], p["hot_edges"], p["resident_vertices"], p["resident_edges"]) == (K, hot_e, R, res_e)
    assert p["max_in_degree"] == int(np.diff(in_ptr).max())
    assert p["dangling"] == int((np.diff(g.ptr.astype(np.int64)) == 0).sum())
    # slots: regular vertices keep their id, the region is a bijection onto n..n+K-1
    hot = cpos >= n
    assert hot.sum() == K and np.array_equal(np.sort(cpos[hot]), n + np.arange(K))
    assert np.array_equal(cpos[~hot], np.nonzero(~hot)[0])


def test_tiles_and_partition(dg, graph):
    g = graph
    for cus, workers in ((256, 0), (4, 0), (1, 0), (256, 3), (256, 100_000)):
        p = dg.plan(g.n, g.ptr, g.idx, g.w, compute_units=cus, workers=workers)
        tile_v = p["tile_v"].astype(np.int64)
        ref, variant = _ref_tiles(p["in_ptr"], workers if workers else cus * PER_CU)
        np.testing.assert_array_equal(tile_v, ref)
        assert p["sweep_variant"] == variant
        T = tile_v.size - 1
        assert p["tiles"] == T
        nv = np.diff(tile_v)
        ne = np.diff(p["in_ptr"].astype(np.int64)[tile_v])
        max_e = TILE_E_NARROW if variant == NARROW else TILE_E
        assert (nv >= 1).all() and (nv <= TILE_V).all()
        assert ((ne <= max_e) | (nv == 1)).all()  # a larger vertex is a tile of its own
        P = workers if workers else cus * PER_CU
        P = max(1, min(P, T))
        if P > 8 and not workers:
            P &= ~7
        assert p["workers"] == P
        work, cost = _ref_workers(tile_v, p["in_ptr"], P)
        np.testing.assert_array_equal(p["work_t"], work)
        assert (np.diff(work) >= 0).all() and work[0] == 0 and work[-1] == T
        # each worker's cost exceeds the ideal share by less than one tile
        cum = np.concatenate([[0.0], np.cumsum(cost)])
        per = cum[work[1:]] - cum[work[:-1]]
        assert per.max() <= cum[-1] / P + cost.max() + 1e-6


BATCH_TILE_E = 4096


def test_batch_tiles(dg, graph):
    """The batched tiles refine the tiles: every tile boundary is one of
    theirs, each run holds at most 4096 in-edges unless it is one vertex,
    and the cut is greedy (a run ends only where its next vertex would take
    it past 4096 in-edges, or at a tile's end)."""
    g = graph
    for variant in ("wide", "narrow"):
        p = dg.plan(g.n, g.ptr, g.idx, g.w, sweep_variant=variant)
        tv = p["tile_v"].astype(np.int64)
        bt = p["btile_v"].astype(np.int64)
        assert p["batch_tiles"] == bt.size - 1 >= p["tiles"]
        assert bt[0] == 0 and bt[-1] == g.n and (np.diff(bt) >= 1).all()
        assert np.isin(tv, bt).all()
        deg = np.diff(p["in_ptr"].astype(np.int64))
        e = np.concatenate([[0], np.cumsum(deg)])
        ne, nv = np.diff(e[bt]), np.diff(bt)
        assert ((ne <= BATCH_TILE_E) | (nv == 1)).all()
        tile_ends = set(tv.tolist())
        for t in range(bt.size - 2):
            end = int(bt[t + 1])
            if end in tile_ends:
                continue
            # an inner cut: the next vertex would not have fitted
            assert ne[t] + deg[end] > BATCH_TILE_E, (variant, t)
    # a hub with more in-edges than a run stays a run of its own
    g = tg.in_star(20_000)
    p = dg.plan(g.n, g.ptr, g.idx, g.w)
    hub = int(np.argmax(np.diff(p["in_ptr"].astype(np.int64))))
    t = int(np.searchsorted(p["btile_v"], hub, side="right")) - 1
    assert p["btile_v"][t] == hub and p["btile_v"][t + 1] == hub + 1
    # in-degrees at the limit: 4096 fits a run, 4097 and 6000 are runs of
    # their own, and the one-edge vertex between them is left alone
    g = tg.hubs_at_run_limit(5)
    p = dg.plan(g.n, g.ptr, g.idx, g.w)
    deg = np.diff(p["in_ptr"].astype(np.int64))
    assert [int(deg[v]) for v in (1000, 1001, 1002, 1003, 25000)] == [4096, 4097, 1, 6000, 4096]
    bt = p["btile_v"].tolist()
    for v in (1000, 1001, 1002, 1003):
        assert v in bt and v + 1 in bt, v
    # no edges: the tiles themselves
    p = dg.plan(3000, np.zeros(3001, np.uint64), np.zeros(0, np.uint32))
    np.testing.assert_array_equal(p["btile_v"], [0, 1024, 2048, 3000])


BATCH_PER_CU = {"sssp": 8, "ppr": 5}  # default batched workgroups per compute unit


def test_batch_partitions(dg, graph):
    """The default batched partitions: per algorithm, its workgroups per
    compute unit rounded down to a multiple of 8, at most one per batched
    tile, split over the batched tiles with the blocked partition's cost
    quantiles."""
    g = graph
    for cus in (256, 4, 1):
        p = dg.plan(g.n, g.ptr, g.idx, g.w, compute_units=cus)
        bt = p["btile_v"].astype(np.int64)
        Tb = bt.size - 1
        for algo, per in BATCH_PER_CU.items():
            P = max(1, min(cus * per, Tb))
            if P > 8:
                P &= ~7
            assert p[f"batch_workers_{algo}"] == P, (algo, cus)
            work, _ = _ref_workers(bt, p["in_ptr"], P)
            np.testing.assert_array_equal(p[f"work_{algo}"], work, err_msg=f"{algo} cus={cus}")


@pytest.mark.parametrize("hot,res", [(0, AUTO), (50, AUTO), (1000, 100), (AUTO, 0), (AUTO, 1), (AUTO, 2049),
                                     (AUTO, 8193), (AUTO, 100_000)])
def test_region_options(dg, hot, res):
    g = gg.rmat(14, seed=14)
    p = dg.plan(g.n, g.ptr, g.idx, g.w, hot_vertices=hot, resident_vertices=res)
    cpos, K, hot_e, R, res_e = _ref_cpos(g, hot, res)
    np.testing.assert_array_equal(p["cpos"], cpos)
    assert (p["hot_vertices"], p["hot_edges"], p["resident_vertices"], p["resident_edges"]) == (K, hot_e, R, res_e)
    assert R <= min(K, 32768)


def test_resident_table_automatic_threshold(dg):
    """Banded graphs of even degree: the 32768 largest sources cover too few
    edges at 4M vertices, so the automatic size keeps no table; an explicit
    size keeps one."""
    g = gg.banded(1 << 20, 16, 4096, 0.01, seed=2)
    p = dg.plan(g.n, g.ptr, g.idx, None)
    assert p["resident_vertices"] == 0 and p["resident_edges"] == 0 and p["hot_vertices"] > 0
    q = dg.plan(g.n, g.ptr, g.idx, None, resident_vertices=6144)
    assert q["resident_vertices"] == 6144
    assert p["weight_bytes"] == 0 and p["in_w"] is None


@pytest.mark.parametrize("wmax,wbytes", [(1, 1), (255, 1), (256, 4), (0xFFFFFFFF, 4)])
def test_weight_width(dg, wmax, wbytes):
    g0 = gg.rmat(10, seed=10)
    rng = np.random.default_rng(1)
    w = rng.integers(0, wmax, size=g0.m, dtype=np.uint64, endpoint=True).astype(np.uint32)
    w[0] = wmax
    g = dataclasses.replace(g0, w=w)
    p = dg.plan(g.n, g.ptr, g.idx, g.w)
    assert p["weight_bytes"] == wbytes
    o = np.argsort(g.idx, kind="stable")
    np.testing.assert_array_equal(p["in_w"], w[o])


def test_csc_input_gives_the_same_plan(dg, graph):
    g = graph
    p = dg.plan(g.n, g.ptr, g.idx, g.w)
    src = np.repeat(np.arange(g.n, dtype=np.uint32), np.diff(g.ptr.astype(np.int64)))
    o = np.argsort(g.idx, kind="stable")
    q = dg.plan(g.n, p["in_ptr"].astype(np.uint64), src[o], g.w[o], layout="csc")
    for k in ("in_ptr", "in_src", "in_w", "cpos", "tile_v", "work_t", "hot_vertices", "resident_vertices",
              "content_hash"):
        np.testing.assert_array_equal(np.asarray(q[k]), np.asarray(p[k]), err_msg=k)


def test_content_hash(dg):
    g = gg.rmat(11, seed=4)
    a = dg.plan(g.n, g.ptr, g.idx, g.w)["content_hash"]
    assert dg.plan(g.n, g.ptr.copy(), g.idx.copy(), g.w.copy())["content_hash"] == a
    w2 = g.w.copy()
    w2[5] ^= 1
    assert dg.plan(g.n, g.ptr, g.idx, w2)["content_hash"] != a
    assert dg.plan(g.n, g.ptr, g.idx, None)["content_hash"] != a
    # the worker count is not part of the content
    assert dg.plan(g.n, g.ptr, g.idx, g.w, workers=7)["content_hash"] == a


def test_edge_cases(dg):
    # one vertex, no edges
    p = dg.plan(1, np.zeros(2, np.uint64), np.zeros(0, np.uint32))
    assert (p["tiles"], p["workers"], p["hot_vertices"], p["dangling"]) == (1, 1, 0, 1)
    np.testing.assert_array_equal(p["tile_v"], [0, 1])
    # many vertices, no edges: full tiles of 1024
    p = dg.plan(3000, np.zeros(3001, np.uint64), np.zeros(0, np.uint32))
    np.testing.assert_array_equal(p["tile_v"], [0, 1024, 2048, 3000])
    # one hub with far more than a tile's in-edges is a tile of its own
    g = tg.in_star(20_000)
    p = dg.plan(g.n, g.ptr, g.idx, g.w)
    deg = np.diff(p["in_ptr"].astype(np.int64))
    hub = int(np.argmax(deg))
    assert deg[hub] > TILE_E
    t = int(np.searchsorted(p["tile_v"], hub, side="right")) - 1
    assert p["tile_v"][t] == hub and p["tile_v"][t + 1] == hub + 1


@pytest.mark.parametrize("variant", ["wide", "wide_inflight", "narrow"])
def test_forced_sweep_variant(dg, variant):
    g = gg.rmat(14, seed=14)
    code = {"wide": WIDE, "wide_inflight": WIDE_INFLIGHT, "narrow": NARROW}[variant]
    p = dg.plan(g.n, g.ptr, g.idx, g.w, sweep_variant=variant)
    ref, v = _ref_tiles(p["in_ptr"], 256 * PER_CU, code)
    assert p["sweep_variant"] == v == code
    np.testing.assert_array_equal(p["tile_v"], ref)


def test_automatic_sweep_variant_by_size(dg):
    """Small graphs take the narrow tiles, mid-size ones the wide tiles with
    all gathers in flight, large ones the paced wide variant."""
    small = gg.rmat(12, seed=3)
    assert dg.plan(small.n, small.ptr, small.idx, small.w)["sweep_variant"] == NARROW
    mid = gg.banded(1 << 20, 16, 4096, 0.01, seed=2)  # 16.8M in-edges: about 4 wide tiles per worker
    p = dg.plan(mid.n, mid.ptr, mid.idx, None)
    assert 2 * 256 <= p["tiles"] <= 8 * 256 and p["sweep_variant"] == WIDE_INFLIGHT
    # the same graph on 64 compute units has 16 wide tiles per worker
    assert dg.plan(mid.n, mid.ptr, mid.idx, None, compute_units=64)["sweep_variant"] == WIDE


def test_validation(dg):
    P = dg.DG_ERR_INVALID_ARGUMENT
    ptr = np.array([0, 1, 2], np.uint64)
    idx = np.array([1, 0], np.uint32)
    cases = [
        dict(n=0, ptr=np.zeros(1, np.uint64), idx=np.zeros(0, np.uint32)),
        dict(n=2, ptr=np.array([1, 1, 2], np.uint64), idx=idx),       # ptr[0] != 0
        dict(n=2, ptr=np.array([0, 2, 1], np.uint64), idx=idx),       # decreasing
        dict(n=2, ptr=np.array([0, 1, 3], np.uint64), idx=idx),       # ptr[n] != m
        dict(n=2, ptr=ptr, idx=np.array([1, 2], np.uint32)),          # idx >= n
    ]
    for c in cases:
        with pytest.raises(dg.DGError) as e:
            dg.plan(c["n"], c["ptr"], c["idx"])
        assert e.value.status == P, c
    with pytest.raises(dg.DGError) as e:
        dg.plan(2, ptr, idx, compute_units=0)
    assert e.value.status == P
    # the C call rejects unknown layout codes and a NULL out pointer
    h = dg.C.c_void_p()
    assert dg.dg_plan_create(2, 2, 7, dg._np_ptr(ptr), dg._np_ptr(idx), None, None, 1, dg.C.byref(h)) == P
    assert dg.dg_plan_create(2, 2, 0, dg._np_ptr(ptr), dg._np_ptr(idx), None, None, 1, None) == P
    # an unknown sweep variant
    bad = dg.dg_graph_opts(0, dg.DG_HOT_AUTO, dg.DG_RESIDENT_AUTO, 4, 0)
    assert dg.dg_plan_create(2, 2, 0, dg._np_ptr(ptr), dg._np_ptr(idx), None, dg.C.byref(bad), 1, dg.C.byref(h)) == P
    assert "sweep_variant" in dg.last_error()
    assert dg.dg_plan_info_get(None, None) == P
    assert dg.dg_plan_arrays(None, None, None, None, None, None, None) == P
    assert dg.dg_plan_destroy(None) == dg.DG_OK
    # weights requested from an unweighted plan
    assert dg.dg_plan_create(2, 2, 0, dg._np_ptr(ptr), dg._np_ptr(idx), None, None, 1, dg.C.byref(h)) == dg.DG_OK
    buf = np.empty(2, np.uint32)
    assert dg.dg_plan_arrays(h, None, None, dg._np_ptr(buf), None, None, None) == P
    dg.dg_plan_destroy(h)
