"""Input generator checks (CPU): determinism and the structure each stand-in
workload is meant to have."""
import numpy as np

import graphgen as gg


def _check_csr(g):
    ptr = g.ptr.astype(np.int64)
    assert ptr[0] == 0 and ptr[-1] == g.m and (np.diff(ptr) >= 0).all()
    assert g.idx.dtype == np.uint32 and g.w.dtype == np.uint32 and g.ptr.dtype == np.uint64
    if g.m:
        assert int(g.idx.max()) < g.n
        assert g.w.min() >= 1 and g.w.max() <= 255
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(ptr))
    key = (src << 32) | g.idx.astype(np.int64)
    assert (np.diff(key) > 0).all(), "edges must be sorted and free of duplicates"


def test_rmat_deterministic_and_structured():
    a = gg.rmat(10, seed=10)
    b = gg.rmat(10, seed=10)
    c = gg.rmat(10, seed=11)
    assert a.sha256() == b.sha256() != c.sha256()
    _check_csr(a)
    assert a.n == 1024 and 0.6 * 16 * 1024 < a.m <= 16 * 1024
    indeg = np.bincount(a.idx, minlength=a.n)
    # skew: the top 1% of vertices by in-degree hold far more than 1% of edges
    top = np.sort(indeg)[::-1][: a.n // 100].sum()
    assert top > 0.08 * a.m


def test_rmat_weights_follow_dedup_order():
    g = gg.rmat(8, seed=3)
    w2 = gg.stream(3, "weights").integers(1, 256, size=g.m, dtype=np.uint32)
    np.testing.assert_array_equal(g.w, w2)


def test_erdos_renyi():
    g = gg.erdos_renyi(5000, 8, seed=4)
    _check_csr(g)
    src = np.repeat(np.arange(g.n), np.diff(g.ptr.astype(np.int64)))
    assert (src != g.idx).all(), "no self-loops"
    assert 0.99 * 40000 < g.m <= 40000


def test_banded_band_and_long_range():
    n, hw = 50_000, 4096
    g = gg.banded(n, 16, hw, 0.01, seed=5)
    _check_csr(g)
    src = np.repeat(np.arange(n), np.diff(g.ptr.astype(np.int64)))
    off = np.abs(g.idx.astype(np.int64) - src)
    long_frac = (off > hw).mean()
    assert (off > 0).all()
    assert 0.003 < long_frac < 0.012
    assert g.m > 0.98 * 16 * n


def test_path_and_sources():
    p = gg.path_graph(5, weight=7)
    _check_csr(p)
    np.testing.assert_array_equal(p.idx, [1, 2, 3, 4])
    g = gg.rmat(9, seed=1)
    s = gg.pick_sources(g, 16, seed=9)
    assert len(set(s.tolist())) == 16
    deg = np.diff(g.ptr.astype(np.int64))
    assert (deg[s] > 0).all()
    np.testing.assert_array_equal(s, gg.pick_sources(g, 16, seed=9))


def test_from_edges_multigraph_keeps_duplicates():
    g = gg.from_edges(3, [0, 0, 1], [1, 1, 2], dedup=False)
    assert g.m == 3
