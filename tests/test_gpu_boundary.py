"""GPU tests of the C ABI's input and statistics paths (needs an MI355X):

* graphs uploaded from device arrays equal graphs uploaded from host arrays
  (same layout facts, bit-identical synchronous results), and malformed
  device arrays are refused after the copy;
* dg_stats.err_bound (the float64 certificate ||T(x) - x||_1 / (1 - alpha)
  computed on the device) equals the oracle's certificate of the returned
  vector and bounds its true L1 error against the oracle's fixed point;
* dg_stats.commits / commit_interval are the commits the delayed sweeps make:
  recomputed from the partition with the rule the header states.
"""
import ctypes as C

import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from tests import graphs as tg

pytestmark = pytest.mark.gpu
ALPHA = 0.85


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


def _np(t):
    return t.cpu().numpy()


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int64)).to(dtype=dtype, device="cuda")


@pytest.mark.parametrize("layout", ["csr", "csc"])
def test_device_arrays_match_host(dg, layout):
    import torch
    g = gg.rmat(13, seed=13)
    if layout == "csr":
        ptr, idx, w = g.ptr, g.idx, g.w
    else:  # transpose on the host: in-edges grouped by destination
        src = np.repeat(np.arange(g.n), np.diff(g.ptr.astype(np.int64)))
        order = np.argsort(g.idx, kind="stable")
        idx = src[order].astype(np.uint32)
        w = g.w[order]
        ptr = np.concatenate([[0], np.cumsum(np.bincount(g.idx, minlength=g.n))]).astype(np.uint64)
    H = dg.Graph(g.n, ptr, idx, w, layout=layout)
    D = dg.Graph(g.n, _dev(ptr, torch.uint64), _dev(idx, torch.uint32), _dev(w, torch.uint32), layout=layout)
    ih, id_ = H.info(), D.info()
    for f, _ in dg.dg_graph_info._fields_:
        assert getattr(ih, f) == getattr(id_, f), f
    # the same layout gives the same synchronous iterates up to the order of
    # the float64 LDS additions (not fixed between runs)
    xh, sh = H.pagerank(tol=1e-9, mode="sync", dtype="f64")
    xd, sd = D.pagerank(tol=1e-9, mode="sync", dtype="f64")
    assert float((xh - xd).abs().sum()) < 1e-13 and abs(sh.sweeps - sd.sweeps) <= 1
    for src in gg.pick_sources(g, 2, seed=4).tolist():
        assert torch.equal(H.sssp(src, mode="async")[0], D.sssp(src, mode="async")[0])
    H.close()
    D.close()


def test_device_arrays_refused_when_malformed(dg):
    import torch
    ptr = _dev(np.array([0, 1, 3, 3]), torch.uint64)
    bad_idx = _dev(np.array([1, 0, 3]), torch.uint32)  # 3 >= n
    with pytest.raises(dg.DGError) as e:
        dg.Graph(3, ptr, bad_idx)
    assert e.value.status == dg.DG_ERR_INVALID_ARGUMENT
    bad_ptr = _dev(np.array([0, 2, 1, 3]), torch.uint64)
    with pytest.raises(dg.DGError) as e:
        dg.Graph(3, bad_ptr, _dev(np.array([1, 0, 2]), torch.uint32))
    assert e.value.status == dg.DG_ERR_INVALID_ARGUMENT


_GRAPHS = {}


def _graph(name):
    if name not in _GRAPHS:
        g = {"rmat14": lambda: gg.rmat(14, seed=14), "dangling": lambda: tg.dangling_heavy(20_000, 3),
             "instar": lambda: tg.in_star(5000)}[name]()
        _GRAPHS[name] = (g, opr.pagerank_fixed_point(g))
    return _GRAPHS[name]


@pytest.mark.parametrize("name", ["rmat14", "dangling", "instar"])
@pytest.mark.parametrize("mode,d,dtype,tol", [("sync", 1, "f64", 1e-6), ("async", 1, "f32", 1e-6),
                                               ("delayed", 64, "f32", 1e-4), ("delayed", 0xFFFFFFFF, "f64", 1e-9)])
def test_err_bound_is_the_certificate(dg, name, mode, d, dtype, tol):
    g, xs = _graph(name)
    G = dg.Graph.from_csr(g)
    x, st = G.pagerank(tol=tol, mode=mode, d=d, dtype=dtype, err_bound=True)
    x = _np(x)
    cert = opr.certificate(g, x)
    err = float(np.abs(x - xs).sum())
    print(f"{name} {mode} d={d} {dtype} tol={tol}: err_bound {st.err_bound:.3e} oracle cert {cert:.3e} "
          f"true error {err:.3e}")
    assert abs(st.err_bound - cert) <= 1e-12 + 1e-9 * cert
    assert st.err_bound >= err - 2e-12  # the oracle's x* is itself exact to ~1e-12
    assert st.err_bound <= (1 + ALPHA) / (1 - ALPHA) * err + 2e-11
    _, st0 = G.pagerank(tol=tol, mode=mode, d=d, dtype=dtype)
    assert st0.err_bound == 0.0  # not requested
    G.close()


def _commits(tile_v, work_t, d):
    c = 0
    for w in range(len(work_t) - 1):
        staged = 0
        t0, t1 = int(work_t[w]), int(work_t[w + 1])
        for t in range(t0, t1):
            nv = int(tile_v[t + 1] - tile_v[t])
            if t + 1 == t1 or staged + nv >= d:
                c += 1
                staged = 0
            else:
                staged += nv
    return c


def test_commit_stats(dg):
    g = gg.rmat(16, seed=16)
    G = dg.Graph.from_csr(g)
    info = G.info()
    p = dg.plan(g.n, g.ptr, g.idx, g.w, compute_units=info.compute_units)
    assert p["tiles"] == info.tiles and p["workers"] == info.workers
    tv, wt = p["tile_v"], p["work_t"]
    assert np.array_equal(G.partition(), tv[wt])
    for d in (1, 64, 1024, 4096, 0xFFFFFFFF):
        _, st = G.pagerank(tol=1e-6, mode="delayed", d=d, dtype="f32")
        want = _commits(tv, wt, min(d, 1 << 31))
        assert st.commits == want, (d, st.commits, want)
        assert st.commit_interval == round(g.n / want)
        assert st.tile_vertices == round(g.n / info.tiles)
        _, sb = G.sssp(0, mode="delayed", d=d)
        assert sb.commits == want
    assert G.pagerank(tol=1e-6, mode="async", dtype="f32")[1].commits == 0
    # any d up to the largest tile commits after every tile
    _, st = G.pagerank(tol=1e-6, mode="delayed", d=1, dtype="f32")
    assert st.commits == info.tiles
    G.close()
