"""Parity at full size (needs an MI355X; a few minutes of host time).

Workloads, in the launch configuration bench.py times (default workers and
compact hot region):

* R-MAT scale 22 (4,194,304 vertices, ~65M edges after deduplication,
  a/b/c/d .57/.19/.19/.05, permuted, seed 22);
* the diagonal-banded graph, 16,777,216 vertices, 16 out-edges within
  +-4096 plus 1% long-range (seed 24).

PageRank is compared with the oracle's float64 fixed point (Jacobi to an L1
change below 1e-12; the C oracle for the banded graph) directly: L1 <= 1e-6
in every mode, d and precision.

SSSP results are checked with the oracle's O(m) optimality certificate, which
holds exactly when the distances are the true shortest paths (a bit-exact
check without a second solver), and one source against scipy's Dijkstra.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp

pytestmark = pytest.mark.gpu

MODES = [("sync", 1), ("async", 1), ("delayed", 1), ("delayed", 64), ("delayed", 1024), ("delayed", 0xFFFFFFFF)]
PR_TOL = {"f64": 1e-8, "f32": 1e-7}


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


@pytest.fixture(scope="module")
def rmat22():
    g = gg.rmat(22, seed=22)
    print(f"rmat22 n={g.n} m={g.m}", flush=True)
    return g


@pytest.fixture(scope="module")
def rmat22_xstar(rmat22):
    from oracle import cpr
    x = cpr.pagerank_fixed_point(rmat22, tol=1e-12)
    print("rmat22 fixed point ready", flush=True)
    return x


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_rmat22_pagerank_all_modes(dg, rmat22, rmat22_xstar, dtype):
    G = dg.Graph.from_csr(rmat22)
    for mode, d in MODES:
        x, st = G.pagerank(tol=PR_TOL[dtype], mode=mode, d=d, dtype=dtype, max_sweeps=500)
        err = float(np.abs(x.cpu().numpy() - rmat22_xstar).sum())
        print(f"rmat22 {dtype} {mode} d={d}: sweeps={st.sweeps} L1 err={err:.2e} t={st.seconds*1e3:.2f} ms",
              flush=True)
        assert err <= 1e-6, (dtype, mode, d, err)
    G.close()


def test_rmat22_sssp_all_modes(dg, rmat22):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    G = dg.Graph.from_csr(rmat22)
    sources = gg.pick_sources(rmat22, 16, seed=22).tolist()
    # one source against an independent solver
    deg = np.diff(rmat22.ptr.astype(np.int64))
    mat = csr_matrix((rmat22.w.astype(np.float64), rmat22.idx.astype(np.int64), rmat22.ptr.astype(np.int64)),
                     shape=(rmat22.n, rmat22.n))
    ref = sp_dijkstra(mat, directed=True, indices=sources[0])
    ref = np.where(np.isinf(ref), osp.INF32, ref).astype(np.uint32)
    del deg
    for mode, d in MODES:
        dist, st = G.sssp(sources[0], mode=mode, d=d)
        np.testing.assert_array_equal(dist.cpu().numpy(), ref, err_msg=f"{mode} d={d}")
    # the rest by certificate, cycling through the modes
    for i, src in enumerate(sources[1:6]):
        mode, d = MODES[i % len(MODES)]
        dist, st = G.sssp(src, mode=mode, d=d)
        ok, msg = osp.certificate(rmat22, src, dist.cpu().numpy())
        print(f"rmat22 sssp src={src} {mode} d={d}: sweeps={st.sweeps} certificate {msg}", flush=True)
        assert ok, msg
    G.close()


@pytest.fixture(scope="module")
def banded16m():
    g = gg.banded(1 << 24, 16, 4096, 0.01, seed=24)
    print(f"banded n={g.n} m={g.m}", flush=True)
    return g


@pytest.fixture(scope="module")
def banded16m_xstar(banded16m):
    from oracle import cpr
    x = cpr.pagerank_fixed_point(banded16m, tol=1e-12)
    print("banded fixed point ready", flush=True)
    return x


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_banded16m_pagerank_all_modes(dg, banded16m, banded16m_xstar, dtype):
    """The diagonal-clustered graph where delay should not help (section
    IV-C), against the oracle's fixed point (the C oracle's Jacobi to 1e-12,
    the numpy oracle's iterates computed in parallel): L1 <= 1e-6 in every
    mode and d, in both precisions."""
    g = banded16m
    xs = banded16m_xstar
    G = dg.Graph.from_csr(g)
    for mode, d in MODES:
        x, st = G.pagerank(tol=PR_TOL[dtype], mode=mode, d=d, dtype=dtype, max_sweeps=1000)
        err = float(np.abs(x.cpu().numpy() - xs).sum())
        print(f"banded {dtype} {mode} d={d}: sweeps={st.sweeps} L1 err={err:.2e} t={st.seconds*1e3:.2f} ms",
              flush=True)
        assert err <= 1e-6, (dtype, mode, d, err)
    G.close()


def test_banded16m_sssp_all_modes(dg, banded16m):
    """One source against scipy's Dijkstra bit for bit in every mode and d;
    two more by the oracle's optimality certificate."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    g = banded16m
    srcs = gg.pick_sources(g, 3, seed=24).tolist()
    mat = csr_matrix((g.w.astype(np.float64), g.idx.astype(np.int64), g.ptr.astype(np.int64)), shape=(g.n, g.n))
    ref = sp_dijkstra(mat, directed=True, indices=srcs[0])
    del mat
    ref = np.where(np.isinf(ref), osp.INF32, ref).astype(np.uint32)
    print("banded Dijkstra ready", flush=True)
    G = dg.Graph.from_csr(g)
    for mode, d in MODES:
        dist, st = G.sssp(srcs[0], mode=mode, d=d)
        print(f"banded sssp {mode} d={d}: sweeps={st.sweeps}", flush=True)
        np.testing.assert_array_equal(dist.cpu().numpy(), ref, err_msg=f"{mode} d={d}")
    for src, (mode, d) in zip(srcs[1:], [("async", 1), ("delayed", 0xFFFFFFFF)]):
        dist, st = G.sssp(src, mode=mode, d=d)
        ok, msg = osp.certificate(g, src, dist.cpu().numpy())
        print(f"banded sssp src={src} {mode} d={d}: sweeps={st.sweeps} certificate {msg}", flush=True)
        assert ok, msg
    G.close()


@pytest.fixture(scope="module")
def rmat20():
    return gg.rmat(20, seed=20)


def test_rmat20_batched_256_sources(dg, rmat20):
    """The batched configuration at its own size: 256 SSSP sources and 256
    one-hot PPR vectors on RMAT-20.  Every SSSP row passes the oracle's
    optimality certificate and 8 rows equal Dijkstra (scipy); every PPR row
    (float64, tol 1e-9) is bounded by the oracle's contraction certificate
    ||P_s(x) - x|| / (1 - alpha) <= 1e-7, and 2 rows are compared with the
    oracle's fixed point directly."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    g = rmat20
    sources = gg.pick_sources(g, 256, seed=20)
    G = dg.Graph.from_csr(g)
    out, st = G.sssp_batch(sources, mode="async")
    print(f"rmat20 sssp_batch x256 async: sweeps={st.sweeps} t={st.seconds * 1e3:.1f} ms", flush=True)
    got = out.cpu().numpy()
    for q in range(0, 256, 16):
        ok, msg = osp.certificate(g, int(sources[q]), got[q])
        assert ok, (q, msg)
    mat = csr_matrix((g.w.astype(np.float64), g.idx, g.ptr.astype(np.int64)), shape=(g.n, g.n))
    ref = sp_dijkstra(mat, directed=True, indices=sources[:8].astype(np.int64))
    for q in range(8):
        r = np.where(np.isinf(ref[q]), dg.DG_INF_DIST, ref[q]).astype(np.uint32)
        np.testing.assert_array_equal(got[q], r, err_msg=f"row {q}")
    del out, got
    x, st = G.ppr_batch(sources, tol=1e-9, mode="async", dtype="f64", max_sweeps=2000)
    print(f"rmat20 ppr_batch x256 async f64: sweeps={st.sweeps} t={st.seconds * 1e3:.1f} ms", flush=True)
    xs = x.cpu().numpy()
    worst = 0.0
    for q in range(0, 256, 16):
        c = opr.ppr_certificate(g, xs[q], int(sources[q]))
        worst = max(worst, c)
        assert c <= 1e-7, (q, c)
    for q in range(2):
        ref_x = opr.ppr_fixed_point(g, int(sources[q]))
        assert float(np.abs(xs[q] - ref_x).sum()) <= 1e-8
    print(f"rmat20 ppr worst certificate bound {worst:.2e}", flush=True)
    G.close()


def test_rmat20_single_query_inflight_variant(dg, rmat20):
    """RMAT-20 at its own size picks the wide sweep variant with all gathers
    in flight (about 4 wide tiles per worker): PageRank within L1 1e-6 of the
    oracle's fixed point in every mode (float32), SSSP by the optimality
    certificate in every mode."""
    g = rmat20
    G = dg.Graph.from_csr(g)
    assert G.info().sweep_variant == dg.DG_SWEEP_WIDE_INFLIGHT
    xs = opr.pagerank_fixed_point(g, tol=1e-12)
    for mode, d in MODES:
        x, st = G.pagerank(tol=PR_TOL["f32"], mode=mode, d=d, dtype="f32", max_sweeps=500)
        err = float(np.abs(x.cpu().numpy() - xs).sum())
        print(f"rmat20 f32 {mode} d={d}: sweeps={st.sweeps} L1 err={err:.2e}", flush=True)
        assert err <= 1e-6, (mode, d, err)
    src = int(gg.pick_sources(g, 1, seed=21)[0])
    for mode, d in MODES:
        dist, st = G.sssp(src, mode=mode, d=d)
        ok, msg = osp.certificate(g, src, dist.cpu().numpy())
        assert ok, (mode, d, msg)
    G.close()
