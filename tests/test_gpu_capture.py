"""GPU tests of captured launches (dg_graph_set_capture): chunks of sweeps
recorded once into HIP graphs and replayed.

The replayed kernels and arguments are those of the eager launches, so:

* Bellman-Ford in every mode gives the oracle's distances, captured and eager,
  bit for bit, with equal sweep counts in synchronous mode, on every replay;
  the recorded chunks are reused across calls (other sources too), with the
  program's own eager work and synchronisations between the replays;
* synchronous PageRank and personalised PageRank agree with the eager run
  to rounding: their sweeps sum in-edges with LDS atomics, whose order varies
  from run to run, so two eager runs already differ in the last bits (float64:
  L1 <= 1e-13; float32: L1 <= 1e-6, the float32 accuracy bar), and the
  sweep counts agree within one;
* the batched calls (many sources) give the eager distances bit for bit and
  the eager personalised scores to rounding in synchronous mode;
* chunk lengths 1 (a call longer than the recorded chunks, whose tail is
  launched one by one), 3 and 64 (longer than the call) stop at the eager
  sweep count; a call that does not converge returns the eager result;
* the setting is validated.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import sssp as osp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


@pytest.fixture(scope="module")
def rmat12():
    return gg.rmat(12, seed=12)


@pytest.fixture()
def graph(dg, rmat12):
    G = dg.Graph.from_csr(rmat12)
    yield G
    G.close()


def _eager_work():
    """Unrelated eager device work and a synchronisation between replays."""
    import torch
    a = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
    b = (a * 3.0 + 1.0).sum()
    torch.cuda.synchronize()
    return float(b)


ROUNDING = {"f64": 1e-13, "f32": 1e-6}  # L1 between two runs of the same sweeps


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_capture_pagerank_sync_replays(graph, dtype):
    print(f"capture pagerank sync {dtype}", flush=True)
    tol = 1e-10 if dtype == "f64" else 1e-6
    ref, st_ref = graph.pagerank(tol=tol, mode="sync", dtype=dtype)
    ref = ref.cpu().numpy()
    graph.set_capture(8)
    for rep in range(3):
        out, st = graph.pagerank(tol=tol, mode="sync", dtype=dtype)
        err = float(np.abs(out.cpu().numpy() - ref).sum())
        assert err <= ROUNDING[dtype], (rep, err)
        assert abs(st.sweeps - st_ref.sweeps) <= 1 and st.converged
        _eager_work()
    graph.set_capture(0)
    out, st = graph.pagerank(tol=tol, mode="sync", dtype=dtype)
    assert float(np.abs(out.cpu().numpy() - ref).sum()) <= ROUNDING[dtype]


def test_capture_ppr_sync(graph):
    print("capture ppr sync", flush=True)
    ref, st_ref = graph.ppr(7, tol=1e-10, mode="sync", dtype="f64")
    ref = ref.cpu().numpy()
    graph.set_capture(16)
    for rep in range(3):
        out, st = graph.ppr(7, tol=1e-10, mode="sync", dtype="f64")
        err = float(np.abs(out.cpu().numpy() - ref).sum())
        assert err <= ROUNDING["f64"], (rep, err)
        assert abs(st.sweeps - st_ref.sweeps) <= 1
        _eager_work()


@pytest.mark.parametrize("mode,d", [("sync", 1), ("async", 1), ("delayed", 64), ("delayed", 0xFFFFFFFF)])
def test_capture_sssp_modes(graph, rmat12, mode, d):
    print(f"capture sssp {mode} d={d}", flush=True)
    ref, ref_sweeps = osp.bellman_ford_sync(rmat12, 3)[:2]
    eo, est = graph.sssp(3, mode=mode, d=d)
    graph.set_capture(8)
    for src in (3, 3, 11):  # the recorded chunks serve other sources too
        out, st = graph.sssp(src, mode=mode, d=d)
        want = ref if src == 3 else osp.bellman_ford_sync(rmat12, src)[0]
        np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=f"{mode} src={src}")
        if src == 3:
            np.testing.assert_array_equal(out.cpu().numpy(), eo.cpu().numpy())
            if mode == "sync":
                assert st.sweeps == est.sweeps == ref_sweeps
        _eager_work()


def test_capture_batched_sync(graph, rmat12):
    print("capture batched sssp/ppr sync", flush=True)
    rng = np.random.default_rng(5)
    src = rng.integers(0, rmat12.n, 80).astype(np.uint32)
    d_ref, s_ref = graph.sssp_batch(src, mode="sync")
    p_ref, ps_ref = graph.ppr_batch(src[:40], tol=1e-9, mode="sync", dtype="f64")
    d_ref, p_ref = d_ref.cpu().numpy(), p_ref.cpu().numpy()
    graph.set_capture(8)
    for rep in range(2):
        d, s = graph.sssp_batch(src, mode="sync")
        np.testing.assert_array_equal(d.cpu().numpy(), d_ref, err_msg=f"sssp replay {rep}")
        assert s.sweeps == s_ref.sweeps
        p, ps = graph.ppr_batch(src[:40], tol=1e-9, mode="sync", dtype="f64")
        err = np.abs(p.cpu().numpy() - p_ref).sum(axis=1).max()
        assert err <= ROUNDING["f64"], (rep, err)
        assert abs(ps.sweeps - ps_ref.sweeps) <= 1
        _eager_work()
    for q in (0, 17, 79):
        np.testing.assert_array_equal(d_ref[q], osp.bellman_ford_sync(rmat12, int(src[q]))[0])


def test_capture_chunk_lengths(dg):
    """A 700-vertex path from its first vertex takes 700 synchronous sweeps:
    with chunks of 1 the recorded chunks end at 256 and the rest is
    launched one by one; chunks of 64 overrun the call's end."""
    print("capture chunk lengths", flush=True)
    g = gg.path_graph(700, weight=3)
    want = np.arange(700, dtype=np.uint64) * 3
    G = dg.Graph.from_csr(g)
    eo, est = G.sssp(0, mode="sync")
    np.testing.assert_array_equal(eo.cpu().numpy(), want)
    for C in (1, 3, 64):
        G.set_capture(C)
        for rep in range(2):
            out, st = G.sssp(0, mode="sync")
            np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=f"C={C} rep {rep}")
            assert st.sweeps == est.sweeps, (C, st.sweeps, est.sweeps)
    G.close()


def test_capture_not_converged_matches_eager(dg):
    print("capture not converged", flush=True)
    g = gg.path_graph(300, weight=2)
    G = dg.Graph.from_csr(g)
    eo, est = G.sssp(0, mode="sync", max_sweeps=50, allow_not_converged=True)
    assert not est.converged
    G.set_capture(8)
    out, st = G.sssp(0, mode="sync", max_sweeps=50, allow_not_converged=True)
    assert not st.converged and st.sweeps == est.sweeps == 50
    np.testing.assert_array_equal(out.cpu().numpy(), eo.cpu().numpy())
    G.close()


def test_capture_validation(dg, graph):
    with pytest.raises(dg.DGError) as e:
        graph.set_capture(65)
    assert e.value.status == dg.DG_ERR_INVALID_ARGUMENT
    graph.set_capture(64)
    graph.set_capture(0)
