"""GPU parity of the batched entry points (64 queries per batch).

* dg_sssp_batch: every row bit-exact against the oracle's Bellman-Ford from
  that source, in every mode, with several batches and a ragged last batch.
* dg_ppr_batch: every row within L1 1e-6 of the oracle's personalised
  PageRank fixed point (float64, change < 1e-12), with float64 storage
  stopping at tol 1e-9 (then the contraction bound alone guarantees
  alpha/(1-alpha) * 1e-9 < 1e-8) and float32 storage stopping at tol 5e-7,
  above its rounding floor (about 1e-7 synchronous, 1-3e-7 under
  asynchronous commits, where each sweep reads a timing-dependent mix of
  values that differ by rounding).
* Edge cases: synchronous batches stopped after k sweeps return the k-th
  Jacobi iterate; 1025 queries (17 launches, a one-lane tail); a batch of
  one query against the single-query entry points; one-vertex, self-loop
  and edgeless graphs; hubs at the batched tiles' limit of 4096 in-edges
  (single-vertex runs, one of them a one-edge vertex between two hubs).
"""
import ctypes as C

import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp
from tests import graphs as tg

pytestmark = pytest.mark.gpu

MODES = [("sync", 1), ("async", 1), ("delayed", 1), ("delayed", 64), ("delayed", 1024), ("delayed", 0xFFFFFFFF)]


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


@pytest.mark.parametrize("name", ["rmat13", "instar", "banded", "runlimit"])
def test_sssp_batch_all_modes(dg, name):
    if name == "rmat13":
        g = gg.rmat(13, seed=13)
    elif name == "instar":
        g = tg.in_star(20_000)  # one hub beyond a tile (16380 in-edges): the wavefront split
    elif name == "runlimit":
        g = tg.hubs_at_run_limit(5)  # single-vertex batched runs at and above 4096 in-edges
    else:
        g = gg.banded(20_000, 16, 512, 0.01, seed=4)
    k = 70  # two batches, the second ragged
    rng = np.random.default_rng(1)
    sources = rng.integers(0, g.n, size=k).astype(np.uint32)
    sources[5] = sources[6]  # a duplicate query
    if name == "runlimit":
        sources[:5] = [1000, 1001, 1002, 1003, 25000]
    refs = {int(s): osp.bellman_ford_sync(g, int(s))[0] for s in set(sources.tolist())}
    G = dg.Graph.from_csr(g)
    # d <= 64 stages in registers (16 rows per wavefront, a commit every
    # ceil(d/4) of its vertices), d > 64 in the shadow array
    for mode, d in MODES + [("delayed", 16), ("delayed", 63), ("delayed", 65)]:
        out, st = G.sssp_batch(sources, mode=mode, d=d)
        got = out.cpu().numpy()
        for q, s in enumerate(sources.tolist()):
            np.testing.assert_array_equal(got[q], refs[s], err_msg=f"{name} {mode} d={d} query {q} src {s}")
        assert st.converged
        print(f"{name} sssp_batch {mode} d={d}: sweeps={st.sweeps} t={st.seconds*1e3:.2f} ms", flush=True)
    # batched rows equal the single-query entry point
    for s in sources[:3].tolist():
        one, _ = G.sssp(s, mode="sync")
        np.testing.assert_array_equal(one.cpu().numpy(), refs[s])
    G.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-9), ("f32", 5e-7)])
@pytest.mark.parametrize("name", ["rmat12", "dangling", "instar", "runlimit"])
def test_ppr_batch_all_modes(dg, name, dtype, tol):
    if name == "rmat12":
        g = gg.rmat(12, seed=12)
    elif name == "dangling":
        g = tg.dangling_heavy(3000, 5)
    elif name == "runlimit":
        g = tg.hubs_at_run_limit(5)
    else:
        g = tg.in_star(20_000)
    k = 67
    rng = np.random.default_rng(2)
    sources = rng.integers(0, g.n, size=k).astype(np.uint32)
    deg = np.diff(g.ptr.astype(np.int64))
    sources[0] = int(np.flatnonzero(deg == 0)[0])  # a dangling restart vertex
    if name == "runlimit":
        sources[1:6] = [1000, 1001, 1002, 1003, 25000]
    refs = {int(s): opr.ppr_fixed_point(g, int(s)) for s in set(sources.tolist())}
    G = dg.Graph.from_csr(g)
    for mode, d in MODES:
        out, st = G.ppr_batch(sources, tol=tol, mode=mode, d=d, dtype=dtype, max_sweeps=5000)
        got = out.cpu().numpy()
        errs = [np.abs(got[q] - refs[s]).sum() for q, s in enumerate(sources.tolist())]
        print(f"{name} ppr_batch {dtype} {mode} d={d}: sweeps={st.sweeps} max L1 err={max(errs):.2e}", flush=True)
        assert max(errs) <= (1e-8 if dtype == "f64" else 1e-6), (mode, d, max(errs))
        assert np.abs(got.sum(axis=1) - 1.0).max() < 1e-9
        assert st.converged
    G.close()


def test_ppr_batch_row_independent_of_mix(dg):
    """Synchronous sweeps are lane-local and each query stops on its own
    change, so a row is the same bit for bit alone and in a mixed batch."""
    g = gg.rmat(12, seed=7)
    rng = np.random.default_rng(5)
    sources = rng.integers(0, g.n, size=100).astype(np.uint32)
    G = dg.Graph.from_csr(g)
    for dtype, tol in (("f32", 5e-7), ("f64", 1e-9)):
        mix, _ = G.ppr_batch(sources, tol=tol, mode="sync", dtype=dtype)
        for q in (0, 37, 99):
            one, _ = G.ppr_batch(sources[q:q + 1], tol=tol, mode="sync", dtype=dtype)
            np.testing.assert_array_equal(mix[q].cpu().numpy(), one[0].cpu().numpy(), err_msg=f"{dtype} query {q}")
    G.close()


def test_batch_validation(dg):
    g = gg.rmat(10, seed=10)
    G = dg.Graph.from_csr(g)
    out = np.zeros(4 * g.n, np.uint32)
    st = dg.dg_stats()
    src = np.array([0, 1, g.n, 2], np.uint32)
    assert dg.dg_sssp_batch(G._h, dg._np_ptr(src), 4, dg.DG_SYNC, 1, 100, dg._np_ptr(out), 0, C.byref(st),
                            None) == dg.DG_ERR_INVALID_ARGUMENT
    src = np.array([0], np.uint32)
    assert dg.dg_sssp_batch(G._h, dg._np_ptr(src), 0, dg.DG_SYNC, 1, 100, dg._np_ptr(out), 0, C.byref(st),
                            None) == dg.DG_ERR_INVALID_ARGUMENT
    outf = np.zeros(g.n, np.float64)
    assert dg.dg_ppr_batch(G._h, dg._np_ptr(src), 1, 1.5, 1e-6, dg.DG_SYNC, 1, dg.DG_F32, 100, dg._np_ptr(outf), 0,
                           C.byref(st), None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_ppr_batch(G._h, dg._np_ptr(src), 1, 0.85, 1e-6, dg.DG_SYNC, 1, 7, 100, dg._np_ptr(outf), 0,
                           C.byref(st), None) == dg.DG_ERR_INVALID_ARGUMENT
    # host outputs through the raw ABI
    s2 = np.array([3, 7], np.uint32)
    out2 = np.zeros(2 * g.n, np.uint32)
    assert dg.dg_sssp_batch(G._h, dg._np_ptr(s2), 2, dg.DG_DELAYED, 64, 2000, dg._np_ptr(out2), 0, C.byref(st),
                            None) == dg.DG_OK
    np.testing.assert_array_equal(out2[:g.n], osp.bellman_ford_sync(g, 3)[0])
    np.testing.assert_array_equal(out2[g.n:], osp.bellman_ford_sync(g, 7)[0])
    outp = np.zeros(2 * g.n, np.float64)
    assert dg.dg_ppr_batch(G._h, dg._np_ptr(s2), 2, 0.85, 1e-9, dg.DG_ASYNC, 1, dg.DG_F64, 5000, dg._np_ptr(outp),
                           0, C.byref(st), None) == dg.DG_OK
    assert np.abs(outp[:g.n] - opr.ppr_fixed_point(g, 3)).sum() < 1e-6
    G.close()


def test_batch_sync_per_sweep_iterates(dg):
    """Synchronous batched sweeps stopped after k sweeps return the oracle's
    k-th Jacobi iterate of every query: Bellman-Ford bit-exact, personalised
    PageRank (float64, normalised like every finished row) within 1e-13
    relative L1."""
    g = gg.rmat(12, seed=21)
    srcs = gg.pick_sources(g, 5, seed=8)
    G = dg.Graph.from_csr(g)
    iters = {int(s): osp.bellman_ford_sync(g, int(s), keep_iterates=True)[2] for s in srcs}
    for k in (1, 2, 3, 5):
        out, st = G.sssp_batch(srcs, mode="sync", max_sweeps=k, allow_not_converged=True)
        got = out.cpu().numpy()
        for q, s in enumerate(srcs.tolist()):
            its = iters[s]
            np.testing.assert_array_equal(got[q], its[min(k, len(its)) - 1], err_msg=f"k={k} query {q}")
        assert st.sweeps == k and not st.converged
    for k in (1, 2, 4):
        out, st = G.ppr_batch(srcs, tol=0.0, mode="sync", dtype="f64", max_sweeps=k, allow_not_converged=True)
        got = out.cpu().numpy()
        for q, s in enumerate(srcs.tolist()):
            ref, n_sw = opr.ppr_jacobi(g, s, tol=0.0, max_sweeps=k)
            assert n_sw == k
            ref = ref / ref.sum()
            assert np.abs(got[q] - ref).sum() <= 1e-13, (k, q)
        assert st.sweeps == k and not st.converged
    G.close()


def test_batch_many_batches_one_lane_tail(dg):
    """1025 queries: 17 launches of 64 lanes, the last holding one query.
    Sampled rows in every batch, the tail included, bit-exact (SSSP) or
    within the rule's bound (PPR)."""
    g = gg.rmat(10, seed=30)
    rng = np.random.default_rng(30)
    k = 1025
    srcs = rng.integers(0, g.n, size=k).astype(np.uint32)
    G = dg.Graph.from_csr(g)
    sample = list(range(0, k, 61)) + [63, 64, 1023, 1024]
    for mode, d in (("sync", 1), ("async", 1), ("delayed", 64)):
        out, st = G.sssp_batch(srcs, mode=mode, d=d)
        got = out.cpu().numpy()
        assert got.shape == (k, g.n) and st.converged
        for q in sample:
            np.testing.assert_array_equal(got[q], osp.bellman_ford_sync(g, int(srcs[q]))[0], err_msg=f"{mode} {q}")
    out, st = G.ppr_batch(srcs, tol=1e-9, mode="delayed", d=64, dtype="f64", max_sweeps=5000)
    got = out.cpu().numpy()
    assert st.converged and np.abs(got.sum(axis=1) - 1.0).max() < 1e-9
    for q in sample:
        assert np.abs(got[q] - opr.ppr_fixed_point(g, int(srcs[q]))).sum() <= 1e-8, q
    G.close()


def test_batch_single_query_matches_single_entry_point(dg):
    """A batch of one query equals the single-query entry points: SSSP bit
    for bit, PPR within the rule's bound of the same fixed point; a batch of
    one source repeated gives identical rows in synchronous mode."""
    g = gg.rmat(12, seed=33)
    s = int(gg.pick_sources(g, 1, seed=9)[0])
    G = dg.Graph.from_csr(g)
    for mode, d in MODES:
        one, _ = G.sssp_batch(np.array([s], np.uint32), mode=mode, d=d)
        single, _ = G.sssp(s, mode=mode, d=d)
        np.testing.assert_array_equal(one[0].cpu().numpy(), single.cpu().numpy(), err_msg=f"{mode} d={d}")
        p, _ = G.ppr_batch(np.array([s], np.uint32), tol=1e-9, mode=mode, d=d, dtype="f64", max_sweeps=5000)
        x, _ = G.ppr(s, tol=1e-9, mode=mode, d=d, dtype="f64", max_sweeps=5000)
        assert np.abs(p[0].cpu().numpy() - x.cpu().numpy()).sum() <= 2e-8, (mode, d)
    rep = np.full(130, s, np.uint32)
    out, _ = G.ppr_batch(rep, tol=1e-9, mode="sync", dtype="f64")
    got = out.cpu().numpy()
    assert (got == got[0]).all()
    G.close()


def test_batch_degenerate_graphs(dg):
    """One vertex without edges, a self-loop only, and an edgeless graph:
    distance 0 at the source and unreachable elsewhere, PPR all mass at the
    restart vertex (a dangling vertex returns its mass there)."""
    G = dg.Graph(1, np.array([0, 0], np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    for mode, d in MODES:
        dist, _ = G.sssp_batch(np.zeros(3, np.uint32), mode=mode, d=d)
        assert (dist.cpu().numpy() == 0).all()
        p, _ = G.ppr_batch(np.zeros(2, np.uint32), tol=1e-12, mode=mode, d=d, dtype="f64")
        assert np.abs(p.cpu().numpy() - 1.0).max() < 1e-15
    G.close()
    G = dg.Graph(1, np.array([0, 1], np.uint64), np.zeros(1, np.uint32), np.array([9], np.uint32))
    p, _ = G.ppr_batch(np.zeros(1, np.uint32), tol=1e-12, mode="async", dtype="f64")
    assert abs(p.cpu().numpy()[0, 0] - 1.0) < 1e-15
    G.close()
    n = 777
    G = dg.Graph(n, np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    srcs = np.array([0, 5, 776], np.uint32)
    for mode, d in MODES:
        dist, _ = G.sssp_batch(srcs, mode=mode, d=d)
        dv = dist.cpu().numpy()
        p, _ = G.ppr_batch(srcs, tol=1e-12, mode=mode, d=d, dtype="f64")
        pv = p.cpu().numpy()
        for q, s in enumerate(srcs.tolist()):
            assert dv[q, s] == 0 and (np.delete(dv[q], s) == dg.DG_INF_DIST).all()
            assert abs(pv[q, s] - 1.0) < 1e-15 and np.abs(np.delete(pv[q], s)).max() == 0.0
    G.close()


def test_batch_commit_counts(dg):
    """dg_stats.commits of a delayed batched call: each wavefront commits
    every ceil(d/4) of its rows and at the end of its block, so d = 1 commits
    every row on its own (n per batch-sweep), d = 64 about n/16 (staged in
    LDS), d = 256 about n/64 (staged in the shadow), and a whole block at
    most once per wavefront; sync and async report 0.  The
    interval is n / commits."""
    g = gg.rmat(12, seed=40)
    srcs = gg.pick_sources(g, 3, seed=1)
    G = dg.Graph.from_csr(g)
    for call in ("sssp", "ppr"):
        def run(mode, d):
            if call == "sssp":
                return G.sssp_batch(srcs, mode=mode, d=d)[1]
            return G.ppr_batch(srcs, tol=1e-9, mode=mode, d=d, dtype="f64")[1]
        for mode in ("sync", "async"):
            st = run(mode, 1)
            assert st.commits == 0 and st.commit_interval == 0
        st = run("delayed", 1)
        assert st.commits == g.n and st.commit_interval == 1, (call, st.commits)
        Tb = G.info().batch_tiles  # the batched calls' own tiles
        assert st.tile_vertices == (g.n + Tb // 2) // Tb
        st = run("delayed", 64)
        waves = 4 * st.workers
        assert g.n / 16 <= st.commits <= g.n / 16 + waves, (call, st.commits)
        assert abs(st.commit_interval - g.n / st.commits) <= 0.5
        st = run("delayed", 256)  # staged in the shadow, a commit every 64 rows per wavefront
        assert g.n / 64 <= st.commits <= g.n / 64 + 4 * st.workers, (call, st.commits)
        st = run("delayed", dg.DG_D_WHOLE)
        assert st.workers <= st.commits <= waves, (call, st.commits)
        print(f"{call}: whole-block commits {st.commits} for {st.workers} workers", flush=True)
    G.close()
