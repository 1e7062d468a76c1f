"""Single-query personalised PageRank (dg_ppr) against the CPU oracle (needs
an MI355X).

* Every mode and d, float64 at tol 1e-9: L1 <= 1e-8 of the oracle's fixed
  point x*_s (the oracle's Jacobi to 1e-12, normalised); float32 at tol
  1.5e-7: L1 <= 1e-6.  The stopping rule bounds a synchronous iterate's error
  by alpha/(1-alpha) tol = 8.5e-7 there; at tol 5e-7 a slowly mixing graph
  (the banded one) stops 2.2e-6 away, as that bound allows.
* Synchronous iterates: after k sweeps the (normalised) result equals the
  oracle's k-th Jacobi iterate to 1e-13 (synchronous sweeps conserve mass, so
  the rescale is 1 up to rounding).
* A dangling restart vertex keeps all the mass: x* = e_s.
* err_bound equals the oracle's certificate of the returned vector.
* Global PageRank through the same kernels is unchanged (bit-identical
  iterates are checked against the stored golden values elsewhere; here the
  two entry points give different results on the same graph).
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from tests import graphs as tg

pytestmark = pytest.mark.gpu
F32_TOL = 1.5e-7
MODES = [("sync", 1), ("async", 1), ("delayed", 1), ("delayed", 64), ("delayed", 0xFFFFFFFF),
         ("delayed_local", 64)]


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


_G = {}


def _graph(name):
    if name not in _G:
        g = {"rmat13": lambda: gg.rmat(13, seed=13), "dangling": lambda: tg.dangling_heavy(6000, 9),
             "banded": lambda: gg.banded(40_000, 8, 512, 0.01, seed=5), "instar": lambda: tg.in_star(3000)}[name]()
        _G[name] = g
    return _G[name]


@pytest.mark.parametrize("name", ["rmat13", "dangling", "banded", "instar"])
def test_ppr_all_modes(dg, name):
    g = _graph(name)
    G = dg.Graph.from_csr(g)
    srcs = gg.pick_sources(g, 2, seed=3).tolist()
    if name == "instar":
        srcs = [0, 5]  # the hub (dangling) and a leaf
    for s in srcs:
        xs = opr.ppr_fixed_point(g, s)
        for mode, d in MODES:
            for dtype, tol, bound in (("f64", 1e-9, 1e-8), ("f32", F32_TOL, 1e-6)):
                x, st = G.ppr(s, tol=tol, mode=mode, d=d, dtype=dtype, max_sweeps=5000)
                err = float(np.abs(x.cpu().numpy() - xs).sum())
                print(f"{name} s={s} {mode} d={d} {dtype}: sweeps={st.sweeps} L1 err={err:.2e}", flush=True)
                assert err <= bound, (name, s, mode, d, dtype, err)
    G.close()


def test_ppr_sync_iterates(dg):
    g = _graph("rmat13")
    s = int(gg.pick_sources(g, 1, seed=7)[0])
    G = dg.Graph.from_csr(g)
    for k in (1, 2, 5, 9):
        x, st = G.ppr(s, tol=0.0, mode="sync", dtype="f64", max_sweeps=k, allow_not_converged=True)
        ref, _ = opr.ppr_jacobi(g, s, tol=0.0, max_sweeps=k)
        ref = ref / ref.sum()
        assert st.sweeps == k
        assert np.abs(x.cpu().numpy() - ref).sum() <= 1e-13
    G.close()


def test_ppr_dangling_restart_and_err_bound(dg):
    g = _graph("dangling")
    G = dg.Graph.from_csr(g)
    s = int(np.flatnonzero(np.diff(g.ptr.astype(np.int64)) == 0)[0])
    x, st = G.ppr(s, tol=1e-12, mode="async", dtype="f64")
    e = np.zeros(g.n)
    e[s] = 1.0
    assert np.abs(x.cpu().numpy() - e).sum() < 1e-14
    s2 = int(gg.pick_sources(g, 1, seed=2)[0])
    for mode, dtype, tol in (("sync", "f64", 1e-6), ("delayed", "f32", 1e-5)):
        x, st = G.ppr(s2, tol=tol, mode=mode, d=64, dtype=dtype, err_bound=True)
        x = x.cpu().numpy()
        cert = opr.ppr_certificate(g, x, s2)
        err = float(np.abs(x - opr.ppr_fixed_point(g, s2)).sum())
        print(f"ppr {mode} {dtype} tol={tol}: err_bound {st.err_bound:.3e} oracle cert {cert:.3e} err {err:.3e}")
        assert abs(st.err_bound - cert) <= 1e-12 + 1e-9 * cert
        assert st.err_bound >= err - 1e-12
    G.close()


def test_ppr_matches_batched_rows(dg):
    g = _graph("rmat13")
    G = dg.Graph.from_csr(g)
    srcs = gg.pick_sources(g, 5, seed=11)
    xb, _ = G.ppr_batch(srcs, tol=1e-10, mode="sync", dtype="f64")
    for q, s in enumerate(srcs.tolist()):
        x, _ = G.ppr(s, tol=1e-10, mode="sync", dtype="f64")
        assert float((x - xb[q]).abs().sum()) < 1e-9
    G.close()


def test_ppr_validation(dg):
    g = _graph("instar")
    G = dg.Graph.from_csr(g)
    with pytest.raises(dg.DGError):
        G.ppr(g.n)
    with pytest.raises(dg.DGError):
        G.ppr(0, damping=1.0)
    G.close()


def test_error_bound_of_any_vector(dg):
    """dg_error_bound equals the oracle's certificates (global and
    personalised) on perturbed vectors, from device and host memory."""
    import torch
    g = _graph("dangling")
    G = dg.Graph.from_csr(g)
    rng = np.random.default_rng(4)
    s = int(gg.pick_sources(g, 1, seed=8)[0])
    for restart in (None, s):
        xs = opr.pagerank_fixed_point(g) if restart is None else opr.ppr_fixed_point(g, s)
        for sc in (1e-3, 1e-7):
            y = np.abs(xs + sc * rng.standard_normal(g.n) / g.n)
            y /= y.sum()
            want = opr.certificate(g, y) if restart is None else opr.ppr_certificate(g, y, s)
            got_h = G.error_bound(y, restart=restart)
            got_d = G.error_bound(torch.from_numpy(y).cuda(), restart=restart)
            assert abs(got_h - want) <= 1e-12 + 1e-9 * want and abs(got_d - want) <= 1e-12 + 1e-9 * want
            assert got_h >= np.abs(y - xs).sum() - 1e-12
    G.close()
