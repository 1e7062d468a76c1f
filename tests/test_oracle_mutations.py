"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each test monkeypatches one oracle function with a plausible bug (a dropped
term, a transposed operand, a wrong index or sign) and checks that at least
one independent pin then fails.  This shows the pins have teeth; the real
oracle passes the same checks in test_oracle_pins.py.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp
from tests import graphs as tg

A = 0.85


def _pr_pins_hold():
    """The closed-form and networkx pins, as one boolean."""
    checks = []
    n = 5
    x = opr.pagerank_fixed_point(tg.in_star(n))
    hub = (1 + (n - 1) * A) / (n + (n - 1) * A)
    checks.append(abs(x[0] - hub) < 1e-9)
    x = opr.pagerank_fixed_point(tg.out_star(n))
    checks.append(abs(x[0] - 1 / (n + A)) < 1e-9)
    x = opr.pagerank_fixed_point(tg.cycle(7))
    checks.append(np.abs(x - 1 / 7).max() < 1e-9)
    x = opr.pagerank_fixed_point(gg.from_edges(2, [0], [1]))
    checks.append(abs(x[0] - 1 / (2 + A)) < 1e-9)
    # unnormalised Jacobi iterate must keep mass 1 by itself
    xs, _, _, _ = opr.pagerank_jacobi(tg.dangling_heavy(40, 1), tol=1e-12)
    checks.append(abs(xs.sum() - 1) < 1e-9)
    return all(checks)


def _mut_no_dangling(x, src, dst, deg, alpha=A):
    n = x.shape[0]
    c = np.where(deg > 0, x / np.maximum(deg, 1), 0.0)
    return (1 - alpha) / n + alpha * np.bincount(dst, weights=c[src], minlength=n)


def _mut_transposed(x, src, dst, deg, alpha=A):
    n = x.shape[0]
    c = np.where(deg > 0, x / np.maximum(deg, 1), 0.0)
    pulled = np.bincount(src, weights=c[dst], minlength=n)
    return (1 - alpha) / n + alpha * (pulled + x[deg == 0].sum() / n)


def _mut_teleport(x, src, dst, deg, alpha=A):
    n = x.shape[0]
    c = np.where(deg > 0, x / np.maximum(deg, 1), 0.0)
    pulled = np.bincount(dst, weights=c[src], minlength=n)
    return (1 - alpha) + alpha * (pulled + x[deg == 0].sum() / n)


def _mut_no_degree(x, src, dst, deg, alpha=A):
    n = x.shape[0]
    c = np.where(deg > 0, x, 0.0)
    pulled = np.bincount(dst, weights=c[src], minlength=n)
    return (1 - alpha) / n + alpha * (pulled + x[deg == 0].sum() / n)


def test_real_oracle_passes():
    assert _pr_pins_hold()


@pytest.mark.parametrize("mutant", [_mut_no_dangling, _mut_transposed, _mut_teleport, _mut_no_degree])
def test_pagerank_mutants_caught(monkeypatch, mutant):
    monkeypatch.setattr(opr, "apply_T", mutant)
    assert not _pr_pins_hold()


def _sssp_pins_hold():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra as sp_dijkstra
    ok = True
    for seed in range(3):
        g = tg.random_graph(40, 100, seed)
        src, dst, w = osp.edge_list(g)
        mat = csr_matrix((w.astype(np.float64), (src, dst)), shape=(g.n, g.n))
        d, sweeps, its = osp.bellman_ford_sync(g, 0, keep_iterates=True)
        ref = sp_dijkstra(mat, directed=True, indices=0)
        ref = np.where(np.isinf(ref), osp.INF32, ref).astype(np.uint32)
        ok &= bool(np.array_equal(d, ref))
        ok &= osp.certificate(g, 0, d)[0]
        for k, it in enumerate(its, start=1):
            ok &= bool(np.array_equal(it, osp.bounded_hop_distances(g, 0, k)))
    p = gg.path_graph(12)
    d, sweeps, _ = osp.bellman_ford_sync(p, 0)
    ok &= bool(np.array_equal(d, np.arange(12))) and sweeps == 12
    return ok


def test_real_sssp_passes():
    assert _sssp_pins_hold()


def _edge_list_weight_off_by_one(g):
    s, d, w = _orig_edge_list(g)
    return s, d, w - 1


def _edge_list_reversed(g):
    s, d, w = _orig_edge_list(g)
    return d, s, w


_orig_edge_list = osp.edge_list


@pytest.mark.parametrize("mutant", [_edge_list_weight_off_by_one, _edge_list_reversed])
def test_sssp_mutants_caught(monkeypatch, mutant):
    monkeypatch.setattr(osp, "edge_list", mutant)
    assert not _sssp_pins_hold()


def test_sssp_extra_sweep_caught(monkeypatch):
    """A Bellman-Ford that forgets to count the confirming sweep breaks the
    path-graph sweep count."""
    orig = osp.bellman_ford_sync

    def short(g, source, max_sweeps=None, keep_iterates=False):
        d, s, its = orig(g, source, max_sweeps, keep_iterates)
        return d, s - 1, its[:-1]

    monkeypatch.setattr(osp, "bellman_ford_sync", short)
    assert not _sssp_pins_hold()


# ------------------------------------------------ error certificates --
#
# The certificates ||T(x) - x|| / (1 - alpha) decide the pass/fail of results
# that have no stored fixed point (large batched and served personalised
# PageRank rows), so each plausible mistake in them must break a pin.


def _cert_pins_hold(cert_fn, fixed_point, graphs):
    """The pins of test_oracle_pins: certificate ~ 0 at the fixed point from a
    dense solve, err <= cert <= (1 + a)/(1 - a) err around it, and exactness
    on a rescaled fixed point."""
    ok = True
    rng = np.random.default_rng(9)
    for g, s in graphs:
        xs = fixed_point(g, s)
        ok &= cert_fn(g, xs, s) < 1e-13
        n = g.n
        pert = [xs + sc * rng.standard_normal(n) / n for sc in (1e-3, 1e-6)] + [xs * (1 + 1e-4), xs * (1 - 3e-7)]
        for x in pert:
            err = np.abs(x - xs).sum()
            c = cert_fn(g, x, s)
            ok &= err <= c * (1 + 1e-9) + 1e-15
            ok &= c <= err * (1 + A) / (1 - A) * (1 + 1e-9) + 1e-15
    return bool(ok)


_PPR_GRAPHS = [(tg.random_graph(120, 500, 11), 3), (tg.dangling_heavy(90, 5), 7)]


def _ppr_holds():
    return _cert_pins_hold(lambda g, x, s: opr.ppr_certificate(g, x, s), opr.ppr_dense, _PPR_GRAPHS)


def _pr_holds():
    graphs = [(tg.random_graph(120, 500, 11), 0), (tg.dangling_heavy(90, 5), 0)]
    return _cert_pins_hold(lambda g, x, s: opr.certificate(g, x), lambda g, s: opr.pagerank_dense(g), graphs)


def test_real_certificates_pass():
    assert _ppr_holds()
    assert _pr_holds()


def _ppr_step(x, src, dst, deg, s, alpha, teleport=True, dangling_to="restart"):
    n = x.shape[0]
    c = np.where(deg > 0, x / np.maximum(deg, 1), 0.0)
    out = alpha * np.bincount(dst, weights=c[src], minlength=n)
    dang = float(x[deg == 0].sum())
    if dangling_to == "restart":
        out[s] += alpha * dang
    else:
        out += alpha * dang / n
    if teleport:
        out[s] += 1.0 - alpha
    return out


def _ppr_cert_mutant(kind):
    def cert(g, x, s, alpha=A):
        src, dst = opr.edge_list(g)
        deg = opr.out_degree(g)
        x = np.asarray(x, dtype=np.float64)
        if kind == "no_factor":
            return float(np.abs(opr.apply_ppr(x, src, dst, deg, s, alpha) - x).sum())
        if kind == "zero":
            return 0.0
        if kind == "plus_alpha":
            return float(np.abs(opr.apply_ppr(x, src, dst, deg, s, alpha) - x).sum()) / (1.0 + alpha)
        if kind == "dangling_uniform":
            y = _ppr_step(x, src, dst, deg, s, alpha, dangling_to="uniform")
        elif kind == "no_teleport":
            y = _ppr_step(x, src, dst, deg, s, alpha, teleport=False)
        return float(np.abs(y - x).sum()) / (1.0 - alpha)
    return cert


@pytest.mark.parametrize("kind", ["no_factor", "zero", "plus_alpha", "dangling_uniform", "no_teleport"])
def test_ppr_certificate_mutants_caught(monkeypatch, kind):
    monkeypatch.setattr(opr, "ppr_certificate", _ppr_cert_mutant(kind))
    assert not _ppr_holds()


def _pr_cert_mutant(kind):
    def cert(g, x, alpha=A):
        src, dst = opr.edge_list(g)
        deg = opr.out_degree(g)
        x = np.asarray(x, dtype=np.float64)
        r = float(np.abs(opr.apply_T(x, src, dst, deg, alpha) - x).sum())
        return {"no_factor": r, "zero": 0.0, "plus_alpha": r / (1.0 + alpha)}[kind]
    return cert


@pytest.mark.parametrize("kind", ["no_factor", "zero", "plus_alpha"])
def test_pr_certificate_mutants_caught(monkeypatch, kind):
    monkeypatch.setattr(opr, "certificate", _pr_cert_mutant(kind))
    assert not _pr_holds()
