"""GPU parity of the access-matrix instrumentation (NEXT f4; section IV,
effects of graph topology): the library's matrix equals, count for count,
the oracle's definition evaluated with the library's own partition."""
import ctypes as C

import numpy as np
import pytest

import graphgen as gg
from oracle import topology as otop
from tests import graphs as tg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


@pytest.mark.parametrize("name", ["rmat14", "banded", "instar", "complete", "few_workers"])
def test_access_matrix_matches_oracle(dg, name):
    kw = {}
    if name == "rmat14":
        g = gg.rmat(14, seed=14)  # has a compact hot region (slots >= n in the index stream)
    elif name == "banded":
        g = gg.banded(200_000, 8, 1024, 0.01, seed=6)
    elif name == "instar":
        g = tg.in_star(5000)
    elif name == "complete":
        g = tg.complete(40)
    else:
        g = gg.rmat(12, seed=3)
        kw = {"workers": 5}
    G = dg.Graph.from_csr(g, **kw)
    info = G.info()
    first = G.partition()
    assert first[0] == 0 and first[-1] == g.n and (np.diff(first.astype(np.int64)) >= 0).all()
    assert first.shape[0] == info.workers + 1
    if name == "rmat14":
        assert info.hot_vertices > 0
    for groups in sorted({1, min(8, info.workers), min(32, info.workers), min(64, info.workers)}):
        counts, st = G.access_matrix(groups)
        ref, same = otop.access_matrix(g, first, groups)
        np.testing.assert_array_equal(counts.astype(np.int64), ref, err_msg=f"{name} groups={groups}")
        assert st.reads == g.m and st.same_worker == same and st.groups == groups
        d, u = otop.shares(ref)
        assert abs(st.diagonal_share - d) < 1e-12 and abs(st.uniform_diagonal - u) < 1e-12
    G.close()


def test_access_matrix_validation(dg):
    g = gg.rmat(10, seed=1)
    G = dg.Graph.from_csr(g)
    st = dg.dg_access_stats()
    for groups in (0, 65, G.info().workers + 1):
        assert dg.dg_access_matrix(G._h, groups, None, C.byref(st), None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_access_matrix(G._h, 4, None, None, None) == dg.DG_ERR_INVALID_ARGUMENT
    G.close()


@pytest.mark.parametrize("name,want", [("banded", "async"), ("rmat14", "delayed"), ("few_workers", "delayed")])
def test_predict_mode(dg, name, want):
    """dg_predict_mode reads the 8-group access matrix (the oracle's shares of
    the same partition) and leaves commits unbuffered exactly when the lift
    of the diagonal reaches DG_PREDICT_CLUSTER_LIFT."""
    kw = {}
    if name == "banded":
        g = gg.banded(200_000, 8, 1024, 0.01, seed=6)
    elif name == "rmat14":
        g = gg.rmat(14, seed=14)
    else:
        g = gg.rmat(12, seed=3)
        kw = {"workers": 5}
    G = dg.Graph.from_csr(g, **kw)
    p = G.predict_mode()
    groups = min(8, G.info().workers)
    ref, same = otop.access_matrix(g, G.partition(), groups)
    d, u = otop.shares(ref)
    assert p["groups"] == groups
    assert abs(p["diagonal_share"] - d) < 1e-12 and abs(p["uniform_diagonal"] - u) < 1e-12
    assert abs(p["lift"] - d / u) < 1e-9 and abs(p["self_share"] - same / g.m) < 1e-12
    assert (p["lift"] >= 2.0) == (p["mode"] == "async")
    assert p["mode"] == want and p["d"] == (64 if want == "delayed" else 0)
    G.close()
