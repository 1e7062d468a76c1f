"""dg_sssp_noalloc against dg_sssp through the C ABI (needs an MI355X).

The no-allocation entry point keeps every buffer of the call in the
library's fixed scratch array.  Two calls in a row, the second on a smaller
graph, must both give dg_sssp's distances bit for bit (and, in synchronous
mode, its sweep count), so nothing a call leaves in the shared array may leak
into the next.  Host and device outputs are both exercised, and a graph whose
call would need more scratch than the array holds is refused cleanly.
"""
import ctypes as C

import numpy as np
import pytest

import graphgen as gg
from tests import graphs as tg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_01409_amd import dg as _dg
    return _dg


MODES = [("sync", 1), ("async", 1), ("delayed", 64), ("delayed", 1 << 20)]


def _host_call(dg, G, src, mode, d):
    out = np.full(G.n, 7, np.uint32)
    st = dg.dg_stats()
    s = dg.dg_sssp_noalloc(G._h, int(src), dg.MODES[mode], int(d), 65535, dg._np_ptr(out), 0, C.byref(st), None)
    assert s == dg.DG_OK, dg.last_error()
    return out, st


@pytest.mark.parametrize("mode,d", MODES)
def test_noalloc_matches_sssp_twice(dg, mode, d):
    import torch
    big = gg.rmat(14, seed=14)
    small = tg.random_graph(3001, 20_000, 7, weights=(1, 255))
    for g in (big, small):  # second call: smaller input into the same scratch
        G = dg.Graph.from_csr(g)
        for src in gg.pick_sources(g, 2, seed=5).tolist():
            ref, sr = G.sssp(src, mode=mode, d=d)
            out, sn = G.sssp_noalloc(src, mode=mode, d=d)
            print(f"{g.name} n={g.n} {mode} d={d} src={src}: sweeps {sn.sweeps} (dg_sssp {sr.sweeps})", flush=True)
            assert torch.equal(out, ref)
            if mode == "sync":
                assert sn.sweeps == sr.sweeps
            assert sn.commits == sr.commits and sn.commit_interval == sr.commit_interval
            host, sh = _host_call(dg, G, src, mode, d)
            np.testing.assert_array_equal(host, ref.cpu().numpy())
        G.close()


def test_noalloc_refuses_beyond_scratch(dg):
    """A graph whose distance arrays alone exceed the fixed array."""
    n = dg.DG_NOALLOC_SCRATCH_BYTES // 8 + 1024  # two uint32 arrays of n slots > the array
    g = gg.path_graph(n)
    G = dg.Graph.from_csr(g)
    with pytest.raises(dg.DGError) as e:
        G.sssp_noalloc(0, mode="sync", max_sweeps=4)
    assert e.value.status == dg.DG_ERR_UNSUPPORTED and "scratch" in str(e.value)
    out, st = G.sssp(0, mode="async", max_sweeps=4, allow_not_converged=True)  # the graph itself is fine
    G.close()


def test_noalloc_validation(dg):
    g = tg.random_graph(100, 400, 3, weights=(1, 9))
    G = dg.Graph.from_csr(g)
    out = np.zeros(g.n, np.uint32)
    st = dg.dg_stats()
    for args, want in [((None, 0, 0, 1, 10), dg.DG_ERR_INVALID_ARGUMENT),
                       ((G._h, g.n, 0, 1, 10), dg.DG_ERR_INVALID_ARGUMENT),
                       ((G._h, 0, 3, 1, 10), dg.DG_ERR_INVALID_ARGUMENT),
                       ((G._h, 0, 2, 0, 10), dg.DG_ERR_INVALID_ARGUMENT),
                       ((G._h, 0, 0, 1, 0), dg.DG_ERR_INVALID_ARGUMENT),
                       ((G._h, 0, 0, 1, 65536), dg.DG_ERR_INVALID_ARGUMENT)]:
        assert dg.dg_sssp_noalloc(*args, dg._np_ptr(out), 0, C.byref(st), None) == want
    G.close()
