"""The stored expected values for the small R-MAT workload still match the
oracle and the generator (catches drift in either)."""
import json
import os

import numpy as np

import graphgen as gg
from oracle import pagerank as opr
from oracle import sssp as osp

HERE = os.path.dirname(os.path.abspath(__file__))


def test_rmat10_golden_matches_oracle():
    with open(os.path.join(HERE, "golden", "rmat10_seed10.json")) as f:
        gold = json.load(f)
    g = gg.rmat(10, seed=10)
    assert g.sha256() == gold["sha256"] and g.m == gold["m"]
    xs = opr.pagerank_fixed_point(g)
    assert np.abs(xs - np.array(gold["pagerank_fixed_point"])).sum() < 1e-13
    d, s, _ = osp.bellman_ford_sync(g, gold["sssp_source"])
    np.testing.assert_array_equal(d, np.array(gold["sssp_dist"], dtype=np.uint32))
    assert s == gold["sssp_sync_sweeps"]
    ok, msg = osp.certificate(g, 0, d)
    assert ok, msg
    assert opr.certificate(g, np.array(gold["pagerank_fixed_point"])) < 1e-10
