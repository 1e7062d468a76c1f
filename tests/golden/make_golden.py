"""Write the stored expected values for the small R-MAT workload.

Calls only the CPU oracle (and the seeded input generator).  Output:
``rmat10_seed10.json`` holding the graph's sha256, the PageRank fixed point
(float64, L1 change < 1e-12 then normalised), the synchronous sweep counts at
tol 1e-6, and the Bellman-Ford distances from vertex 0 with the synchronous
sweep count.

Workload: R-MAT scale 10, edge factor 16, a/b/c/d = 0.57/0.19/0.19/0.05,
ids permuted, directed, duplicates removed, weights uniform in [1, 255],
seed 10; PageRank damping 0.85 from 1/N.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
from oracle import pagerank as opr  # noqa: E402
from oracle import sssp as osp  # noqa: E402


def main():
    g = gg.rmat(10, seed=10)
    xs = opr.pagerank_fixed_point(g, tol=1e-12)
    _, sweeps_pr, _, _ = opr.pagerank_jacobi(g, tol=1e-6)
    _, sweeps_pr7, _, _ = opr.pagerank_jacobi(g, tol=1e-7)
    d, sweeps_bf, _ = osp.bellman_ford_sync(g, 0)
    out = {
        "workload": "rmat scale 10, ef 16, abcd .57/.19/.19/.05, permuted, dedup, w U[1,255], seed 10",
        "sha256": g.sha256(),
        "n": g.n,
        "m": g.m,
        "alpha": 0.85,
        "pagerank_fixed_point": [float(v) for v in xs],
        "pagerank_sync_sweeps_tol1e-6": sweeps_pr,
        "pagerank_sync_sweeps_tol1e-7": sweeps_pr7,
        "sssp_source": 0,
        "sssp_dist": [int(v) for v in d],
        "sssp_sync_sweeps": sweeps_bf,
    }
    path = os.path.join(HERE, "rmat10_seed10.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
