"""CPU checks of bench.py's host-side parts: it refuses more than one GPU,
and its algorithmic-byte model (the numerator of roofline.achieved) counts
what each sweep must move: per edge the source index, the gathered value
and, for SSSP, the stored weight; per vertex the offset and the per-vertex
reads and writes of the update."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N22, M22 = 4_194_304, 65_243_650  # RMAT-22, seed 22


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_algorithmic_bytes_per_sweep():
    sys.path.insert(0, ROOT)
    import bench
    n, m = N22, M22
    # PageRank: 4-byte index + gathered contribution per edge; offset,
    # out-degree, old score, new score and new contribution per vertex
    assert bench.pr_bytes_per_sweep(n, m, "f32") == 8 * m + 20 * n == 605_835_280
    assert bench.pr_bytes_per_sweep(n, m, "f64") == 12 * m + 32 * n
    # Bellman-Ford: index + weight + gathered distance per edge; offset, old
    # and new distance per vertex; byte weights when every weight fits a byte
    assert bench.bf_bytes_per_sweep(n, m, 1) == 9 * m + 12 * n == 637_524_498
    assert bench.bf_bytes_per_sweep(n, m, 4) == 12 * m + 12 * n


def test_oracle_worker_and_cpu_baseline():
    """The bench's oracle leg on a small graph of the same family: its
    reference x* is the oracle's fixed point, its Bellman-Ford distances
    equal scipy's Dijkstra, and the CPU-baseline record is well formed."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench
    import graphgen as gg
    from oracle import pagerank as opr
    orc = bench.oracle_worker(10, 2)
    g = gg.rmat(10, seed=10)
    assert np.abs(orc["xstar"] - opr.pagerank_fixed_point(g)).sum() < 1e-9
    sw6, t6 = orc["pr_tol1e-6"]
    sw7, t7 = orc["pr_tol1e-7"]
    assert 0 < sw6 <= sw7 <= orc["ref_sweeps"] and 0 < t6 <= t7
    assert len(orc["bf"]) == 2 and all(d["equal_to_bf"] for d in orc["dijkstra"])
    cpu = bench.cpu_baseline(orc, g.m)
    assert cpu["kind"] == "oracle" and cpu["cores"] == 1 and cpu["unit"] == "GTEPS"
    assert abs(cpu["value"] - round(g.m * sw6 / t6 / 1e9, 4)) < 1e-12
