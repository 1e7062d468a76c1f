"""The committed profile summaries agree on how byte counters are turned
into bytes (CPU only): FETCH_SIZE reads half of a plain copy's bytes on this
GPU, so every summary that converts FETCH_SIZE multiplies by 2.0, and the
traffic file bench.py reads carries the same factor."""
import glob
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fetch_size_calibration_is_the_same_everywhere():
    files = glob.glob(os.path.join(ROOT, "profiles", "*.md"))
    converting = [f for f in files if re.search(r"FETCH_SIZE[^\n]*x 1024", open(f).read())]
    assert converting, "no summary converts FETCH_SIZE"
    for f in converting:
        text = open(f).read()
        assert re.search(r"FETCH_SIZE x 1024 x 2\.0", text), f
        assert not re.search(r"FETCH_SIZE x 1024 / ", text), f
    with open(os.path.join(ROOT, "profiles", "pr_sweep_f32_delayed_rmat22_traffic.json")) as fh:
        tr = json.load(fh)
    assert abs(tr["fetch_scale_from_copy"] - 2.0) < 1e-3 and tr["write_scale_from_copy"] == 1.0
    want = tr["fetch_kib_per_launch_raw"] * 1024 * tr["fetch_scale_from_copy"] + tr["write_kib_per_launch_raw"] * 1024
    assert abs(tr["hbm_bytes_per_launch"] - want) < 2


def test_traffic_file_matches_the_kernel_source():
    """The traffic file bench.py reports beside its roofline was measured on the
    sweep kernel source as it stands (its sha256 prefix), so a changed kernel
    is re-profiled before the file is used again."""
    import hashlib
    with open(os.path.join(ROOT, "profiles", "pr_sweep_f32_delayed_rmat22_traffic.json")) as fh:
        tr = json.load(fh)
    src = os.path.join(ROOT, "paper_2110_01409_amd", "csrc", "sweep_kernels.hip")
    with open(src, "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()[:16]
    assert tr["kernel_sha256_16"] == h
    with open(os.path.join(ROOT, "profiles", "sweeps_delayed_rmat22.md")) as fh:
        assert h in fh.read()
