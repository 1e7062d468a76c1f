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


def _rows(text, header):
    """Cells of the markdown table that starts with `header` (first cell kept as text)."""
    lines = text[text.index(header):].splitlines()[2:]
    out = []
    for ln in lines:
        if not ln.startswith("|"):
            break
        out.append([c.strip() for c in ln.strip("|").split("|")])
    return out


def test_batched_summaries_add_up():
    """The derived columns of the batched summaries follow from their raw
    ones: fabric bytes per batch-sweep = (FETCH_SIZE x 2.0 + WRITE_SIZE) KiB
    over the 4 batches of a dispatch, and achieved TB/s = algorithmic bytes of
    the 4 batches / median duration, against 8 TB/s."""
    with open(os.path.join(ROOT, "profiles", "batch_rmat22.md")) as fh:
        text = fh.read()
    alg22 = {"mbf": 19.18, "mppr": 20.18}  # GB per batch-sweep (SSSP, PPR)
    rows = _rows(text, "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB |")
    assert len(rows) == 6
    for r in rows:
        f, w, fgb, wgb, tot, alg, ratio = (float(x) for x in r[1:8])
        assert abs(f * 1024 * 2.0 / 4 / 1e9 - fgb) <= 0.006 and abs(w * 1024 / 4 / 1e9 - wgb) <= 0.006, r
        assert abs(fgb + wgb - tot) <= 0.011 and alg == alg22["mbf" if "mbf" in r[0] else "mppr"], r
        assert abs(tot / alg - ratio) <= 0.006, r
    rows = _rows(text, "| kernel | mode | sweeps | median ms (4 batches) | ms per batch |")
    assert len(rows) == 6
    for r in rows:
        ms, per, tbs, frac = (float(x) for x in r[3:7])
        alg = alg22["mbf" if "mbf" in r[0] else "mppr"]
        # the table rounds the median to 0.01 ms
        assert abs(ms / 4 - per) <= 0.006 and abs(alg * 4 / ms - tbs) <= 0.006 + tbs * 0.005 / ms, r
        assert abs(tbs / 8 - frac) <= 0.006, r
    with open(os.path.join(ROOT, "profiles", "batch_rmat20.md")) as fh:
        text = fh.read()
    n, m = 1048576, 16084292
    alg20 = {"mbf": (m * 261 + n * 512) / 1e9, "mppr": (m * 260 + n * 768) / 1e9}
    rows = _rows(text, "| kernel | mode | sweeps | median ms (4 batches) | algorithmic TB/s |")
    assert len(rows) == 6
    for r in rows:
        ms, tbs, frac = (float(x) for x in r[3:6])
        alg = alg20["mbf" if "mbf" in r[0] else "mppr"]
        # the table rounds the median to 0.01 ms
        assert abs(alg * 4 / ms - tbs) <= 0.006 + tbs * 0.005 / ms and abs(tbs / 8 - frac) <= 0.006, r
