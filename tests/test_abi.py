"""The C-ABI library loads, exports every symbol include/dg.h declares, and
validates arguments on the host before any HIP call (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")


@pytest.fixture(scope="module")
def dg():
    from paper_2110_01409_amd import dg as _dg
    return _dg


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(dg_[a-z_]+)\s*\(", src))
    return {n for n in names if not n.endswith("_fn")}


def test_exports_match_header(dg):
    declared = _declared()
    assert declared == set(dg.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", dg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dg_[a-z_]+)\b", out))
    missing = declared - exported
    assert not missing, missing
    for name in declared:
        assert hasattr(dg.lib, name)


def test_status_strings(dg):
    for s in range(6):
        assert dg.status_str(s).startswith("DG_")
    assert "gfx950" in dg.version()


def _create(dg, n, ptr, idx, w=None, layout=None):
    h = C.c_void_p()
    ptr = np.ascontiguousarray(ptr, np.uint64)
    idx = np.ascontiguousarray(idx, np.uint32)
    wp = None if w is None else dg._np_ptr(np.ascontiguousarray(w, np.uint32))
    s = dg.dg_graph_create(n, idx.shape[0], dg.DG_CSR if layout is None else layout, dg._np_ptr(ptr),
                           dg._np_ptr(idx), wp, None, None, C.byref(h))
    return s, h


@pytest.mark.parametrize("case", ["n0", "ptr0", "decreasing", "ptr_end", "idx_range", "layout", "null_ptr"])
def test_create_validation(dg, case):
    ptr = np.array([0, 1, 3, 3], np.uint64)
    idx = np.array([1, 0, 2], np.uint32)
    n = 3
    layout = None
    if case == "n0":
        n = 0
    elif case == "ptr0":
        ptr = ptr + 1
    elif case == "decreasing":
        ptr = np.array([0, 2, 1, 3], np.uint64)
    elif case == "ptr_end":
        ptr = np.array([0, 1, 2, 2], np.uint64)
    elif case == "idx_range":
        idx = np.array([1, 0, 3], np.uint32)
    elif case == "layout":
        layout = 7
    if case == "null_ptr":
        h = C.c_void_p()
        s = dg.dg_graph_create(3, 3, dg.DG_CSR, None, dg._np_ptr(idx), None, None, None, C.byref(h))
    else:
        s, h = _create(dg, n, ptr, idx, layout=layout)
    assert s == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.last_error()
    assert not h.value


def test_valid_graph_without_device(dg):
    """A well-formed graph passes validation; on a machine without a GPU the
    call then fails cleanly with DG_ERR_DEVICE (with a GPU it succeeds)."""
    import torch
    s, h = _create(dg, 3, [0, 1, 3, 3], [1, 0, 2], [5, 6, 7])
    if torch.cuda.is_available():
        assert s == dg.DG_OK
        dg.dg_graph_destroy(h)
    else:
        assert s == dg.DG_ERR_DEVICE and "device" in dg.last_error()


@pytest.mark.parametrize("case", ["flag2", "null_ptr", "null_idx", "n0", "m_huge"])
def test_create_device_arrays_validation(dg, case):
    """arrays_on_device: the checks that need no read of the arrays come
    before any device call, so they hold on a machine without a GPU."""
    ptr = np.array([0, 1, 3, 3], np.uint64)
    idx = np.array([1, 0, 2], np.uint32)
    n, m = 3, 3
    opts = dg.dg_graph_opts(0, dg.DG_HOT_AUTO, dg.DG_RESIDENT_AUTO, 0, 2 if case == "flag2" else 1)
    pp, ip = dg._np_ptr(ptr), dg._np_ptr(idx)
    if case == "null_ptr":
        pp = None
    elif case == "null_idx":
        ip = None
    elif case == "n0":
        n = 0
    elif case == "m_huge":
        m = 0xFFFFFFFF
    h = C.c_void_p()
    s = dg.dg_graph_create(n, m, dg.DG_CSR, pp, ip, None, C.byref(opts), None, C.byref(h))
    assert s == dg.DG_ERR_INVALID_ARGUMENT, dg.last_error()
    assert dg.last_error() and not h.value


def test_create_device_arrays_needs_device_memory(dg):
    """Host pointers flagged as device arrays: DG_ERR_DEVICE without a GPU,
    DG_ERR_INVALID_ARGUMENT (not device memory) with one."""
    import torch
    ptr = np.array([0, 1, 3, 3], np.uint64)
    idx = np.array([1, 0, 2], np.uint32)
    opts = dg.dg_graph_opts(0, dg.DG_HOT_AUTO, dg.DG_RESIDENT_AUTO, 0, 1)
    h = C.c_void_p()
    s = dg.dg_graph_create(3, 3, dg.DG_CSR, dg._np_ptr(ptr), dg._np_ptr(idx), None, C.byref(opts), None,
                           C.byref(h))
    if torch.cuda.is_available():
        assert s == dg.DG_ERR_INVALID_ARGUMENT and "device memory" in dg.last_error()
    else:
        assert s == dg.DG_ERR_DEVICE
    assert not h.value


def test_plan_refuses_device_arrays(dg):
    ptr = np.array([0, 1, 3, 3], np.uint64)
    idx = np.array([1, 0, 2], np.uint32)
    opts = dg.dg_graph_opts(0, dg.DG_HOT_AUTO, dg.DG_RESIDENT_AUTO, 0, 1)
    h = C.c_void_p()
    s = dg.dg_plan_create(3, 3, dg.DG_CSR, dg._np_ptr(ptr), dg._np_ptr(idx), None, C.byref(opts), 8, C.byref(h))
    assert s == dg.DG_ERR_INVALID_ARGUMENT and "arrays_on_device" in dg.last_error()
    assert not h.value


def test_call_validation_null_graph(dg):
    out = np.zeros(4, np.float64)
    st = dg.dg_stats()
    assert dg.dg_pagerank(None, 0.85, 1e-6, 0, 1, 0, 10, dg._np_ptr(out), 0, C.byref(st), None) == \
        dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_sssp(None, 0, 0, 1, 10, dg._np_ptr(out), 0, C.byref(st), None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_graph_destroy(None) == dg.DG_OK
    assert dg.dg_graph_info_get(None, None) == dg.DG_ERR_INVALID_ARGUMENT


def test_allocator_hooks_must_pair(dg):
    alloc = dg.ALLOC_FN(lambda n, s, c: None)
    assert dg.lib.dg_set_allocator(alloc, dg.FREE_FN(), None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.lib.dg_set_allocator(dg.ALLOC_FN(), dg.FREE_FN(), None) == dg.DG_OK


def _descs(dg, graphs):
    keep, arr = [], (dg.dg_graph_desc * max(1, len(graphs)))()
    for i, (n, ptr, idx, w) in enumerate(graphs):
        ptr = np.ascontiguousarray(ptr, np.uint64)
        idx = np.ascontiguousarray(idx, np.uint32)
        w = None if w is None else np.ascontiguousarray(w, np.uint32)
        keep.append((ptr, idx, w))
        arr[i] = dg.dg_graph_desc(n, idx.shape[0], ptr.ctypes.data, idx.ctypes.data,
                                  None if w is None else w.ctypes.data)
    return arr, keep


GOOD = (3, [0, 1, 3, 3], [1, 0, 2], [5, 6, 7])


@pytest.mark.parametrize("case", ["empty", "n0", "ptr_end", "idx_range", "mixed_weights", "decreasing"])
def test_set_create_validation(dg, case):
    graphs = [GOOD, GOOD]
    if case == "n0":
        graphs = [GOOD, (0, [0], [], None)]
    elif case == "ptr_end":
        graphs = [GOOD, (3, [0, 1, 2, 2], [1, 0, 2], [1, 1, 1])]
    elif case == "idx_range":
        graphs = [GOOD, (3, [0, 1, 3, 3], [1, 0, 3], [1, 1, 1])]
    elif case == "mixed_weights":
        graphs = [GOOD, (3, [0, 1, 3, 3], [1, 0, 2], None)]
    elif case == "decreasing":
        graphs = [GOOD, (3, [0, 2, 1, 3], [1, 0, 2], [1, 1, 1])]
    arr, keep = _descs(dg, graphs)
    h = C.c_void_p()
    s = dg.dg_set_create(0 if case == "empty" else len(graphs), arr, None, None, C.byref(h))
    assert s == dg.DG_ERR_INVALID_ARGUMENT, dg.last_error()
    assert dg.last_error()
    assert not h.value


def test_set_valid_without_device(dg):
    import torch
    arr, keep = _descs(dg, [GOOD, (1, [0, 0], [], [])])
    h = C.c_void_p()
    s = dg.dg_set_create(2, arr, None, None, C.byref(h))
    if torch.cuda.is_available():
        assert s == dg.DG_OK
        dg.dg_set_destroy(h)
    else:
        assert s == dg.DG_ERR_DEVICE and "device" in dg.last_error()


def test_set_call_validation_null(dg):
    out = np.zeros(4, np.float64)
    st = dg.dg_stats()
    assert dg.dg_set_pagerank(None, 0.85, 1e-6, 0, 1, 0, 10, 0, dg._np_ptr(out), 0, None, C.byref(st), None) == \
        dg.DG_ERR_INVALID_ARGUMENT
    src = np.zeros(1, np.uint32)
    assert dg.dg_set_sssp(None, dg._np_ptr(src), 0, 1, 10, 0, dg._np_ptr(out), 0, None, C.byref(st), None) == \
        dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_set_destroy(None) == dg.DG_OK
    assert dg.dg_set_info_get(None, None) == dg.DG_ERR_INVALID_ARGUMENT


def test_topology_call_validation_null(dg):
    st = dg.dg_access_stats()
    assert dg.dg_access_matrix(None, 8, None, C.byref(st), None) == dg.DG_ERR_INVALID_ARGUMENT
    out = np.zeros(4, np.uint32)
    assert dg.dg_graph_partition(None, dg._np_ptr(out), None) == dg.DG_ERR_INVALID_ARGUMENT


def test_tune_call_validation_null(dg):
    t = dg.dg_tuning()
    assert dg.dg_tune(None, 0, 0, 1e-6, 0, 0, C.byref(t), None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_graph_repartition(None, 8, None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_graph_repartition_batch(None, dg.DG_ALGO_SSSP, 8, None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_graph_set_capture(None, 8) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_set_set_capture(None, 8) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_set_repartition(None, 8, None) == dg.DG_ERR_INVALID_ARGUMENT
    pr = dg.dg_prediction()
    assert dg.dg_predict_mode(None, C.byref(pr), None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_set_tune(None, 0, 0, 1e-6, None, 0, C.byref(t), None) == dg.DG_ERR_INVALID_ARGUMENT


def test_tune_cache_roundtrip(dg, tmp_path):
    """The tuning cache is host-only: save, clear and load a file, with a
    malformed line reported and skipped."""
    p = tmp_path / "tune.txt"
    dg.tune_cache_clear()
    dg.tune_cache_save(p)
    assert p.read_text().startswith("#")
    p.write_text("# comment\n"
                 "00000000deadbeef 0 0 1e-06 0 640 2 64 13 0.0065\n"
                 "00000000deadbee0 1 0 0 5 256 1 1 12 0.0043 3 16384\n"
                 "00000000deadbee1 0 1 1e-08 0 120 0 1 21 0.0004 3 4096 16\n"
                 "00000000deadbee2 0 1 1e-08 0 120 0 1 21 0.0004 3 4096 65\n"
                 "not a valid line\n")
    assert dg.dg_tune_cache_load(os.fsencode(str(p))) == dg.DG_ERR_INVALID_ARGUMENT
    assert "2 malformed" in dg.last_error()  # the text line, and a capture chunk beyond 64
    q = tmp_path / "again.txt"
    dg.tune_cache_save(q)
    lines = sorted(ln for ln in q.read_text().splitlines() if not ln.startswith("#"))
    assert len(lines) == 3 and lines[2].split()[:8] == ["00000000deadbeef", "0", "0", "9.9999999999999995e-07",
                                                        "0", "640", "2", "64"]
    # a line without the mapping columns loads with the automatic mapping and one launch per sweep; one with
    # them keeps them
    assert lines[2].split()[10:] == ["0", str(0xFFFFFFFF), "0"]
    assert lines[0].split()[10:] == ["3", "16384", "0"]
    assert lines[1].split()[10:] == ["3", "4096", "16"]
    dg.tune_cache_clear()
    dg.tune_cache_save(q)
    assert [ln for ln in q.read_text().splitlines() if not ln.startswith("#")] == []
    assert dg.dg_tune_cache_load(b"/nonexistent/dir/x") == dg.DG_ERR_INVALID_ARGUMENT


def test_server_call_validation_null(dg):
    h = C.c_void_p()
    opts = dg.dg_server_opts(0, 0, dg.DG_ASYNC, 64, 0.85, 1e-6, dg.DG_F32)
    assert dg.dg_server_create(None, 1, C.byref(opts), None, C.byref(h)) == dg.DG_ERR_INVALID_ARGUMENT
    rid = C.c_uint64()
    assert dg.dg_server_submit(None, 0, 0, 0, C.byref(rid)) == dg.DG_ERR_INVALID_ARGUMENT
    cnt = C.c_uint32()
    assert dg.dg_server_step(None, None, 0, C.byref(cnt)) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_server_fetch(None, 1, None, 0, None) == dg.DG_ERR_INVALID_ARGUMENT
    assert dg.dg_server_destroy(None) == dg.DG_OK


@pytest.mark.parametrize("args", [(1000, 0, 256, 4), (3 << 20, 0, 256, 4), (1 << 33, 0, 256, 4), (1 << 20, 2, 256, 4),
                                  (1 << 20, 0, 0, 4), (1 << 20, 0, 17, 4), (1 << 20, 0, 256, 0),
                                  (1 << 20, 0, 4096, 65536)])
def test_probe_gather_validation(dg, args):
    sec = C.c_double(-1.0)
    assert dg.dg_probe_gather(*args, C.byref(sec), None) == dg.DG_ERR_INVALID_ARGUMENT
    assert sec.value == -1.0 and dg.last_error()
