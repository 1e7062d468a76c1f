"""Python binding of the C ABI in include/dg.h (argument marshalling only).

The ``dg_*`` functions are the C entry points (every symbol of the header,
listed in ``EXPORTS``), loaded with ctypes from the in-tree ``libdg.so``.  Every step of a sweep runs in the HIP
library; PyTorch only provides device memory (its caching allocator is
registered as the library's allocator) and the stream.

``Graph`` wraps a graph handle and ``GraphSet`` a set handle, with keyword
defaults.  If the library is missing,
importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DG_LIBRARY names another build of the same library (the host-sanitizer
# build the CPU tests use); by default the in-tree libdg.so.
LIB_PATH = os.environ.get("DG_LIBRARY") or os.path.join(_HERE, "libdg.so")

DG_OK, DG_ERR_INVALID_ARGUMENT, DG_ERR_OUT_OF_MEMORY, DG_ERR_DEVICE, DG_ERR_NOT_CONVERGED, DG_ERR_UNSUPPORTED = range(6)
DG_SYNC, DG_ASYNC, DG_DELAYED, DG_DELAYED_LOCAL = 0, 1, 2, 3
DG_CSR, DG_CSC = 0, 1
DG_F32, DG_F64 = 0, 1
DG_D_WHOLE = 0xFFFFFFFF
DG_INF_DIST = 0xFFFFFFFF

MODES = {"sync": DG_SYNC, "async": DG_ASYNC, "delayed": DG_DELAYED, "delayed_local": DG_DELAYED_LOCAL}
DTYPES = {"f32": DG_F32, "f64": DG_F64}

# Every symbol declared in include/dg.h.
EXPORTS = ("dg_set_allocator", "dg_graph_create", "dg_graph_destroy", "dg_graph_info_get", "dg_pagerank", "dg_ppr",
           "dg_error_bound",
           "dg_sssp", "dg_sssp_batch", "dg_ppr_batch", "dg_set_create", "dg_set_destroy", "dg_set_info_get",
           "dg_set_pagerank", "dg_set_sssp", "dg_graph_partition", "dg_access_matrix", "dg_graph_repartition",
           "dg_graph_repartition_batch",
           "dg_tune", "dg_tune_batch", "dg_graph_set_mapping", "dg_graph_set_capture", "dg_set_set_capture",
           "dg_set_repartition", "dg_set_tune", "dg_predict_mode",
           "dg_tune_cache_clear", "dg_tune_cache_save", "dg_tune_cache_load", "dg_server_create",
           "dg_server_destroy", "dg_server_submit", "dg_server_step", "dg_server_fetch", "dg_server_status_get",
           "dg_plan_create", "dg_plan_info_get", "dg_plan_arrays", "dg_plan_batch_tiles", "dg_plan_destroy", "dg_probe_gather", "dg_sssp_noalloc",
           "dg_status_str", "dg_last_error", "dg_version")
DG_NOALLOC_SCRATCH_BYTES = 100663296
DG_QUERY_SSSP, DG_QUERY_PPR = 0, 1
QUERIES = {"sssp": DG_QUERY_SSSP, "ppr": DG_QUERY_PPR}
DG_ALGO_PAGERANK, DG_ALGO_SSSP = 0, 1
DG_TUNE_NO_CACHE, DG_TUNE_KEEP_WORKERS = 1, 2
MODE_NAMES = {0: "sync", 1: "async", 2: "delayed"}


class dg_stats(C.Structure):
    _fields_ = [("sweeps", C.c_uint32), ("workers", C.c_uint32), ("tile_vertices", C.c_uint32),
                ("commit_interval", C.c_uint32), ("residual", C.c_double), ("seconds", C.c_double),
                ("edges_traversed", C.c_uint64), ("err_bound", C.c_double), ("request", C.c_uint32),
                ("commits", C.c_uint32)]


DG_STATS_ERR_BOUND = 1


class dg_graph_info(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint64), ("workers", C.c_uint32), ("tiles", C.c_uint32),
                ("max_in_degree", C.c_uint32), ("dangling", C.c_uint32), ("has_weights", C.c_uint32),
                ("compute_units", C.c_uint32), ("hot_vertices", C.c_uint32), ("hot_edges", C.c_uint64),
                ("resident_vertices", C.c_uint32), ("resident_edges", C.c_uint64), ("weight_bytes", C.c_uint32),
                ("device_bytes", C.c_uint64), ("sweep_variant", C.c_uint32), ("batch_tiles", C.c_uint32)]


class dg_plan_info(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint64), ("workers", C.c_uint32), ("tiles", C.c_uint32),
                ("max_in_degree", C.c_uint32), ("dangling", C.c_uint32), ("hot_vertices", C.c_uint32),
                ("hot_edges", C.c_uint64), ("resident_vertices", C.c_uint32), ("resident_edges", C.c_uint64),
                ("weight_bytes", C.c_uint32), ("content_hash", C.c_uint64), ("sweep_variant", C.c_uint32),
                ("batch_tiles", C.c_uint32), ("batch_workers_sssp", C.c_uint32), ("batch_workers_ppr", C.c_uint32)]


class dg_graph_opts(C.Structure):
    _fields_ = [("workers", C.c_uint32), ("hot_vertices", C.c_uint32), ("resident_vertices", C.c_uint32),
                ("sweep_variant", C.c_uint32), ("arrays_on_device", C.c_uint32)]


DG_HOT_AUTO = 0xFFFFFFFF
DG_RESIDENT_AUTO = 0xFFFFFFFF
DG_SWEEP_AUTO, DG_SWEEP_WIDE, DG_SWEEP_WIDE_INFLIGHT, DG_SWEEP_NARROW = 0, 1, 2, 3
SWEEP_VARIANTS = {"auto": DG_SWEEP_AUTO, "wide": DG_SWEEP_WIDE, "wide_inflight": DG_SWEEP_WIDE_INFLIGHT,
                  "narrow": DG_SWEEP_NARROW}


class dg_graph_desc(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint64), ("ptr", C.c_void_p), ("idx", C.c_void_p),
                ("w", C.c_void_p)]


class dg_access_stats(C.Structure):
    _fields_ = [("reads", C.c_uint64), ("same_worker", C.c_uint64), ("diagonal", C.c_uint64),
                ("groups", C.c_uint32), ("workers", C.c_uint32), ("self_share", C.c_double),
                ("diagonal_share", C.c_double), ("uniform_diagonal", C.c_double)]


class dg_prediction(C.Structure):
    _fields_ = [("mode", C.c_int), ("d", C.c_uint32), ("groups", C.c_uint32), ("reserved", C.c_uint32),
                ("diagonal_share", C.c_double), ("uniform_diagonal", C.c_double), ("lift", C.c_double),
                ("self_share", C.c_double)]


class dg_tuning(C.Structure):
    _fields_ = [("workers", C.c_uint32), ("mode", C.c_int), ("d", C.c_uint32), ("sweeps", C.c_uint32),
                ("seconds", C.c_double), ("predicted_seconds", C.c_double), ("candidates", C.c_uint32),
                ("from_cache", C.c_uint32), ("graph_hash", C.c_uint64), ("sweep_variant", C.c_uint32),
                ("resident_vertices", C.c_uint32), ("repeats", C.c_uint32), ("capture_chunk", C.c_uint32),
                ("seconds_min", C.c_double), ("seconds_max", C.c_double), ("default_seconds", C.c_double),
                ("default_seconds_min", C.c_double), ("default_seconds_max", C.c_double)]


class dg_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_batches", C.c_uint32), ("mode", C.c_int), ("d", C.c_uint32),
                ("damping", C.c_double), ("tol", C.c_double), ("dtype", C.c_int)]


class dg_request_info(C.Structure):
    _fields_ = [("graph", C.c_uint32), ("kind", C.c_int), ("source", C.c_uint32), ("sweeps", C.c_uint32),
                ("state", C.c_uint32), ("submit_step", C.c_uint64), ("admit_step", C.c_uint64),
                ("finish_step", C.c_uint64)]


class dg_server_status(C.Structure):
    _fields_ = [("queued", C.c_uint32), ("running", C.c_uint32), ("finished", C.c_uint32), ("batches", C.c_uint32),
                ("state_bytes", C.c_uint64), ("steps", C.c_uint64)]


class dg_set_opts(C.Structure):
    _fields_ = [("workers", C.c_uint32)]


class dg_set_info(C.Structure):
    _fields_ = [("graphs", C.c_uint32), ("n", C.c_uint64), ("m", C.c_uint64), ("tiles", C.c_uint32),
                ("workers", C.c_uint32), ("has_weights", C.c_uint32), ("device_bytes", C.c_uint64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2110_01409_amd.build` "
                          "(or __graft_entry__.build()) first")
    # PyTorch first: the library then binds to the HIP runtime PyTorch loaded
    # (its libamdhip64 satisfies the library's dependency), so device
    # pointers and streams from torch are valid in the library.  Loaded the
    # other way round, the process holds two HIP runtimes and the library
    # finds no device.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "dg_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, P]),
        "dg_graph_create": (C.c_int, [C.c_uint32, C.c_uint64, C.c_int, P, P, P, C.POINTER(dg_graph_opts), P,
                                      C.POINTER(C.c_void_p)]),
        "dg_graph_destroy": (C.c_int, [P]),
        "dg_plan_create": (C.c_int, [C.c_uint32, C.c_uint64, C.c_int, P, P, P, C.POINTER(dg_graph_opts), C.c_uint32,
                                     C.POINTER(C.c_void_p)]),
        "dg_plan_info_get": (C.c_int, [P, C.POINTER(dg_plan_info)]),
        "dg_plan_arrays": (C.c_int, [P, P, P, P, P, P, P]),
        "dg_plan_batch_tiles": (C.c_int, [P, P, P, P]),
        "dg_plan_destroy": (C.c_int, [P]),
        "dg_graph_info_get": (C.c_int, [P, C.POINTER(dg_graph_info)]),
        "dg_pagerank": (C.c_int, [P, C.c_double, C.c_double, C.c_int, C.c_uint32, C.c_int, C.c_uint32, P, C.c_int,
                                  C.POINTER(dg_stats), P]),
        "dg_ppr": (C.c_int, [P, C.c_uint32, C.c_double, C.c_double, C.c_int, C.c_uint32, C.c_int, C.c_uint32, P,
                             C.c_int, C.POINTER(dg_stats), P]),
        "dg_error_bound": (C.c_int, [P, C.c_double, C.c_uint32, P, C.c_int, C.POINTER(C.c_double), P]),
        "dg_sssp": (C.c_int, [P, C.c_uint32, C.c_int, C.c_uint32, C.c_uint32, P, C.c_int, C.POINTER(dg_stats), P]),
        "dg_sssp_noalloc": (C.c_int, [P, C.c_uint32, C.c_int, C.c_uint32, C.c_uint32, P, C.c_int,
                                      C.POINTER(dg_stats), P]),
        "dg_sssp_batch": (C.c_int, [P, P, C.c_uint32, C.c_int, C.c_uint32, C.c_uint32, P, C.c_int,
                                    C.POINTER(dg_stats), P]),
        "dg_ppr_batch": (C.c_int, [P, P, C.c_uint32, C.c_double, C.c_double, C.c_int, C.c_uint32, C.c_int, C.c_uint32, P,
                                   C.c_int, C.POINTER(dg_stats), P]),
        "dg_set_create": (C.c_int, [C.c_uint32, P, C.POINTER(dg_set_opts), P, C.POINTER(C.c_void_p)]),
        "dg_set_destroy": (C.c_int, [P]),
        "dg_set_info_get": (C.c_int, [P, C.POINTER(dg_set_info)]),
        "dg_set_pagerank": (C.c_int, [P, C.c_double, C.c_double, C.c_int, C.c_uint32, C.c_int, C.c_uint32,
                                      C.c_uint32, P, C.c_int, P, C.POINTER(dg_stats), P]),
        "dg_set_sssp": (C.c_int, [P, P, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, P, C.c_int, P,
                                  C.POINTER(dg_stats), P]),
        "dg_graph_partition": (C.c_int, [P, P, P]),
        "dg_access_matrix": (C.c_int, [P, C.c_uint32, P, C.POINTER(dg_access_stats), P]),
        "dg_graph_repartition": (C.c_int, [P, C.c_uint32, P]),
        "dg_graph_repartition_batch": (C.c_int, [P, C.c_int, C.c_uint32, P]),
        "dg_tune": (C.c_int, [P, C.c_int, C.c_int, C.c_double, C.c_uint32, C.c_uint32, C.POINTER(dg_tuning), P]),
        "dg_tune_batch": (C.c_int, [P, C.c_int, C.c_int, C.c_double, P, C.c_uint32, C.c_uint32,
                                    C.POINTER(dg_tuning), P]),
        "dg_graph_set_mapping": (C.c_int, [P, C.c_uint32, C.c_uint32, C.c_uint32, P]),
        "dg_graph_set_capture": (C.c_int, [P, C.c_uint32]),
        "dg_set_set_capture": (C.c_int, [P, C.c_uint32]),
        "dg_set_repartition": (C.c_int, [P, C.c_uint32, P]),
        "dg_set_tune": (C.c_int, [P, C.c_int, C.c_int, C.c_double, P, C.c_uint32, C.POINTER(dg_tuning), P]),
        "dg_predict_mode": (C.c_int, [P, C.POINTER(dg_prediction), P]),
        "dg_tune_cache_clear": (C.c_int, []),
        "dg_tune_cache_save": (C.c_int, [C.c_char_p]),
        "dg_tune_cache_load": (C.c_int, [C.c_char_p]),
        "dg_server_create": (C.c_int, [P, C.c_uint32, C.POINTER(dg_server_opts), P, C.POINTER(C.c_void_p)]),
        "dg_server_destroy": (C.c_int, [P]),
        "dg_server_submit": (C.c_int, [P, C.c_uint32, C.c_int, C.c_uint32, C.POINTER(C.c_uint64)]),
        "dg_server_step": (C.c_int, [P, P, C.c_uint32, C.POINTER(C.c_uint32)]),
        "dg_server_fetch": (C.c_int, [P, C.c_uint64, P, C.c_int, C.POINTER(dg_request_info)]),
        "dg_server_status_get": (C.c_int, [P, C.POINTER(dg_server_status)]),
        "dg_probe_gather": (C.c_int, [C.c_uint64, C.c_int, C.c_uint32, C.c_uint32, C.POINTER(C.c_double), P]),
        "dg_status_str": (C.c_char_p, [C.c_int]),
        "dg_last_error": (C.c_char_p, []),
        "dg_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_str(s: int) -> str:
    return lib.dg_status_str(s).decode()


def last_error() -> str:
    return lib.dg_last_error().decode()


def version() -> str:
    return lib.dg_version().decode()


# Thin same-name wrappers of the C entry points.
def dg_set_allocator(alloc, free_fn, ctx=None):
    return lib.dg_set_allocator(alloc, free_fn, ctx)


def dg_graph_create(n, m, layout, ptr, idx, w, opts, stream, out):
    return lib.dg_graph_create(n, m, layout, ptr, idx, w, opts, stream, out)


def dg_graph_destroy(g):
    return lib.dg_graph_destroy(g)


def dg_plan_create(n, m, layout, ptr, idx, w, opts, compute_units, out):
    return lib.dg_plan_create(n, m, layout, ptr, idx, w, opts, compute_units, out)


def dg_plan_info_get(p, info):
    return lib.dg_plan_info_get(p, info)


def dg_plan_arrays(p, in_ptr, in_src, in_w, cpos, tile_v, work_t):
    return lib.dg_plan_arrays(p, in_ptr, in_src, in_w, cpos, tile_v, work_t)


def dg_plan_batch_tiles(p, btile_v, work_sssp, work_ppr):
    return lib.dg_plan_batch_tiles(p, btile_v, work_sssp, work_ppr)


def dg_plan_destroy(p):
    return lib.dg_plan_destroy(p)


def dg_graph_info_get(g, info):
    return lib.dg_graph_info_get(g, info)


def dg_pagerank(g, damping, tol, mode, d, dtype, max_sweeps, out, out_on_device, stats, stream):
    return lib.dg_pagerank(g, damping, tol, mode, d, dtype, max_sweeps, out, out_on_device, stats, stream)


DG_NO_RESTART = 0xFFFFFFFF


def dg_error_bound(g, damping, restart, scores, scores_on_device, out_bound, stream):
    return lib.dg_error_bound(g, damping, restart, scores, scores_on_device, out_bound, stream)


def dg_ppr(g, src, damping, tol, mode, d, dtype, max_sweeps, out, out_on_device, stats, stream):
    return lib.dg_ppr(g, src, damping, tol, mode, d, dtype, max_sweeps, out, out_on_device, stats, stream)


def dg_sssp(g, src, mode, d, max_sweeps, out, out_on_device, stats, stream):
    return lib.dg_sssp(g, src, mode, d, max_sweeps, out, out_on_device, stats, stream)


def dg_sssp_noalloc(g, src, mode, d, max_sweeps, out, out_on_device, stats, stream):
    return lib.dg_sssp_noalloc(g, src, mode, d, max_sweeps, out, out_on_device, stats, stream)


def dg_sssp_batch(g, sources, k, mode, d, max_sweeps, out, out_on_device, stats, stream):
    return lib.dg_sssp_batch(g, sources, k, mode, d, max_sweeps, out, out_on_device, stats, stream)


def dg_ppr_batch(g, sources, k, damping, tol, mode, d, dtype, max_sweeps, out, out_on_device, stats, stream):
    return lib.dg_ppr_batch(g, sources, k, damping, tol, mode, d, dtype, max_sweeps, out, out_on_device, stats,
                            stream)


def dg_set_create(count, graphs, opts, stream, out):
    return lib.dg_set_create(count, graphs, opts, stream, out)


def dg_set_destroy(s):
    return lib.dg_set_destroy(s)


def dg_set_info_get(s, info):
    return lib.dg_set_info_get(s, info)


def dg_set_pagerank(s, damping, tol, mode, d, dtype, max_sweeps, flags, out, out_on_device, out_sweeps, stats,
                    stream):
    return lib.dg_set_pagerank(s, damping, tol, mode, d, dtype, max_sweeps, flags, out, out_on_device, out_sweeps,
                               stats, stream)


def dg_set_sssp(s, sources, mode, d, max_sweeps, flags, out, out_on_device, out_sweeps, stats, stream):
    return lib.dg_set_sssp(s, sources, mode, d, max_sweeps, flags, out, out_on_device, out_sweeps, stats, stream)


def dg_graph_partition(g, out_first_vertex, stream):
    return lib.dg_graph_partition(g, out_first_vertex, stream)


def dg_access_matrix(g, groups, out_counts, stats, stream):
    return lib.dg_access_matrix(g, groups, out_counts, stats, stream)


def dg_graph_repartition(g, workers, stream):
    return lib.dg_graph_repartition(g, workers, stream)


def dg_graph_repartition_batch(g, algo, workers, stream):
    return lib.dg_graph_repartition_batch(g, algo, workers, stream)


def dg_tune(g, algo, dtype, tol, src, flags, out, stream):
    return lib.dg_tune(g, algo, dtype, tol, src, flags, out, stream)


def dg_tune_cache_clear():
    return lib.dg_tune_cache_clear()


def dg_tune_cache_save(path):
    return lib.dg_tune_cache_save(path)


def dg_tune_cache_load(path):
    return lib.dg_tune_cache_load(path)


def dg_server_create(graphs, count, opts, stream, out):
    return lib.dg_server_create(graphs, count, opts, stream, out)


def dg_server_destroy(srv):
    return lib.dg_server_destroy(srv)


def dg_server_submit(srv, graph, kind, source, out_id):
    return lib.dg_server_submit(srv, graph, kind, source, out_id)


def dg_server_step(srv, out_finished, cap, out_count):
    return lib.dg_server_step(srv, out_finished, cap, out_count)


def dg_server_fetch(srv, rid, out, out_on_device, info):
    return lib.dg_server_fetch(srv, rid, out, out_on_device, info)


def dg_server_status_get(srv, status):
    return lib.dg_server_status_get(srv, status)


def dg_probe_gather(table_bytes, streamed, per_thread, workgroups, out_seconds, stream):
    return lib.dg_probe_gather(table_bytes, streamed, per_thread, workgroups, out_seconds, stream)


def probe_gather(table_bytes, streamed=False, per_thread=256, workgroups=1024, stream=None):
    """Seconds of one launch of workgroups x 256 x per_thread random 4-byte
    loads from a table of table_bytes (best of three), and the load count."""
    sec = C.c_double()
    _check(dg_probe_gather(int(table_bytes), 1 if streamed else 0, int(per_thread), int(workgroups), C.byref(sec),
                           _stream_handle(stream)))
    return sec.value, int(workgroups) * 256 * int(per_thread)


def dg_tune_batch(g, algo, dtype, tol, sources, k, flags, out, stream):
    return lib.dg_tune_batch(g, algo, dtype, tol, sources, k, flags, out, stream)


def dg_graph_set_mapping(g, variant, resident, workers, stream):
    return lib.dg_graph_set_mapping(g, variant, resident, workers, stream)


def dg_graph_set_capture(g, chunk_sweeps):
    return lib.dg_graph_set_capture(g, chunk_sweeps)


def dg_set_set_capture(s, chunk_sweeps):
    return lib.dg_set_set_capture(s, chunk_sweeps)


def dg_predict_mode(g, out, stream):
    return lib.dg_predict_mode(g, out, stream)


def dg_set_repartition(s, workers, stream):
    return lib.dg_set_repartition(s, workers, stream)


def dg_set_tune(s, algo, dtype, tol, sources, flags, out, stream):
    return lib.dg_set_tune(s, algo, dtype, tol, sources, flags, out, stream)


def tune_cache_save(path):
    _check(dg_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path):
    _check(dg_tune_cache_load(os.fsencode(path)))


def tune_cache_clear():
    _check(dg_tune_cache_clear())


def _check(status, allow=()):
    if status != DG_OK and status not in allow:
        raise DGError(status, last_error())
    return status


# ------------------------------------------------------ torch as allocator --

_torch_hooks = None


def plan(n, ptr, idx, w=None, layout="csr", compute_units=256, workers=0, hot_vertices=DG_HOT_AUTO,
         resident_vertices=DG_RESIDENT_AUTO, sweep_variant="auto"):
    """The layout dg_graph_create would upload, built on the host only
    (dg_plan_*): a dict of the plan's facts and its arrays as numpy arrays
    (in_ptr, in_src, in_w or None, cpos, tile_v, work_t; btile_v, the tiles
    of the batched calls, and work_sssp / work_ppr, their default batched
    partitions)."""
    ptr = np.ascontiguousarray(ptr, dtype=np.uint64)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    wa = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
    opts = dg_graph_opts(int(workers), int(hot_vertices), int(resident_vertices), SWEEP_VARIANTS[sweep_variant])
    h = C.c_void_p()
    _check(dg_plan_create(int(n), int(idx.shape[0]), DG_CSR if layout == "csr" else DG_CSC, _np_ptr(ptr),
                          _np_ptr(idx), None if wa is None else _np_ptr(wa), C.byref(opts), int(compute_units),
                          C.byref(h)))
    try:
        info = dg_plan_info()
        _check(dg_plan_info_get(h, C.byref(info)))
        out = {f: getattr(info, f) for f, _ in dg_plan_info._fields_}
        arr = {"in_ptr": np.empty(info.n + 1, np.uint32), "in_src": np.empty(info.m, np.uint32),
               "in_w": np.empty(info.m, np.uint32) if wa is not None else None,
               "cpos": np.empty(info.n, np.uint32), "tile_v": np.empty(info.tiles + 1, np.uint32),
               "work_t": np.empty(info.workers + 1, np.uint32)}
        _check(dg_plan_arrays(h, *[None if a is None else _np_ptr(a) for a in arr.values()]))
        arr["btile_v"] = np.empty(info.batch_tiles + 1, np.uint32)
        arr["work_sssp"] = np.empty(info.batch_workers_sssp + 1, np.uint32)
        arr["work_ppr"] = np.empty(info.batch_workers_ppr + 1, np.uint32)
        _check(dg_plan_batch_tiles(h, _np_ptr(arr["btile_v"]), _np_ptr(arr["work_sssp"]), _np_ptr(arr["work_ppr"])))
        out.update(arr)
        return out
    finally:
        dg_plan_destroy(h)


def use_torch_allocator():
    """Route the library's device allocations through torch's caching
    allocator (idempotent)."""
    global _torch_hooks
    if _torch_hooks is not None:
        return
    import torch

    def _alloc(nbytes, stream, ctx):
        try:
            dev = torch.cuda.current_device()
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:  # the library reports DG_ERR_OUT_OF_MEMORY
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
    _check(lib.dg_set_allocator(hooks[0], hooks[1], None))
    _torch_hooks = hooks


def _stream_handle(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _is_device_tensor(a):
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


@dataclasses.dataclass
class Stats:
    sweeps: int
    workers: int
    tile_vertices: int
    commit_interval: int
    residual: float
    seconds: float
    edges_traversed: int
    converged: bool
    err_bound: float = 0.0
    commits: int = 0

    @property
    def gteps(self) -> float:
        return self.edges_traversed / self.seconds / 1e9 if self.seconds > 0 else float("nan")


def _stats(s: dg_stats, converged: bool) -> Stats:
    return Stats(s.sweeps, s.workers, s.tile_vertices, s.commit_interval, s.residual, s.seconds,
                 s.edges_traversed, converged, s.err_bound, s.commits)


VARIANT_NAMES = {1: "wide", 2: "wide_inflight", 3: "narrow"}


def _tuning(t):
    return {"workers": t.workers, "mode": MODE_NAMES[t.mode], "d": t.d, "sweeps": t.sweeps,
            "seconds": t.seconds, "seconds_min": t.seconds_min, "seconds_max": t.seconds_max,
            "predicted_seconds": t.predicted_seconds, "candidates": t.candidates,
            "from_cache": bool(t.from_cache), "graph_hash": t.graph_hash,
            "sweep_variant": VARIANT_NAMES.get(t.sweep_variant, "auto"),
            "resident_vertices": t.resident_vertices, "repeats": t.repeats, "capture_chunk": t.capture_chunk,
            "default_seconds": t.default_seconds, "default_seconds_min": t.default_seconds_min,
            "default_seconds_max": t.default_seconds_max}


class Graph:
    """A graph resident in device memory.

    ``Graph(n, ptr, idx, w=None, layout="csr")`` copies host arrays (ptr
    uint64[n+1], idx uint32[m], w uint32[m] or None) to the device and builds
    the in-edge form.  ``Graph.from_csr(g)`` takes a ``graphgen.CSRGraph``.
    The keyword options are those of dg_graph_opts: ``workers``,
    ``hot_vertices``, ``resident_vertices`` and ``sweep_variant`` ("auto",
    "wide", "wide_inflight" or "narrow"); ``info().sweep_variant`` reports
    the variant in use.
    """

    def __init__(self, n, ptr, idx, w=None, layout="csr", stream=None, torch_allocator=True, workers=0,
                 hot_vertices=DG_HOT_AUTO, resident_vertices=DG_RESIDENT_AUTO, sweep_variant="auto"):
        dev = _is_device_tensor(ptr)
        if dev:
            # device arrays (torch tensors of the required dtypes, contiguous)
            import torch
            for a, want in ((ptr, torch.uint64), (idx, torch.uint32), (w, torch.uint32)):
                if a is not None and (not _is_device_tensor(a) or a.dtype != want or not a.is_contiguous()):
                    raise TypeError("device input needs contiguous device tensors: ptr uint64, idx and w uint32")
            pp, ip = C.c_void_p(ptr.data_ptr()), C.c_void_p(idx.data_ptr())
            wp = None if w is None else C.c_void_p(w.data_ptr())
            m = int(idx.shape[0])
        else:
            ptr = np.ascontiguousarray(ptr, dtype=np.uint64)
            idx = np.ascontiguousarray(idx, dtype=np.uint32)
            wa = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
            pp, ip, wp = _np_ptr(ptr), _np_ptr(idx), None if wa is None else _np_ptr(wa)
            m = int(idx.shape[0])
        if torch_allocator:
            use_torch_allocator()
        h = C.c_void_p()
        lay = DG_CSR if layout == "csr" else DG_CSC
        opts = dg_graph_opts(int(workers), int(hot_vertices), int(resident_vertices), SWEEP_VARIANTS[sweep_variant],
                             1 if dev else 0)
        _check(dg_graph_create(int(n), m, lay, pp, ip, wp, C.byref(opts), _stream_handle(stream), C.byref(h)))
        self._h = h
        self.n = int(n)
        self.m = m
        self._dependents = []  # objects holding device state allocated through this graph

    @classmethod
    def from_csr(cls, g, **kw):
        return cls(g.n, g.ptr, g.idx, g.w, layout="csr", **kw)

    def info(self) -> dg_graph_info:
        inf = dg_graph_info()
        _check(dg_graph_info_get(self._h, C.byref(inf)))
        return inf

    def pagerank(self, damping=0.85, tol=1e-6, mode="delayed", d=64, dtype="f32", max_sweeps=10_000,
                 out=None, stream=None, allow_not_converged=False, err_bound=False):
        """Returns (scores float64 tensor on the device, Stats); with
        err_bound=True, Stats.err_bound holds the device-computed certificate
        ||T(x) - x||_1 / (1 - damping)."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        st = dg_stats()
        st.request = DG_STATS_ERR_BOUND if err_bound else 0
        s = _check(dg_pagerank(self._h, float(damping), float(tol), MODES[mode], int(d), DTYPES[dtype],
                               int(max_sweeps), C.c_void_p(out.data_ptr()), 1, C.byref(st),
                               _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, _stats(st, s == DG_OK)

    def error_bound(self, scores, restart=None, damping=0.85, stream=None):
        """dg_error_bound of a float64 score vector (device tensor or numpy
        array): an upper bound on its L1 distance to the fixed point of
        PageRank, or of personalised PageRank with this restart vertex."""
        b = C.c_double()
        rs = DG_NO_RESTART if restart is None else int(restart)
        if _is_device_tensor(scores):
            import torch
            assert scores.dtype == torch.float64 and scores.is_contiguous() and scores.numel() == self.n
            _check(dg_error_bound(self._h, float(damping), rs, C.c_void_p(scores.data_ptr()), 1, C.byref(b),
                                  _stream_handle(stream)))
        else:
            a = np.ascontiguousarray(scores, dtype=np.float64)
            assert a.size == self.n
            _check(dg_error_bound(self._h, float(damping), rs, _np_ptr(a), 0, C.byref(b), _stream_handle(stream)))
        return b.value

    def ppr(self, src, damping=0.85, tol=1e-6, mode="delayed", d=64, dtype="f32", max_sweeps=10_000, out=None,
            stream=None, allow_not_converged=False, err_bound=False):
        """Personalised PageRank of restart vertex src (dg_ppr): float64
        scores on the device, Stats."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        st = dg_stats()
        st.request = DG_STATS_ERR_BOUND if err_bound else 0
        s = _check(dg_ppr(self._h, int(src), float(damping), float(tol), MODES[mode], int(d), DTYPES[dtype],
                          int(max_sweeps), C.c_void_p(out.data_ptr()), 1, C.byref(st), _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, _stats(st, s == DG_OK)

    def sssp(self, src, mode="delayed", d=64, max_sweeps=None, out=None, stream=None, allow_not_converged=False):
        """Returns (distances uint32 tensor on the device, Stats)."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.uint32, device="cuda")
        if max_sweeps is None:
            max_sweeps = min(self.n + 1, 1_000_000)
        st = dg_stats()
        s = _check(dg_sssp(self._h, int(src), MODES[mode], int(d), int(max_sweeps), C.c_void_p(out.data_ptr()), 1,
                           C.byref(st), _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, _stats(st, s == DG_OK)

    def sssp_noalloc(self, src, mode="delayed", d=64, max_sweeps=None, out=None, stream=None,
                     allow_not_converged=False):
        """dg_sssp_noalloc: as sssp, with no allocation inside the call (the
        library's fixed scratch array).  ``out`` (uint32 [n], device) is
        allocated here when not given, before the call."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.uint32, device="cuda")
        if max_sweeps is None:
            max_sweeps = min(self.n + 1, 65535)
        st = dg_stats()
        s = _check(dg_sssp_noalloc(self._h, int(src), MODES[mode], int(d), int(max_sweeps),
                                   C.c_void_p(out.data_ptr()), 1, C.byref(st), _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, _stats(st, s == DG_OK)

    def sssp_batch(self, sources, mode="delayed", d=64, max_sweeps=None, out=None, stream=None,
                   allow_not_converged=False):
        """Distances from every source: uint32 tensor [k, n] on the device, Stats."""
        import torch
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        k = int(src.shape[0])
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.uint32, device="cuda")
        if max_sweeps is None:
            max_sweeps = min(self.n + 1, 100_000)
        st = dg_stats()
        s = _check(dg_sssp_batch(self._h, _np_ptr(src), k, MODES[mode], int(d), int(max_sweeps),
                                 C.c_void_p(out.data_ptr()), 1, C.byref(st), _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, _stats(st, s == DG_OK)

    def ppr_batch(self, sources, damping=0.85, tol=1e-6, mode="delayed", d=64, dtype="f32", max_sweeps=10_000,
                  out=None, stream=None, allow_not_converged=False):
        """Personalised PageRank per restart vertex: float64 tensor [k, n], Stats."""
        import torch
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        k = int(src.shape[0])
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.float64, device="cuda")
        st = dg_stats()
        s = _check(dg_ppr_batch(self._h, _np_ptr(src), k, float(damping), float(tol), MODES[mode], int(d),
                                DTYPES[dtype], int(max_sweeps), C.c_void_p(out.data_ptr()), 1, C.byref(st),
                                _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, _stats(st, s == DG_OK)

    def repartition(self, workers=0, stream=None):
        """Rebuild the blocked partition over `workers` workers (0 = default)."""
        _check(dg_graph_repartition(self._h, int(workers), _stream_handle(stream)))

    def repartition_batch(self, algo, workers=0, stream=None):
        """Rebuild the batched partition of algo ("sssp" or "ppr") over
        `workers` workgroups per batch (0 = default)."""
        _check(dg_graph_repartition_batch(self._h, DG_ALGO_SSSP if algo == "sssp" else DG_ALGO_PAGERANK, int(workers),
                                          _stream_handle(stream)))

    def tune(self, algo="pagerank", dtype="f32", tol=1e-6, src=0, use_cache=True, keep_workers=False, stream=None):
        """Choose workers, mode and d (the graph keeps the chosen partition).
        Returns a dict with the choice and its measured time."""
        t = dg_tuning()
        flags = (0 if use_cache else DG_TUNE_NO_CACHE) | (DG_TUNE_KEEP_WORKERS if keep_workers else 0)
        _check(dg_tune(self._h, DG_ALGO_PAGERANK if algo == "pagerank" else DG_ALGO_SSSP, DTYPES[dtype],
                       float(tol), int(src), flags, C.byref(t), _stream_handle(stream)))
        return _tuning(t)

    def tune_batch(self, algo, sources, dtype="f32", tol=1e-6, stream=None):
        """dg_tune_batch on a sample of sources ("sssp" or "ppr"); the graph
        keeps the chosen batched partition.  Returns the choice as a dict."""
        t = dg_tuning()
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        _check(dg_tune_batch(self._h, DG_ALGO_PAGERANK if algo == "ppr" else DG_ALGO_SSSP, DTYPES[dtype], float(tol),
                             _np_ptr(src), int(src.shape[0]), 0, C.byref(t), _stream_handle(stream)))
        return _tuning(t)

    def set_mapping(self, sweep_variant="auto", resident_vertices=DG_RESIDENT_AUTO, workers=0, stream=None):
        """dg_graph_set_mapping: sweep variant, resident-table limit, workers."""
        _check(dg_graph_set_mapping(self._h, SWEEP_VARIANTS[sweep_variant], int(resident_vertices), int(workers),
                                    _stream_handle(stream)))

    def set_capture(self, chunk_sweeps):
        """dg_graph_set_capture: replay recorded chunks of this many sweeps
        (0: launch every sweep on its own)."""
        _check(dg_graph_set_capture(self._h, int(chunk_sweeps)))

    def predict_mode(self, stream=None):
        """dg_predict_mode: the commit mode the access matrix suggests, as a dict."""
        p = dg_prediction()
        _check(dg_predict_mode(self._h, C.byref(p), _stream_handle(stream)))
        return {"mode": MODE_NAMES[p.mode], "d": p.d, "groups": p.groups, "diagonal_share": p.diagonal_share,
                "uniform_diagonal": p.uniform_diagonal, "lift": p.lift, "self_share": p.self_share}

    def partition(self, stream=None):
        """First vertex of each worker's block: uint32 array [workers + 1]."""
        out = np.zeros(self.info().workers + 1, np.uint32)
        _check(dg_graph_partition(self._h, _np_ptr(out), _stream_handle(stream)))
        return out

    def access_matrix(self, groups=32, stream=None):
        """Reads of one pull sweep by reading worker group (rows) into values
        owned by group (columns): (uint64 array [groups, groups], dg_access_stats)."""
        out = np.zeros((groups, groups), np.uint64)
        st = dg_access_stats()
        _check(dg_access_matrix(self._h, int(groups), _np_ptr(out), C.byref(st), _stream_handle(stream)))
        return out, st

    def close(self):
        if getattr(self, "_h", None):
            # A server's batch state is allocated through the graph: release it
            # first.  The references are strong so that this also holds when the
            # garbage collector finalizes a graph and its server in either order.
            for dep in list(getattr(self, "_dependents", [])):
                dep.close()
            dg_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class GraphSet:
    """Many graphs resident together (one union graph) and swept in one
    launch per sweep.

    ``GraphSet(graphs)`` takes ``graphgen.CSRGraph`` objects (all weighted or
    all unweighted).  Results are flat tensors over the union of the graphs'
    vertices, each graph's PageRank normalised on its own; ``offsets[i]`` is
    graph i's first vertex and ``split(t)`` cuts a result into per-graph
    views.
    """

    def __init__(self, graphs, workers=0, stream=None, torch_allocator=True):
        if torch_allocator:
            use_torch_allocator()
        self._keep = []
        descs = (dg_graph_desc * len(graphs))()
        for i, g in enumerate(graphs):
            ptr = np.ascontiguousarray(g.ptr, dtype=np.uint64)
            idx = np.ascontiguousarray(g.idx, dtype=np.uint32)
            w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.uint32)
            self._keep.append((ptr, idx, w))
            descs[i] = dg_graph_desc(int(g.n), int(idx.shape[0]), ptr.ctypes.data, idx.ctypes.data,
                                     None if w is None else w.ctypes.data)
        h = C.c_void_p()
        opts = dg_set_opts(int(workers))
        _check(dg_set_create(len(graphs), descs, C.byref(opts), _stream_handle(stream), C.byref(h)))
        self._keep = None  # the library copied the arrays
        self._h = h
        self.sizes = [int(g.n) for g in graphs]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])

    def info(self) -> dg_set_info:
        i = dg_set_info()
        _check(dg_set_info_get(self._h, C.byref(i)))
        return i

    def split(self, t):
        return [t[self.offsets[i]:self.offsets[i + 1]] for i in range(len(self.sizes))]

    def set_capture(self, chunk_sweeps):
        """dg_set_set_capture: replay recorded chunks of this many sweeps
        (0: launch every sweep on its own)."""
        _check(dg_set_set_capture(self._h, int(chunk_sweeps)))

    def repartition(self, workers=0, stream=None):
        """dg_set_repartition: per-graph worker blocks for `workers` workgroups."""
        _check(dg_set_repartition(self._h, int(workers), _stream_handle(stream)))

    def tune(self, algo="pagerank", sources=None, dtype="f64", tol=1e-6, stream=None):
        """dg_set_tune ("pagerank" or "sssp" with one local source per graph);
        the set keeps the chosen partition.  Returns the choice as a dict."""
        t = dg_tuning()
        src = None
        if algo == "sssp":
            src = np.ascontiguousarray(sources, dtype=np.uint32)
        _check(dg_set_tune(self._h, DG_ALGO_SSSP if algo == "sssp" else DG_ALGO_PAGERANK, DTYPES[dtype], float(tol),
                           None if src is None else _np_ptr(src), 0, C.byref(t), _stream_handle(stream)))
        return _tuning(t)

    def pagerank(self, damping=0.85, tol=1e-6, mode="delayed", d=64, dtype="f64", max_sweeps=10_000, stream=None,
                 allow_not_converged=False):
        """Per-graph PageRank: (float64 tensor [n], per-graph sweeps, Stats)."""
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        sw = np.zeros(len(self.sizes), np.uint32)
        st = dg_stats()
        s = _check(dg_set_pagerank(self._h, float(damping), float(tol), MODES[mode], int(d), DTYPES[dtype],
                                   int(max_sweeps), 0, C.c_void_p(out.data_ptr()), 1,
                                   _np_ptr(sw), C.byref(st), _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, sw, _stats(st, s == DG_OK)

    def sssp(self, sources, mode="delayed", d=64, max_sweeps=None, stream=None, allow_not_converged=False):
        """Per-graph Bellman-Ford from sources[i] (local ids): (uint32 tensor
        [n] of distances, per-graph sweeps, Stats)."""
        import torch
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        if max_sweeps is None:
            max_sweeps = min(self.n + 1, 1_000_000)
        out = torch.empty(self.n, dtype=torch.uint32, device="cuda")
        sw = np.zeros(len(self.sizes), np.uint32)
        st = dg_stats()
        s = _check(dg_set_sssp(self._h, _np_ptr(src), MODES[mode], int(d), int(max_sweeps),
                               0, C.c_void_p(out.data_ptr()), 1, _np_ptr(sw),
                               C.byref(st), _stream_handle(stream)),
                   allow=(DG_ERR_NOT_CONVERGED,) if allow_not_converged else ())
        return out, sw, _stats(st, s == DG_OK)

    def close(self):
        if getattr(self, "_h", None):
            dg_set_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over resident ``Graph`` objects (continuous batching).

    ``submit(graph, kind, source)`` queues a query ("sssp" or "ppr") and
    returns its id; ``step()`` runs one sweep boundary and returns the ids
    finished so far; ``fetch(id)`` returns the result tensor (uint32
    distances or float64 scores) and the request's info.
    """

    def __init__(self, graphs, mode="async", d=64, damping=0.85, tol=1e-6, dtype="f32", hbm_budget=0,
                 max_batches=0, stream=None):
        self._graphs = list(graphs)  # keep them alive
        for g in self._graphs:
            g._dependents.append(self)
        arr = (C.c_void_p * len(self._graphs))(*[g._h.value for g in self._graphs])
        opts = dg_server_opts(int(hbm_budget), int(max_batches), MODES[mode], int(d), float(damping), float(tol),
                              DTYPES[dtype])
        h = C.c_void_p()
        _check(dg_server_create(arr, len(self._graphs), C.byref(opts), _stream_handle(stream), C.byref(h)))
        self._h = h
        self._buf = np.zeros(4096, np.uint64)

    def submit(self, graph, kind, source):
        rid = C.c_uint64()
        _check(dg_server_submit(self._h, int(graph), QUERIES[kind], int(source), C.byref(rid)))
        return int(rid.value)

    def step(self):
        cnt = C.c_uint32()
        _check(dg_server_step(self._h, _np_ptr(self._buf), self._buf.shape[0], C.byref(cnt)))
        return self._buf[:cnt.value].astype(np.int64).tolist()

    def info(self, rid):
        info = dg_request_info()
        _check(dg_server_fetch(self._h, int(rid), None, 0, C.byref(info)))
        return {"graph": info.graph, "kind": "sssp" if info.kind == DG_QUERY_SSSP else "ppr", "source": info.source,
                "sweeps": info.sweeps, "state": info.state, "submit_step": info.submit_step,
                "admit_step": info.admit_step, "finish_step": info.finish_step}

    def fetch(self, rid, out=None):
        """Result of a finished request (into `out`, a device tensor of at
        least n elements of the result's size, if given) and its info."""
        import torch
        inf = self.info(rid)
        n = self._graphs[inf["graph"]].n
        if out is None:
            out = torch.empty(n, dtype=torch.uint32 if inf["kind"] == "sssp" else torch.float64, device="cuda")
        elif out.numel() * out.element_size() < n * (4 if inf["kind"] == "sssp" else 8) or not out.is_cuda:
            raise ValueError("out is too small or not on the device")
        info = dg_request_info()
        _check(dg_server_fetch(self._h, int(rid), C.c_void_p(out.data_ptr()), 1, C.byref(info)))
        return out, inf

    def status(self):
        st = dg_server_status()
        _check(dg_server_status_get(self._h, C.byref(st)))
        return {"queued": st.queued, "running": st.running, "finished": st.finished, "batches": st.batches,
                "state_bytes": st.state_bytes, "steps": st.steps}

    def close(self):
        if getattr(self, "_h", None):
            dg_server_destroy(self._h)
            self._h = None
        for g in getattr(self, "_graphs", []):
            if self in getattr(g, "_dependents", []):
                g._dependents.remove(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
