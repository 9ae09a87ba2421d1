"""ctypes binding of libfbpq (include/fbpq.h): the same entry points, argument
marshalling only. Every step of the search runs in the library's HIP kernels.

Arrays are numpy arrays in host memory, or torch tensors on the index's GPU for
fbpq_search_device (torch provides device memory and the stream). A missing or
unloadable library raises at import time: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfbpq.so")

FBPQ_OK = 0
FBPQ_E_INVALID = -1
FBPQ_E_IO = -2
FBPQ_E_FORMAT = -3
FBPQ_E_OOM = -4
FBPQ_E_DEVICE = -5
FBPQ_E_STATE = -6
FBPQ_E_CAPACITY = -7
FBPQ_E_TIMEOUT = -8
FBPQ_E_CANCELLED = -9
FBPQ_KC = 256
FBPQ_K_MAX = 1024

EXPORTS = ("fbpq_index_create", "fbpq_load_index", "fbpq_index_file_check", "fbpq_build_tables",
           "fbpq_search", "fbpq_search_uneven", "fbpq_search_device", "fbpq_search_device_noalloc",
           "fbpq_search_device_async", "fbpq_search_device_finish",
           "fbpq_debug_visit",
           "fbpq_debug_dists", "fbpq_debug_tables", "fbpq_debug_rank", "fbpq_info",
           "fbpq_table_bytes", "fbpq_set_option", "fbpq_profile_read", "fbpq_stats_read", "fbpq_autotune",
           "fbpq_autotune_cached",
           "fbpq_free_index", "fbpq_last_error", "fbpq_server_create", "fbpq_server_create2",
           "fbpq_server_submit", "fbpq_server_cancel", "fbpq_server_poll", "fbpq_server_counts",
           "fbpq_server_stats", "fbpq_server_first_error", "fbpq_server_destroy", "fbpq_probe_lds_gather")
STAGES = ("half_keys", "prefix", "prefix_fb", "traverse", "layout", "lq", "score", "select", "scan2",
          "traverse_wide", "scan_wide", "rotate")
SERVER_STATS = ("submitted", "completed", "failed", "timeout", "cancelled", "rejected", "batches", "batched",
                "peak_reserved", "peak_batch_reserved", "budget", "lane_budget", "pending")
STATS = ("cell_scan", "fused_topk", "two_pass", "prefix_wave", "prefix_wg", "retried", "graph_replays",
         "wide", "wide_bands", "wide_evals", "wide_loads", "cand_cell_scan", "cand_two_pass", "cand_wide",
         "fused_rescan", "win_admitted", "win_lost")


class FbpqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fbpq error {code}: {msg}")
        self.code = code


class IndexDesc(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("T", ctypes.c_int32), ("M", ctypes.c_int32),
                ("Kc", ctypes.c_int32), ("N", ctypes.c_int64), ("C1", ctypes.c_void_p),
                ("C2", ctypes.c_void_p), ("R", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("codes", ctypes.c_void_p), ("ids", ctypes.c_void_p), ("QL", ctypes.c_void_p),
                ("SL", ctypes.c_void_p), ("Rot", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("T", ctypes.c_int32), ("M", ctypes.c_int32),
                ("Kc", ctypes.c_int32), ("N", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("norm_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("tables_ready", ctypes.c_int32), ("device", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("nlanes", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("D", ctypes.c_int32), ("ws_budget", ctypes.c_int64), ("max_pending", ctypes.c_int64),
                ("timeout_s", ctypes.c_double), ("fake_ns_per_cand", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run paper_1404_1831_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "fbpq_index_create": ([P, ctypes.c_int, P], ctypes.c_int),
        "fbpq_load_index": ([ctypes.c_char_p, ctypes.c_int, P], ctypes.c_int),
        "fbpq_index_file_check": ([ctypes.c_char_p, P], ctypes.c_int),
        "fbpq_build_tables": ([P], ctypes.c_int),
        "fbpq_search": ([P, P, i64, i64, i32, P, P], ctypes.c_int),
        "fbpq_search_uneven": ([P, P, i64, P, P, i32, P, P], ctypes.c_int),
        "fbpq_search_device": ([P, P, i64, P, P, i32, P, P, P], ctypes.c_int),
        "fbpq_search_device_noalloc": ([P, P, i64, P, P, i32, P, P, P], ctypes.c_int),
        "fbpq_search_device_async": ([P, P, i64, P, P, i64, i32, P, P, P, P], ctypes.c_int),
        "fbpq_search_device_finish": ([P], ctypes.c_int),
        "fbpq_debug_visit": ([P, P, i64, i64, P, i64, P, P, i64, P], ctypes.c_int),
        "fbpq_debug_dists": ([P, P, i64, i64, P, P, i64, P], ctypes.c_int),
        "fbpq_debug_tables": ([P, P, P, P, P, P], ctypes.c_int),
        "fbpq_debug_rank": ([P, P, i64, i32, P, P], ctypes.c_int),
        "fbpq_info": ([P, P], ctypes.c_int),
        "fbpq_table_bytes": ([i64, i64, i64, P, P], ctypes.c_int),
        "fbpq_set_option": ([P, ctypes.c_char_p, i64], ctypes.c_int),
        "fbpq_profile_read": ([P, i32, i32, P, P], ctypes.c_int),
        "fbpq_stats_read": ([P, P, i32, i32], ctypes.c_int),
        "fbpq_autotune": ([P, P, i64, P, P, i32, P, P, P, i32, P], ctypes.c_int),
        "fbpq_autotune_cached": ([P, P, i64, P, P, i32, P, P, P, i32, ctypes.c_char_p, P, P], ctypes.c_int),
        "fbpq_free_index": ([P], None),
        "fbpq_server_create": ([P, i32, i32, i32, P], ctypes.c_int),
        "fbpq_server_create2": ([P, P, P], ctypes.c_int),
        "fbpq_server_submit": ([P, P, i64, i32, i64], ctypes.c_int),
        "fbpq_server_cancel": ([P, i64], ctypes.c_int),
        "fbpq_server_stats": ([P, P, i32], ctypes.c_int),
        "fbpq_server_poll": ([P, i32, ctypes.c_double, P, P, P, P, P, P], ctypes.c_int),
        "fbpq_server_counts": ([P, P, P, P], ctypes.c_int),
        "fbpq_server_first_error": ([P], ctypes.c_char_p),
        "fbpq_server_destroy": ([P], None),
        "fbpq_last_error": ([], ctypes.c_char_p),
        "fbpq_probe_lds_gather": ([ctypes.c_int, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(rc: int) -> None:
    if rc != FBPQ_OK:
        raise FbpqError(rc, lib.fbpq_last_error().decode())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def fbpq_last_error() -> str:
    return lib.fbpq_last_error().decode()


def fbpq_table_bytes(T: int, M: int, Kc: int = FBPQ_KC):
    tb, nb = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.fbpq_table_bytes(T, M, Kc, ctypes.byref(tb), ctypes.byref(nb)))
    return tb.value, nb.value


def fbpq_index_file_check(path: str) -> Info:
    info = Info()
    _check(lib.fbpq_index_file_check(path.encode(), ctypes.byref(info)))
    return info


def fbpq_index_create(ix, device: int = 0) -> ctypes.c_void_p:
    """ix: any object with D, T, M, Kc, C1, C2, R, offsets, codes, ids (numpy),
    optionally local codebooks QL, SL ([T][M/2][Kc][D/M] float32) and an OPQ
    rotation Rot ([D][D] float32)."""
    keep = [np.ascontiguousarray(ix.C1, np.float32), np.ascontiguousarray(ix.C2, np.float32),
            np.ascontiguousarray(ix.R, np.float32), np.ascontiguousarray(ix.offsets, np.int64),
            np.ascontiguousarray(ix.codes, np.uint8), np.ascontiguousarray(ix.ids, np.uint32)]
    ql, sl, rot = getattr(ix, "QL", None), getattr(ix, "SL", None), getattr(ix, "Rot", None)
    ptrs = [_p(a) for a in keep]
    for a in (ql, sl, rot):
        if a is not None:
            keep.append(np.ascontiguousarray(a, np.float32))
            ptrs.append(_p(keep[-1]))
        else:
            ptrs.append(None)
    d = IndexDesc(ix.D, ix.T, ix.M, ix.Kc, keep[4].shape[0], *ptrs)
    h = ctypes.c_void_p()
    _check(lib.fbpq_index_create(ctypes.byref(d), device, ctypes.byref(h)))
    return h


def fbpq_load_index(path: str, device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib.fbpq_load_index(path.encode(), device, ctypes.byref(h)))
    return h


def fbpq_build_tables(h) -> None:
    _check(lib.fbpq_build_tables(h))


def fbpq_info(h) -> Info:
    info = Info()
    _check(lib.fbpq_info(h, ctypes.byref(info)))
    return info


def fbpq_set_option(h, key: str, value: int) -> None:
    _check(lib.fbpq_set_option(h, key.encode(), int(value)))


def fbpq_profile_read(h, stage: int, reset: bool = False):
    """(milliseconds, launches) accumulated for a kernel stage while profiling."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib.fbpq_profile_read(h, int(stage), int(reset), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def fbpq_stats_read(h, reset: bool = False) -> dict:
    """Path counters (option "stats" must be on), by name."""
    out = np.zeros(len(STATS), np.int64)
    _check(lib.fbpq_stats_read(h, _p(out), len(STATS), int(reset)))
    return dict(zip(STATS, out.tolist()))


def _tune_dict(out) -> dict:
    return {"prefix": int(out[0]), "items": int(out[1]), "us_per_search": int(out[2]), "persist": int(out[3]),
            "tile": int(out[4]), "pwaves": int(out[5])}


def fbpq_autotune(h, d_q, L, k, k_max: int, d_ids, d_dists, stream, reps: int = 3) -> dict:
    """Tune the first layer, the scan form and the persistent scan's shape on a
    device batch (torch tensors); returns the choice."""
    nq = d_q.shape[0]
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int64), (nq,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    out = np.zeros(6, np.int64)
    _check(lib.fbpq_autotune(h, ctypes.c_void_p(d_q.data_ptr()), nq, _p(L), _p(k), int(k_max),
                             ctypes.c_void_p(d_ids.data_ptr()), ctypes.c_void_p(d_dists.data_ptr()),
                             ctypes.c_void_p(stream.cuda_stream), int(reps), _p(out)))
    return _tune_dict(out)


def fbpq_autotune_cached(h, d_q, L, k, k_max: int, d_ids, d_dists, stream, cache_path: str, reps: int = 3) -> dict:
    """fbpq_autotune through a JSON-lines cache file; the dict says whether the
    choice came from the cache."""
    nq = d_q.shape[0]
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int64), (nq,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    out = np.zeros(6, np.int64)
    hit = ctypes.c_int32()
    _check(lib.fbpq_autotune_cached(h, ctypes.c_void_p(d_q.data_ptr()), nq, _p(L), _p(k), int(k_max),
                                    ctypes.c_void_p(d_ids.data_ptr()), ctypes.c_void_p(d_dists.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream), int(reps), cache_path.encode(), _p(out),
                                    ctypes.byref(hit)))
    d = _tune_dict(out)
    d["from_cache"] = bool(hit.value)
    return d


def fbpq_free_index(h) -> None:
    lib.fbpq_free_index(h)


def fbpq_search(h, q: np.ndarray, L: int, k: int):
    q = np.ascontiguousarray(q, np.float32)
    nq = q.shape[0]
    ids = np.empty((nq, k), np.int64)
    d = np.empty((nq, k), np.float32)
    _check(lib.fbpq_search(h, _p(q), nq, int(L), int(k), _p(ids), _p(d)))
    return ids, d


def fbpq_search_rc(h, q: np.ndarray, L: int, k: int):
    """fbpq_search returning (code, ids, dists) instead of raising: with
    FBPQ_E_CAPACITY the rows it could not serve hold (-2, NaN), the others are complete."""
    q = np.ascontiguousarray(q, np.float32)
    nq = q.shape[0]
    ids = np.empty((nq, k), np.int64)
    d = np.empty((nq, k), np.float32)
    rc = lib.fbpq_search(h, _p(q), nq, int(L), int(k), _p(ids), _p(d))
    return rc, ids, d


def fbpq_search_uneven_rc(h, q: np.ndarray, L, k, k_max: int):
    """fbpq_search_uneven returning (code, ids, dists) instead of raising."""
    q = np.ascontiguousarray(q, np.float32)
    nq = q.shape[0]
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int64), (nq,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    ids = np.empty((nq, k_max), np.int64)
    d = np.empty((nq, k_max), np.float32)
    rc = lib.fbpq_search_uneven(h, _p(q), nq, _p(L), _p(k), int(k_max), _p(ids), _p(d))
    return rc, ids, d


def fbpq_search_uneven(h, q: np.ndarray, L, k, k_max: int):
    q = np.ascontiguousarray(q, np.float32)
    nq = q.shape[0]
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int64), (nq,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    ids = np.empty((nq, k_max), np.int64)
    d = np.empty((nq, k_max), np.float32)
    _check(lib.fbpq_search_uneven(h, _p(q), nq, _p(L), _p(k), int(k_max), _p(ids), _p(d)))
    return ids, d


def fbpq_search_device(h, d_q, L: np.ndarray, k: np.ndarray, k_max: int, d_ids, d_dists,
                       stream=None) -> None:
    """d_q, d_ids, d_dists: contiguous torch tensors on the index's GPU
    (float32 [nq, D], int64 [nq, k_max], float32 [nq, k_max]); L, k: host arrays."""
    nq = d_q.shape[0]
    assert d_q.is_contiguous() and d_ids.is_contiguous() and d_dists.is_contiguous()
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int64), (nq,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    st = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
    _check(lib.fbpq_search_device(h, ctypes.c_void_p(d_q.data_ptr()), nq, _p(L), _p(k), int(k_max),
                                  ctypes.c_void_p(d_ids.data_ptr()), ctypes.c_void_p(d_dists.data_ptr()),
                                  st))


def fbpq_search_device_async(h, d_q, d_L, d_k, L_max: int, k_max: int, d_ids, d_dists, d_pending,
                             stream=None) -> None:
    """Queues a search without waiting: every array a contiguous torch tensor on
    the index's GPU (d_L int64 [nq], d_k int32 [nq], d_pending int32 [2])."""
    nq = d_q.shape[0]
    for t in (d_q, d_L, d_k, d_ids, d_dists, d_pending):
        assert t.is_contiguous()
    st = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
    v = ctypes.c_void_p
    _check(lib.fbpq_search_device_async(h, v(d_q.data_ptr()), nq, v(d_L.data_ptr()), v(d_k.data_ptr()), int(L_max),
                                        int(k_max), v(d_ids.data_ptr()), v(d_dists.data_ptr()),
                                        v(d_pending.data_ptr()), st))


def fbpq_search_device_finish(h) -> int:
    """Runs the deeper rounds of the last asynchronous search, if it has any;
    returns FBPQ_OK or FBPQ_E_CAPACITY (rows it could not serve are (-2, NaN))."""
    rc = lib.fbpq_search_device_finish(h)
    if rc not in (FBPQ_OK, FBPQ_E_CAPACITY):
        _check(rc)
    return rc


def fbpq_search_device_noalloc(h, d_q, L: np.ndarray, k: np.ndarray, k_max: int, d_ids, d_dists,
                               stream=None) -> int:
    """fbpq_search_device with every workspace buffer in the library's static
    scratch array (no device allocation); returns the code (FBPQ_E_CAPACITY:
    the search needs more than the scratch holds)."""
    nq = d_q.shape[0]
    assert d_q.is_contiguous() and d_ids.is_contiguous() and d_dists.is_contiguous()
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int64), (nq,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    st = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
    rc = lib.fbpq_search_device_noalloc(h, ctypes.c_void_p(d_q.data_ptr()), nq, _p(L), _p(k), int(k_max),
                                        ctypes.c_void_p(d_ids.data_ptr()), ctypes.c_void_p(d_dists.data_ptr()),
                                        st)
    if rc not in (FBPQ_OK, FBPQ_E_CAPACITY):
        _check(rc)
    return rc


def fbpq_debug_visit(h, q: np.ndarray, L: int, cells_cap: int, pos_cap: int):
    """Per query: (cells [n][2] of (cell id, points taken), positions) in visit order."""
    q = np.ascontiguousarray(q, np.float32)
    nq = q.shape[0]
    cells = np.zeros((nq, cells_cap, 2), np.int64)
    ncells = np.zeros(nq, np.int64)
    pos = np.zeros((nq, pos_cap), np.int64)
    npos = np.zeros(nq, np.int64)
    _check(lib.fbpq_debug_visit(h, _p(q), nq, int(L), _p(cells), cells_cap, _p(ncells), _p(pos),
                                pos_cap, _p(npos)))
    return [(cells[r, :ncells[r]], pos[r, :npos[r]]) for r in range(nq)]


def fbpq_debug_dists(h, q: np.ndarray, L: int, cap: int):
    """Per query: (storage positions, FP32 FBPQ distances) of all candidates."""
    q = np.ascontiguousarray(q, np.float32)
    nq = q.shape[0]
    pos = np.zeros((nq, cap), np.int64)
    d = np.zeros((nq, cap), np.float32)
    n = np.zeros(nq, np.int64)
    _check(lib.fbpq_debug_dists(h, _p(q), nq, int(L), _p(pos), _p(d), cap, _p(n)))
    return [(pos[r, :n[r]], d[r, :n[r]]) for r in range(nq)]


def fbpq_debug_tables(h):
    info = fbpq_info(h)
    T, M = info.T, info.M
    CR1 = np.empty((T, M // 2, FBPQ_KC), np.float32)
    CR2 = np.empty((T, M // 2, FBPQ_KC), np.float32)
    nR = np.empty((M, FBPQ_KC), np.float32)
    nC1 = np.empty(T, np.float32)
    nC2 = np.empty(T, np.float32)
    _check(lib.fbpq_debug_tables(h, _p(CR1), _p(CR2), _p(nR), _p(nC1), _p(nC2)))
    return CR1, CR2, nR, nC1, nC2


def fbpq_debug_rank(h, q: np.ndarray, P: int):
    q = np.ascontiguousarray(q, np.float32)
    nq = q.shape[0]
    keys = np.empty((nq, 2, P), np.float64)
    idx = np.empty((nq, 2, P), np.int32)
    _check(lib.fbpq_debug_rank(h, _p(q), nq, int(P), _p(keys), _p(idx)))
    return keys, idx


def fbpq_probe_lds_gather(device: int = 0) -> float:
    """Chip-wide random 4-byte LDS reads per second (the scans' lookup pattern)."""
    r = ctypes.c_double()
    _check(lib.fbpq_probe_lds_gather(int(device), ctypes.byref(r)))
    return r.value


def fbpq_server_create(h, max_batch: int, nlanes: int, k_max: int) -> ctypes.c_void_p:
    s = ctypes.c_void_p()
    _check(lib.fbpq_server_create(h, int(max_batch), int(nlanes), int(k_max), ctypes.byref(s)))
    return s


def fbpq_server_create2(h, max_batch: int, nlanes: int, k_max: int, D: int = 0, ws_budget: int = 0,
                        max_pending: int = 0, timeout_s: float = 0.0, fake_ns_per_cand: float = 0.0):
    """Server with admission limits; h None with fake_ns_per_cand > 0: host test backend."""
    cfg = ServerConfig(int(max_batch), int(nlanes), int(k_max), int(D), int(ws_budget), int(max_pending),
                       float(timeout_s), float(fake_ns_per_cand))
    s = ctypes.c_void_p()
    rc = lib.fbpq_server_create2(h, ctypes.byref(cfg), ctypes.byref(s))
    if rc != FBPQ_OK:
        raise FbpqError(rc, "fbpq_server_create2 failed: " + lib.fbpq_last_error().decode())
    return s


def fbpq_server_submit(s, q: np.ndarray, L: int, k: int, tag: int) -> int:
    """Queues a request; returns FBPQ_OK, or FBPQ_E_CAPACITY when admission refuses it."""
    q = np.ascontiguousarray(q, np.float32)
    rc = lib.fbpq_server_submit(s, _p(q), int(L), int(k), int(tag))
    if rc not in (FBPQ_OK, FBPQ_E_CAPACITY):
        _check(rc)
    return rc


def fbpq_server_cancel(s, tag: int) -> int:
    """FBPQ_OK if the queued request was taken out, FBPQ_E_STATE if none is queued under tag."""
    return lib.fbpq_server_cancel(s, int(tag))


def fbpq_server_stats(s) -> dict:
    out = np.zeros(len(SERVER_STATS), np.int64)
    _check(lib.fbpq_server_stats(s, _p(out), out.size))
    return dict(zip(SERVER_STATS, (int(x) for x in out)))


def fbpq_server_poll(s, max_n: int, k_max: int, D: int = 0, wait_s: float = 0.0):
    """(tags, ids [n][k_max], dists, times [n][3], status) of finished requests."""
    tags = np.empty(max_n, np.int64)
    ids = np.empty((max_n, k_max), np.int64)
    d = np.empty((max_n, k_max), np.float32)
    times = np.empty((max_n, 3), np.float64)
    st = np.empty(max_n, np.int32)
    n = ctypes.c_int32()
    _check(lib.fbpq_server_poll(s, int(max_n), float(wait_s), _p(tags), _p(ids), _p(d), _p(times), _p(st),
                                ctypes.byref(n)))
    k = n.value
    return tags[:k], ids[:k], d[:k], times[:k], st[:k]


def fbpq_server_counts(s):
    p, b, n = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.fbpq_server_counts(s, ctypes.byref(p), ctypes.byref(b), ctypes.byref(n)))
    return p.value, b.value, n.value


def fbpq_server_first_error(s) -> str:
    return lib.fbpq_server_first_error(s).decode()


def fbpq_server_destroy(s) -> None:
    lib.fbpq_server_destroy(s)

