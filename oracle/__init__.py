"""FBPQ oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

ctypes binding of the plain FP64 C oracle in fbpq_oracle.c (Multi-D-ADC with
explicit displacement reconstruction, Section 2.3 of the paper, and the same
search with the local codebooks of HBPQ, Section 3.2). An index with an OPQ
rotation (`Rot`, Section 2.1) lives in the rotated space: every function that
takes queries rotates them first (`rotate`), so they take queries in the
original space. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package. It never imports the GPU package.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fbpq_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FP contraction, no fast-math."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.orc_half_dists.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P]
        lib.orc_half_dists.restype = None
        lib.orc_rank.argtypes = [P, ctypes.c_int, P]
        lib.orc_rank.restype = ctypes.c_int
        lib.orc_rank_lists.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P]
        lib.orc_rank_lists.restype = ctypes.c_int
        lib.orc_point_dist.argtypes = [ctypes.c_int] * 4 + [P, P, P, P, i32, i32, P]
        lib.orc_point_dist.restype = ctypes.c_double
        ix_args = [ctypes.c_int] * 4 + [i64, P, P, P, P, P, P]
        lib.orc_visit.argtypes = ix_args + [P, i64, P, i64, P, P, i64]
        lib.orc_visit.restype = i64
        lib.orc_rotate.argtypes = [ctypes.c_int, P, P, i64, P]
        lib.orc_rotate.restype = None
        lib.orc_search.argtypes = ix_args + [P, i64, P, P, i32, P, P, P, P, ctypes.c_int]
        lib.orc_search.restype = ctypes.c_int
        lix_args = [ctypes.c_int] * 4 + [i64] + [P] * 7  # QL and SL in place of R
        lib.orc_search_local.argtypes = lix_args + [P, i64, P, P, i32, P, P, P, P, ctypes.c_int]
        lib.orc_search_local.restype = ctypes.c_int
        lib.orc_point_dist_local.argtypes = [ctypes.c_int] * 4 + [P, P, P, P, P, i32, i32, P]
        lib.orc_point_dist_local.restype = ctypes.c_double
        lib.orc_point_dists.argtypes = [ctypes.c_int] * 4 + [i64] + [P] * 7 + [P, i64, P, P]
        lib.orc_point_dists.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ix_args(ix):
    """Arguments of the C entry points. With local codebooks (ix.QL set) the
    codebook arguments are QL, SL (the *_local entry points), else R."""
    local = getattr(ix, "QL", None) is not None
    books = ((np.ascontiguousarray(ix.QL, np.float32), np.ascontiguousarray(ix.SL, np.float32)) if local
             else (np.ascontiguousarray(ix.R, np.float32),))
    keep = (np.ascontiguousarray(ix.C1, np.float32), np.ascontiguousarray(ix.C2, np.float32)) + books + (
        np.ascontiguousarray(ix.offsets, np.int64), np.ascontiguousarray(ix.codes, np.uint8),
        np.ascontiguousarray(ix.ids, np.uint32))
    return keep, [ix.D, ix.T, ix.M, ix.Kc, ix.N] + [_p(a) for a in keep]


def rotate(Rot: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Queries in the rotated space of an OPQ index: q' = Rot q per row, each
    coordinate an FP64 fused multiply-add chain over b = 0..D-1, rounded to FP32."""
    Rot = np.ascontiguousarray(Rot, np.float32)
    Q = np.ascontiguousarray(Q, np.float32)
    D = Rot.shape[0]
    assert Rot.shape == (D, D) and Q.shape[-1] == D
    flat = Q.reshape(-1, D)
    out = np.empty_like(flat)
    _load().orc_rotate(D, _p(Rot), _p(flat), flat.shape[0], _p(out))
    return out.reshape(Q.shape)


def _in_space(ix, Q: np.ndarray) -> np.ndarray:
    """Queries in the index's space: rotated when the index has an OPQ rotation."""
    Rot = getattr(ix, "Rot", None)
    return np.ascontiguousarray(Q, np.float32) if Rot is None else rotate(Rot, Q)


def half_dists(q: np.ndarray, Ch: np.ndarray) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float32)
    Ch = np.ascontiguousarray(Ch, np.float32)
    d = np.empty(Ch.shape[0], np.float64)
    _load().orc_half_dists(_p(q), _p(Ch), Ch.shape[0], Ch.shape[1], _p(d))
    return d


def rank(d: np.ndarray) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    o = np.empty(d.size, np.int32)
    if _load().orc_rank(_p(d), d.size, _p(o)) != 0:
        raise MemoryError("orc_rank: no memory for the sort")
    return o


def rank_lists(ix, q: np.ndarray):
    """(d1, d2, u, v) of one query: FP64 half distances and rank lists."""
    q = _in_space(ix, q)
    T = ix.T
    d1, d2 = np.empty(T), np.empty(T)
    u, v = np.empty(T, np.int32), np.empty(T, np.int32)
    C1 = np.ascontiguousarray(ix.C1, np.float32)
    C2 = np.ascontiguousarray(ix.C2, np.float32)
    if _load().orc_rank_lists(ix.D, T, _p(C1), _p(C2), _p(q), _p(d1), _p(d2), _p(u), _p(v)) != 0:
        raise MemoryError("orc_rank_lists: no memory for the sort")
    return d1, d2, u, v


def point_dist(ix, q: np.ndarray, i: int, j: int, code: np.ndarray) -> float:
    q = _in_space(ix, q)
    code = np.ascontiguousarray(code, np.uint8)
    C1 = np.ascontiguousarray(ix.C1, np.float32)
    C2 = np.ascontiguousarray(ix.C2, np.float32)
    R = np.ascontiguousarray(ix.R, np.float32)
    return _load().orc_point_dist(ix.D, ix.T, ix.M, ix.Kc, _p(C1), _p(C2), _p(R), _p(q),
                                  int(i), int(j), _p(code))


def point_dists(ix, q: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """FP64 distances from q, given in the index's (rotated, if any) space, to
    the stored points at storage positions pos, by explicit reconstruction
    (through the local codebooks when the index has them)."""
    q = np.ascontiguousarray(q, np.float32)
    pos = np.ascontiguousarray(pos, np.int64)
    local = getattr(ix, "QL", None) is not None
    arrs = [np.ascontiguousarray(ix.C1, np.float32), np.ascontiguousarray(ix.C2, np.float32),
            np.ascontiguousarray(ix.R, np.float32),
            np.ascontiguousarray(ix.QL, np.float32) if local else None,
            np.ascontiguousarray(ix.SL, np.float32) if local else None,
            np.ascontiguousarray(ix.offsets, np.int64), np.ascontiguousarray(ix.codes, np.uint8)]
    out = np.empty(pos.size, np.float64)
    ptrs = [(_p(a) if a is not None else None) for a in arrs]
    rc = _load().orc_point_dists(ix.D, ix.T, ix.M, ix.Kc, ix.N, *ptrs, _p(q), pos.size, _p(pos), _p(out))
    if rc != 0:
        raise ValueError("storage position out of range")
    return out


def point_dist_local(ix, q: np.ndarray, i: int, j: int, code: np.ndarray) -> float:
    """FP64 distance to the reconstruction with the local codebooks of ix."""
    q = _in_space(ix, q)
    code = np.ascontiguousarray(code, np.uint8)
    C1 = np.ascontiguousarray(ix.C1, np.float32)
    C2 = np.ascontiguousarray(ix.C2, np.float32)
    QL = np.ascontiguousarray(ix.QL, np.float32)
    SL = np.ascontiguousarray(ix.SL, np.float32)
    return _load().orc_point_dist_local(ix.D, ix.T, ix.M, ix.Kc, _p(C1), _p(C2), _p(QL), _p(SL), _p(q),
                                        int(i), int(j), _p(code))


def visit(ix, q: np.ndarray, L: int, cells_cap: int = 1 << 20):
    """Visited cells [(cell id, points taken)] and candidate storage positions."""
    if getattr(ix, "QL", None) is not None:
        import dataclasses
        ix = dataclasses.replace(ix, QL=None, SL=None)  # the traversal does not read codebooks
    keep, args = _ix_args(ix)
    q = _in_space(ix, q)
    Leff = max(0, min(int(L), ix.N))
    cells = np.zeros((cells_cap, 2), np.int64)
    nc = np.zeros(1, np.int64)
    pos = np.zeros(max(Leff, 1), np.int64)
    n = _load().orc_visit(*args, _p(q), int(L), _p(cells), cells_cap, _p(nc), _p(pos), pos.size)
    if n < 0:
        raise RuntimeError(f"orc_visit failed ({n})")
    ncell = int(nc[0])
    if ncell > cells_cap:
        raise RuntimeError("cells_cap too small")
    return cells[:ncell].copy(), pos[:n].copy()


def host_threads() -> int:
    """Host cores this process may run on (its CPU affinity), at most 16: the
    share of host cores that goes with one GPU on the machines the GPU runs
    use, and enough for every oracle workload here."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# threads of `search` when the caller names none (None: host_threads())
DEFAULT_THREADS = None


def search(ix, Q: np.ndarray, L, k, kmax: int | None = None, nthreads: int | None = None):
    """Top-k (ids int64, dists float64, ncand, ncells) for every query.

    L and k are scalars or per-query arrays; outputs are [nq][kmax] padded with
    (-1, +inf)."""
    keep, args = _ix_args(ix)
    Q = _in_space(ix, np.asarray(Q, np.float32).reshape(-1, ix.D))
    nq = Q.shape[0]
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, np.int64), (nq,)))
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    if kmax is None:
        kmax = int(k.max()) if nq else 1
    ids = np.empty((nq, kmax), np.int64)
    d = np.empty((nq, kmax), np.float64)
    ncand = np.empty(nq, np.int64)
    ncells = np.empty(nq, np.int64)
    if nthreads is None:
        nthreads = DEFAULT_THREADS or host_threads()
    nthreads = max(1, min(int(nthreads), max(nq, 1)))
    fn = _load().orc_search_local if getattr(ix, "QL", None) is not None else _load().orc_search
    rc = fn(*args, _p(Q), nq, _p(L), _p(k), kmax, _p(ids), _p(d), _p(ncand), _p(ncells), nthreads)
    if rc != 0:
        raise RuntimeError("orc_search failed")
    return ids, d, ncand, ncells
