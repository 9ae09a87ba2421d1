"""Comparison helpers for the GPU parity tests (GPU path vs FP64 oracle).

Tolerance for an FP32 FBPQ distance d32 against the FP64 oracle distance d64
of the same candidate: |d32 - d64| <= 1e-4 * d64 + 1e-6 * (||q||^2 + ||x^||^2).
The relative term is the bound the search is held to; the absolute floor covers
cancellation when the distance is tiny next to the norms, since FP32 rounding
of the table entries scales with ||q||^2 and ||x^||^2 (x^ = the reconstruction
of equation approximation).
"""

from __future__ import annotations

import sys

import numpy as np

REL = 1e-4
ABS_NORM = 1e-6


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def recon(ix, pos: np.ndarray) -> np.ndarray:
    """FP64 reconstructions [len(pos), D] of stored points (equation
    approximation; with local codebooks, equation residual of Section 3.2),
    for the norm term of the tolerance."""
    cell = np.searchsorted(ix.offsets, pos, side="right") - 1
    i, j = cell // ix.T, cell % ix.T
    x = np.concatenate([ix.C1[i], ix.C2[j]], 1).astype(np.float64)
    ds, mh = ix.D // ix.M, ix.M // 2
    for m in range(ix.M):
        if getattr(ix, "QL", None) is None:
            w = ix.R[m][ix.codes[pos, m]]
        elif m < mh:
            w = ix.QL[i, m, ix.codes[pos, m]]
        else:
            w = ix.SL[j, m - mh, ix.codes[pos, m]]
        x[:, m * ds:(m + 1) * ds] += w
    return x


def tol(ix, q: np.ndarray, pos: np.ndarray, d64: np.ndarray) -> np.ndarray:
    x = recon(ix, pos)
    q = q.astype(np.float64)
    return REL * np.abs(d64) + ABS_NORM * ((q @ q) + (x * x).sum(1))


def oracle_dists(ix, q: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """The oracle's FP64 distances (explicit reconstruction) from q, in the
    index's space, to the stored points at positions pos."""
    import oracle
    return oracle.point_dists(ix, q, pos)


def pos_of_ids(ix, ids: np.ndarray) -> np.ndarray:
    inv = np.empty(ix.N, np.int64)
    inv[ix.ids.astype(np.int64)] = np.arange(ix.N)
    return inv[ids]


def assert_topk(ix, Q, k_req, g_ids, g_d, o_ids, o_d, ncand=None):
    """GPU top-k equals the oracle's up to near-ties at the k boundary.

    Per query: padded positions agree; the i-th GPU distance is within tolerance
    of the i-th oracle distance; every GPU id's own FP64 distance is within
    tolerance of its GPU distance; ids differ only where their FP64 distances
    lie within tolerance of the k-th oracle distance.
    """
    nq = Q.shape[0]
    k_req = np.broadcast_to(np.asarray(k_req), (nq,))
    for r in range(nq):
        k = int(k_req[r])
        gi, gd, oi, od = g_ids[r, :k], g_d[r, :k], o_ids[r, :k], o_d[r, :k]
        valid_o = oi >= 0
        valid_g = gi >= 0
        assert np.array_equal(valid_o, valid_g), (r, "padding differs", valid_o.sum(), valid_g.sum())
        assert np.all(np.isinf(gd[~valid_g])) and np.all(g_ids[r, k:] == -1)
        n = int(valid_g.sum())
        if n == 0:
            continue
        gi, gd, oi, od = gi[:n], gd[:n].astype(np.float64), oi[:n], od[:n]
        assert len(set(gi.tolist())) == n, (r, "duplicate ids")
        assert np.all(np.diff(gd) >= 0), (r, "GPU distances not sorted")
        gpos = pos_of_ids(ix, gi)
        g64 = oracle_dists(ix, Q[r], gpos)
        t = tol(ix, Q[r], gpos, g64)
        assert np.all(np.abs(gd - g64) <= t), (r, "distance out of tolerance",
                                               np.max(np.abs(gd - g64) / np.maximum(t, 1e-30)))
        opos = pos_of_ids(ix, oi)
        to = tol(ix, Q[r], opos, od)
        assert np.all(np.abs(np.sort(g64) - od) <= 2 * np.maximum(t, to)), (r, "sorted distances differ")
        if not np.array_equal(gi, oi):
            kth = od[-1]
            tk = to[-1]
            for x in set(gi.tolist()) ^ set(oi.tolist()):
                dx = oracle_dists(ix, Q[r], pos_of_ids(ix, np.array([x])))[0]
                assert abs(dx - kth) <= 2 * tk + 1e-9, (r, "id mismatch away from the k-th distance", x, dx, kth)
            same = set(gi.tolist()) == set(oi.tolist())
            if same:
                # same set, different order: only among near-equal distances
                assert np.all(np.abs(g64 - od) <= 2 * np.maximum(t, to)), (r, "order differs beyond ties")
