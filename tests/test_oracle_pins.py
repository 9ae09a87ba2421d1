"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact integer
arithmetic, a brute-force enumeration, the true Euclidean distance of points
the index stores losslessly, the textbook PQ-ADC of equation (adc) in the T=1
case, and the algebraic identities of equations (distance) and
(decomposition). A dropped term, a wrong sign or index, a transposed operand or
a wrong tie order in the oracle fails at least one of them.
"""

import numpy as np
import pytest

import oracle
import synth


def _exact_half(q, Ch):
    return ((q[None, :].astype(np.int64) - Ch.astype(np.int64)) ** 2).sum(1)


def test_half_dists_exact_on_integers():
    rng = np.random.default_rng(0)
    Ch = rng.integers(-300, 300, (97, 64)).astype(np.float32)
    q = rng.integers(0, 256, 64).astype(np.float32)
    d = oracle.half_dists(q, Ch)
    assert np.array_equal(d, _exact_half(q, Ch).astype(np.float64))


def test_rank_ties_by_index():
    rng = np.random.default_rng(1)
    d = rng.integers(0, 5, 200).astype(np.float64)
    o = oracle.rank(d)
    ref = np.lexsort((np.arange(d.size), d))
    assert np.array_equal(o, ref)


def _brute_visit(ix, q, L):
    """All T*T cells sorted by (key, a, b), then concatenated until min(L, N)."""
    T, h = ix.T, ix.D // 2
    d1 = _exact_half(q[:h], ix.C1)
    d2 = _exact_half(q[h:], ix.C2)
    u = np.lexsort((np.arange(T), d1))
    v = np.lexsort((np.arange(T), d2))
    A, B = np.meshgrid(np.arange(T), np.arange(T), indexing="ij")
    A, B = A.ravel(), B.ravel()
    key = d1[u[A]] + d2[v[B]]
    order = np.lexsort((B, A, key))
    Leff = min(L, ix.N)
    cells, pos, total = [], [], 0
    for o in order:
        if total >= Leff:
            break
        c = int(u[A[o]]) * T + int(v[B[o]])
        beg, end = int(ix.offsets[c]), int(ix.offsets[c + 1])
        take = min(end - beg, Leff - total)
        cells.append((c, take))
        pos.extend(range(beg, beg + take))
        total += take
    return np.array(cells, np.int64).reshape(-1, 2), np.array(pos, np.int64)


@pytest.mark.parametrize("T", [1, 2, 3, 8, 16])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_traversal_matches_bruteforce(T, seed):
    rng = np.random.default_rng(100 + seed)
    counts = rng.integers(0, 4, T * T) * (rng.random(T * T) < 0.6)
    if counts.sum() == 0:
        counts[0] = 1
    # small-integer centroids: many exactly equal keys exercise the (a, b) tie order
    ix = synth.tiny_index(T, counts, M=2, D=4, seed=seed)
    q = rng.integers(0, 6, 4).astype(np.float32)
    N = ix.N
    for L in sorted({1, 2, max(1, N // 3), max(1, N - 1), N, N + 5}):
        cells, pos = oracle.visit(ix, q, L)
        bc, bp = _brute_visit(ix, q, L)
        assert np.array_equal(cells, bc), (T, seed, L)
        assert np.array_equal(pos, bp), (T, seed, L)
        assert pos.size == min(L, N)


def test_traversal_forced_ties_duplicate_centroids():
    T = 6
    C1 = np.zeros((T, 2), np.float32)
    C1[3:] = 1.0  # rows 0-2 and 3-5 are duplicates
    C2 = np.zeros((T, 2), np.float32)
    C2[::2] = 2.0
    counts = np.ones(T * T, np.int64)
    counts[7] = 0
    counts[20] = 5
    ix = synth.tiny_index(T, counts, M=2, D=4, seed=3, C1=C1, C2=C2)
    q = np.array([0, 0, 1, 1], np.float32)
    for L in range(1, ix.N + 2):
        cells, pos = oracle.visit(ix, q, L)
        bc, bp = _brute_visit(ix, q, L)
        assert np.array_equal(cells, bc) and np.array_equal(pos, bp), L


def test_traversal_keys_nondecreasing_gmm():
    means = synth.gmm_means(0)
    base = synth.sample_points(20000, means, 1)
    ix = synth.build_index(base, 16, 8, train_n=5000)
    q = synth.make_queries(1, means, 2)[0]
    d1, d2, u, v = oracle.rank_lists(ix, q)
    cells, pos = oracle.visit(ix, q, 3000)
    inv_u = np.empty(ix.T, np.int64)
    inv_u[u] = np.arange(ix.T)
    inv_v = np.empty(ix.T, np.int64)
    inv_v[v] = np.arange(ix.T)
    i, j = cells[:, 0] // ix.T, cells[:, 0] % ix.T
    key = d1[i] + d2[j]
    a, b = inv_u[i], inv_v[j]
    assert np.all((np.diff(key) > 0) | ((np.diff(key) == 0) & (
        (np.diff(a) > 0) | ((np.diff(a) == 0) & (np.diff(b) > 0)))))
    assert pos.size == 3000 and cells[:-1, 1].sum() + cells[-1, 1] == 3000


def test_lossless_equals_exact_knn():
    # 600 stored vectors repeat earlier ones exactly (equal distances) and ids
    # are shuffled, so the (distance, id) order is not the storage order
    ix = synth.lossless_index(N=3000, T=8, M=4, D=16, seed=7, dup=600, shuffle_ids=True)
    rng = np.random.default_rng(5)
    Q = ix.base[ix.ids[-rng.integers(1, 600, 6)]] + rng.integers(-1, 2, (6, 16)).astype(np.float32)
    k = 25
    ids, d, ncand, _ = oracle.search(ix, Q, ix.N + 10, k, nthreads=2)
    X = ix.base.astype(np.float64)
    for r in range(Q.shape[0]):
        dd = ((X - Q[r].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.arange(ix.N), dd))[:k]
        assert np.array_equal(ids[r], order)
        assert np.array_equal(d[r], dd[order])
        assert ncand[r] == ix.N


def test_T1_is_textbook_pq_adc():
    """One cell with zero centroids: the search is exhaustive PQ-ADC,
    sum_m ||q_m - R_m(b_m)||^2 read from per-subspace tables (equation adc)."""
    ix = synth.random_index(N=2000, T=1, M=8, D=32, seed=9)
    ix.C1[:] = 0
    ix.C2[:] = 0
    rng = np.random.default_rng(2)
    Q = (rng.random((5, 32)) * 50).astype(np.float32)
    k = 17
    ids, d, _, _ = oracle.search(ix, Q, 10 ** 9, k, nthreads=1)
    ds = 32 // 8
    for r in range(5):
        q = Q[r].astype(np.float64)
        lut = np.stack([((q[m * ds:(m + 1) * ds][None] - ix.R[m].astype(np.float64)) ** 2).sum(1)
                        for m in range(8)])
        adc = lut[np.arange(8)[None, :], ix.codes.astype(np.int64)].sum(1)
        order = np.lexsort((ix.ids.astype(np.int64), adc))[:k]
        assert np.array_equal(ids[r], ix.ids[order].astype(np.int64))
        np.testing.assert_allclose(d[r], adc[order], rtol=1e-12)


def test_decomposition_identity():
    """Oracle distance (O(D) reconstruction) equals the expansion of equation
    (distance) with the norm split of equation (decomposition), all in FP64."""
    means = synth.gmm_means(0)
    base = synth.sample_points(20000, means, 1)
    ix = synth.build_index(base, 16, 8, train_n=5000)
    q = synth.make_queries(1, means, 2)[0].astype(np.float64)
    cells, pos = oracle.visit(ix, q.astype(np.float32), 2000)
    cell_of = np.searchsorted(ix.offsets, pos, side="right") - 1
    D, M, h, ds = ix.D, ix.M, ix.D // 2, ix.D // ix.M
    C1, C2, R = (a.astype(np.float64) for a in (ix.C1, ix.C2, ix.R))
    for p, c in list(zip(pos, cell_of))[::37]:
        i, j = divmod(int(c), ix.T)
        code = ix.codes[p]
        r = np.concatenate([R[m, code[m]] for m in range(M)])
        cvec = np.concatenate([C1[i], C2[j]])
        norm = (C1[i] @ C1[i] + C2[j] @ C2[j] + sum(R[m, code[m]] @ R[m, code[m]] for m in range(M))
                + 2 * sum(C1[i][m * ds:(m + 1) * ds] @ R[m, code[m]] for m in range(M // 2))
                + 2 * sum(C2[j][(m - M // 2) * ds:(m - M // 2 + 1) * ds] @ R[m, code[m]]
                          for m in range(M // 2, M)))
        expansion = q @ q - 2 * (q @ cvec) - 2 * (q @ r) + norm
        got = oracle.point_dist(ix, q.astype(np.float32), i, j, code)
        assert abs(got - expansion) <= 1e-10 * max(1.0, q @ q), (got, expansion)


def test_search_equals_lexsort_of_visited():
    means = synth.gmm_means(0)
    base = synth.sample_points(30000, means, 1)
    ix = synth.build_index(base, 32, 8, train_n=5000)
    Q = synth.make_queries(4, means, 2)
    L, k = 4000, 50
    ids, d, ncand, _ = oracle.search(ix, Q, L, k, nthreads=3)
    for r in range(4):
        _, pos = oracle.visit(ix, Q[r], L)
        assert ncand[r] == pos.size == L
        cell_of = np.searchsorted(ix.offsets, pos, side="right") - 1
        i, j = cell_of // ix.T, cell_of % ix.T
        rec = np.concatenate([ix.C1[i], ix.C2[j]], 1).astype(np.float64)
        ds = ix.D // ix.M
        for m in range(ix.M):
            rec[:, m * ds:(m + 1) * ds] += ix.R[m][ix.codes[pos, m]]
        dd = ((rec - Q[r].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((ix.ids[pos], dd))[:k]
        assert np.array_equal(ids[r], ix.ids[pos][order].astype(np.int64))
        np.testing.assert_allclose(d[r], dd[order], rtol=1e-12)


def test_padding_when_fewer_candidates():
    ix = synth.random_index(N=30, T=4, M=2, D=4, seed=4)
    q = np.zeros(4, np.float32)
    ids, d, ncand, _ = oracle.search(ix, q[None], 7, 12, kmax=15)
    assert ncand[0] == 7
    assert np.all(ids[0, 7:] == -1) and np.all(np.isinf(d[0, 7:]))
    assert np.all(ids[0, :7] >= 0) and np.all(np.diff(d[0, :7]) >= 0)


def test_empty_index_and_threads_agree():
    ix = synth.random_index(N=5000, T=8, M=4, D=16, seed=12, empty_frac=0.5)
    rng = np.random.default_rng(3)
    Q = (rng.random((9, 16)) * 100).astype(np.float32)
    L = rng.integers(1, 6000, 9)
    k = rng.integers(1, 20, 9).astype(np.int32)
    a = oracle.search(ix, Q, L, k, kmax=20, nthreads=1)
    b = oracle.search(ix, Q, L, k, kmax=20, nthreads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---- local codebooks (HBPQ, Section 3.2) -----------------------------------------

def test_local_lossless_equals_exact_knn():
    """Points built from local codebooks that differ per centroid: the search
    with those codebooks returns the exact kNN (equation residual); the same
    index searched with the two codebook sets exchanged does not."""
    import dataclasses
    ix = synth.lossless_local_index(N=3000, T=8, M=4, D=16, seed=13, dup=300)
    rng = np.random.default_rng(6)
    Q = ix.base[ix.ids[-rng.integers(1, 300, 6)]] + rng.integers(-1, 2, (6, 16)).astype(np.float32)
    k = 25
    ids, d, ncand, _ = oracle.search(ix, Q, ix.N + 10, k, nthreads=2)
    X = ix.base.astype(np.float64)
    for r in range(Q.shape[0]):
        dd = ((X - Q[r].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.arange(ix.N), dd))[:k]
        assert np.array_equal(ids[r], order)
        assert np.array_equal(d[r], dd[order])
        assert ncand[r] == ix.N
    swapped = dataclasses.replace(ix, QL=ix.SL, SL=ix.QL)
    s_ids, s_d, _, _ = oracle.search(swapped, Q, ix.N + 10, k, nthreads=2)
    assert not np.array_equal(s_d, d)


def test_local_with_global_codebooks_is_the_global_search():
    """Local codebooks that all equal the global ones reduce the search to
    Multi-D-ADC: same ids and bit-identical distances."""
    import dataclasses
    ix = synth.random_index(N=4000, T=16, M=8, D=32, seed=21)
    mh = ix.M // 2
    QL = np.ascontiguousarray(np.broadcast_to(ix.R[:mh][None], (ix.T,) + ix.R[:mh].shape), np.float32)
    SL = np.ascontiguousarray(np.broadcast_to(ix.R[mh:][None], (ix.T,) + ix.R[mh:].shape), np.float32)
    loc = dataclasses.replace(ix, QL=QL, SL=SL)
    rng = np.random.default_rng(3)
    Q = rng.normal(0, 30, (8, ix.D)).astype(np.float32)
    for L in (1, 500, 3000, 10_000):
        g_ids, g_d, g_n, _ = oracle.search(ix, Q, L, 20)
        l_ids, l_d, l_n, _ = oracle.search(loc, Q, L, 20)
        assert np.array_equal(g_ids, l_ids) and np.array_equal(g_d, l_d) and np.array_equal(g_n, l_n)


def test_local_point_dist_uses_row_and_column_codebooks():
    """One stored point of the lossless local index: its distance to itself is
    0, and the distance to any query equals the exact Euclidean distance."""
    ix = synth.lossless_local_index(N=500, T=6, M=4, D=16, seed=14)
    rng = np.random.default_rng(9)
    cells = np.repeat(np.arange(ix.T * ix.T), np.diff(ix.offsets))
    for s in rng.integers(0, ix.N, 10):
        i, j = divmod(int(cells[s]), ix.T)
        x = ix.base[ix.ids[s]]
        assert oracle.point_dist_local(ix, x, i, j, ix.codes[s]) == 0.0
        q = rng.integers(-50, 50, ix.D).astype(np.float32)
        assert oracle.point_dist_local(ix, q, i, j, ix.codes[s]) == float(((q.astype(np.float64) - x) ** 2).sum())


# ---- OPQ rotation of the queries (Section 2.1; the optimized variants) --------------

def test_rotation_identity_is_the_plain_search():
    """An identity rotation leaves every query bit-identical, so the search is
    the unrotated one to the last bit."""
    import dataclasses
    ix = synth.random_index(N=3000, T=16, M=4, D=16, seed=11)
    Q = np.random.default_rng(3).normal(0, 20, (8, 16)).astype(np.float32)
    rix = dataclasses.replace(ix, Rot=np.eye(16, dtype=np.float32))
    a = oracle.search(ix, Q, 700, 15, nthreads=2)
    b = oracle.search(rix, Q, 700, 15, nthreads=2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_rotation_by_permutation_permutes_the_query():
    """Rot[a][b] = 1 where b = p(a): coordinate a of the rotated query is
    coordinate p(a) of the query, exactly (this fixes q' = Rot q, not Rot^T q)."""
    import dataclasses
    ix = synth.random_index(N=3000, T=16, M=4, D=16, seed=12)
    rng = np.random.default_rng(4)
    Q = rng.normal(0, 20, (8, 16)).astype(np.float32)
    p = rng.permutation(16)
    P = np.zeros((16, 16), np.float32)
    P[np.arange(16), p] = 1.0
    assert np.array_equal(oracle.rotate(P, Q), Q[:, p])
    a = oracle.search(dataclasses.replace(ix, Rot=P), Q, 900, 12, nthreads=2)
    b = oracle.search(ix, Q[:, p], 900, 12, nthreads=2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert not np.array_equal(oracle.rotate(P.T.copy(), Q), Q[:, p])


def test_rotated_lossless_index_is_exact_knn_in_the_original_space():
    """A lossless index in the rotated space holds x' = Rot x; searched with
    queries of the original space and L >= N it returns the exact kNN of the
    original points x = Rot^T x' (a rotation keeps distances)."""
    import dataclasses
    ix = synth.lossless_index(N=3000, T=8, M=4, D=16, seed=9, dup=200)
    Rot = synth.random_rotation(16, seed=5)
    rix = dataclasses.replace(ix, Rot=Rot)
    X = ix.base.astype(np.float64) @ Rot.astype(np.float64)  # rows x = Rot^T x'
    rng = np.random.default_rng(7)
    Q = (X[rng.integers(0, ix.N, 6)] + rng.normal(0, 1.5, (6, 16))).astype(np.float32)
    k = 20
    ids, d, ncand, _ = oracle.search(rix, Q, ix.N + 5, k, nthreads=2)
    for r in range(Q.shape[0]):
        dd = ((X - Q[r].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.arange(ix.N), dd))[:k]
        assert np.array_equal(ids[r], order), r
        assert np.allclose(d[r], dd[order], rtol=1e-5, atol=1e-3), r
        assert ncand[r] == ix.N
    # the transposed rotation is a different search
    wrong = oracle.search(dataclasses.replace(ix, Rot=Rot.T.copy()), Q, ix.N + 5, k, nthreads=2)[0]
    assert not np.array_equal(wrong, ids)


def test_random_rotation_is_orthogonal_and_seeded():
    """The generator's rotation is orthogonal (to FP32 rounding) and fixed by its seed."""
    R = synth.random_rotation(128, seed=23)
    assert R.shape == (128, 128) and R.dtype == np.float32
    G = R.astype(np.float64) @ R.T.astype(np.float64)
    assert np.abs(G - np.eye(128)).max() < 1e-5
    assert np.array_equal(R, synth.random_rotation(128, seed=23))
    assert not np.array_equal(R, synth.random_rotation(128, seed=24))


def test_point_dists_lossless_and_consistent():
    """Batch point distances: on a lossless index (codewords equal the
    displacements) they are the exact squared distances to the stored points,
    and they equal the one-point entry for every position."""
    ix = synth.lossless_index(N=400, T=4, M=4, D=16, seed=7)
    rng = np.random.default_rng(3)
    q = rng.integers(0, 40, 16).astype(np.float32)
    pos = np.arange(ix.N)
    d = oracle.point_dists(ix, q, pos)
    pts = ix.base[np.asarray(ix.ids, np.int64)].astype(np.float64)
    assert np.array_equal(d, ((pts - q.astype(np.float64)) ** 2).sum(1))
    for p in rng.integers(0, ix.N, 20):
        cell = int(np.searchsorted(ix.offsets, p, side="right") - 1)
        one = oracle.point_dist(ix, q, cell // ix.T, cell % ix.T, ix.codes[p])
        assert one == d[p]
