"""GPU parity: the HIP search through the C ABI against the FP64 oracle.

Visited-cell lists and candidate positions must be bit-exact, sorted prefixes of
the half lists bit-exact (FP64 keys and indices), per-candidate distances and
the top-k within the tolerance of tests/parity.py.
"""

import numpy as np
import pytest

import oracle
import synth
from parity import assert_topk, log, oracle_dists, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fb():
    from paper_1404_1831_amd import fbpq  # raises if the library is not built
    return fbpq


def _open(fb, ix, **opts):
    h = fb.fbpq_index_create(ix, 0)
    fb.fbpq_build_tables(h)
    for k, v in opts.items():
        fb.fbpq_set_option(h, k, v)
    return h


@pytest.fixture(scope="module")
def gmm_small():
    # 100k SIFT-like points, T=64 per half (4096 cells), M=8: the plain-FBPQ workload
    means = synth.gmm_means(0)
    base = synth.sample_points(100000, means, 1)
    ix = synth.build_index(base, 64, 8)
    Q = synth.make_queries(100, means, 2)
    return ix, Q


@pytest.fixture(scope="module")
def gmm_m16():
    means = synth.gmm_means(0)
    base = synth.sample_points(60000, means, 1)
    ix = synth.build_index(base, 128, 16, train_n=10000)
    Q = synth.make_queries(40, means, 2)
    return ix, Q


def test_tables_match_fp64(fb, gmm_m16):
    ix, _ = gmm_m16
    log("tables: T=128 M=16")
    h = _open(fb, ix)
    CR1, CR2, nR, nC1, nC2 = fb.fbpq_debug_tables(h)
    fb.fbpq_free_index(h)
    C1, C2, R = (a.astype(np.float64) for a in (ix.C1, ix.C2, ix.R))
    M, ds = ix.M, ix.D // ix.M
    for k in range(M // 2):
        ref1 = 2 * C1[:, k * ds:(k + 1) * ds] @ R[k].T
        ref2 = 2 * C2[:, k * ds:(k + 1) * ds] @ R[M // 2 + k].T
        np.testing.assert_allclose(CR1[:, k], ref1, rtol=1e-6, atol=1e-6 * np.abs(ref1).max())
        np.testing.assert_allclose(CR2[:, k], ref2, rtol=1e-6, atol=1e-6 * np.abs(ref2).max())
    np.testing.assert_allclose(nR, (R * R).sum(2), rtol=1e-6)
    np.testing.assert_allclose(nC1, (C1 * C1).sum(1), rtol=1e-6)
    np.testing.assert_allclose(nC2, (C2 * C2).sum(1), rtol=1e-6)


@pytest.mark.parametrize("P", [64, 17, 1])
def test_rank_prefix_bitexact(fb, gmm_small, P):
    ix, Q = gmm_small
    log(f"rank prefix: T=64 P={P}")
    h = _open(fb, ix)
    keys, idx = fb.fbpq_debug_rank(h, Q[:30], P)
    fb.fbpq_free_index(h)
    for r in range(30):
        d1, d2, u, v = oracle.rank_lists(ix, Q[r])
        assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P])
        assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]])


def test_rank_prefix_ties(fb):
    # integer centroids with many duplicates: equal keys ordered by index
    ix = synth.random_index(N=2000, T=300, M=4, D=16, seed=3, int_valued=True)
    ix.C1[100:200] = ix.C1[:100]
    rng = np.random.default_rng(4)
    Q = rng.integers(0, 32, (8, 16)).astype(np.float32)
    log("rank prefix ties: T=300")
    h = _open(fb, ix)
    for P in (300, 128, 5):
        keys, idx = fb.fbpq_debug_rank(h, Q, P)
        for r in range(8):
            d1, d2, u, v = oracle.rank_lists(ix, Q[r])
            assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P]), P
            assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]])
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("block_min", [1, 0])
def test_rank_prefix_block_minima_ties(fb, block_min):
    # T = 4096 and 8192 integer centroids, 2048 of them copies of others (their
    # keys tied with another centroid's, in other blocks): prefixes from the
    # block minima of the key kernel (4 and 8 samples per lane) equal the
    # oracle's, ties ordered by index
    for T in (4096, 8192):
        ix = synth.random_index(N=3000, T=T, M=4, D=16, seed=3, int_valued=True)
        ix.C1[2048:4096] = ix.C1[:2048]
        ix.C2[1024:2048] = ix.C2[:1024]
        rng = np.random.default_rng(6)
        Q = rng.integers(0, 32, (24, 16)).astype(np.float32)
        log(f"rank prefix from block minima: T={T} duplicated centroids block_min={block_min}")
        h = _open(fb, ix, block_min=block_min, stats=1)
        for P in (128, 64, 7):
            keys, idx = fb.fbpq_debug_rank(h, Q, P)
            for r in range(Q.shape[0]):
                d1, d2, u, v = oracle.rank_lists(ix, Q[r])
                assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P]), (T, P, r)
                assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]])
        st = fb.fbpq_stats_read(h)
        fb.fbpq_free_index(h)
        assert st["prefix_wave"] > 0


def _check_visit(fb, h, ix, Q, L, cap=1 << 16):
    cap = min(ix.T * ix.T + 1, cap)
    got = fb.fbpq_debug_visit(h, Q, L, cells_cap=cap, pos_cap=max(1, min(L, ix.N)))
    for r in range(Q.shape[0]):
        cells, pos = oracle.visit(ix, Q[r], L, cells_cap=max(cap, 1 << 20))
        gc, gp = got[r]
        assert np.array_equal(gc, cells), (r, L, gc.shape, cells.shape)
        assert np.array_equal(gp, pos), (r, L)


@pytest.mark.parametrize("L", [10000, 1, 777, 100000, 250000])
def test_visit_bitexact_gmm(fb, gmm_small, L):
    ix, Q = gmm_small
    log(f"visit: N=1e5 T=64 L={L}")
    h = _open(fb, ix)
    _check_visit(fb, h, ix, Q[:50], L)
    fb.fbpq_free_index(h)


def test_visit_retries_prefix_and_cells(fb, gmm_small):
    ix, Q = gmm_small
    log("visit with prefix=1, max_cells=64 (forced second rounds)")
    h = _open(fb, ix, prefix=1, max_cells=64)
    _check_visit(fb, h, ix, Q[:20], 10000)
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("T,seed", [(1, 0), (2, 1), (3, 2), (8, 3), (16, 4), (40, 5)])
def test_visit_tiny_with_ties_and_empty_cells(fb, T, seed):
    rng = np.random.default_rng(200 + seed)
    counts = rng.integers(0, 5, T * T) * (rng.random(T * T) < 0.5)
    if counts.sum() == 0:
        counts[0] = 2
    ix = synth.tiny_index(T, counts, M=2, D=4, seed=seed)
    Q = rng.integers(0, 6, (6, 4)).astype(np.float32)
    log(f"visit tiny: T={T} N={ix.N}")
    h = _open(fb, ix)
    for L in sorted({1, 2, max(1, ix.N // 2), ix.N, ix.N + 3}):
        _check_visit(fb, h, ix, Q, L)
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("items", [1, 0])
def test_candidate_distances_within_tolerance(fb, gmm_small, items):
    ix, Q = gmm_small
    L = 10000
    log(f"per-candidate FBPQ distances: N=1e5 T=64 M=8 L=1e4 items={items}")
    h = _open(fb, ix, items=items)
    got = fb.fbpq_debug_dists(h, Q[:20], L, cap=L)
    fb.fbpq_free_index(h)
    for r in range(20):
        pos, d32 = got[r]
        _, opos = oracle.visit(ix, Q[r], L)
        assert np.array_equal(np.sort(pos), np.sort(opos))
        d64 = oracle_dists(ix, Q[r], pos)
        t = tol(ix, Q[r], pos, d64)
        err = np.abs(d32.astype(np.float64) - d64)
        assert np.all(err <= t), (r, float((err / t).max()))


def test_candidate_distances_m16_chunked(fb, gmm_m16):
    ix, Q = gmm_m16
    L = 5000
    log("per-candidate distances: T=128 M=16 L=5000 chunk=1024")
    h = _open(fb, ix, chunk=1024)
    got = fb.fbpq_debug_dists(h, Q[:10], L, cap=L)
    fb.fbpq_free_index(h)
    for r in range(10):
        pos, d32 = got[r]
        _, opos = oracle.visit(ix, Q[r], L)
        assert np.array_equal(np.sort(pos), np.sort(opos))
        d64 = oracle_dists(ix, Q[r], pos)
        assert np.all(np.abs(d32 - d64) <= tol(ix, Q[r], pos, d64))


@pytest.mark.parametrize("items", [1, 0])
def test_search_cfg0_topk(fb, gmm_small, items):
    ix, Q = gmm_small
    L, k = 10000, 10
    log(f"search: N=1e5 T=64 M=8 nq=100 L=1e4 k=10 items={items}")
    h = _open(fb, ix, items=items)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    g2_ids, g2_d = fb.fbpq_search(h, Q, L, k)
    fb.fbpq_free_index(h)
    assert np.array_equal(g_ids, g2_ids) and np.array_equal(g_d, g2_d), "not deterministic"
    o_ids, o_d, ncand, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)
    # recall@10 against exact NN equals the oracle's
    X = ix.base.astype(np.float64)
    exact = np.array([np.argmin(((X - q.astype(np.float64)) ** 2).sum(1)) for q in Q])
    r_gpu = np.mean([exact[i] in g_ids[i] for i in range(len(Q))])
    r_orc = np.mean([exact[i] in o_ids[i] for i in range(len(Q))])
    log(f"recall@10 gpu={r_gpu:.3f} oracle={r_orc:.3f}")
    assert r_gpu == r_orc


@pytest.mark.parametrize("chunk,items", [(8192, 1), (8192, 0), (512, 0)])
def test_search_m16_k100_chunks(fb, gmm_m16, chunk, items):
    ix, Q = gmm_m16
    L, k = 6000, 100
    log(f"search: T=128 M=16 L=6000 k=100 chunk={chunk} items={items}")
    h = _open(fb, ix, chunk=chunk, items=items)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


def test_search_uneven_L_k(fb, gmm_small):
    ix, Q = gmm_small
    rng = np.random.default_rng(9)
    L = rng.integers(1, 30000, Q.shape[0])
    L[:3] = [1, ix.N, ix.N + 100]
    k = rng.choice([1, 10, 100], Q.shape[0]).astype(np.int32)
    log("search uneven L/k: N=1e5 T=64")
    h = _open(fb, ix)
    g_ids, g_d = fb.fbpq_search_uneven(h, Q, L, k, 100)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k, kmax=100)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


def test_lossless_exact_knn_with_ties(fb):
    ix = synth.lossless_index(N=5000, T=16, M=4, D=16, seed=7, dup=1000, shuffle_ids=True)
    rng = np.random.default_rng(5)
    Q = ix.base[ix.ids[-rng.integers(1, 1000, 12)]] + rng.integers(-1, 2, (12, 16)).astype(np.float32)
    k = 30
    log("lossless with duplicates: N=5000 T=16 M=4 L>N")
    h = _open(fb, ix)
    g_ids, g_d = fb.fbpq_search(h, Q, ix.N + 1, k)
    fb.fbpq_free_index(h)
    X = ix.base.astype(np.float64)
    for r in range(12):
        dd = ((X - Q[r].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.arange(ix.N), dd))[:k]
        # integer data: FP32 FBPQ distances are exact here, ties break by id
        assert np.array_equal(g_ids[r], order), r
        assert np.array_equal(g_d[r].astype(np.float64), dd[order]), r


def test_padding_k_above_L_and_empty(fb):
    ix = synth.random_index(N=400, T=8, M=4, D=16, seed=12, empty_frac=0.6)
    rng = np.random.default_rng(1)
    Q = (rng.random((5, 16)) * 100).astype(np.float32)
    log("padding: L=7 k=20; nq=0")
    h = _open(fb, ix)
    g_ids, g_d = fb.fbpq_search(h, Q, 7, 20)
    o_ids, o_d, _, _ = oracle.search(ix, Q, 7, 20)
    assert_topk(ix, Q, 20, g_ids, g_d, o_ids, o_d)
    assert np.all(g_ids[:, 7:] == -1) and np.all(np.isinf(g_d[:, 7:]))
    e_ids, e_d = fb.fbpq_search(h, Q[:0], 7, 20)
    assert e_ids.shape == (0, 20)
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("M,D", [(2, 16), (4, 16), (16, 32), (32, 64)])
def test_code_lengths(fb, M, D):
    ix = synth.random_index(N=3000, T=12, M=M, D=D, seed=M)
    rng = np.random.default_rng(M)
    Q = (rng.random((6, D)) * 100).astype(np.float32)
    log(f"code length M={M} D={D}")
    h = _open(fb, ix)
    g_ids, g_d = fb.fbpq_search(h, Q, 900, 25)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, 900, 25)
    assert_topk(ix, Q, 25, g_ids, g_d, o_ids, o_d)


def test_T1_single_cell(fb):
    ix = synth.random_index(N=3000, T=1, M=8, D=32, seed=9)
    rng = np.random.default_rng(2)
    Q = (rng.random((4, 32)) * 50).astype(np.float32)
    log("T=1 (exhaustive PQ-ADC)")
    h = _open(fb, ix)
    g_ids, g_d = fb.fbpq_search(h, Q, 10 ** 9, 40)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, 10 ** 9, 40)
    assert_topk(ix, Q, 40, g_ids, g_d, o_ids, o_d)


def test_load_index_file_matches_create(fb, gmm_small, tmp_path):
    ix, Q = gmm_small
    p = str(tmp_path / "ix.bin")
    synth.write_index(p, ix)
    log("load from file")
    h1 = _open(fb, ix)
    h2 = fb.fbpq_load_index(p, 0)
    fb.fbpq_build_tables(h2)
    a = fb.fbpq_search(h1, Q[:20], 5000, 10)
    b = fb.fbpq_search(h2, Q[:20], 5000, 10)
    info = fb.fbpq_info(h2)
    fb.fbpq_free_index(h1)
    fb.fbpq_free_index(h2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert info.tables_ready == 1 and info.table_bytes == 64 * 8 * 256 * 4


@pytest.mark.parametrize("nth", [1, 4, 12])
def test_device_error_poisons_handle(fb, gmm_small, nth):
    # A failed HIP call (reported on the host in place of the nth checked call
    # after the option is set; no kernel misbehaves) ends that search with
    # FBPQ_E_DEVICE and poisons the handle: every later call refuses with the
    # same code, the handle still frees, and a fresh handle on the same index
    # gives the results of before.
    ix, Q = gmm_small
    h = _open(fb, ix)
    ids0, d0 = fb.fbpq_search(h, Q[:8], 2000, 10)
    fb.fbpq_set_option(h, "inject_device_error", nth)
    failed = None
    for _ in range(nth):  # each search makes at least one checked call
        try:
            fb.fbpq_search(h, Q[:8], 2000, 10)
        except fb.FbpqError as ex:
            failed = ex
            break
    assert failed is not None and failed.code == fb.FBPQ_E_DEVICE
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_search(h, Q[:8], 2000, 10)
    assert e.value.code == fb.FBPQ_E_DEVICE
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_set_option(h, "prefix", 64)
    assert e.value.code == fb.FBPQ_E_DEVICE
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_info(h)
    assert e.value.code == fb.FBPQ_E_DEVICE
    fb.fbpq_free_index(h)
    h = _open(fb, ix)
    ids1, d1 = fb.fbpq_search(h, Q[:8], 2000, 10)
    fb.fbpq_free_index(h)
    assert np.array_equal(ids0, ids1) and np.array_equal(d0, d1)


def test_errors(fb, gmm_small):
    ix, Q = gmm_small
    h = fb.fbpq_index_create(ix, 0)
    with pytest.raises(fb.FbpqError) as e:
        fb.fbpq_search(h, Q[:2], 100, 10)
    assert e.value.code == fb.FBPQ_E_STATE
    fb.fbpq_build_tables(h)
    for L, k in ((0, 10), (100, 0), (100, 2000)):
        with pytest.raises(fb.FbpqError) as e:
            fb.fbpq_search(h, Q[:2], L, k)
        assert e.value.code == fb.FBPQ_E_INVALID
    fb.fbpq_free_index(h)


# ---- wavefront prefix select (T >= 256, P <= 256) -------------------------------

@pytest.fixture(scope="module")
def gmm_wide():
    """GMM indexes with T = 256, 1000 and 4096 centroids per half (built on the GPU)."""
    import torch
    dev = torch.device("cuda:0")
    means = synth.gmm_means(0)
    base = synth.sample_points(200000, means, 1, dev)
    out = {}
    for T in (256, 1000, 4096):
        out[T] = synth.build_index(base, T, 8, train_n=20000, keep_base=False)
    Q = synth.make_queries(40, means, 2)
    return out, Q


@pytest.mark.parametrize("T,P", [(256, 128), (256, 255), (1000, 1), (1000, 100), (4096, 128), (4096, 256)])
def test_rank_prefix_wave_bitexact(fb, gmm_wide, T, P):
    idxs, Q = gmm_wide
    ix = idxs[T]
    log(f"rank prefix (wavefront select): T={T} P={P}")
    h = _open(fb, ix, stats=1)
    keys, idx = fb.fbpq_debug_rank(h, Q, P)
    st = fb.fbpq_stats_read(h)
    fb.fbpq_free_index(h)
    log(f"  counters {st}")
    assert st["prefix_wave"] + st["prefix_wg"] == 2 * Q.shape[0]
    assert st["prefix_wave"] > 0
    for r in range(Q.shape[0]):
        d1, d2, u, v = oracle.rank_lists(ix, Q[r])
        assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P]), r
        assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]]), r


@pytest.mark.parametrize("scale,shift", [(1.0, 0.0), (1e-4, -0.0128), (300.0, -38400.0)])
@pytest.mark.parametrize("split", [1, 0])
def test_split_keys_prefix_bitexact(fb, gmm_wide, scale, shift, split):
    # The approximate keys from two-part FP16 half-centroids (split = 1) or FP32
    # products (split = 0), on data whose magnitudes span small values, the
    # SIFT-like range and values beyond the FP16 range (each side scaled by a
    # power of two on the device), with negative coordinates: the FP64
    # prefixes equal the oracle's bit for bit either way.
    import dataclasses
    idxs, Q = gmm_wide
    ix = idxs[4096]
    ixs = dataclasses.replace(ix, C1=(ix.C1 * scale + shift).astype(np.float32),
                              C2=(ix.C2 * scale + shift).astype(np.float32))
    Qs = (Q * scale + shift).astype(np.float32)
    P = 128
    log(f"split keys: T=4096 P={P} scale={scale} shift={shift} split={split}")
    h = _open(fb, ixs, split_keys=split)
    keys, idx = fb.fbpq_debug_rank(h, Qs, P)
    fb.fbpq_free_index(h)
    for r in range(Qs.shape[0]):
        d1, d2, u, v = oracle.rank_lists(ixs, Qs[r])
        assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P]), r
        assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]]), r


@pytest.mark.parametrize("nq,T", [(300, 4096), (32800, 4096), (300, 1000)])
@pytest.mark.parametrize("split", [1, 0])
def test_rank_prefix_full_workgroups(fb, gmm_wide, nq, T, split):
    # Batches of at least 128 queries fill whole workgroups of four 32-row
    # groups, which in the split form share each 16-centroid strip through LDS
    # (the 40-query batches above never fill one). 300 queries also leave a
    # workgroup with one full and one partial row group; 32,800 queries take
    # the 512-centroid chunks and leave one full row group alone; at T = 1000
    # the last chunk of every row is partial and takes the general loop. The FP64
    # prefixes equal the oracle's bit for bit on every row checked, and most
    # rows take the wavefront select (wrong approximate keys push rows off it).
    idxs, _ = gmm_wide
    ix = idxs[T]
    Q = synth.make_queries(nq, synth.gmm_means(0), 5)
    P = 64
    log(f"rank prefix, full workgroups: T={T} nq={nq} P={P} split={split}")
    h = _open(fb, ix, split_keys=split, stats=1)
    keys, idx = fb.fbpq_debug_rank(h, Q, P)
    st = fb.fbpq_stats_read(h)
    fb.fbpq_free_index(h)
    log(f"  counters {st}")
    assert st["prefix_wave"] + st["prefix_wg"] == 2 * nq
    assert st["prefix_wave"] > nq
    rows = range(nq) if nq <= 300 else sorted(set(range(0, nq, 211)) | set(range(nq - 40, nq)))
    for r in rows:
        d1, d2, u, v = oracle.rank_lists(ix, Q[r])
        assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P]), r
        assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]]), r


def test_search_T1000_visit_and_topk(fb, gmm_wide):
    idxs, Q = gmm_wide
    ix = idxs[1000]
    L, k = 3000, 20
    log("search: N=2e5 T=1000 M=8 L=3000 k=20")
    h = _open(fb, ix, stats=1)
    _check_visit(fb, h, ix, Q[:12], L)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    log(f"  counters {fb.fbpq_stats_read(h)}")
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


# ---- threshold-stepping traversal ------------------------------------------------
# pop_budget=0 sends every query to the threshold kernel, pop_budget=1 defers
# every query the first batch of pops does not finish.

@pytest.mark.parametrize("budget", [0, 1])
@pytest.mark.parametrize("L", [1, 777, 10000, 250000])
def test_visit_threshold_steps_gmm(fb, gmm_small, budget, L):
    ix, Q = gmm_small
    log(f"visit by threshold steps: N=1e5 T=64 L={L} pop_budget={budget}")
    h = _open(fb, ix, pop_budget=budget, stats=1)
    _check_visit(fb, h, ix, Q[:30], L)
    if budget == 0:
        assert fb.fbpq_stats_read(h)["wide"] >= 30
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("budget", [0, 1])
def test_visit_threshold_steps_retries(fb, gmm_small, budget):
    ix, Q = gmm_small
    log(f"visit by threshold steps with prefix=1, max_cells=64, pop_budget={budget}")
    h = _open(fb, ix, prefix=1, max_cells=64, pop_budget=budget, stats=1)
    _check_visit(fb, h, ix, Q[:20], 10000)
    assert fb.fbpq_stats_read(h)["retried"] > 0
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("T,seed", [(2, 1), (3, 2), (8, 3), (16, 4), (40, 5)])
def test_visit_threshold_steps_ties(fb, T, seed):
    # integer centroids and queries: many cells share one key
    rng = np.random.default_rng(200 + seed)
    counts = rng.integers(0, 5, T * T) * (rng.random(T * T) < 0.5)
    if counts.sum() == 0:
        counts[0] = 2
    ix = synth.tiny_index(T, counts, M=2, D=4, seed=seed)
    Q = rng.integers(0, 6, (6, 4)).astype(np.float32)
    log(f"visit tiny by threshold steps: T={T} N={ix.N}")
    h = _open(fb, ix, pop_budget=0)
    for L in sorted({1, 2, max(1, ix.N // 2), ix.N, ix.N + 3}):
        _check_visit(fb, h, ix, Q, L)
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("budget", [0, 1])
def test_visit_one_key_band_in_chunks(fb, budget):
    # every centroid of a half is the same point: all 4096 cells share one key,
    # so the band is walked in (a, b) order in chunks of 2048 cells
    T = 64
    rng = np.random.default_rng(77)
    counts = rng.integers(0, 3, T * T)
    C1 = np.tile(np.array([[1.0, 2.0]], np.float32), (T, 1))
    C2 = np.tile(np.array([[0.0, 3.0]], np.float32), (T, 1))
    ix = synth.tiny_index(T, counts, M=2, D=4, seed=9, C1=C1, C2=C2)
    Q = rng.integers(0, 6, (3, 4)).astype(np.float32)
    log(f"visit one-key band: T={T} N={ix.N} pop_budget={budget}")
    h = _open(fb, ix, pop_budget=budget)
    for L in (1, ix.N // 3, ix.N - 1, ix.N):
        _check_visit(fb, h, ix, Q, L)
    fb.fbpq_free_index(h)


@pytest.mark.parametrize("budget", [512, 0])
def test_search_threshold_steps_topk(fb, gmm_small, budget):
    ix, Q = gmm_small
    L, k = 20000, 100
    log(f"search: N=1e5 T=64 L={L} k={k} pop_budget={budget}")
    h = _open(fb, ix, pop_budget=budget)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


@pytest.mark.parametrize("P", [3000, 4096])
def test_long_prefix_rank_visit_and_topk(fb, gmm_wide, P):
    # prefixes longer than the one-at-a-time traversal holds (T = 4096)
    idxs, Q = gmm_wide
    ix = idxs[4096]
    log(f"long prefix: N=2e5 T=4096 P={P}")
    h = _open(fb, ix, prefix=P, stats=1)
    keys, idx = fb.fbpq_debug_rank(h, Q[:6], P)
    for r in range(6):
        d1, d2, u, v = oracle.rank_lists(ix, Q[r])
        assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P]), r
        assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]]), r
    _check_visit(fb, h, ix, Q[:4], 3000, cap=1 << 20)  # sparse cells: about 10^5 visited
    L, k = 5000, 10
    g_ids, g_d = fb.fbpq_search(h, Q[:16], L, k)
    assert fb.fbpq_stats_read(h)["wide"] >= 16
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q[:16], L, k)
    assert_topk(ix, Q[:16], k, g_ids, g_d, o_ids, o_d)


@pytest.mark.parametrize("items", [1, 0])
def test_wide_scan_sparse_cells(fb, gmm_wide, items):
    # T = 1000 with 2e5 points: about 0.2 points per cell, so L = 20000 gives a
    # query more than 8192 candidates in sparse cells (the HBM two-pass scan)
    idxs, Q = gmm_wide
    ix = idxs[1000]
    L, k = 20000, 50
    log(f"wide two-pass scan: N=2e5 T=1000 L={L} k={k} items={items}")
    h = _open(fb, ix, items=items, stats=1)
    got = fb.fbpq_debug_dists(h, Q[:4], L, cap=L)
    for r in range(4):
        pos, d32 = got[r]
        _, opos = oracle.visit(ix, Q[r], L)
        assert np.array_equal(np.sort(pos), np.sort(opos)), r
        d64 = oracle_dists(ix, Q[r], pos)
        err = np.abs(d32.astype(np.float64) - d64)
        assert np.all(err <= tol(ix, Q[r], pos, d64)), r
    fb.fbpq_stats_read(h, reset=True)
    g_ids, g_d = fb.fbpq_search(h, Q[:12], L, k)
    st = fb.fbpq_stats_read(h)
    fb.fbpq_free_index(h)
    log(f"  counters {st}")
    assert st["two_pass"] >= 12
    o_ids, o_d, _, _ = oracle.search(ix, Q[:12], L, k)
    assert_topk(ix, Q[:12], k, g_ids, g_d, o_ids, o_d)


# ---- local codebooks (HBPQ, Section 3.2) ----------------------------------------

def test_local_lossless_exact_knn(fb):
    # integer data: every table entry and distance is exact in FP32, so the
    # top-k equals the brute-force kNN of the raw vectors bit for bit
    ix = synth.lossless_local_index(N=3000, T=8, M=4, D=16, seed=13, dup=300)
    rng = np.random.default_rng(6)
    Q = ix.base[ix.ids[-rng.integers(1, 300, 8)]] + rng.integers(-1, 2, (8, 16)).astype(np.float32)
    k = 25
    log("local codebooks: lossless index, L >= N")
    h = _open(fb, ix, stats=1)
    g_ids, g_d = fb.fbpq_search(h, Q, ix.N + 10, k)
    assert fb.fbpq_stats_read(h)["two_pass"] >= Q.shape[0]
    fb.fbpq_free_index(h)
    X = ix.base.astype(np.float64)
    for r in range(Q.shape[0]):
        dd = ((X - Q[r].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.arange(ix.N), dd))[:k]
        assert np.array_equal(g_ids[r], order), r
        assert np.array_equal(g_d[r].astype(np.float64), dd[order]), r


@pytest.mark.parametrize("L", [1, 777, 10000, 250000])
def test_local_gmm_distances_and_topk(fb, gmm_small, L):
    ix, Q = gmm_small
    lix = synth.with_local_codebooks(ix)
    k = 20
    log(f"local codebooks: N=1e5 T=64 M=8 L={L}")
    h = _open(fb, lix)
    got = fb.fbpq_debug_dists(h, Q[:8], L, cap=min(L, lix.N))
    for r in range(8):
        pos, d32 = got[r]
        _, opos = oracle.visit(lix, Q[r], L)
        assert np.array_equal(np.sort(pos), np.sort(opos)), r
        d64 = oracle_dists(lix, Q[r], pos)
        err = np.abs(d32.astype(np.float64) - d64)
        assert np.all(err <= tol(lix, Q[r], pos, d64)), (r, float((err / tol(lix, Q[r], pos, d64)).max()))
    g_ids, g_d = fb.fbpq_search(h, Q[:40], L, k)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(lix, Q[:40], L, k)
    assert_topk(lix, Q[:40], k, g_ids, g_d, o_ids, o_d)


def test_local_long_rows_in_chunks(fb):
    # 16 cells of 1500 points over T = 4: a row holds 6000 candidates, cut
    # into tasks of 2048; the table of each task is folded by its wavefront
    ix = synth.with_local_codebooks(_dense_index(False), seed=5, scale=1.0)
    rng = np.random.default_rng(8)
    Q = rng.integers(0, 6, (16, 4)).astype(np.float32)
    L, k = 20000, 50
    log("local codebooks: rows of 6000 candidates")
    h = _open(fb, ix)
    got = fb.fbpq_debug_dists(h, Q[:4], L, cap=ix.N)
    for r in range(4):
        pos, d32 = got[r]
        d64 = oracle_dists(ix, Q[r], pos)
        assert len(pos) == min(L, ix.N)
        assert np.all(np.abs(d32.astype(np.float64) - d64) <= tol(ix, Q[r], pos, d64)), r
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


# ---- the Multi-D-ADC baseline: explicit O(D) reconstruction on the GPU -----------

@pytest.mark.parametrize("which,L", [("small", 777), ("small", 10000), ("m16", 5000)])
def test_adc_od_baseline_matches_oracle(fb, gmm_small, gmm_m16, which, L):
    ix, Q = gmm_small if which == "small" else gmm_m16
    k = 20
    log(f"O(D) baseline: {which} L={L}")
    h = _open(fb, ix, adc_od=1, stats=1)
    got = fb.fbpq_debug_dists(h, Q[:6], L, cap=min(L, ix.N))
    for r in range(6):
        pos, d32 = got[r]
        _, opos = oracle.visit(ix, Q[r], L)
        assert np.array_equal(np.sort(pos), np.sort(opos)), r
        d64 = oracle_dists(ix, Q[r], pos)
        assert np.all(np.abs(d32.astype(np.float64) - d64) <= tol(ix, Q[r], pos, d64)), r
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    assert fb.fbpq_stats_read(h)["two_pass"] >= Q.shape[0]
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


# ---- D = 384, the GIST-like width: wider halves, the same code length -------------

@pytest.fixture(scope="module")
def gmm_d384():
    # 40k mixture points of D = 384 with T = 256 per half and M = 8 (48
    # coordinates per subspace): the half keys take the multi-slab path (D/2 =
    # 192 coordinates), the prefixes the wavefront select, and the O(D) scan
    # reads its codebooks from memory (one half of them is 196 KB, beyond LDS)
    means = synth.gmm_means(0, D=384)
    base = synth.sample_points(40000, means, 1)
    ix = synth.build_index(base, 256, 8, train_n=10000)
    Q = synth.make_queries(30, means, 2)
    return ix, Q


@pytest.mark.parametrize("P", [64, 200])
def test_d384_rank_prefix_bitexact(fb, gmm_d384, P):
    ix, Q = gmm_d384
    log(f"rank prefix: D=384 T=256 P={P}")
    h = _open(fb, ix, stats=1)
    keys, idx = fb.fbpq_debug_rank(h, Q, P)
    st = fb.fbpq_stats_read(h)
    fb.fbpq_free_index(h)
    assert st["prefix_wave"] > 0
    for r in range(Q.shape[0]):
        d1, d2, u, v = oracle.rank_lists(ix, Q[r])
        assert np.array_equal(idx[r, 0], u[:P]) and np.array_equal(idx[r, 1], v[:P]), r
        assert np.array_equal(keys[r, 0], d1[u[:P]]) and np.array_equal(keys[r, 1], d2[v[:P]]), r


@pytest.mark.parametrize("adc_od,L", [(0, 3000), (0, 20000), (1, 3000), (1, 20000)])
def test_d384_search_matches_oracle(fb, gmm_d384, adc_od, L):
    ix, Q = gmm_d384
    k = 20
    log(f"D=384 search: adc_od={adc_od} L={L}")
    h = _open(fb, ix, adc_od=adc_od)
    got = fb.fbpq_debug_dists(h, Q[:6], L, cap=min(L, ix.N))
    for r in range(6):
        pos, d32 = got[r]
        _, opos = oracle.visit(ix, Q[r], L)
        assert np.array_equal(np.sort(pos), np.sort(opos)), r
        d64 = oracle_dists(ix, Q[r], pos)
        assert np.all(np.abs(d32.astype(np.float64) - d64) <= tol(ix, Q[r], pos, d64)), r
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


def test_d320_adc_od_uneven_groups(fb):
    # D = 320, M = 8: three of the four subspaces of a half fit in LDS at once,
    # so the O(D) scan takes each half in groups {0, 1, 2} and {3}
    means = synth.gmm_means(0, D=320)
    ix = synth.build_index(synth.sample_points(20000, means, 1), 64, 8, train_n=8000)
    Q = synth.make_queries(16, means, 2)
    L, k = 4000, 20
    log("O(D) baseline: D=320, uneven subspace groups")
    h = _open(fb, ix, adc_od=1)
    got = fb.fbpq_debug_dists(h, Q[:4], L, cap=L)
    for r in range(4):
        pos, d32 = got[r]
        d64 = oracle_dists(ix, Q[r], pos)
        assert len(pos) == L
        assert np.all(np.abs(d32.astype(np.float64) - d64) <= tol(ix, Q[r], pos, d64)), r
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


# ---- OPQ: queries rotated into the index's space ------------------------------

def _rotated(ix, Q, seed=23):
    # the index's space is the rotated one; queries arrive in the original
    # space, Q_orig = Rot^T Q (so that Rot Q_orig falls back near the data)
    import dataclasses
    Rot = synth.random_rotation(ix.D, seed=seed)
    Qo = (Q.astype(np.float64) @ Rot.astype(np.float64)).astype(np.float32)
    return dataclasses.replace(ix, Rot=Rot), Qo


@pytest.mark.parametrize("L", [777, 10000])
def test_rotation_prefix_visit_dists_topk(fb, gmm_small, L):
    ix0, Q0 = gmm_small
    ix, Q = _rotated(ix0, Q0[:30])
    Qr = oracle.rotate(ix.Rot, Q)  # the queries the index sees
    k = 20
    log(f"OPQ rotation: T=64 D=128 L={L}")
    h = _open(fb, ix)
    keys, idx = fb.fbpq_debug_rank(h, Q[:10], 64)
    for r in range(10):
        d1, d2, u, v = oracle.rank_lists(ix, Q[r])
        assert np.array_equal(idx[r, 0], u[:64]) and np.array_equal(idx[r, 1], v[:64]), r
        assert np.array_equal(keys[r, 0], d1[u[:64]]) and np.array_equal(keys[r, 1], d2[v[:64]]), r
    _check_visit(fb, h, ix, Q[:6], L)
    got = fb.fbpq_debug_dists(h, Q[:6], L, cap=min(L, ix.N))
    for r in range(6):
        pos, d32 = got[r]
        d64 = oracle_dists(ix, Qr[r], pos)
        assert np.all(np.abs(d32.astype(np.float64) - d64) <= tol(ix, Qr[r], pos, d64)), r
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Qr, k, g_ids, g_d, o_ids, o_d)
    # device entry point with a captured first round: every replay sees the
    # rotated queries at the same address
    import torch
    fb.fbpq_set_option(h, "graph", 1)
    dev = torch.device("cuda:0")
    d_q = torch.from_numpy(Q).to(dev)
    Ls, ks = np.full(Q.shape[0], L, np.int64), np.full(Q.shape[0], k, np.int32)
    d_ids = torch.empty((Q.shape[0], k), dtype=torch.int64, device=dev)
    d_d = torch.empty((Q.shape[0], k), dtype=torch.float32, device=dev)
    for rep in range(3):  # the same buffers: the second and third calls replay
        d_ids.fill_(-7)
        d_d.zero_()
        fb.fbpq_search_device(h, d_q, Ls, ks, k, d_ids, d_d, torch.cuda.current_stream(dev))
        torch.cuda.synchronize()
        assert np.array_equal(d_ids.cpu().numpy(), g_ids), rep
        assert np.array_equal(d_d.cpu().numpy(), g_d), rep
    fb.fbpq_free_index(h)


def test_load_index_with_local_codebooks_and_rotation(fb, tmp_path):
    # the optional file sections reach the device: a file index searches bit
    # for bit like the same arrays given to fbpq_index_create, and both match
    # the oracle (local codebooks and an OPQ rotation together)
    import dataclasses
    base = synth.random_index(N=3000, T=16, M=4, D=16, seed=21)
    ix = dataclasses.replace(synth.with_local_codebooks(base, seed=8), Rot=synth.random_rotation(16, seed=9))
    path = str(tmp_path / "ix.bin")
    synth.write_index(path, ix)
    Q = np.random.default_rng(2).normal(0, 20, (12, 16)).astype(np.float32)
    L, k = 900, 10
    log("file index with local codebooks and a rotation")
    h1 = _open(fb, ix)
    a_ids, a_d = fb.fbpq_search(h1, Q, L, k)
    fb.fbpq_free_index(h1)
    h2 = fb.fbpq_load_index(path, 0)
    fb.fbpq_build_tables(h2)
    b_ids, b_d = fb.fbpq_search(h2, Q, L, k)
    fb.fbpq_free_index(h2)
    assert np.array_equal(a_ids, b_ids) and np.array_equal(a_d, b_d)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, oracle.rotate(ix.Rot, Q), k, b_ids, b_d, o_ids, o_d)


# ---- the selection fused into the cell scan and its fallbacks --------------------

def _dense_index(const_codes: bool):
    # 16 cells of 1500 points each: every query takes the cell scan
    ix = synth.tiny_index(4, np.full(16, 1500), M=2, D=4, seed=21)
    if const_codes:
        ix.codes[:] = 7  # every point of a cell at the same distance: ties far beyond the window
    return ix


@pytest.mark.parametrize("const_codes,k", [(False, 10), (False, 100), (False, 256), (False, 300),
                                           (False, 1024), (True, 10), (True, 100)])
def test_fused_topk_and_fallbacks(fb, const_codes, k):
    ix = _dense_index(const_codes)
    rng = np.random.default_rng(8)
    Q = rng.integers(0, 6, (24, 4)).astype(np.float32)
    L = 8000
    log(f"fused top-k: dense cells, const_codes={const_codes} k={k}")
    h = _open(fb, ix, stats=1)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    st = fb.fbpq_stats_read(h)
    fb.fbpq_free_index(h)
    log(f"  counters {st}")
    assert st["cell_scan"] == Q.shape[0] and st["two_pass"] == 0
    if k > 256:
        assert st["fused_topk"] == 0 and st["fused_rescan"] == 0  # k above the sample count: streamed
    else:
        # every query is either selected in the scan or scored again, streamed
        assert st["fused_topk"] + st["fused_rescan"] == Q.shape[0]
        if const_codes:
            assert st["fused_rescan"] > 0  # a whole cell ties at the bound: window overflow
        elif k <= 100:
            assert st["fused_topk"] > 0
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


@pytest.mark.parametrize("k,L", [(256, 30000), (100, 60000), (1, 20000)])
def test_window_compaction_and_bounds(fb, gmm_small, k, L):
    # k = 256 gives each wavefront's bound its loosest form (the largest of its
    # 64 samples), so the window passes half full and is compacted; long lists
    # take the bounds at growing intervals. Every query is either selected in
    # the scan or scored again, and the top-k equals the oracle's.
    ix, Q = gmm_small
    Q = Q[:24]
    log(f"window: N=1e5 T=64 M=8 nq=24 L={L} k={k}")
    h = _open(fb, ix, stats=1, items=1)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    st = fb.fbpq_stats_read(h)
    fb.fbpq_free_index(h)
    log(f"  counters {st}")
    assert st["fused_topk"] + st["fused_rescan"] == st["cell_scan"] == Q.shape[0]
    assert st["fused_topk"] > 0
    if k == 256:
        assert st["win_admitted"] > 512 * Q.shape[0]  # more than half a window per query
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


# ---- the full batched workload, in the launch configuration the benchmark times ---

def test_full_batched_10M_sampled(fb):
    import torch
    dev = torch.device("cuda:0")
    means = synth.gmm_means(0)
    base = synth.sample_points(10_000_000, means, 1, dev)
    ix = synth.build_index(base, 4096, 16, keep_base=False)
    del base
    nq, L, k = 10000, 10000, 100
    Q = synth.make_queries(nq, means, 2, dev)
    log(f"full batch: N={ix.N} T=4096 M=16 nq={nq} L={L} k={k}")
    h = _open(fb, ix, stats=1)
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, k, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, k, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    fb.fbpq_search_device(h, d_q, np.full(nq, L, np.int64), np.full(nq, k, np.int32), k, d_ids, d_d, stream)
    torch.cuda.synchronize()
    st = fb.fbpq_stats_read(h)
    log(f"  counters {st}")
    g_ids, g_d = d_ids.cpu().numpy(), d_d.cpu().numpy()
    sample = np.random.default_rng(17).choice(nq, 48, replace=False)
    _check_visit(fb, h, ix, Q[sample[:6]], L)
    fb.fbpq_free_index(h)
    assert st["prefix_wave"] + st["prefix_wg"] == 2 * nq
    assert st["cell_scan"] + st["two_pass"] == nq
    o_ids, o_d, _, _ = oracle.search(ix, Q[sample], L, k)
    assert_topk(ix, Q[sample], k, g_ids[sample], g_d[sample], o_ids, o_d)


# ---- graph capture of the first round -------------------------------------------

@pytest.mark.parametrize("T,min_replays", [(256, 3), (1000, 3)])
def test_graph_replays_match_eager(fb, gmm_wide, T, min_replays):
    # cells hold few points here: most queries need a retry round with a
    # longer prefix, whose larger buffers force one recapture
    import torch
    idxs, _ = gmm_wide
    ix = idxs[T]
    dev = torch.device("cuda:0")
    means = synth.gmm_means(0)
    nq, L, k = 64, 3000, 20
    log(f"graph replays: N=2e5 T={T} M=8 nq=64 L=3000 k=20")
    hg = _open(fb, ix, stats=1, graph=1)
    he = _open(fb, ix)
    d_q = torch.empty(nq, ix.D, dtype=torch.float32, device=dev)
    d_ids = torch.empty(nq, k, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, k, dtype=torch.float32, device=dev)
    e_ids = torch.empty_like(d_ids)
    e_d = torch.empty_like(d_d)
    Ls, ks = np.full(nq, L, np.int64), np.full(nq, k, np.int32)
    stream = torch.cuda.current_stream(dev)
    for rep in range(5):
        Q = synth.make_queries(nq, means, 100 + rep)
        d_q.copy_(torch.from_numpy(Q))
        fb.fbpq_search_device(hg, d_q, Ls, ks, k, d_ids, d_d, stream)
        # the program's own eager work between replays
        scratch = torch.randn(1 << 20, device=dev).sum()
        torch.cuda.synchronize()
        fb.fbpq_search_device(he, d_q, Ls, ks, k, e_ids, e_d, stream)
        torch.cuda.synchronize()
        assert torch.equal(d_ids, e_ids) and torch.equal(d_d, e_d), rep
        assert float(scratch) == float(scratch)
    st = fb.fbpq_stats_read(hg)
    fb.fbpq_free_index(hg)
    fb.fbpq_free_index(he)
    log(f"  counters {st}")
    assert st["graph_replays"] >= min_replays


def test_autotune_then_parity(fb, gmm_wide):
    import torch
    idxs, Q = gmm_wide
    ix = idxs[256]
    dev = torch.device("cuda:0")
    nq, L, k = Q.shape[0], 2000, 10
    log("autotune: N=2e5 T=256 M=8 nq=40 L=2000 k=10")
    h = _open(fb, ix)
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, k, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, k, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    choice = fb.fbpq_autotune(h, d_q, L, k, k, d_ids, d_d, stream, reps=2)
    log(f"  chosen {choice}")
    assert choice["prefix"] in (16, 32, 64, 128, 256) and choice["items"] in (0, 1) and choice["us_per_search"] > 0
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


@pytest.mark.timeout(400)
def test_full_uneven_100M_sampled(fb):
    """N = 1e8, T = 16384, M = 8, 2e4 queries, L log-uniform in [1e3, 1e5], k in {1, 10, 100}."""
    import torch
    dev = torch.device("cuda:0")
    means = synth.gmm_means(0)
    base = synth.sample_points(100_000_000, means, 1, dev)
    ix = synth.build_index(base, 16384, 8, keep_base=False)
    del base
    torch.cuda.empty_cache()
    nq, kmax = 20000, 100
    Q = synth.make_queries(nq, means, 2, dev)
    L, k = synth.draw_L_k(nq, 3)
    log(f"full uneven batch: N={ix.N} T=16384 M=8 nq={nq} mean L={L.mean():.0f}")
    h = _open(fb, ix, stats=1)
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, kmax, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, kmax, dtype=torch.float32, device=dev)
    fb.fbpq_search_device(h, d_q, L, k, kmax, d_ids, d_d, torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    st = fb.fbpq_stats_read(h)
    log(f"  counters {st}")
    g_ids, g_d = d_ids.cpu().numpy(), d_d.cpu().numpy()
    sample = np.random.default_rng(19).choice(nq, 24, replace=False)
    _check_visit(fb, h, ix, Q[sample[:4]], int(L[sample[:4]].max()))
    fb.fbpq_free_index(h)
    assert st["prefix_wave"] + st["prefix_wg"] == 2 * nq
    assert st["cell_scan"] + st["two_pass"] == nq
    o_ids, o_d, _, _ = oracle.search(ix, Q[sample], L[sample], k[sample], kmax=kmax)
    assert_topk(ix, Q[sample], k[sample], g_ids[sample], g_d[sample], o_ids, o_d)


# ---- served form ----------------------------------------------------------------

@pytest.mark.parametrize("rot", [False, True])
def test_server_continuous_batching(fb, gmm_small, rot):
    # rot: the index lives in a rotated space (OPQ) and the serving lanes share
    # its rotation; requests arrive in the original space
    import time
    ix, Q0 = gmm_small
    means = synth.gmm_means(0)
    nreq, kmax = (120 if rot else 300), 100
    Q = synth.make_queries(nreq, means, 7)
    if rot:
        ix, Q = _rotated(ix, Q)
    rng = np.random.default_rng(31)
    L = rng.integers(1, 30000, nreq)
    k = rng.choice([1, 10, 100], nreq).astype(np.int32)
    log(f"server: N=1e5 T=64 M=8, {nreq} requests, 2 lanes, batches of at most 64, rotation={rot}")
    h = _open(fb, ix)
    s = fb.fbpq_server_create(h, 64, 2, kmax)
    got = {}
    try:
        for i in range(nreq):
            fb.fbpq_server_submit(s, Q[i], int(L[i]), int(k[i]), i)
            if i % 50 == 49:
                time.sleep(0.002)  # arrivals in bursts
        deadline = time.time() + 60
        while len(got) < nreq and time.time() < deadline:
            tags, ids, d, times, st = fb.fbpq_server_poll(s, 128, kmax, wait_s=0.2)
            for j, t in enumerate(tags):
                assert st[j] == 0
                assert times[j, 0] <= times[j, 1] <= times[j, 2]
                got[int(t)] = (ids[j], d[j])
        pending, batches, batched = fb.fbpq_server_counts(s)
    finally:
        fb.fbpq_server_destroy(s)
        fb.fbpq_free_index(h)
    log(f"  {batches} batches for {batched} requests")
    assert len(got) == nreq and batched == nreq and pending == 0
    assert batches < nreq  # requests were batched together
    g_ids = np.stack([got[i][0] for i in range(nreq)])
    g_d = np.stack([got[i][1] for i in range(nreq)])
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k, kmax=kmax)
    assert_topk(ix, oracle.rotate(ix.Rot, Q) if rot else Q, k, g_ids, g_d, o_ids, o_d)


@pytest.fixture(scope="module")
def sparse_t8192():
    """3000 points in random cells of a T = 8192 multi-index (6.7e7 cells): a
    query with L = 50 visits about 1.3e6 cells, and most of them need more than
    4096 ranks of one half list (prefixes beyond what the LDS-resident
    traversal and layouts hold)."""
    ix = synth.random_index(N=3000, T=8192, M=4, D=16, seed=21)
    rng = np.random.default_rng(5)
    Q = (rng.random((8, 16)) * 100).astype(np.float32)
    return ix, Q


def _cut_needs_ranks(ix, q, L, P):
    """True when the oracle's traversal of q needs cells outside the P x P
    window of the sorted half lists: its last visited cell's key reaches the
    smallest key outside the window."""
    cells, _ = oracle.visit(ix, q, L, cells_cap=1 << 22)
    d1, d2, u, v = oracle.rank_lists(ix, q)
    last = int(cells[-1, 0])
    cut_key = d1[last // ix.T] + d2[last % ix.T]
    kb = min(d1[u[P - 1]] + d2[v[0]], d1[u[0]] + d2[v[P - 1]])
    return cut_key >= kb


def test_long_prefix_beyond_lds_visit_and_topk(fb, sparse_t8192):
    ix, Q = sparse_t8192
    L, k = 50, 10
    log(f"long prefix in HBM: N=3000 T=8192 M=4 L={L} (retry rounds up to P=8192)")
    need = [_cut_needs_ranks(ix, Q[r], L, 4096) for r in range(Q.shape[0])]
    log(f"  queries needing more than 4096 ranks: {sum(need)} of {len(need)}")
    assert sum(need) >= 2
    h = _open(fb, ix, stats=1)
    _check_visit(fb, h, ix, Q[:4], L, cap=1 << 22)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    st = fb.fbpq_stats_read(h)
    log(f"  counters {st}")
    fb.fbpq_free_index(h)
    assert st["retried"] > 0
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


@pytest.mark.parametrize("L", [1, 20, 200])
def test_full_prefix_in_hbm(fb, sparse_t8192, L):
    # P = T = 8192 from the first round: the complete sorted lists, every query
    # traversed by the long-prefix kernel
    ix, Q = sparse_t8192
    k = 10
    log(f"full prefix in HBM: N=3000 T=8192 P=8192 L={L}")
    h = _open(fb, ix, prefix=8192, stats=1)
    keys, idx = fb.fbpq_debug_rank(h, Q[:2], 8192)
    for r in range(2):
        d1, d2, u, v = oracle.rank_lists(ix, Q[r])
        assert np.array_equal(idx[r, 0], u) and np.array_equal(idx[r, 1], v), r
        assert np.array_equal(keys[r, 0], d1[u]) and np.array_equal(keys[r, 1], d2[v]), r
    if L <= 50:
        _check_visit(fb, h, ix, Q[:2], L, cap=1 << 22)
    g_ids, g_d = fb.fbpq_search(h, Q, L, k)
    st = fb.fbpq_stats_read(h)
    fb.fbpq_free_index(h)
    assert st["wide"] >= Q.shape[0]
    o_ids, o_d, _, _ = oracle.search(ix, Q, L, k)
    assert_topk(ix, Q, k, g_ids, g_d, o_ids, o_d)


def test_capacity_rows_contract(fb, sparse_t8192):
    """With the prefix capped at 4096 ranks, exactly the queries whose
    traversal needs a longer prefix end with (-2, NaN) and the search returns
    FBPQ_E_CAPACITY; every other row equals the oracle's."""
    ix, Q = sparse_t8192
    L, k, cap = 50, 10, 4096
    need = np.array([_cut_needs_ranks(ix, Q[r], L, cap) for r in range(Q.shape[0])])
    log(f"capacity contract: T=8192 prefix_cap={cap}, {int(need.sum())} of {need.size} queries over the cap")
    assert 0 < need.sum() < need.size
    h = _open(fb, ix, prefix_cap=cap)
    rc, g_ids, g_d = fb.fbpq_search_rc(h, Q, L, k)
    fb.fbpq_free_index(h)
    assert rc == fb.FBPQ_E_CAPACITY
    failed = np.all(g_ids == -2, axis=1)
    assert np.array_equal(failed, need)
    assert np.all(np.isnan(g_d[failed]))
    ok = ~failed
    o_ids, o_d, _, _ = oracle.search(ix, Q[ok], L, k)
    assert_topk(ix, Q[ok], k, g_ids[ok], g_d[ok], o_ids, o_d)


def _dev_search(fb, h, Q, L, k, kmax, Lmax=None, async_=False):
    import torch
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    nq = Q.shape[0]
    dq = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).to(dev)
    ids = torch.full((nq, kmax), -7, dtype=torch.int64, device=dev)
    d = torch.full((nq, kmax), -7.0, dtype=torch.float32, device=dev)
    if not async_:
        fb.fbpq_search_device(h, dq, L, k, kmax, ids, d, st)
        torch.cuda.synchronize()
        return ids.cpu().numpy(), d.cpu().numpy()
    pend = torch.full((2,), -1, dtype=torch.int32, device=dev)
    dL = torch.from_numpy(np.ascontiguousarray(L, np.int64)).to(dev)
    dk = torch.from_numpy(np.ascontiguousarray(k, np.int32)).to(dev)
    fb.fbpq_search_device_async(h, dq, dL, dk, Lmax, kmax, ids, d, pend, st)
    return ids, d, pend, (dq, dL, dk)


def test_async_entry_equals_blocking(fb, gmm_small):
    """Device budgets, no wait: the same rows as the blocking device entry, bit
    for bit; out-of-range budgets are clamped and counted."""
    import torch
    ix, Q = gmm_small
    nq, kmax, Lmax = Q.shape[0], 20, 20000
    rng = np.random.default_rng(12)
    L = rng.integers(1, Lmax + 1, nq).astype(np.int64)
    k = rng.integers(1, kmax + 1, nq).astype(np.int32)
    L[3], L[5], k[7] = 0, 50000, 30
    log("async device entry: N=1e5 T=64, 100 queries, 3 budgets out of range")
    h = _open(fb, ix)
    r_ids, r_d = _dev_search(fb, h, Q, np.clip(L, 1, Lmax), np.clip(k, 1, kmax), kmax)
    ids, d, pend, keep = _dev_search(fb, h, Q, L, k, kmax, Lmax, async_=True)
    torch.cuda.synchronize()
    p = pend.cpu().numpy()
    assert p[0] == 0 and p[1] == 3
    assert fb.fbpq_search_device_finish(h) == fb.FBPQ_OK
    assert np.array_equal(ids.cpu().numpy(), r_ids)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), r_d.view(np.uint32))
    fb.fbpq_free_index(h)


def test_async_entry_deeper_rounds(fb, sparse_t8192):
    """A first round that leaves queries for deeper traversal: d_pending says
    how many, and finish (or the next search) completes them on the stream."""
    import torch
    ix, Q = sparse_t8192
    L, k = np.full(8, 50, np.int64), np.full(8, 10, np.int32)
    log("async device entry with deeper rounds: T=8192, L=50")
    h = _open(fb, ix)
    r_ids, r_d = _dev_search(fb, h, Q, L, k, 10)
    for implicit in (False, True):
        ids, d, pend, keep = _dev_search(fb, h, Q, L, k, 10, 50, async_=True)
        torch.cuda.synchronize()
        assert pend.cpu().numpy()[0] > 0
        if implicit:
            _dev_search(fb, h, Q[:1], L[:1], k[:1], 10)  # the next search finishes the previous one first
        else:
            assert fb.fbpq_search_device_finish(h) == fb.FBPQ_OK
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), r_ids)
        assert np.array_equal(d.cpu().numpy().view(np.uint32), r_d.view(np.uint32))
    fb.fbpq_free_index(h)


@pytest.fixture(scope="module")
def gmm_dense():
    # 4e5 points in T = 64 per half: dense cells (the cell scan's queries)
    means = synth.gmm_means(0)
    base = synth.sample_points(400000, means, 1)
    ix = synth.build_index(base, 64, 8, train_n=20000)
    Q = synth.make_queries(300, means, 2)
    return ix, Q


def test_persistent_scan_bitexact(fb, gmm_dense):
    """Every tile size and workgroup shape of the persistent scan gives the
    per-query scan's rows bit for bit, on a batch of uneven budgets."""
    ix, Q = gmm_dense
    nq, kmax = Q.shape[0], 100
    L, k = synth.draw_L_k(nq, 3, 100, 100000, (1, 10, 100))
    log("persistent scan: N=4e5 T=64 M=8, 300 queries, L log-uniform in [1e2, 1e5], k in {1, 10, 100}")
    h = _open(fb, ix, stats=1)
    r_ids, r_d = _dev_search(fb, h, Q, L, k, kmax)
    assert fb.fbpq_stats_read(h, reset=True)["cell_scan"] > 0
    for tile in (64, 2048, 8192, 1 << 30):
        for w in (2, 4, 8):
            fb.fbpq_set_option(h, "persist", 1)
            fb.fbpq_set_option(h, "tile", tile)
            fb.fbpq_set_option(h, "pwaves", w)
            ids, d = _dev_search(fb, h, Q, L, k, kmax)
            assert np.array_equal(ids, r_ids), (tile, w)
            assert np.array_equal(d.view(np.uint32), r_d.view(np.uint32)), (tile, w)
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q[:60], L[:60], k[:60], kmax=kmax)
    assert_topk(ix, Q[:60], k[:60], r_ids[:60], r_d[:60], o_ids, o_d)


def test_autotune_cache(fb, gmm_dense, tmp_path):
    import torch
    ix, Q = gmm_dense
    dev = torch.device("cuda:0")
    nq, kmax = Q.shape[0], 100
    L, k = synth.draw_L_k(nq, 3, 100, 100000, (1, 10, 100))
    log("autotune with a cache: N=4e5 T=64 M=8, 300 queries")
    cache = str(tmp_path / "tune.jsonl")
    d_q = torch.from_numpy(Q).to(dev).contiguous()
    d_ids = torch.empty(nq, kmax, dtype=torch.int64, device=dev)
    d_d = torch.empty(nq, kmax, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream(dev)
    h = _open(fb, ix)
    first = fb.fbpq_autotune_cached(h, d_q, L, k, kmax, d_ids, d_d, st, cache, reps=2)
    fb.fbpq_free_index(h)
    h = _open(fb, ix)
    second = fb.fbpq_autotune_cached(h, d_q, L, k, kmax, d_ids, d_d, st, cache, reps=2)
    log(f"  tuned {first}, then {second}")
    assert not first["from_cache"] and second["from_cache"]
    for key in ("prefix", "items", "persist", "tile", "pwaves"):
        assert first[key] == second[key]
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and '"key": "D=128 T=64 M=8' in lines[0]
    ids, d = _dev_search(fb, h, Q, L, k, kmax)  # the tuned setting is on the handle
    fb.fbpq_free_index(h)
    o_ids, o_d, _, _ = oracle.search(ix, Q[:60], L[:60], k[:60], kmax=kmax)
    assert_topk(ix, Q[:60], k[:60], ids[:60], d[:60], o_ids, o_d)


def test_wide_scan_long_prefix(fb):
    """Far queries on a sparse Zipf-sized index (1e9 points over 16384^2 cells,
    M=8) at L = 1e5: the visited diagram spans more than 4096 rows or columns
    with about one point per cell, so the query takes the two-pass wide scan
    after the long-prefix traversal. Every candidate's distance and the top-k
    against the oracle (this case once scored from stale memory)."""
    import torch

    log("wide scan, long prefix: Zipf index N=1e9 T=16384 M=8, two far queries, L=100000")
    ix = synth.zipf_index(1_000_000_000, 16384, 8, device="cuda:0")
    torch.cuda.empty_cache()
    Q = synth.make_queries(160000, synth.gmm_means(0), 2)[[58183, 114151]]
    L, k = 100000, 10
    h = _open(fb, ix)
    try:
        o_ids, o_d, _, _ = oracle.search(ix, Q, np.full(2, L, np.int64), k)
        for r in range(2):
            cells, _ = oracle.visit(ix, Q[r], L, 1 << 20)
            rows = np.unique(cells[:, 0] // ix.T).size
            cols = np.unique(cells[:, 0] % ix.T).size
            log(f"query {r}: {len(cells)} cells, {rows} rows, {cols} columns")
            assert max(rows, cols) > 4096 and L < 128 * len(cells)
            (dp, dd), = fb.fbpq_debug_dists(h, Q[r:r + 1], L, L)
            assert dp.size == L
            od = oracle_dists(ix, Q[r], dp)
            bad = np.abs(dd.astype(np.float64) - od) > tol(ix, Q[r], dp, od)
            assert not bad.any(), f"query {r}: {int(bad.sum())} of {L} candidate distances off"
        g_ids, g_d = fb.fbpq_search_uneven(h, Q, np.full(2, L, np.int64), np.full(2, k, np.int32), k)
        for r in range(2):
            q = Q[r].astype(np.float64)
            # the distance tolerance of tests/parity.py with |x| bounded by |q| + sqrt(d)
            t = 1e-4 * o_d[r] + 1e-6 * (q @ q + (np.sqrt(q @ q) + np.sqrt(np.maximum(o_d[r], 0))) ** 2)
            assert np.all(np.abs(g_d[r].astype(np.float64) - o_d[r]) <= t)
            firm = o_d[r] < o_d[r][k - 1] - 2 * t[k - 1]
            assert set(o_ids[r][firm].tolist()) <= set(g_ids[r].tolist())
    finally:
        fb.fbpq_free_index(h)
        del ix
        torch.cuda.empty_cache()
