"""The no-allocation search entry (fbpq_search_device_noalloc) against the
allocating one (fbpq_search_device), through the C ABI on the GPU.

Two calls in a row on the same handle, the second with a smaller batch (and
smaller L), each compared with fbpq_search_device on the same inputs; the
entry must also refuse a search larger than its scratch with FBPQ_E_CAPACITY.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fb():
    from paper_1404_1831_amd import fbpq  # raises if the library is not built
    return fbpq


@pytest.fixture(scope="module")
def small():
    means = synth.gmm_means(0)
    base = synth.sample_points(100000, means, 1)
    ix = synth.build_index(base, 64, 8)
    Q = synth.make_queries(100, means, 2)
    return ix, Q


def _run(fb, h, Q, L, k, kmax, noalloc):
    import torch
    dev = torch.device("cuda:0")
    dq = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).to(dev)
    ids = torch.full((Q.shape[0], kmax), -7, dtype=torch.int64, device=dev)
    d = torch.full((Q.shape[0], kmax), -7.0, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream()
    if noalloc:
        rc = fb.fbpq_search_device_noalloc(h, dq, L, k, kmax, ids, d, stream=st)
    else:
        fb.fbpq_search_device(h, dq, L, k, kmax, ids, d, stream=st)
        rc = fb.FBPQ_OK
    torch.cuda.synchronize()
    return rc, ids.cpu().numpy(), d.cpu().numpy()


def test_noalloc_matches_allocating_entry(fb, small):
    ix, Q = small
    h = fb.fbpq_index_create(ix, 0)
    fb.fbpq_build_tables(h)
    try:
        rng = np.random.default_rng(9)
        for nq, Lhi in ((100, 10000), (37, 3000)):  # the second call is smaller
            L = rng.integers(1, Lhi + 1, nq).astype(np.int64)
            k = rng.integers(1, 21, nq).astype(np.int32)
            print(f"no-alloc search: N=1e5 T=64 M=8 nq={nq} L<={Lhi}", flush=True)
            rc, g_ids, g_d = _run(fb, h, Q[:nq], L, k, 20, True)
            assert rc == fb.FBPQ_OK
            _, a_ids, a_d = _run(fb, h, Q[:nq], L, k, 20, False)
            assert np.array_equal(g_ids, a_ids)
            assert np.array_equal(g_d.view(np.uint32), a_d.view(np.uint32))
    finally:
        fb.fbpq_free_index(h)


def test_noalloc_refuses_over_scratch(fb, small):
    ix, Q = small
    h = fb.fbpq_index_create(ix, 0)
    fb.fbpq_build_tables(h)
    try:
        # 4000 queries at L = 10^5: distance rows alone need 1.6 GB
        Qb = np.repeat(Q, 40, axis=0)
        print("no-alloc search over the scratch limit: nq=4000 L=1e5", flush=True)
        rc, ids, _ = _run(fb, h, Qb, np.full(Qb.shape[0], 100000), np.full(Qb.shape[0], 10), 10, True)
        assert rc == fb.FBPQ_E_CAPACITY
        assert np.all(ids == -7)  # nothing written
        # the handle still searches normally afterwards
        rc, g_ids, _ = _run(fb, h, Q[:8], np.full(8, 500), np.full(8, 5), 5, True)
        assert rc == fb.FBPQ_OK and np.all(g_ids[:, 0] >= 0)
    finally:
        fb.fbpq_free_index(h)
