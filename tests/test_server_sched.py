"""Scheduler of the served form on the host test backend (CPU only).

The server's lanes run a host backend here (fbpq_server_create2 with a null
index): a batch sleeps a fixed time per candidate and answers request (q, k)
with ids j + 1000 * round(q[0]) and distances q[1] + j. Batching, admission by
workspace, back-pressure, timeouts and cancellation are the code the GPU lanes
use. Each test checks that every request completes exactly once, with its own
result, and that the limits hold.
"""

import threading
import time

import numpy as np
import pytest

fb = pytest.importorskip("paper_1404_1831_amd.fbpq")

D, KMAX = 8, 10


def _q(tag):
    q = np.zeros(D, np.float32)
    q[0] = tag
    q[1] = 0.5 * tag
    return q


def _drain(s, want, timeout=30.0):
    got = {}
    t_end = time.time() + timeout
    while len(got) < want and time.time() < t_end:
        tags, ids, d, times, st = fb.fbpq_server_poll(s, 256, KMAX, wait_s=0.05)
        for i, t in enumerate(tags):
            assert int(t) not in got, f"request {t} completed twice"
            got[int(t)] = (ids[i].copy(), d[i].copy(), times[i].copy(), int(st[i]))
    return got


def _check_result(tag, k, res):
    ids, d, _, st = res
    assert st == fb.FBPQ_OK
    assert np.array_equal(ids[:k], 1000 * tag + np.arange(k))
    assert np.allclose(d[:k], 0.5 * tag + np.arange(k))
    assert np.all(ids[k:] == -1)


def test_concurrent_submit_and_poll_strand_nothing():
    """Submissions from one thread while another polls: each request finishes
    within a bound of its own batch time (a stranded request would wait for
    the poll deadline)."""
    s = fb.fbpq_server_create2(None, 16, 2, KMAX, D=D, fake_ns_per_cand=200.0)
    n = 150
    Ls = 1000 + (np.arange(n) * 7919) % 20000
    ks = 1 + np.arange(n) % KMAX
    try:
        def submit():
            for i in range(n):
                assert fb.fbpq_server_submit(s, _q(i), int(Ls[i]), int(ks[i]), i) == fb.FBPQ_OK
                time.sleep(0.002)

        th = threading.Thread(target=submit)
        th.start()
        got = _drain(s, n)
        th.join()
        assert len(got) == n
        for i in range(n):
            _check_result(i, int(ks[i]), got[i])
            t_sub, t_start, t_done = got[i][2]
            # one batch of at most 16 requests of at most 2^15 candidates takes < 0.11 s
            assert t_done - t_sub < 1.0, f"request {i} waited {t_done - t_sub:.2f} s"
        st = fb.fbpq_server_stats(s)
        assert st["submitted"] == n and st["completed"] == n and st["batched"] == n
    finally:
        fb.fbpq_server_destroy(s)


def test_batches_hold_one_budget_class_in_arrival_order():
    s = fb.fbpq_server_create2(None, 64, 1, KMAX, D=D, fake_ns_per_cand=20.0)
    try:
        # block the lane, then queue a mix of classes
        fb.fbpq_server_submit(s, _q(0), 2_000_000, 1, 0)
        time.sleep(0.01)
        Ls = [3000, 70000, 3500, 70000, 2100, 130000, 3900]
        for i, L in enumerate(Ls, start=1):
            fb.fbpq_server_submit(s, _q(i), L, 3, i)
        got = _drain(s, len(Ls) + 1)
        assert len(got) == len(Ls) + 1
        batch = {t: (r[2][1], r[2][2]) for t, r in got.items()}
        cls = {i: int(np.log2(L)) for i, L in enumerate(Ls, start=1)}
        for a in cls:
            for b in cls:
                if a < b:
                    assert (batch[a] == batch[b]) == (cls[a] == cls[b]), (a, b)
        # the oldest queued request's class runs first
        assert batch[1][0] <= min(batch[i][0] for i in cls)
    finally:
        fb.fbpq_server_destroy(s)


def test_workspace_budget_and_refusal():
    # reservation of the host backend: 64 B per candidate + 4096
    budget = 2 * (64 * 50_000 + 4096)
    s = fb.fbpq_server_create2(None, 32, 2, KMAX, D=D, ws_budget=budget, fake_ns_per_cand=50.0)
    try:
        lane = budget // 2
        # too large for a lane's share: refused, nothing queued
        assert fb.fbpq_server_submit(s, _q(999), 60_000, 2, 999) == fb.FBPQ_E_CAPACITY
        n = 40
        for i in range(n):
            assert fb.fbpq_server_submit(s, _q(i), 20_000 + 37 * i, 2, i) == fb.FBPQ_OK
        got = _drain(s, n)
        assert len(got) == n and 999 not in got
        for i in range(n):
            _check_result(i, 2, got[i])
        st = fb.fbpq_server_stats(s)
        assert st["rejected"] == 1
        assert st["lane_budget"] == lane
        assert 0 < st["peak_batch_reserved"] <= lane
        assert st["peak_reserved"] <= budget
        # a lane's share holds at most two such requests: batches of <= 2
        assert st["batches"] >= n // 2
    finally:
        fb.fbpq_server_destroy(s)


def test_back_pressure_refuses_over_max_pending():
    s = fb.fbpq_server_create2(None, 1, 1, KMAX, D=D, max_pending=4, fake_ns_per_cand=1000.0)
    try:
        assert fb.fbpq_server_submit(s, _q(0), 100_000, 1, 0) == fb.FBPQ_OK  # runs (0.1 s)
        time.sleep(0.02)
        rcs = [fb.fbpq_server_submit(s, _q(i), 10, 1, i) for i in range(1, 9)]
        assert rcs[:4] == [fb.FBPQ_OK] * 4
        assert rcs[4:] == [fb.FBPQ_E_CAPACITY] * 4
        got = _drain(s, 5)
        assert sorted(got) == [0, 1, 2, 3, 4]
        assert fb.fbpq_server_stats(s)["rejected"] == 4
    finally:
        fb.fbpq_server_destroy(s)


def test_timeout_and_cancel():
    s = fb.fbpq_server_create2(None, 1, 1, KMAX, D=D, timeout_s=0.15, fake_ns_per_cand=1000.0)
    try:
        assert fb.fbpq_server_submit(s, _q(0), 300_000, 1, 0) == fb.FBPQ_OK  # 0.3 s on the lane
        time.sleep(0.02)
        for i in range(1, 6):
            assert fb.fbpq_server_submit(s, _q(i), 10, 1, i) == fb.FBPQ_OK
        assert fb.fbpq_server_cancel(s, 3) == fb.FBPQ_OK
        assert fb.fbpq_server_cancel(s, 3) == fb.FBPQ_E_STATE  # no longer queued
        assert fb.fbpq_server_cancel(s, 12345) == fb.FBPQ_E_STATE
        got = _drain(s, 6)
        assert len(got) == 6
        assert got[0][3] == fb.FBPQ_OK
        assert got[3][3] == fb.FBPQ_E_CANCELLED
        for i in (1, 2, 4, 5):
            # queued behind a 0.3 s batch with a 0.15 s deadline: never searched
            assert got[i][3] == fb.FBPQ_E_TIMEOUT, (i, got[i][3])
            assert np.all(got[i][0] == -1)
            assert got[i][2][2] - got[i][2][0] < 0.25  # completed at the deadline, not after the batch
        st = fb.fbpq_server_stats(s)
        assert st["timeout"] == 4 and st["cancelled"] == 1 and st["completed"] == 1
    finally:
        fb.fbpq_server_destroy(s)


def test_destroy_finishes_queued_requests():
    s = fb.fbpq_server_create2(None, 4, 2, KMAX, D=D, fake_ns_per_cand=100.0)
    for i in range(20):
        fb.fbpq_server_submit(s, _q(i), 5000, 1, i)
    t0 = time.time()
    fb.fbpq_server_destroy(s)  # drains the queue, then joins the lanes
    assert time.time() - t0 < 10.0


def test_bad_configs():
    with pytest.raises(fb.FbpqError):
        fb.fbpq_server_create2(None, 4, 2, KMAX, D=D)  # no index and no test backend
    with pytest.raises(fb.FbpqError):
        fb.fbpq_server_create2(None, 0, 2, KMAX, D=D, fake_ns_per_cand=1.0)
    with pytest.raises(fb.FbpqError):
        fb.fbpq_server_create2(None, 4, 17, KMAX, D=D, fake_ns_per_cand=1.0)
