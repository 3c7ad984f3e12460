"""Scheduler logic of the serving loop on the CPU, through the C ABI with
the fake executor (no device work; each batch takes a modelled time per
work item).  Covers admission by budget, queue limits, first-come-first-
served order, batch splitting of large requests, the latency stamps, and
the failure path (a batch failed by injection fails only its requests and
releases their budget)."""
import os
import time

import pytest

from paper_2312_15073_amd import _lib as L

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="libmfa.so not built")

ADDR = 0x1000      # any non-null address: the fake executor never dereferences


def server(mfa, **kw):
    return mfa.Server(**kw)


@pytest.fixture(scope="module")
def mfa():
    import paper_2312_15073_amd as m
    return m


def test_budget_and_argument_errors(mfa):
    with server(mfa, hbm_budget_bytes=28 * 1000, queue_cap=4, fake_item_us=1.0) as s:
        mid = s.add_model(None)
        with pytest.raises(mfa.MFAError) as e:
            s.submit_points(mid, ADDR, ADDR, n=1001)          # 28,028 bytes > budget
        assert e.value.status == L.MFA_E_BUDGET
        with pytest.raises(mfa.MFAError) as e:
            s.submit_points(mid + 5, ADDR, ADDR, n=10)
        assert e.value.status == L.MFA_E_ARG
        with pytest.raises(mfa.MFAError) as e:
            s.submit_points(mid, ADDR, ADDR, n=0)
        assert e.value.status == L.MFA_E_ARG
        with pytest.raises(mfa.MFAError) as e:
            s.poll(12345)
        assert e.value.status == L.MFA_E_NOTFOUND


def test_queue_full_returns_busy(mfa):
    # one item per request at 20 ms: the queue fills faster than it drains
    with server(mfa, hbm_budget_bytes=1 << 30, queue_cap=3, max_batch_items=1,
                fake_item_us=20000.0) as s:
        mid = s.add_model(None)
        tickets, busy = [], 0
        for _ in range(12):
            try:
                tickets.append(s.submit_points(mid, ADDR, ADDR, n=10))
            except mfa.MFAError as e:
                assert e.status == L.MFA_E_BUSY
                busy += 1
        assert busy > 0
        for t in tickets:
            assert s.wait(t)["done"] == 1


def test_fifo_completion_and_stamps(mfa):
    with server(mfa, hbm_budget_bytes=1 << 30, queue_cap=256, max_batch_items=4,
                fake_item_us=200.0) as s:
        mid = s.add_model(None)
        tickets = [s.submit_points(mid, ADDR, ADDR, n=256 * (1 + k % 3)) for k in range(40)]
        st = [s.wait(t) for t in tickets]
    done = [x["t_done"] for x in st]
    assert done == sorted(done)                         # first come, first served
    for x in st:
        assert x["status"] == 0 and x["done"] == 1
        assert x["t_submit"] <= x["t_admit"] <= x["t_start"] <= x["t_done"]


def test_budget_limits_concurrent_admission(mfa):
    # each request needs 28 KB of a 60 KB budget: at most two admitted at once
    with server(mfa, hbm_budget_bytes=60_000, queue_cap=64, max_batch_items=64,
                fake_item_us=2000.0) as s:
        mid = s.add_model(None)
        tickets = [s.submit_points(mid, ADDR, ADDR, n=1000) for _ in range(6)]
        st = [s.wait(t) for t in tickets]
    for k in range(2, 6):
        assert st[k]["t_admit"] >= st[k - 2]["t_done"] - 1e-9


def test_large_request_is_split_across_batches(mfa):
    # a 64-item frame with 8-item batches, then a 1-item query behind it:
    # the query is admitted only after the frame but the frame spans 8 batches
    with server(mfa, hbm_budget_bytes=1 << 30, queue_cap=16, max_batch_items=8,
                fake_item_us=1000.0) as s:
        mid = s.add_model(None)
        t0 = time.perf_counter()
        big = s.submit_render(mid, None, None, 128, 128, ADDR)     # 8 x 8 tiles
        small = s.submit_points(mid, ADDR, ADDR, n=100)
        a, b = s.wait(big), s.wait(small)
        wall = time.perf_counter() - t0
    assert a["t_done"] - a["t_start"] >= 0.064 * 0.9           # 64 items x 1 ms
    assert b["t_done"] >= a["t_done"] - 0.002                  # shares the last batch at most
    assert wall < 5.0


def test_destroy_drains_queue(mfa):
    s = server(mfa, hbm_budget_bytes=1 << 30, queue_cap=64, fake_item_us=500.0)
    mid = s.add_model(None)
    tickets = [s.submit_points(mid, ADDR, ADDR, n=512) for _ in range(10)]
    s.close()                                                  # returns after all are done
    assert len(tickets) == 10


def test_failed_batch_fails_only_its_requests_and_releases_budget(mfa):
    # one-item requests, one item per batch: batch k holds request k.  The
    # second batch fails as a device error would: its request completes with
    # MFA_E_DEVICE, the requests before and after it complete normally (the
    # failure is not sticky), and its budget is released, which the last
    # request (needing the whole budget) shows by being admitted at all.
    budget = 28 * 256
    with server(mfa, hbm_budget_bytes=budget, queue_cap=16, max_batch_items=1,
                fake_item_us=500.0, fake_fail_batch=2) as s:
        mid = s.add_model(None)
        tickets = [s.submit_points(mid, ADDR, ADDR, n=100) for _ in range(4)]
        tickets.append(s.submit_points(mid, ADDR, ADDR, n=256))     # the whole budget
        stats = []
        for t in tickets:
            try:
                st = s.wait(t)
            except mfa.MFAError as e:
                assert e.status == L.MFA_E_DEVICE
                st = s.poll(t)
            stats.append(st)
    assert [x["done"] for x in stats] == [1] * 5
    assert [x["status"] for x in stats] == [0, L.MFA_E_DEVICE, 0, 0, 0]
    assert stats[4]["t_admit"] >= max(x["t_done"] for x in stats[:4]) - 1e-9


def test_failure_of_a_split_request_marks_the_whole_request(mfa):
    # a 9-item frame over 4-item batches spans batches 1..3; batch 2 fails:
    # the frame fails as a whole (its other batches succeed), the queries
    # queued behind it (batch 3 or later) succeed
    with server(mfa, hbm_budget_bytes=1 << 30, queue_cap=16, max_batch_items=4,
                fake_item_us=300.0, fake_fail_batch=2) as s:
        mid = s.add_model(None)
        frame = s.submit_render(mid, None, None, 48, 48, ADDR)      # 3 x 3 tiles
        q1 = s.submit_points(mid, ADDR, ADDR, n=200)
        with pytest.raises(mfa.MFAError) as e:
            s.wait(frame)
        assert e.value.status == L.MFA_E_DEVICE
        st = s.poll(frame)
        assert st["done"] == 1 and st["status"] == L.MFA_E_DEVICE
        assert s.wait(q1)["status"] == 0
        q2 = s.submit_points(mid, ADDR, ADDR, n=200)
        assert s.wait(q2)["status"] == 0
