"""Scheduling logic of the serving loop, driven on the CPU by its fake
executor (every clock step takes a fixed time, no GPU work): FIFO admission
into slots, slot reuse, queue limits, latency accounting, statistics and
configuration errors."""
import ctypes
import time

import pytest

from paper_2003_01178_amd import crystal as cx

STEP_NS = 20_000_000          # 20 ms per clock step


def pred_plan(n_rows=1000, n_groups=1):
    """A valid template over fake (never dereferenced) column pointers."""
    q = cx.StarQueryC()
    q.cols[0] = 4096
    q.n_cols, q.n_rows, q.n_preds = 1, n_rows, 1
    q.preds[0] = cx.Pred(0, cx.Range(0, 0))
    q.agg, q.n_groups = cx.AGG_COUNT, n_groups
    return q


def wait_for(fn, timeout=10.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        if fn():
            return True
        time.sleep(0.002)
    return False


def test_fifo_admission_slot_reuse_and_queue_limit():
    srv = cx.Server([dict(plan=pred_plan(1000))], slots=1, segment_rows=256, max_queue=2, inflight=1,
                    fake_step_ns=STEP_NS)
    try:
        assert srv.stats()["n_segments"] == 4
        t1 = srv.submit(0, preds=[(0, 1)])
        assert wait_for(lambda: srv.stats()["admitted"] == 1)
        t2 = srv.submit(0, preds=[(0, 1)])
        t3 = srv.submit(0, preds=[(0, 1)])
        assert srv.submit(0, preds=[(0, 1)]) is None           # queue of two is full
        assert srv.stats()["rejected"] == 1
        lat = {}
        order = []

        def poll_all():
            for t in (t1, t2, t3):
                if t in lat:
                    continue
                done, res, ns = srv.poll(t, 0)
                if done:
                    lat[t] = ns
                    order.append(t)
                    assert res.tolist() == [0]
            return len(lat) == 3
        assert wait_for(poll_all, timeout=20)
        assert order == [t1, t2, t3]                             # one slot: strictly one after another
        cycle = 4 * STEP_NS
        assert lat[t1] >= 0.9 * cycle
        assert lat[t2] >= lat[t1] + 0.9 * cycle - 0.2 * cycle   # waited for the slot
        st = srv.stats()
        assert st["admitted"] == 3 and st["completed"] == 3 and st["queued"] == 0
        assert st["busy_slot_steps"] == 12
        with pytest.raises(cx.CrystalError):
            srv.poll(t1, 0)                                      # a ticket is released once read
    finally:
        srv.close()


def test_slots_run_concurrently_and_join_mid_cycle():
    srv = cx.Server([dict(plan=pred_plan(4096))], slots=4, segment_rows=1024, max_queue=64, inflight=1,
                    fake_step_ns=STEP_NS)
    try:
        a = srv.submit(0, preds=[(0, 1)])
        assert wait_for(lambda: srv.stats()["steps"] >= 2)     # a is half way through its cycle
        b = srv.submit(0, preds=[(0, 1)])                      # joins mid-cycle
        res = {}

        def both():
            for t in (a, b):
                if t not in res:
                    done, _, ns = srv.poll(t, 0)
                    if done:
                        res[t] = ns
            return len(res) == 2
        assert wait_for(both, timeout=10)
        st = srv.stats()
        # b shared steps with a: fewer clock steps than two back-to-back cycles
        assert st["steps"] < 8
        assert st["busy_slot_steps"] == 8
    finally:
        srv.close()


def test_two_templates_and_many_queries():
    srv = cx.Server([dict(plan=pred_plan(2000)), dict(plan=pred_plan(2000, n_groups=3))], slots=16,
                    segment_rows=500, max_queue=1000, inflight=2, fake_step_ns=2_000_000)
    try:
        tickets = [(srv.submit(k % 2, preds=[(0, k)]), k % 2) for k in range(100)]
        assert all(t is not None for t, _ in tickets)
        done = set()

        def all_done():
            for t, tp in tickets:
                if t in done:
                    continue
                ok, res, _ = srv.poll(t, tp)
                if ok:
                    assert res.size == (1 if tp == 0 else 3)
                    done.add(t)
            return len(done) == len(tickets)
        assert wait_for(all_done, timeout=30)
        st = srv.stats()
        assert st["completed"] == 100 and st["admitted"] == 100
    finally:
        srv.close()


def test_invalid_configurations():
    lib = cx.load()
    for kw in [dict(segment_rows=250), dict(slots=17), dict(slots=0), dict(inflight=0)]:
        args = dict(slots=2, segment_rows=256, max_queue=4, inflight=1, fake_step_ns=STEP_NS)
        args.update(kw)
        with pytest.raises(cx.CrystalError) as e:
            cx.Server([dict(plan=pred_plan(1000))], **args)
        assert e.value.code == cx.EINVAL
    with pytest.raises(cx.CrystalError):                       # templates over different fact tables
        cx.Server([dict(plan=pred_plan(1000)), dict(plan=pred_plan(999))], slots=2, segment_rows=256,
                  max_queue=4, fake_step_ns=STEP_NS)
    srv = cx.Server([dict(plan=pred_plan(1000))], slots=2, segment_rows=256, max_queue=4, fake_step_ns=STEP_NS)
    try:
        with pytest.raises(cx.CrystalError):
            srv.submit(3, preds=[(0, 1)])                      # no such template
        with pytest.raises(cx.CrystalError):
            srv.poll(12345, 0)                                 # unknown ticket
    finally:
        srv.close()
    assert lib.crystal_server_create(None, None) == cx.EINVAL



def test_poll_capacity_is_checked_against_the_tickets_template():
    """The result size comes from the ticket's own template: a buffer sized
    for a smaller template is rejected (nothing copied, the ticket kept),
    and the binding sizes its buffer from the ticket."""
    srv = cx.Server([dict(plan=pred_plan(512, n_groups=7000)), dict(plan=pred_plan(512, n_groups=1))], slots=2,
                    segment_rows=256, max_queue=8, inflight=1, fake_step_ns=1_000_000)
    try:
        lib = cx.load()
        tk = srv.submit(0, preds=[(0, 1)])
        assert wait_for(lambda: srv.stats()["completed"] == 1)
        small = (ctypes.c_int64 * 1)()
        done, lat = ctypes.c_int32(), ctypes.c_int64()
        assert lib.crystal_server_poll(srv.h, tk, small, 1, ctypes.byref(done), ctypes.byref(lat)) == cx.EINVAL
        with pytest.raises(cx.CrystalError) as e:
            srv.poll(tk, 1)                                    # the other template's size: too small
        assert e.value.code == cx.EINVAL
        ok, res, ns = srv.poll(tk)                             # sized from the ticket: 7000 values
        assert ok and res.size == 7000 and ns > 0
        # released once read: the ticket is unknown now
        assert lib.crystal_server_poll(srv.h, tk, None, 0, ctypes.byref(done), ctypes.byref(lat)) == cx.EINVAL
    finally:
        srv.close()


def test_deadline_drops_queued_and_running_queries():
    """One slot, 4 segments of 20 ms: a running query whose deadline falls
    mid-cycle is dropped and frees its slot; a queued query that cannot get
    the slot before its deadline is dropped from the queue; both poll as
    CRYSTAL_ETIMEDOUT, and a query without a deadline behind them completes."""
    srv = cx.Server([dict(plan=pred_plan(1000))], slots=1, segment_rows=256, max_queue=8, inflight=1,
                    fake_step_ns=STEP_NS)
    try:
        a = srv.submit(0, preds=[(0, 1)], deadline_ns=int(2.5 * STEP_NS))    # times out while running
        b = srv.submit(0, preds=[(0, 1)], deadline_ns=int(1.5 * STEP_NS))    # times out in the queue
        c = srv.submit(0, preds=[(0, 1)])
        outcome = {}

        def poll_all():
            for t in (a, b, c):
                if t in outcome:
                    continue
                try:
                    done, res, ns = srv.poll(t)
                    if done:
                        outcome[t] = ("done", ns)
                except cx.CrystalError as e:
                    outcome[t] = (e.code, None)
            return len(outcome) == 3
        assert wait_for(poll_all, timeout=20)
        assert outcome[a][0] == cx.ETIMEDOUT
        assert outcome[b][0] == cx.ETIMEDOUT
        assert outcome[c][0] == "done"
        # c took the slot once a was dropped, not after a's full cycle
        assert outcome[c][1] < 4 * STEP_NS + 4 * STEP_NS
        st = srv.stats()
        assert st["timed_out"] == 2 and st["completed"] == 1 and st["admitted"] == 2
    finally:
        srv.close()


def test_cancel_queued_running_and_finished():
    srv = cx.Server([dict(plan=pred_plan(1000))], slots=1, segment_rows=256, max_queue=8, inflight=1,
                    fake_step_ns=STEP_NS)
    try:
        a = srv.submit(0, preds=[(0, 1)])
        b = srv.submit(0, preds=[(0, 1)])
        assert wait_for(lambda: srv.stats()["steps"] >= 1)          # a is running, b queued
        srv.cancel(b)                                               # queued
        srv.cancel(a)                                               # running: frees the slot
        d = srv.submit(0, preds=[(0, 1)])
        t0 = time.time()
        assert wait_for(lambda: srv.poll(d)[0], timeout=20)
        assert time.time() - t0 < 4 * 4 * STEP_NS / 1e9             # d did not wait for a's cycle
        e = srv.submit(0, preds=[(0, 1)])
        assert wait_for(lambda: srv.stats()["completed"] == 2, timeout=20)
        srv.cancel(e)                                               # finished, not polled: discarded
        for t in (a, b, e):
            with pytest.raises(cx.CrystalError) as err:
                srv.poll(t)
            assert err.value.code == cx.EINVAL                      # released
        with pytest.raises(cx.CrystalError):
            srv.cancel(12345)
        st = srv.stats()
        assert st["cancelled"] == 3 and st["completed"] == 2
    finally:
        srv.close()
