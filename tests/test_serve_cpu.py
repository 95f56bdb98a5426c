"""The streaming service's scheduler on the CPU, with a fake executor.

The fake executor keeps each stream's history on the host and computes a
tick's outputs with the CPU oracle after a simulated service time, so
admission, per-stream ordering, budget accounting, cancellation and failure
handling are tested without a GPU; the concatenated outputs of every stream
must still equal the oracle's one-shot transform of its concatenated input.
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1201_5380_amd import synth
from paper_1201_5380_amd.serve import CANCELLED, DONE, FAILED, REJECTED, Server


class FakePlan:
    def __init__(self, nchans, nbits, dms, dt=64e-6, f_top=1581.8):
        self.nchans, self.nbits = nchans, nbits
        self.df = -400.0 / nchans
        self.table, self.max_delay = oracle.delay_table(nchans, dt, f_top, self.df, dms)
        self.ndm = len(dms)
        self.row_bytes = nchans * nbits // 8


class FakeExecutor:
    def __init__(self, plans, service_s=0.002, fail_on=None):
        self.plans = plans
        self.hist = [np.zeros((0, p.row_bytes), np.uint8) for p in plans]
        self.service_s = service_s
        self.fail_on = fail_on or set()
        self.launched = []
        self.max_concurrent_bytes = 0

    def request_bytes(self, sid, nsamps):
        p = self.plans[sid]
        return nsamps * p.row_bytes + p.ndm * nsamps * 4

    def launch(self, reqs):
        ids = [r.stream_id for r in reqs]
        assert len(set(ids)) == len(ids), "a tick holds one chunk per stream"
        if any(r.seq in self.fail_on for r in reqs):
            raise RuntimeError("injected failure")
        self.launched.append([(r.stream_id, r.seq) for r in reqs])
        for r in reqs:
            p = self.plans[r.stream_id]
            x = np.concatenate([self.hist[r.stream_id], r.data])
            n = x.shape[0]
            if n > p.max_delay:
                r.out = oracle.dedisperse(x, n, p.nchans, p.nbits, p.table, p.max_delay)
                r.n_out = n - p.max_delay
                self.hist[r.stream_id] = x[n - p.max_delay:]
            else:
                r.out, r.n_out = None, 0
                self.hist[r.stream_id] = x
        ev = threading.Event()
        threading.Timer(self.service_s, ev.set).start()
        return ev

    @staticmethod
    def wait(handle):
        handle.wait()


def _plans():
    return [FakePlan(64, 8, synth.dm_list_linear(6, 60.0)),
            FakePlan(32, 2, synth.dm_list_linear(5, 200.0)),
            FakePlan(64, 8, synth.dm_list_linear(3, 10.0))]


def test_outputs_equal_one_shot_and_order_kept():
    plans = _plans()
    ex = FakeExecutor(plans)
    srv = Server(ex, len(plans), budget_bytes=10**9, max_tick=2).start()
    rng = np.random.default_rng(0)
    sent = [[] for _ in plans]
    reqs = []
    for k in range(40):
        sid = int(rng.integers(0, len(plans)))
        p = plans[sid]
        L = int(rng.integers(1, 2 * p.max_delay + 50))
        maxc = 255 if p.nbits == 8 else 3
        codes = rng.integers(0, maxc + 1, size=(L, p.nchans), dtype=np.uint8)
        data = synth.pack(codes, p.nbits).reshape(L, p.row_bytes)
        sent[sid].append(data)
        reqs.append(srv.submit(sid, data))
        if k % 7 == 0:
            time.sleep(0.003)
    srv.drain(timeout=30)
    srv.stop()
    assert all(r.status == DONE for r in reqs)
    for sid, p in enumerate(plans):
        mine = [r for r in reqs if r.stream_id == sid]
        assert [r.seq for r in mine] == list(range(len(mine)))
        # per-stream launch order follows sequence numbers
        order = [seq for tick in ex.launched for (s, seq) in tick if s == sid]
        assert order == sorted(order)
        outs = [r.out[:, : r.n_out] for r in mine if r.n_out]
        x = np.concatenate(sent[sid])
        want = oracle.dedisperse(x, x.shape[0], p.nchans, p.nbits, p.table, p.max_delay)
        assert np.array_equal(np.concatenate(outs, axis=1), want)
    st = srv.stats()
    assert st["requests_done"] == 40 and st["ticks"] >= 20 and st["mean_tick_size"] <= 2


def test_budget_never_exceeded_and_requests_wait():
    plans = _plans()
    ex = FakeExecutor(plans, service_s=0.02)
    one = ex.request_bytes(0, 100)
    srv = Server(ex, len(plans), budget_bytes=2 * one + 1, max_tick=4).start()
    data = np.zeros((100, plans[0].row_bytes), np.uint8)
    reqs = [srv.submit(0, data) for _ in range(6)]
    srv.drain(timeout=30)
    srv.stop()
    assert all(r.status == DONE for r in reqs)
    assert srv.peak_used <= 2 * one + 1
    assert srv.used == 0


class ResidentExecutor(FakeExecutor):
    """A fake executor whose streams hold device memory between requests."""

    def __init__(self, plans, resident, **kw):
        super().__init__(plans, **kw)
        self.resident = resident

    def resident_bytes(self):
        return self.resident


def test_budget_counts_the_streams_resident_memory():
    """History and scratch the streams hold are charged before any request:
    with them, only one request fits where two would fit without."""
    plans = _plans()
    ex = ResidentExecutor(plans, resident=0, service_s=0.02)
    one = ex.request_bytes(0, 100)
    resident = one // 2
    ex.resident = resident
    srv = Server(ex, len(plans), budget_bytes=2 * one + 1, max_tick=4).start()
    assert srv.budget == 2 * one + 1 - resident
    data = np.zeros((100, plans[0].row_bytes), np.uint8)
    reqs = [srv.submit(0, data) for _ in range(2)] + [srv.submit(1, np.zeros((100, plans[1].row_bytes), np.uint8))]
    srv.drain(timeout=30)
    srv.stop()
    assert all(r.status == DONE for r in reqs)
    st = srv.stats()
    assert st["resident_bytes"] == resident
    assert st["peak_device_bytes"] == resident + srv.peak_used <= 2 * one + 1
    # two requests of stream 0 never ran side by side: one plus the resident bytes fill the budget
    assert srv.peak_used < 2 * one
    # a chunk that fits the whole budget but not what the streams leave is rejected
    srv2 = Server(ResidentExecutor(plans, resident=one), len(plans), budget_bytes=2 * one - 1)
    assert srv2.submit(0, data).status == REJECTED
    with pytest.raises(ValueError):
        Server(ResidentExecutor(plans, resident=10**6), len(plans), budget_bytes=10**6)


def test_rejections():
    plans = _plans()
    srv = Server(FakeExecutor(plans), len(plans), budget_bytes=10**6)
    d = np.zeros((10, plans[0].row_bytes), np.uint8)
    assert srv.submit(0, d, seq=3).status == REJECTED                     # out of order
    assert srv.submit(0, d.astype(np.int16)).status == REJECTED           # malformed
    assert srv.submit(0, np.zeros((0, plans[0].row_bytes), np.uint8)).status == REJECTED
    big = np.zeros((10**5, plans[0].row_bytes), np.uint8)
    r = srv.submit(0, big)
    assert r.status == REJECTED and "budget" in r.reason
    ok = srv.submit(0, d)
    assert ok.status == "queued" and ok.seq == 0
    assert srv.submit(0, d, seq=0).status == REJECTED                     # duplicate


def test_cancel_before_admission_and_failure_releases_memory():
    plans = _plans()
    ex = FakeExecutor(plans, fail_on={1})
    srv = Server(ex, len(plans), budget_bytes=10**9)
    d = np.zeros((20, plans[0].row_bytes), np.uint8)
    a = srv.submit(0, d)
    b = srv.submit(0, d)
    c = srv.submit(0, d)
    assert srv.cancel(c)
    srv.start()
    srv.drain(timeout=30)
    srv.stop()
    assert a.status == DONE and b.status == FAILED and c.status == CANCELLED
    assert srv.used == 0 and not srv.cancel(a)
    st = srv.stats()
    assert st["failed"] == 1 and st["cancelled"] == 1


def test_on_done_sees_every_request_before_drain_returns():
    """The completion callback runs once per finished request, before the
    request's done event and before drain() returns; a consumer may drop the
    output there."""
    plans = _plans()
    ex = FakeExecutor(plans, service_s=0.01)
    seen = []

    def consume(r):
        assert not r.done.is_set() and r.status == DONE
        assert (r.out is not None) == (r.n_out > 0)
        seen.append((r.stream_id, r.seq, r.n_out))
        r.out = None
        if r.seq == 1 and r.stream_id == 0:
            raise RuntimeError("consumer failure")

    srv = Server(ex, len(plans), budget_bytes=10**9, max_tick=2, on_done=consume).start()
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(12):
        sid = i % len(plans)
        n = int(rng.integers(20, 60))
        reqs.append(srv.submit(sid, np.zeros((n, plans[sid].row_bytes), np.uint8)))
    srv.drain(timeout=30)
    srv.stop()
    assert sorted(seen) == sorted((r.stream_id, r.seq, r.n_out) for r in reqs)
    assert all(r.status == DONE and r.out is None and r.done.is_set() for r in reqs)
    # a raising consumer is recorded and the server keeps going
    assert [(r.stream_id, r.seq) for r, _ in srv.callback_errors] == [(0, 1)]
