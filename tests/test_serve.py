"""CPU tests of the continuous-batching scheduler with a simulated device."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1501_02565_amd.serve import FakeExecutor, Request, Server, SimClock, percentile_ms


def _stream(n=300, seed=0, mean_gap=0.002):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(mean_gap, n))
    sizes = [(240, 320), (480, 640), (436, 1024), (1080, 1920)]
    out = []
    for i in range(n):
        H, W = sizes[rng.integers(0, len(sizes))]
        out.append(Request(i, float(t[i]), H, W, int(rng.integers(500, 5000)), 100))
    return out


def _serve(reqs, slots=2, budget=400 << 20, **kw):
    clk = SimClock()
    ex = FakeExecutor(clk, slots=slots, **kw)
    srv = Server(ex, budget, clock=clk, sleep=clk.sleep)
    return srv.run(reqs, t0=0.0), srv, ex


def test_every_request_served_in_arrival_order():
    reqs, srv, ex = _serve(_stream())
    assert all(r.status == "done" for r in reqs)
    adm = [r.admitted for r in sorted(reqs, key=lambda r: r.rid)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))          # FIFO admission
    for r in reqs:
        assert r.arrival <= r.admitted <= r.done


def test_batches_respect_the_slot_budget():
    reqs, srv, ex = _serve(_stream(), budget=100 << 20)
    by_batch = {}
    for r in reqs:
        if r.status == "done":
            by_batch.setdefault(r.batch, []).append(r)
    assert any(r.status == "rejected" for r in reqs)      # 1920x1080 > 50 MB
    for b in by_batch.values():
        assert sum(ex.request_bytes(r) for r in b) <= srv.slot_budget


def test_continuous_batching_admits_mid_flight_arrivals():
    """Under load, batches start while another is running, and requests
    that arrived during a batch are served by a later batch without waiting
    for the queue to drain."""
    reqs, srv, ex = _serve(_stream(400, mean_gap=0.0003), slots=2)
    assert srv.batches > 1
    assert srv.overlap_events > 0
    # mid-flight admission: a request that arrived while another batch was
    # running on the other slot was started before that batch ended (it did
    # not wait for the running work to drain)
    log = {b: (start, end, set(ids)) for b, (_, ids, start, end) in enumerate(ex.log)}
    mid = 0
    for r in reqs:
        if r.status != "done":
            continue
        start = log[r.batch][0]
        for s0, e0, ids0 in log.values():
            if r.rid not in ids0 and s0 < r.arrival < e0 and start < e0:
                mid += 1
                break
    assert mid > 0
    assert max(len(ids) for _, ids, _, _ in ex.log) > 1


def test_without_a_free_slot_arrivals_wait():
    """With one slot, a request that arrives while a batch runs starts only
    after that batch has finished (the check above is not vacuous)."""
    reqs, srv, ex = _serve(_stream(200, mean_gap=0.0003), slots=1)
    log = {b: (start, end) for b, (_, ids, start, end) in enumerate(ex.log)}
    for r in reqs:
        if r.status != "done":
            continue
        start = log[r.batch][0]
        for s0, e0 in log.values():
            if s0 < r.arrival < e0:
                assert start >= e0


def test_oversized_request_is_rejected():
    reqs = [Request(0, 0.0, 4000, 4000, 1000, 100), Request(1, 0.001, 240, 320, 500, 50)]
    out, srv, ex = _serve(reqs, budget=64 << 20)
    assert out[0].status == "rejected" and out[0].done is None
    assert out[1].status == "done"


def test_latency_percentiles():
    reqs, srv, ex = _serve(_stream())
    p50 = percentile_ms([r.latency for r in reqs], 50)
    p99 = percentile_ms([r.latency for r in reqs], 99)
    assert 0 < p50 <= p99


def test_executor_failure_propagates():
    class Boom(FakeExecutor):
        def submit(self, slot, reqs):
            raise RuntimeError("device failure")
    clk = SimClock()
    srv = Server(Boom(clk), 1 << 30, clock=clk, sleep=clk.sleep)
    with pytest.raises(RuntimeError, match="device failure"):
        srv.run(_stream(5), t0=0.0)
