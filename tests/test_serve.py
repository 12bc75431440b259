"""Serving scheduler on a simulated device (CPU only)."""
import pytest

from paper_1401_7494_amd import serve, synth


class SimClock:
    """Deterministic clock: sleeping advances time."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def make(reqs, budget, max_inflight=8, rate=1e11):
    clk = SimClock()
    ex = serve.FakeExecutor(clk, rate_ups=rate)
    srv = serve.Server(ex, budget, max_inflight, clock=clk, sleep=clk.sleep)
    return srv.run(reqs), ex


def test_every_request_completes_once_and_in_budget():
    reqs = synth.poisson_requests(60, rate_per_s=20.0, seed=1405)
    rep, ex = make(reqs, budget=200 * serve.GIB)
    assert sorted(c.rid for c in rep.completed) == list(range(60))
    assert rep.peak_bytes <= 200 * serve.GIB
    assert all(c.done_s >= c.admitted_s >= c.arrival_s for c in rep.completed)
    s = rep.summary()
    assert s["p99_latency_ms"] >= s["p50_latency_ms"] > 0 and s["aggregate_gups"] > 0


def test_requests_overlap_when_memory_allows():
    reqs = [synth.Request(i, 0.0, 256, 124, "f32", i) for i in range(6)]
    rep, _ = make(reqs, budget=200 * serve.GIB, max_inflight=4)
    assert rep.peak_inflight == 4  # admitted together, not one by one


def test_budget_limits_concurrency_and_admits_as_memory_frees():
    ex_fp = serve.FakeExecutor(lambda: 0.0).footprint(synth.Request(0, 0.0, 512, 496, "f32", 0))
    reqs = [synth.Request(i, 0.0, 512, 496, "f32", i) for i in range(5)]
    rep, _ = make(reqs, budget=2 * ex_fp + 1, max_inflight=8)
    assert rep.peak_inflight == 2 and rep.peak_bytes <= 2 * ex_fp + 1
    # later requests were admitted when earlier ones finished, not at arrival
    adm = sorted(c.admitted_s for c in rep.completed)
    assert adm[2] > 0 and len(rep.completed) == 5


def test_small_requests_are_not_blocked_behind_a_large_one():
    big = serve.FakeExecutor(lambda: 0.0).footprint(synth.Request(0, 0.0, 512, 496, "f32", 0))
    reqs = [synth.Request(0, 0.0, 512, 496, "f32", 0),   # fills the budget
            synth.Request(1, 0.001, 512, 496, "f32", 1),  # must wait
            synth.Request(2, 0.002, 128, 124, "f16", 2)]  # small: fits beside the first
    small = serve.FakeExecutor(lambda: 0.0).footprint(reqs[2])
    rep, _ = make(reqs, budget=big + small + 1)
    by = {c.rid: c for c in rep.completed}
    assert by[2].admitted_s < by[1].admitted_s


def test_oversized_requests_are_rejected_not_queued_forever():
    reqs = [synth.Request(0, 0.0, 512, 496, "f32", 0), synth.Request(1, 0.0, 128, 124, "f32", 1)]
    rep, _ = make(reqs, budget=2 * serve.GIB)
    assert [r.rid for r in rep.rejected] == [0] and [c.rid for c in rep.completed] == [1]


@pytest.mark.parametrize("max_inflight", [1, 3])
def test_inflight_limit_is_respected(max_inflight):
    reqs = [synth.Request(i, 0.0, 128, 124, "f32", i) for i in range(7)]
    rep, _ = make(reqs, budget=200 * serve.GIB, max_inflight=max_inflight)
    assert rep.peak_inflight == max_inflight and len(rep.completed) == 7


def test_cancelled_requests_leave_the_queue_and_free_their_memory():
    fp = serve.FakeExecutor(lambda: 0.0).footprint(synth.Request(0, 0.0, 512, 496, "f32", 0))
    reqs = [synth.Request(0, 0.0, 512, 496, "f32", 0, cancel_s=0.01),  # running when withdrawn
            synth.Request(1, 0.0, 512, 496, "f32", 1, cancel_s=0.005),  # still waiting: never runs
            synth.Request(2, 0.0, 512, 496, "f32", 2)]
    # one fits at a time; each takes 512^3 * 496 / 1e11 = 0.67 s
    rep, ex = make(reqs, budget=fp + 1)
    assert [c.rid for c in rep.completed] == [2]
    how = {rid: where for rid, where, _ in rep.cancelled}
    assert how == {0: "inflight", 1: "waiting"}
    assert 1 not in ex.started and ex.discarded == [0]
    by = {c.rid: c for c in rep.completed}
    assert by[2].admitted_s < 0.1  # admitted once the cancelled request's memory was freed, not after 0.67 s
    assert rep.summary()["cancelled"] == 2


def test_cancel_from_outside_the_loop():
    clk = SimClock()
    ex = serve.FakeExecutor(clk, rate_ups=1e11)
    srv = serve.Server(ex, 200 * serve.GIB, 8, clock=clk, sleep=clk.sleep)
    reqs = [synth.Request(i, 0.0, 256, 124, "f32", i) for i in range(3)]
    srv.cancel(1)
    rep = srv.run(reqs)
    assert sorted(c.rid for c in rep.completed) == [0, 2]
    assert [rid for rid, _, _ in rep.cancelled] == [1]


def test_cancel_from_another_thread_while_serving():
    """Server.cancel from a second thread while run() is going (real clock): the withdrawn request
    never completes, every other one does."""
    import threading
    import time

    ex = serve.FakeExecutor(time.perf_counter, rate_ups=2e10)  # 256^3 x 124 views: ~0.1 s each
    srv = serve.Server(ex, 200 * serve.GIB, max_inflight=1)
    reqs = [synth.Request(i, 0.0, 256, 124, "f32", i) for i in range(4)]
    out = {}
    t = threading.Thread(target=lambda: out.setdefault("rep", srv.run(reqs)))
    t.start()
    time.sleep(0.02)
    srv.cancel(2)  # still waiting behind requests 0 and 1
    t.join(timeout=30)
    rep = out["rep"]
    assert sorted(c.rid for c in rep.completed) == [0, 1, 3]
    assert [(rid, where) for rid, where, _ in rep.cancelled] == [(2, "waiting")]
