"""Host logic of the serving loop on a virtual clock (no GPU).

Fake executors take a fixed time per request; the clock only moves when a
batch runs or the scheduler sleeps, so every latency, batch and deferral is
known exactly.
"""
import pytest

from paper_2102_03494_amd.serve import Request, Scheduler, percentile

pytestmark = pytest.mark.filterwarnings("ignore")


class Clock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExec:
    """A class's executor: one batch in flight, done `per_request * size` after it starts."""

    def __init__(self, clock, per_request, max_batch, budget_batch=None):
        self.clock, self.cost_per_request, self.max_batch = clock, per_request, max_batch
        self.budget_batch = budget_batch if budget_batch is not None else max_batch
        self.batches = []

    def fits(self, b):
        return b <= self.budget_batch

    def start(self, batch):
        self.batches.append([r.rid for r in batch])
        return self.clock.t + self.cost_per_request * len(batch)

    def done(self, end):
        return self.clock.t >= end - 1e-12


POLL = 1e-3


def _sched(execs, policy, clk, concurrent=False):
    return Scheduler(execs, policy, clk.now, clk.sleep, poll_s=POLL, concurrent=concurrent)


def test_percentile_interpolates():
    assert percentile([], 50) is None
    assert percentile([3.0], 99) == 3.0
    assert percentile([1.0, 2.0, 3.0, 4.0], 50) == 2.5
    assert abs(percentile(list(range(101)), 99) - 99.0) < 1e-12


def test_single_class_batches_and_latency():
    clk = Clock()
    ex = FakeExec(clk, 0.1, max_batch=2)
    reqs = [Request(i, "a", t) for i, t in enumerate([0.0, 0.0, 0.0, 0.5])]
    rep = _sched({"a": ex}, "fifo", clk).run(reqs, window_s=1.0, cap_s=10.0)
    # t=0: three waiting, batch of 2 (r0, r1) ends at 0.2; r2 deferred once;
    # then r2 alone ends at 0.3; sleep to 0.5; r3 ends at 0.6
    assert ex.batches == [[0, 1], [2], [3]]
    assert [r.t_done for r in reqs] == pytest.approx([0.2, 0.2, 0.3, 0.6], abs=2 * POLL)
    c = rep["classes"]["a"]
    assert c["completed"] == 4 and c["batches"] == 3 and c["deferrals"] == 1
    assert rep["peak_backlog"] == 3 and rep["backlog_at_end"] == 0
    assert c["p50_latency_s"] == pytest.approx(0.2, abs=2 * POLL)


def test_budget_limits_the_batch_and_counts_deferrals():
    clk = Clock()
    ex = FakeExec(clk, 0.01, max_batch=8, budget_batch=3)
    reqs = [Request(i, "a", 0.0) for i in range(7)]
    rep = _sched({"a": ex}, "sjf", clk).run(reqs, 1.0, 10.0)
    assert [len(b) for b in ex.batches] == [3, 3, 1]
    # 4 left waiting after the first batch, 1 after the second
    assert rep["classes"]["a"]["deferrals"] == 5


def test_concurrent_classes_run_side_by_side():
    """With concurrency a cheap class keeps completing while a long batch of another class is in flight."""
    for policy in ("sjf", "fifo"):
        clk = Clock()
        dear = FakeExec(clk, 5.0, max_batch=1)
        cheap = FakeExec(clk, 0.01, max_batch=4)
        reqs = [Request(0, "dear", 0.0)] + [Request(1 + i, "cheap", 0.5 * i) for i in range(6)]
        rep = _sched({"dear": dear, "cheap": cheap}, policy, clk, concurrent=True).run(reqs, 10.0, 100.0)
        assert reqs[0].t_done == pytest.approx(5.0, abs=2 * POLL)
        for r in reqs[1:]:
            assert r.t_done - r.t_arrival < 0.02, (policy, r.rid)
        assert rep["classes"]["cheap"]["p99_latency_s"] < 0.02
        assert rep["classes"]["dear"]["completed"] == 1


def test_sjf_starts_the_cheap_class_first():
    clk = Clock()
    order = []

    class Recorder(FakeExec):
        def start(self, batch):
            order.append(batch[0].cls)
            return super().start(batch)

    execs = {"dear": Recorder(clk, 1.0, 1), "cheap": Recorder(clk, 0.01, 4)}
    reqs = [Request(0, "dear", 0.0), Request(1, "cheap", 0.0)]
    _sched(execs, "sjf", clk).run(reqs, 1.0, 100.0)
    assert order == ["cheap", "dear"]
    order.clear()
    clk2 = Clock()
    for e in execs.values():
        e.clock = clk2
    _sched(execs, "fifo", clk2).run([Request(0, "dear", 0.0), Request(1, "cheap", 0.0)], 1.0, 100.0)
    assert order == ["dear", "cheap"]


def test_cap_reports_backlog_and_window_stops_admission():
    clk = Clock()
    ex = FakeExec(clk, 1.0, max_batch=1)
    reqs = [Request(i, "a", 0.1 * i) for i in range(10)] + [Request(99, "a", 5.0)]  # the last is after the window
    rep = _sched({"a": ex}, "fifo", clk).run(reqs, window_s=1.0, cap_s=3.0)
    c = rep["classes"]["a"]
    assert c["completed"] == 3
    assert rep["backlog_at_end"] == 7  # arrived inside the window, never served
    assert reqs[-1].t_done is None


def test_request_that_never_fits_is_rejected():
    clk = Clock()
    ex = FakeExec(clk, 0.1, max_batch=4, budget_batch=0)
    rep = _sched({"a": ex}, "fifo", clk).run([Request(0, "a", 0.0)], 1.0, 10.0)
    assert rep["rejected"] == 1 and rep["classes"]["a"]["completed"] == 0


def test_serial_mode_runs_one_batch_at_a_time():
    clk = Clock()
    dear = FakeExec(clk, 5.0, max_batch=1)
    cheap = FakeExec(clk, 0.01, max_batch=4)
    reqs = [Request(0, "dear", 0.0), Request(1, "cheap", 1.0)]
    _sched({"dear": dear, "cheap": cheap}, "sjf", clk).run(reqs, 10.0, 100.0)
    assert reqs[0].t_done == pytest.approx(5.0, abs=2 * POLL)
    assert reqs[1].t_done == pytest.approx(5.01, abs=3 * POLL)  # waited for the long batch


# ---- continuous batching (ContinuousServer) ------------------------------------
from paper_2102_03494_amd.serve import ContinuousServer  # noqa: E402


class FakeEngine:
    """An engine whose requests each need `steps` ticks; a tick advances every
    in-flight request by one step (up to `slots` in flight) and takes
    `tick_s` of device time after the previous tick of any engine."""

    def __init__(self, dev, steps, slots, tick_s):
        self.dev, self.steps, self.slots, self.tick_s = dev, steps, slots, tick_s
        self.waiting, self.flight = [], {}
        self.ticks = []

    def submit(self, r):
        self.waiting.append(r)

    def has_work(self):
        return bool(self.waiting or self.flight)

    def backlog(self):
        return len(self.waiting) + len(self.flight)

    def tick(self):
        while self.waiting and len(self.flight) < self.slots:
            r = self.waiting.pop(0)
            self.flight[r.rid] = [r, 0]
        if not self.flight:
            return None
        done = []
        for rid in list(self.flight):
            self.flight[rid][1] += 1
            if self.flight[rid][1] == self.steps:
                done.append(self.flight.pop(rid)[0])
        self.ticks.append(sorted(self.flight) + [x.rid for x in done])
        self.dev["busy_until"] = max(self.dev["busy_until"], self.dev["clock"].t) + self.tick_s
        return done


def _server(engines, clk, dev, ahead=1, order=None):
    return ContinuousServer(engines, lambda cls: dev["busy_until"], lambda tok: clk.t >= tok - 1e-12,
                            clk.now, clk.sleep, poll_s=POLL, ahead=ahead, order=order)


def test_continuous_admits_arrivals_into_running_work():
    """A request arriving while another is in flight joins at the next tick:
    both advance together, and the later one finishes `steps` ticks after it
    joined instead of after the first request's whole run."""
    clk = Clock()
    dev = {"busy_until": 0.0, "clock": clk}
    eng = FakeEngine(dev, steps=10, slots=8, tick_s=0.01)
    reqs = [Request(0, "a", 0.0), Request(1, "a", 0.035)]
    rep = _server({"a": eng}, clk, dev).run(reqs, window_s=1.0, cap_s=5.0)
    c = rep["classes"]["a"]
    assert c["completed"] == 2 and rep["backlog_at_end"] == 0
    # request 1 appears in a tick while request 0 is still in flight
    assert any(0 in t and 1 in t for t in eng.ticks)
    lat0, lat1 = reqs[0].t_done - reqs[0].t_arrival, reqs[1].t_done - reqs[1].t_arrival
    assert lat0 == pytest.approx(0.10, abs=3 * POLL)
    assert lat1 == pytest.approx(0.10, abs=0.01 + 3 * POLL)


def test_continuous_interleaves_classes_and_respects_slots():
    """Two classes alternate ticks (neither waits for the other's requests to
    finish), and at most `slots` requests of a class are in flight."""
    clk = Clock()
    dev = {"busy_until": 0.0, "clock": clk}
    short = FakeEngine(dev, steps=3, slots=2, tick_s=0.001)
    long_ = FakeEngine(dev, steps=50, slots=1, tick_s=0.004)
    reqs = [Request(i, "s", 0.002 * i) for i in range(5)] + [Request(100, "l", 0.0)]
    rep = _server({"s": short, "l": long_}, clk, dev, order=["s", "l"]).run(reqs, window_s=1.0, cap_s=5.0)
    assert rep["classes"]["s"]["completed"] == 5 and rep["classes"]["l"]["completed"] == 1
    assert max(len(t) for t in short.ticks) <= 2
    # every short request finishes before the long one
    assert max(r.t_done for r in reqs[:5]) < reqs[5].t_done
