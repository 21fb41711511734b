"""Serving loop logic on the CPU with a fake executor: every request completes, the
HBM budget is never exceeded, waiting requests are admitted as slots free up, and
classes do not block each other."""
import pytest

from paper_2105_01612_amd.serve import Request, Server
from paper_2105_01612_amd import workload as wl


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5           # every poll advances time by 10 us
        return self.t


class FakeBackend:
    """Service time proportional to voxels; slot bytes 3 * 24 B per voxel."""

    def __init__(self, clock, rate=2e10):
        self.clock, self.rate = clock, rate
        self.created = 0
        self.destroyed = 0
        self.live = 0
        self.log = []

    def slot_bytes(self, n):
        return 3 * 24 * n ** 3

    def create(self, n):
        self.created += 1
        self.live += 1
        return {"n": n, "until": None}

    def submit(self, h, req):
        h["until"] = self.clock.t + req.n ** 3 / self.rate
        h["req"] = req
        self.log.append(("submit", req.rid, self.clock.t))

    def done(self, h):
        return h["until"] is not None and self.clock.t >= h["until"]

    def result(self, h):
        return h["req"].rid

    def destroy(self, h):
        self.destroyed += 1
        self.live -= 1


def make_requests(count, rate, sizes, seed=4000):
    arr = wl.poisson_arrivals(count, rate, seed)
    ns = wl.request_sizes(count, seed, sizes)
    return [Request(i, int(n), float(t), i % 2) for i, (t, n) in enumerate(zip(arr, ns))]


def test_all_complete_within_budget():
    clock = FakeClock()
    be = FakeBackend(clock)
    budget = 3 * 24 * (2 * 128 ** 3 + 2 * 64 ** 3)
    srv = Server(be, budget)
    reqs = make_requests(300, 2000.0, (32, 64, 128))
    seen = []
    stats = srv.run(reqs, clock=clock, on_complete=lambda r, res: seen.append((r.rid, res)))
    assert stats["completed"] == 300
    assert sorted(rid for rid, _ in seen) == list(range(300))
    assert all(rid == res for rid, res in seen)
    assert srv.peak_used <= budget
    for r in reqs:
        assert r.arrival <= r.admitted <= r.done
        assert r.done - r.admitted >= r.n ** 3 / be.rate - 1e-12
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_saturated_queue_drains_in_class_fifo_order():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = Server(be, 3 * 24 * 64 ** 3 * 2, max_slots_per_class=2)
    reqs = [Request(i, 64, 0.0) for i in range(20)]
    srv.run(reqs, clock=clock)
    order = [rid for kind, rid, _ in be.log if kind == "submit"]
    assert order == list(range(20))
    assert max(len(v) for v in srv.slots.values()) <= 2


def test_other_classes_are_not_blocked():
    """A big request that waits for budget does not stop small requests behind it."""
    clock = FakeClock()
    be = FakeBackend(clock, rate=1e9)
    budget = 3 * 24 * (128 ** 3 + 32 ** 3)
    srv = Server(be, budget)
    reqs = [Request(0, 128, 0.0), Request(1, 128, 0.0), Request(2, 32, 0.0), Request(3, 32, 0.0)]
    srv.run(reqs, clock=clock)
    assert reqs[2].done < reqs[1].admitted      # small ones finish while the second big one waits


def test_idle_slots_of_other_classes_are_evicted():
    clock = FakeClock()
    be = FakeBackend(clock)
    budget = 3 * 24 * 128 ** 3
    srv = Server(be, budget)
    reqs = [Request(0, 64, 0.0), Request(1, 128, 0.0005), Request(2, 64, 0.001)]
    srv.run(reqs, clock=clock)
    assert be.destroyed >= 1 and srv.peak_used <= budget


def test_request_larger_than_budget_is_refused():
    clock = FakeClock()
    srv = Server(FakeBackend(clock), 100)
    with pytest.raises(ValueError):
        srv.run([Request(0, 64, 0.0)], clock=clock)


@pytest.mark.parametrize("order", ["fifo", "sjf"])
def test_inflight_cap_is_respected(order):
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = Server(be, budget_bytes=10 ** 12, max_inflight=3, order=order)
    reqs = make_requests(300, 5e4, (16, 24, 32, 48))
    busy_max = {"n": 0}
    orig = be.submit

    def submit(h, r):
        orig(h, r)
        live = sum(1 for ss in srv.slots.values() for sl in ss if sl.req is not None)
        busy_max["n"] = max(busy_max["n"], live)

    be.submit = submit
    res = srv.run(reqs, clock=clock)
    assert res["completed"] == 300
    assert busy_max["n"] <= 3


def test_sjf_admits_smallest_first():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = Server(be, budget_bytes=10 ** 12, max_inflight=1, order="sjf")
    reqs = [Request(0, 48, 0.0), Request(1, 16, 0.0), Request(2, 32, 0.0)]
    srv.run(reqs, clock=clock)
    assert [rid for (what, rid, _) in be.log if what == "submit"] == [1, 2, 0]
