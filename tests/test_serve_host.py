"""Scheduler logic of the serving loop on the CPU, with a fake backend that
models slots, a byte budget and step progress (no GPU): FIFO admission by
footprint, requests wait while the budget is full, every request finishes
exactly once, latency is measured from arrival, the request stream is
seeded."""

import numpy as np

from paper_1812_05711_amd.serve import make_requests, serve


class FakeBackend:
    def __init__(self, budget, max_slots, bytes_per_node=164):
        self.budget, self.max_slots, self.bpn = budget, max_slots, bytes_per_node
        self.used = 0
        self.slots = {}
        self.admitted = []
        self.finished = []

    def footprint(self, req):
        return req["params"]["nx"] * req["params"]["ny"] * self.bpn

    def admit(self, req):
        fp = self.footprint(req)
        if len(self.slots) >= self.max_slots or self.used + fp > self.budget:
            return None
        slot = next(i for i in range(self.max_slots) if i not in self.slots)
        self.slots[slot] = [req, 0]
        self.used += fp
        self.admitted.append(req["id"])
        return slot

    def step(self, n):
        for s in self.slots.values():
            s[1] = min(s[0]["steps"], s[1] + n)

    def poll(self):
        return [k for k, (r, d) in self.slots.items() if d >= r["steps"]]

    def finish(self, slot, req):
        r, _ = self.slots.pop(slot)
        assert r is req
        self.used -= self.footprint(req)
        self.finished.append(req["id"])


class FakeClock:
    """Time advances by a fixed cost per batched chunk of steps."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def test_request_stream_is_seeded_and_shaped():
    a = make_requests(500, rate=50.0, seed=3)
    b = make_requests(500, rate=50.0, seed=3)
    assert [r["arrival"] for r in a] == [r["arrival"] for r in b]
    gaps = np.diff([0.0] + [r["arrival"] for r in a])
    assert abs(gaps.mean() - 1 / 50) < 0.004
    ny = np.array([r["params"]["ny"] for r in a])
    for size, w in zip((64, 128, 256, 512), (0.4, 0.3, 0.2, 0.1)):
        assert abs(np.mean(ny == size) - w) < 0.06
    assert {r["params"]["nx"] for r in a} <= {80, 160, 320, 625}


def test_fifo_admission_by_footprint_and_latency():
    reqs = make_requests(60, rate=200.0, seed=5, steps=300)
    clock = FakeClock()
    # budget for about two of the largest requests: forces queueing
    be = FakeBackend(budget=2 * 625 * 512 * 164, max_slots=8)

    class Timed:
        def __init__(self, inner):
            self.inner = inner

        def __getattr__(self, k):
            return getattr(self.inner, k)

        def step(self, n):
            self.inner.step(n)
            clock.t += 1e-2 * n / 100

    records, summary = serve(reqs, Timed(be), chunk=100, clock=clock, sleep=clock.sleep)
    assert sorted(r["id"] for r in records) == list(range(60))
    assert be.admitted == sorted(be.admitted)  # first come, first served
    assert be.used == 0 and not be.slots
    for r in records:
        assert r["latency"] >= 0 and r["admitted"] >= r["arrival"] and r["done"] >= r["admitted"]
    assert summary["max_queue"] > 0  # the budget made requests wait
    assert summary["requests"] == 60 and summary["p99_s"] >= summary["p50_s"] > 0


def test_request_larger_than_the_budget_is_refused():
    """A request whose footprint exceeds the whole budget can never be
    admitted: it is refused once nothing runs, and the loop still ends."""
    reqs = make_requests(12, rate=100.0, seed=7, steps=200)
    clock = FakeClock()
    big = max(reqs, key=lambda r: r["params"]["nx"] * r["params"]["ny"])
    be = FakeBackend(budget=be_bytes(big) - 1, max_slots=4)

    class Timed:
        def __init__(self, inner):
            self.inner = inner

        def __getattr__(self, k):
            return getattr(self.inner, k)

        def step(self, n):
            self.inner.step(n)
            clock.t += 1e-3 * n / 100

    records, summary = serve(reqs, Timed(be), chunk=100, clock=clock, sleep=clock.sleep, max_wall=1e3)
    too_big = sorted(r["id"] for r in reqs if be.footprint(r) > be.budget)
    assert too_big and summary["refused"] == too_big
    assert sorted(r["id"] for r in records) == sorted(set(range(12)) - set(too_big))
    assert be.used == 0 and not be.slots


def be_bytes(req, bytes_per_node=164):
    return req["params"]["nx"] * req["params"]["ny"] * bytes_per_node
