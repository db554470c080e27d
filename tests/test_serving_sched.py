"""Host-side scheduling of the serving loop, driven by a scripted executor with a virtual
clock (a test double for admission/latency bookkeeping only; no simulation runs here)."""
import numpy as np
import pytest

from paper_1705_10045_amd import inputs as I
from paper_1705_10045_amd import serve


class FakeExecutor:
    """Slots and a byte budget like the pool; each run() advances every admitted request by
    `steps_per_run` steps and costs time proportional to the admitted node count."""

    def __init__(self, clock, slots=4, budget=10 ** 9, steps_per_run=100, ns_per_node=1.0):
        self.clock, self.slots, self.budget = clock, slots, budget
        self.spr, self.ns = steps_per_run, ns_per_node
        self.active = {}
        self.next = 1
        self.max_bytes = 0
        self.max_slots = 0

    @staticmethod
    def footprint(req):
        return 2 * 2 * 19 * req["edge"] ** 3 * 4

    def used(self):
        return sum(self.footprint(r) for r, _ in self.active.values())

    def submit(self, req):
        if len(self.active) >= self.slots or self.used() + self.footprint(req) > self.budget:
            return None
        t = self.next
        self.next += 1
        self.active[t] = (req, req["steps"])
        self.max_bytes = max(self.max_bytes, self.used())
        self.max_slots = max(self.max_slots, len(self.active))
        return t

    def run(self):
        work = sum(r["edge"] ** 3 for r, left in self.active.values() if left > 0)
        self.clock.t += work * self.spr * self.ns * 1e-9 + 1e-5
        for t, (r, left) in list(self.active.items()):
            self.active[t] = (r, max(0, left - self.spr))

    def poll(self, ticket):
        return self.active[ticket][1] == 0, 0

    def collect(self, ticket):
        self.active.pop(ticket)
        return None, 0


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def test_all_requests_complete_within_limits():
    reqs = I.serving_requests(64, steps_range=(100, 1000))
    clock = Clock()
    ex = FakeExecutor(clock, slots=8, budget=3 * 10 ** 9)
    arr = serve.poisson_arrivals(len(reqs), rate=50.0)
    rep = serve.serve(reqs, arr, ex, clock=clock, sleep=clock.sleep)
    assert rep["completed"] == 64 and rep["failed"] == 0
    assert ex.max_slots <= 8 and ex.max_bytes <= 3 * 10 ** 9
    assert rep["peak_in_flight"] <= 8
    # a request cannot finish before its own arrival plus its service rounds
    for i, r in enumerate(reqs):
        assert rep["latency_s"][i] > 0
    assert rep["p50_s"] <= rep["p99_s"]
    assert rep["node_updates"] == sum(r["edge"] ** 3 * r["steps"] for r in reqs)


def test_continuous_batching_admits_while_others_run():
    """Requests arriving while others are in flight are admitted at the next replay boundary,
    not after the batch drains."""
    reqs = [dict(id=i, edge=32, Tr=0.8, kind="droplet", steps=1000, seed=i, noise=0.01)
            for i in range(4)]
    clock = Clock()
    ex = FakeExecutor(clock, slots=4, steps_per_run=100)
    arr = np.array([0.0, 0.0, 0.001, 0.002])
    rep = serve.serve(reqs, arr, ex, clock=clock, sleep=clock.sleep)
    assert rep["peak_in_flight"] == 4
    # the late arrivals finish shortly after the first ones, not one full service time later
    lat = rep["latency_s"]
    assert max(lat) < 1.5 * min(lat[:2])


def test_admission_skips_requests_that_do_not_fit_yet():
    """First fit in arrival order: a large request that does not fit does not block smaller
    ones behind it; it is admitted once memory frees up."""
    big = dict(id=0, edge=128, Tr=0.8, kind="slab", steps=300, seed=1, noise=0.01)
    small = [dict(id=i, edge=32, Tr=0.8, kind="droplet", steps=300, seed=i, noise=0.01)
             for i in range(1, 5)]
    reqs = small[:1] + [big] + small[1:]
    clock = Clock()
    budget = FakeExecutor.footprint(big) + FakeExecutor.footprint(small[0]) - 1
    ex = FakeExecutor(clock, slots=8, budget=budget, steps_per_run=100)
    arr = np.zeros(len(reqs))
    rep = serve.serve(reqs, arr, ex, clock=clock, sleep=clock.sleep)
    assert rep["completed"] == 5
    # the big one had to wait for the small ones (it cannot share the budget with them)
    assert rep["latency_s"][1] > max(rep["latency_s"][i] for i in (0, 2, 3, 4))


def test_request_larger_than_pool_is_reported():
    reqs = [dict(id=0, edge=128, Tr=0.8, kind="slab", steps=100, seed=1, noise=0.01)]
    clock = Clock()
    ex = FakeExecutor(clock, budget=10 ** 6)
    with pytest.raises(RuntimeError):
        serve.serve(reqs, np.zeros(1), ex, clock=clock, sleep=clock.sleep)


def test_poisson_arrivals_rate_and_determinism():
    a = serve.poisson_arrivals(20000, rate=10.0, seed=3)
    assert a[0] == 0 and np.all(np.diff(a) >= 0)
    assert np.mean(np.diff(a)) == pytest.approx(0.1, rel=0.03)
    assert np.array_equal(a, serve.poisson_arrivals(20000, rate=10.0, seed=3))


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert serve.percentile(v, 50) == 50 and serve.percentile(v, 99) == 99
    assert serve.percentile([3.0], 99) == 3.0


class _FakePool:
    """Pool stand-in: a byte budget and slots, no device."""

    def __init__(self, budget, slots):
        self.budget, self.slots, self.used, self.next = budget, slots, 0, 1
        self.submitted = []

    def stats(self):
        return {"active": 0, "bytes_in_use": self.used, "budget": self.budget,
                "free_slots": self.slots}

    def submit(self, params, rho0, u0, T0, steps):
        need = serve.request_bytes_lower_bound(rho0.shape[0])
        if self.slots < 1 or self.budget - self.used < need:
            return None
        self.slots -= 1
        self.used += need
        self.submitted.append(rho0.shape[0])
        self.next += 1
        return self.next - 1


def test_pool_executor_declines_without_building_fields(monkeypatch):
    built = []
    real = I.request_fields

    def counting(req, params=None):
        built.append(req["id"])
        return real(req, params)

    monkeypatch.setattr(I, "request_fields", counting)
    small = dict(id=0, edge=8, Tr=0.8, kind="droplet", steps=3, seed=I.SEED + 1, noise=0.01)
    big = dict(id=1, edge=12, Tr=0.8, kind="slab", steps=3, seed=I.SEED + 2, noise=0.01)
    pool = _FakePool(budget=serve.request_bytes_lower_bound(8) + 10, slots=4)
    ex = serve.PoolExecutor(pool)
    assert ex.submit(big) is None and built == []      # cannot fit: fields never built
    assert ex.submit(small) == 1 and built == [0]
    assert ex.submit(small | {"id": 2}) is None and built == [0]
    pool.budget = 10 ** 9
    assert ex.submit(big) == 2 and built == [0, 1]
    assert pool.submitted == [8, 12]
