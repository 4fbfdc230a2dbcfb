"""Host logic of the serving loop (arena, admission, continuous batching),
driven by a fake backend that lives only in this test."""
import pytest

from paper_2404_01159_amd.serve import Arena, Request, Server, latency_summary
from workloads import serving_specs


def test_arena_first_fit_alignment_and_merge():
    a = Arena(4096)
    x = a.alloc(100)
    y = a.alloc(300)
    z = a.alloc(256)
    assert (x, y, z) == (0, 256, 768)
    assert a.alloc(4096) is None
    a.release(y)
    assert a.alloc(512) == 256  # first fit reuses the hole
    a.release(x)
    a.release(256)
    a.release(z)
    assert a.free == [(0, 4096)] and a.in_use == 0


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Counts generations per run; each step costs `tick` seconds."""

    def __init__(self, clock, tick=0.001):
        self.clock, self.tick = clock, tick
        self.active = set()
        self.gens = {}
        self.max_seen = 0
        self.admit_order = []

    def footprint(self, req):
        return req.K * req.d * 8

    def create(self, req, off, nb):
        return req.rid

    def admit(self, run):
        self.active.add(run)
        self.gens[run] = 0
        self.admit_order.append(run)
        self.max_seen = max(self.max_seen, len(self.active))

    def retire(self, run):
        self.active.remove(run)

    def step(self):
        for r in self.active:
            self.gens[r] += 1
        self.clock.t += self.tick


def reqs(n, rate, gens=10, seed=0):
    return [Request(s["rid"], s["arrival"], s["problem"], s["m"], s["d"], s["N"], s["K"],
                    s["seed"], gens) for s in serving_specs(n, rate, seed, gens)]


def test_every_request_completes_within_budget_and_slots():
    clock = FakeClock()
    be = FakeBackend(clock)
    rs = reqs(40, rate=200.0)
    budget = max(r.K * r.d * 8 for r in rs) * 3
    srv = Server(be, budget, max_runs=5)
    res = srv.serve(rs, clock=clock, sleep=clock.sleep)
    assert sorted(r.rid for r in res) == list(range(40))
    assert all(be.gens[r] == 10 for r in range(40))
    assert be.max_seen <= 5 and srv.peak_runs <= 5
    assert srv.arena.in_use == 0
    # arrival order is kept at admission
    assert be.admit_order == sorted(be.admit_order, key=lambda i: (rs[i].arrival, i))
    for r in res:
        assert r.admitted >= r.arrival - 1e-12
        assert r.latency >= 10 * be.tick - 1e-12
    s = latency_summary(res)
    assert s["runs"] == 40 and s["p99_s"] >= s["p50_s"] > 0


def test_memory_pressure_queues_requests():
    clock = FakeClock()
    be = FakeBackend(clock)
    rs = reqs(20, rate=0.0)  # all at t = 0
    big = max(r.K * r.d * 8 for r in rs)
    srv = Server(be, big + 512, max_runs=64)
    res = srv.serve(rs, clock=clock, sleep=clock.sleep)
    assert len(res) == 20
    assert be.max_seen < 20  # the budget forced queueing


def test_multi_tick_steps_keep_generation_counts():
    """A backend that takes several ticks per step gets them only once no
    request waits, never past a run's last generation."""
    clock = FakeClock()

    class MultiBackend(FakeBackend):
        multi_tick = True

        def __init__(self, clock):
            super().__init__(clock)
            self.steps = []

        def step(self, n=1):
            self.steps.append(n)
            for _ in range(n):
                super().step()

    be = MultiBackend(clock)
    rs = reqs(12, rate=0.0)
    for i, r in enumerate(rs):
        rs[i] = Request(r.rid, r.arrival, r.problem, r.m, r.d, r.N, r.K, r.seed, 5 + i % 4)
    big = max(r.K * r.d * 8 for r in rs)
    srv = Server(be, 64 * big, max_runs=64)
    res = srv.serve(rs, clock=clock, sleep=clock.sleep)
    assert sorted(r.rid for r in res) == list(range(12))
    assert all(be.gens[r.rid] == r.gens for r in rs)
    assert max(be.steps) > 1 and srv.ticks == sum(be.steps) == 8


def test_oversized_request_is_rejected():
    clock = FakeClock()
    rs = reqs(3, rate=0.0)
    with pytest.raises(ValueError):
        Server(FakeBackend(clock), 1024, max_runs=4).serve(rs, clock=clock, sleep=clock.sleep)


def test_serving_specs_shapes():
    specs = serving_specs(256, 20.0, seed=0)
    assert len(specs) == 256
    for s in specs:
        assert s["m"] in (2, 3, 5, 8) and 30 <= s["d"] <= 2000
        assert 100 <= s["K"] <= 10011 and s["N"] == s["K"] and s["problem"] in (1, 2, 3)
    arr = [s["arrival"] for s in specs]
    assert arr == sorted(arr) and 8 < arr[-1] < 18  # ~256 / 20 s
