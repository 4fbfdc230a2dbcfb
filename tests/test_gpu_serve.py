"""Served runs: continuous batching with memory-budget admission.  Every
generation a served run makes inside the serving loop is compared with the
oracle from the run's state before that tick, and each served run's final
state equals the same run advanced alone."""
import numpy as np
import pytest

from parity import check_generation, new_stats

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2404_01159_amd as P

    return P


def test_served_runs_equal_alone(P):
    # runs of every reproduction operator, served together
    from paper_2404_01159_amd.serve import DeviceBackend, Request, Server, latency_summary

    rng = np.random.default_rng(3)
    specs = [(1, 3, 40, 105, 105), (2, 2, 33, 60, 64), (3, 5, 64, 126, 126),
             (2, 8, 90, 120, 120), (1, 3, 300, 300, 300), (3, 2, 31, 200, 200)]
    ops = ["ga", "de", "ga", "pso", "cso", "ga", "rand", "ga"]
    reqs = []
    for i in range(12):
        pb, m, d, N, K = specs[i % len(specs)]
        reqs.append(Request(i, 0.004 * i, pb, m, d, N, K, seed=500 + i,
                            gens=int(rng.integers(8, 25)), op=ops[i % len(ops)]))
    foot = max(P.footprint(r.problem, r.m, r.d, r.N, r.K, P.default_params(r.op, t_max=100))
               for r in reqs)
    be = DeviceBackend(arena_bytes=3 * foot + 4096, max_runs=4, keep_state=True)
    srv = Server(be, 3 * foot + 4096, max_runs=4)
    res = srv.serve(reqs)
    assert sorted(r.rid for r in res) == list(range(12))
    assert srv.peak_runs <= 4
    s = latency_summary(res)
    assert s["p99_s"] >= s["p50_s"] > 0
    for r in reqs:
        alone = P.Run(r.problem, r.m, r.d, r.N, r.K, seed=r.seed,
                      params=P.default_params(r.op, t_max=100))
        alone.run(r.gens)
        a, b = alone.get_state(), be.states[r.rid]
        for k in ("X", "F", "valid", "V", "gamma", "t"):
            assert np.array_equal(a[k], b[k], equal_nan=True), (r.rid, k)
        alone.close()


def test_served_generations_match_oracle(P):
    """Runs admitted and retired by the serving loop (arrivals, a memory budget
    for two or three runs at a time): every tick, each resident run's
    generation is checked against the oracle stage by stage from its state
    before the tick."""
    import oracle as O

    from paper_2404_01159_amd.serve import DeviceBackend, Request, Server

    O.lib()

    class CheckedBackend(DeviceBackend):
        multi_tick = False  # checked tick by tick

        def __init__(self, *a, **kw):
            super().__init__(*a, **kw)
            self.live = {}
            self.stats = new_stats()
            self.per_run = {}

        def create(self, req, offset, nbytes):
            run = super().create(req, offset, nbytes)
            self.live[req.rid] = (run, self.params(req))
            return run

        def retire(self, run):
            self.live = {k: v for k, v in self.live.items() if v[0] is not run}
            super().retire(run)

        def step(self):
            before = {rid: run.get_state() for rid, (run, _) in self.live.items()}
            super().step()
            for rid, (run, prm) in self.live.items():
                check_generation(O, run, prm, before[rid], run.get_offspring(),
                                 run.get_selection(), run.get_state(), self.stats)
                self.per_run[rid] = self.per_run.get(rid, 0) + 1

    specs = [(1, 3, 40, 105, 105), (2, 2, 33, 60, 64), (3, 5, 64, 126, 126),
             (2, 8, 90, 120, 120), (1, 3, 300, 300, 300), (3, 2, 31, 200, 200)]
    reqs = [Request(i, 0.002 * i, *specs[i % len(specs)], seed=900 + i, gens=6 + (i % 4))
            for i in range(8)]
    foot = max(P.footprint(r.problem, r.m, r.d, r.N, r.K, P.default_params(t_max=100))
               for r in reqs)
    be = CheckedBackend(arena_bytes=3 * foot + 4096, max_runs=3, t_max=30)
    srv = Server(be, 3 * foot + 4096, max_runs=3)
    res = srv.serve(reqs)
    assert sorted(r.rid for r in res) == list(range(8))
    assert be.per_run == {r.rid: r.gens for r in reqs}
    st = be.stats
    assert st["straddles"] <= max(2, 1e-6 * st["genes"]), st
    assert st["near_ties"] <= max(1, 1e-4 * st["vectors"]), st
    assert st["adaptations"] >= 1
    print(f"served vs oracle: {st}")
