"""Served runs: continuous batching with memory-budget admission; each
served run's final state equals the same run advanced alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2404_01159_amd as P

    return P


def test_served_runs_equal_alone(P):
    from paper_2404_01159_amd.serve import DeviceBackend, Request, Server, latency_summary

    rng = np.random.default_rng(3)
    specs = [(1, 3, 40, 105, 105), (2, 2, 33, 60, 64), (3, 5, 64, 126, 126),
             (2, 8, 90, 120, 120), (1, 3, 300, 300, 300), (3, 2, 31, 200, 200)]
    reqs = []
    for i in range(12):
        pb, m, d, N, K = specs[i % len(specs)]
        reqs.append(Request(i, 0.004 * i, pb, m, d, N, K, seed=500 + i,
                            gens=int(rng.integers(8, 25))))
    foot = max(P.footprint(r.problem, r.m, r.d, r.N, r.K, P.default_params(t_max=100))
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
                      params=P.default_params(t_max=100))
        alone.run(r.gens)
        a, b = alone.get_state(), be.states[r.rid]
        for k in ("X", "F", "valid", "V", "gamma", "t"):
            assert np.array_equal(a[k], b[k], equal_nan=True), (r.rid, k)
        alone.close()
