"""Batched runs against the oracle, and alone == in the mix.

Runs of different problems, objective counts, dimensions and sizes are
advanced together by rvea_batch_step.  Every batched generation of every run
is compared with the oracle stage by stage from the run's state before the
batch step (Alg. 2, Appendix B, Alg. 1, adaptation), while runs join and
leave at different ticks, with captured graphs and with eager launches.  Each
run must also end bit-identical to the same run advanced alone.
"""
import numpy as np
import pytest

from parity import check_generation, new_stats

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPECS = [
    # problem, m, d, N, K, seed
    (1, 3, 40, 105, 105, 1),
    (2, 2, 31, 60, 64, 2),
    (3, 5, 130, 126, 126, 3),
    (1, 8, 300, 120, 120, 4),
    (2, 3, 700, 300, 300, 5),
    (3, 3, 12, 91, 91, 6),
    (1, 3, 2048, 100, 105, 7),  # long rows, few pairs: each pair split over segments
]


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2404_01159_amd as P

    return P


@pytest.fixture(scope="module")
def O():
    import oracle as O

    O.lib()
    return O


def make(P, spec, t_max=30):
    problem, m, d, N, K, seed = spec
    return P.Run(problem, m, d, N, K, seed=seed, params=P.default_params(t_max=t_max))


@pytest.mark.parametrize("graphs", [True, False])
def test_batched_generations_match_oracle(P, O, graphs):
    """Each batched generation of each run equals the oracle's generation
    from the run's state before the batch step; runs join at different ticks
    and leave after different numbers of generations."""
    prm = P.default_params(t_max=30)  # adaptation every 3 generations
    runs = [make(P, s) for s in SPECS]
    join_at = [0, 2, 0, 4, 1, 3, 2]
    gens = [10, 8, 11, 5, 9, 7, 6]
    batch = P.Batch(8)
    batch.set_graphs(graphs)
    stats = new_stats()
    done = [0] * len(runs)
    active = []
    tick = 0
    while any(done[i] < gens[i] for i in range(len(runs))):
        for i in range(len(runs)):
            if i not in active and done[i] == 0 and tick >= join_at[i]:
                batch.admit(runs[i])
                active.append(i)
        before = {i: runs[i].get_state() for i in active}
        batch.step()
        for i in active:
            r = runs[i]
            check_generation(O, r, prm, before[i], r.get_offspring(), r.get_selection(),
                             r.get_state(), stats)
            done[i] += 1
        for i in list(active):
            if done[i] == gens[i]:
                batch.retire(runs[i])
                active.remove(i)
        tick += 1
    assert stats["generations"] == sum(gens)
    assert stats["adaptations"] >= len(runs)
    assert stats["straddles"] <= max(2, 1e-6 * stats["genes"]), stats
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
    print(f"batched vs oracle (graphs={graphs}): {stats}")
    for r in runs:
        r.close()


def same(a, b):
    sa, sb = a.get_state(), b.get_state()
    for k in ("X", "F", "valid", "V", "gamma", "t"):
        if not np.array_equal(sa[k], sb[k], equal_nan=True):
            return k
    return None


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_equals_alone(P, graphs):
    G = 23
    alone = [make(P, s) for s in SPECS]
    for r in alone:
        r.run(G)
    mixed = [make(P, s) for s in SPECS]
    batch = P.Batch(16)
    batch.set_graphs(graphs)
    for r in mixed:
        batch.admit(r)
    batch.step(G)
    batch.synchronize()
    for a, b in zip(alone, mixed):
        assert same(a, b) is None, same(a, b)


def test_device_filling_batch_equals_alone(P):
    """A batch whose full-scan runs fill the device by themselves (here
    twenty-two 10,011-vector runs with the index switched off and two m = 5
    runs: over 2,048 association workgroups with wide chunks, and over 8 x
    2,048 gamma blocks) associates with wide vector chunks and gives the
    gamma passes their own chunking and eight blocks per workgroup: every
    run still ends bit-identical to the same run alone (own chunking),
    adaptations included."""
    G = 12  # an adaptation at generation 10
    specs = [(1 + i % 3, 3, 12, 10011, 10011, 40 + i) for i in range(22)]
    specs += [(2, 5, 30, 3876, 3876, 60), (3, 5, 20, 3000, 3060, 61)]

    def build():
        out = []
        for pb, m, d, N, K, seed in specs:
            r = P.Run(pb, m, d, N, K, seed=seed, params=P.default_params(t_max=100))
            if m == 3:
                r.set_index(False)
            out.append(r)
        return out

    alone = build()
    for r in alone:
        r.run(G)
    mixed = build()
    batch = P.Batch(32)
    for r in mixed:
        batch.admit(r)
    print("device-filling batch", flush=True)
    batch.step(G)
    batch.synchronize()
    for a, b in zip(alone, mixed):
        assert same(a, b) is None, same(a, b)
    for r in mixed:
        batch.retire(r)
    batch.close()
    for r in alone + mixed:
        r.close()


def test_staggered_join_and_leave(P):
    """Runs join at different generations, leave early, and the single-run
    path continues them afterwards."""
    alone = [make(P, s) for s in SPECS]
    mixed = [make(P, s) for s in SPECS]
    gens = [20, 15, 25, 9, 17, 12, 10]
    for r, g in zip(alone, gens):
        r.run(g)
    batch = P.Batch(8)
    done = [0] * len(SPECS)
    join_at = [0, 3, 0, 5, 1, 8, 2]
    tick = 0
    active = set()
    while any(done[i] < gens[i] for i in range(len(SPECS))):
        for i in range(len(SPECS)):
            if i not in active and done[i] < gens[i] and tick >= join_at[i]:
                batch.admit(mixed[i])
                active.add(i)
        batch.step()
        for i in list(active):
            done[i] += 1
            if done[i] == gens[i]:
                batch.retire(mixed[i])
                active.discard(i)
        tick += 1
    for i, (a, b) in enumerate(zip(alone, mixed)):
        assert same(a, b) is None, (i, same(a, b))
    # retired runs continue alone
    alone[0].run(4)
    mixed[0].run(4)
    assert same(alone[0], mixed[0]) is None


def test_batch_rejects_single_run_calls(P):
    from paper_2404_01159_amd.rvea import RveaError

    r = make(P, SPECS[0])
    b = P.Batch(2)
    b.admit(r)
    with pytest.raises(RveaError):
        r.step()
    with pytest.raises(RveaError):
        r.run(1)
    with pytest.raises(RveaError):
        b.admit(r)
    r2, r3 = make(P, SPECS[1]), make(P, SPECS[2])
    b.admit(r2)
    with pytest.raises(RveaError):
        b.admit(r3)  # full
    b.step()
    assert r.get_state()["t"] == 1


def test_batch_with_general_distribution_indices(P, O):
    """A run with other distribution indices and crossover rate (the general
    offspring variant) batched beside default runs: every generation of each
    against the oracle, and equal to the same runs alone."""
    prm_g = P.default_params(t_max=30, eta_c=15.0, eta_m=5.0, p_c=0.7, p_m=2.0)
    prm_d = P.default_params(t_max=30)
    specs = [(1, 3, 300, 105, 105, 21, prm_g), (2, 3, 64, 91, 91, 22, prm_d),
             (3, 2, 2048, 64, 64, 23, prm_g)]
    mixed = [P.Run(pb, m, d, N, K, seed=sd, params=pr) for pb, m, d, N, K, sd, pr in specs]
    alone = [P.Run(pb, m, d, N, K, seed=sd, params=pr) for pb, m, d, N, K, sd, pr in specs]
    batch = P.Batch(4)
    for r in mixed:
        batch.admit(r)
    stats = new_stats()
    for _ in range(7):
        before = [r.get_state() for r in mixed]
        batch.step()
        for r, st, sp in zip(mixed, before, specs):
            check_generation(O, r, sp[6], st, r.get_offspring(), r.get_selection(), r.get_state(),
                             stats)
    for r in alone:
        r.run(7)
    for a, b in zip(alone, mixed):
        assert same(a, b) is None, same(a, b)
    assert stats["straddles"] <= max(2, 1e-6 * stats["genes"]), stats
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
