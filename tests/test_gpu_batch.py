"""Batched runs: every run's result is the same alone and in the mix.

Runs of different problems, objective counts, dimensions and sizes are
advanced together by rvea_batch_step; each must end bit-identical to the same
run advanced alone (single-run path, itself checked against the oracle in
test_gpu_parity.py), also when runs join and leave at different generations
and whether the batch replays captured graphs or launches eagerly.
"""
import numpy as np
import pytest

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
]


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2404_01159_amd as P

    return P


def make(P, spec, t_max=30):
    problem, m, d, N, K, seed = spec
    return P.Run(problem, m, d, N, K, seed=seed, params=P.default_params(t_max=t_max))


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


def test_staggered_join_and_leave(P):
    """Runs join at different generations, leave early, and the single-run
    path continues them afterwards."""
    alone = [make(P, s) for s in SPECS]
    mixed = [make(P, s) for s in SPECS]
    gens = [20, 15, 25, 9, 17, 12]
    for r, g in zip(alone, gens):
        r.run(g)
    batch = P.Batch(8)
    done = [0] * len(SPECS)
    join_at = [0, 3, 0, 5, 1, 8]
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
