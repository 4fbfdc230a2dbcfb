"""HIP path vs the FP64 oracle, stage by stage, through the C ABI.

Stages follow Alg. 2: initialization, offspring (mating + SBX + PM,
Appendix B), evaluation, selection (Alg. 1) and adaptation.  Each stage is
compared from identical state: the oracle is fed the GPU's state before the
stage.  Rules are in tests/parity.py.
"""
import numpy as np
import pytest

from parity import (gene_mismatches, lockstep, new_stats, objectives_close, ora_params,
                    survivor_near_ties)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


INIT_CASES = [
    # problem, m, d, N, K
    (2, 3, 12, 105, 105),
    (1, 3, 13, 50, 105),
    (3, 2, 7, 9, 10),
    (1, 5, 30, 126, 126),
    (2, 8, 20, 120, 120),
    (3, 3, 257, 91, 91),
]


@pytest.mark.parametrize("case", INIT_CASES)
def test_init_matches_oracle(P, O, case):
    problem, m, d, N, K = case
    run = P.Run(problem, m, d, N, K, seed=11)
    st = run.get_state()
    H = O.lattice_H(K, m)
    assert np.array_equal(st["X"][:N], O.init(11, N, d))
    assert np.all(st["X"][N:] == 0) and np.array_equal(st["valid"], (np.arange(K) < N))
    objectives_close(st["F"][:N], O.evaluate(problem, m, st["X"][:N]))
    assert np.all(np.isnan(st["F"][N:]))
    V0 = O.unit_vectors(H, m)
    assert np.array_equal(st["V0"], V0) and np.array_equal(st["V"], V0)
    assert np.allclose(st["gamma"], O.gamma(V0), rtol=1e-14, atol=0)
    assert st["t"] == 0
    run.close()


LOCKSTEP_CASES = [
    # problem, m, d, N, K, seed, gens
    (2, 3, 12, 105, 105, 0, 100),
    (1, 3, 30, 105, 105, 3, 25),
    (3, 2, 11, 31, 40, 5, 20),
    (1, 5, 33, 126, 126, 7, 12),
    (2, 8, 17, 120, 120, 9, 12),
    (3, 3, 1001, 91, 91, 2, 12),
    (2, 3, 4000, 60, 66, 4, 11),  # long rows, few pairs: each pair split over segments
]


@pytest.mark.parametrize("case", LOCKSTEP_CASES)
def test_generation_lockstep(P, O, case):
    problem, m, d, N, K, seed, gens = case
    prm = P.default_params(t_max=max(gens, 10))
    run = P.Run(problem, m, d, N, K, seed=seed, params=prm)
    stats = lockstep(O, run, prm, gens, new_stats())
    assert stats["straddles"] <= max(2, 1e-6 * stats["genes"]), stats
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
    assert stats["adaptations"] >= 1
    run.close()


def test_arbitrary_state_and_parameters(P, O):
    problem, m, d, N, K = 1, 3, 21, 55, 91
    prm = P.default_params(t_max=60, p_c=0.7, p_m=3.0, eta_c=15.0, eta_m=5.0, lb=-2.0, ub=3.0,
                           fr=0.05)
    run = P.Run(problem, m, d, N, K, seed=123, params=prm)
    from workloads import population, valid_mask, objectives

    X = population(1, K, d, lb=-2.0, ub=3.0)
    valid = valid_mask(2, K, 0.6)
    F = objectives(3, K, m)
    F[valid == 0] = np.nan
    H = O.lattice_H(K, m)
    V = O.unit_vectors(H, m) * np.array([1.0, 2.0, 0.5])
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    run.set_state(X, F, valid, V=V, gamma=None, t=37)
    st = run.get_state()
    assert st["t"] == 37 and np.array_equal(st["valid"], valid)
    assert np.array_equal(st["X"][valid == 1], X[valid == 1])
    assert np.array_equal(st["V"], V)
    assert np.allclose(st["gamma"], O.gamma(V), rtol=1e-14, atol=0)
    stats = lockstep(O, run, prm, 6, new_stats())
    assert stats["straddles"] <= 2 and stats["adaptations"] >= 1
    run.close()


@pytest.mark.parametrize("case", [
    # problem, m, d, N, K: the smallest lattices, a single child, odd N
    (2, 2, 2, 1, 2),
    (1, 3, 3, 1, 3),
    (3, 2, 5, 3, 4),
    (1, 4, 4, 2, 4),
])
def test_tiny_runs_match_oracle(P, O, case):
    problem, m, d, N, K = case
    prm = P.default_params(t_max=12)
    run = P.Run(problem, m, d, N, K, seed=17, params=prm)
    stats = lockstep(O, run, prm, 12, new_stats())
    assert stats["straddles"] <= 2 and stats["near_ties"] <= 1, stats
    run.close()


def test_nonfinite_rows_are_dropped(P, O):
    problem, m, d, N, K = 2, 3, 12, 105, 105
    run = P.Run(problem, m, d, N, K, seed=4)
    st = run.get_state()
    F = st["F"].copy()
    F[[3, 17], 1] = np.nan
    F[40, 0] = np.inf
    run.set_state(st["X"], F, st["valid"], t=0)
    stats = lockstep(O, run, P.default_params(), 1, new_stats())
    assert run.counters()["nonfinite_rows"] == 3
    assert stats["near_ties"] == 0
    run.close()


def test_crowded_vectors(P, O):
    """Adapted vectors crowded far below binary32 resolution (axis ranges
    1 : 1e-3, 4,096 vectors, m = 2): gamma of every vector and one full
    selection still match the oracle; rows whose candidate tiles exceed the
    re-rank's capacity take the exact full scan."""
    problem, m, d, N, K = 2, 2, 12, 4096, 4096
    prm = P.default_params(t_max=50)
    run = P.Run(problem, m, d, N, K, seed=3, params=prm)
    st = run.get_state()
    V = O.unit_vectors(K - 1, m) * np.array([1.0, 1e-3])
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = st["F"].copy()
    F[:, 0] *= 1e3
    run.set_state(st["X"], F, st["valid"], V=V, gamma=None, t=3)
    st2 = run.get_state()
    assert np.allclose(st2["gamma"], O.gamma(V), rtol=1e-13, atol=0)
    stats = lockstep(O, run, prm, 1, new_stats())
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
    assert run.counters()["full_rescans"] > 0
    run.close()


def test_headline_size_stages(P, O):
    """Full 10,011-vector, d=500 shape: two generations, the second adapting."""
    problem, m, d, N, K = 1, 3, 500, 10011, 10011
    prm = P.default_params()
    run = P.Run(problem, m, d, N, K, seed=0, params=prm)
    stats = lockstep(O, run, prm, 1, new_stats())
    st = run.get_state()
    run.set_state(st["X"], st["F"], st["valid"], V=st["V"], gamma=st["gamma"], t=9)
    stats = lockstep(O, run, prm, 1, stats)
    assert stats["adaptations"] == 1
    assert stats["straddles"] <= max(2, 1e-6 * stats["genes"]), stats
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
    c = run.counters()
    assert c["full_rescans"] == 0
    run.close()


def test_big_population_sampled(P, O):
    """100,128 vectors, d=5,000: outputs checked one by one on samples, and
    selection invariants checked over every vector."""
    problem, m, d, N, K, seed = 3, 3, 5000, 100128, 100128, 0
    prm = P.default_params(t_max=50)
    run = P.Run(problem, m, d, N, K, seed=seed, params=prm)
    rng = np.random.default_rng(0)
    # initialization, sampled slots
    slots = np.sort(rng.choice(K, 48, replace=False))
    Xs, Fs = run.get_rows(slots)
    assert np.array_equal(Xs, O.init_rows(seed, slots, d))
    objectives_close(Fs, O.evaluate(problem, m, Xs))
    st = run.get_state(genes=False)
    V0 = O.unit_vectors(446, 3)
    assert np.array_equal(st["V0"], V0)
    g_rows = np.sort(rng.choice(K, 64, replace=False))
    assert np.allclose(st["gamma"][g_rows], O.gamma_rows(V0, g_rows), rtol=1e-14, atol=0)
    # one generation: sampled offspring pairs
    run.step()
    Pn = (N + 1) // 2
    parents_all, _ = O.mate(seed, 1, st["valid"], N)
    pairs = np.sort(rng.choice(Pn, 24, replace=False))
    Xg1, Fg1 = run.get_rows(pairs, offspring=True)
    Xg2, Fg2 = run.get_rows(pairs + Pn, offspring=True)
    used = np.unique(parents_all[pairs].ravel())
    Xp, _ = run.get_rows(used)
    remap = {int(s_): i for i, s_ in enumerate(used)}
    table = np.zeros((Pn, 2), np.int32)  # pair counter = global pair index
    table[pairs] = [[remap[int(a)], remap[int(b)]] for a, b in parents_all[pairs]]
    c1, c2 = O.reproduce_pairs(ora_params(O, prm), seed, 1, Xp, table, N, pairs)
    assert gene_mismatches(Xg1, c1) == 0 and gene_mismatches(Xg2, c2) == 0
    objectives_close(Fg1, O.evaluate(problem, m, Xg1))
    objectives_close(Fg2, O.evaluate(problem, m, Xg2))
    # selection: sampled rows one by one against the oracle ...
    F_off = run.get_offspring(genes=False)["F"]
    run.select()
    sel = run.get_selection()
    Fm = np.vstack([st["F"], F_off]).astype(np.float64)
    z = Fm.min(axis=0)
    assert np.array_equal(sel["zstar"].astype(np.float64), z)
    rows = np.sort(rng.choice(K + N, 256, replace=False))
    a, th, ap = O.assoc_rows(m, K, 1, prm.t_max, prm.alpha, Fm[rows], z, V0, st["gamma"])
    assert np.array_equal(sel["assoc"][rows], a)
    assert np.allclose(sel["apd"][rows], ap, rtol=1e-12, atol=0)
    # ... and invariants over every vector: the survivor of j is the lowest
    # row among the minimal APDs of the rows associated with j, -1 if none,
    # with APDs compared above their lowest kb bits (kb = bits of a row
    # index), as the packed (APD, row) minimum compares them
    s, A, D = sel["surv"], sel["assoc"], sel["apd"]

    def lowest_minimal(keys):
        order = np.lexsort((np.arange(K + N), keys, A))
        A_s = A[order]
        first = np.ones(len(order), bool)
        first[1:] = A_s[1:] != A_s[:-1]
        want = np.full(K, -1)
        heads = np.nonzero(first & (A_s >= 0))[0]
        want[A_s[heads]] = order[heads]
        return want

    kb = int(K + N).bit_length()
    assert np.array_equal(s, lowest_minimal(D.view(np.uint64) >> np.uint64(kb)))
    # against the exact minimum of the full APDs the differences are near-ties
    nt = survivor_near_ties(s, lowest_minimal(D), D, A, K)
    assert nt <= max(1, 1e-4 * K), nt
    print(f"100,128 vectors: {nt} survivors decided below the packed key's resolution")
    assert run.counters()["full_rescans"] == 0
    run.close()


def test_igd_matches_oracle_over_ten_seeds(P, O):
    problem, m, d, N, K = 2, 3, 12, 105, 105
    prm = P.default_params()
    Fs = O.front(problem, m, O.front_H(m))
    g_gpu, g_ora = [], []
    for seed in range(10):
        run = P.Run(problem, m, d, N, K, seed=seed, params=prm)
        run.run(100)
        st = run.get_state()
        g_gpu.append(O.igd(st["F"][st["valid"] == 1].astype(np.float64), Fs))
        run.close()
        ost = O.run(ora_params(O, prm), problem, m, d, N, K, seed, 100)
        g_ora.append(O.igd(ost.F[ost.valid == 1], Fs))
    mg, mo = np.mean(g_gpu), np.mean(g_ora)
    assert abs(mg - mo) <= 0.05 * mo, (g_gpu, g_ora)


def test_headline_igd_matches_oracle_over_ten_seeds(P, O):
    """Full runs at the 10,011-vector workload (linear-front multimodal
    problem, m = 3, d = 500, N = K = 10,011, 100 generations, default
    parameters) for seeds 0-9: the mean IGD of the final survivors to the
    known front (App. C.2) matches the oracle's whole runs within 5%."""
    import time

    problem, m, d, N, K = 1, 3, 500, 10011, 10011
    prm = P.default_params()
    Fs = O.front(problem, m, O.front_H(m))
    g_gpu, g_ora = [], []
    for seed in range(10):
        t0 = time.perf_counter()
        run = P.Run(problem, m, d, N, K, seed=seed, params=prm)
        run.run(100)
        st = run.get_state(genes=False)
        run.close()
        g_gpu.append(O.igd(st["F"][st["valid"] == 1].astype(np.float64), Fs))
        t1 = time.perf_counter()
        ost = O.run(ora_params(O, prm), problem, m, d, N, K, seed, 100)
        g_ora.append(O.igd(ost.F[ost.valid == 1], Fs))
        print(f"seed {seed}: IGD gpu {g_gpu[-1]:.6g} oracle {g_ora[-1]:.6g} "
              f"({t1 - t0:.1f} s gpu, {time.perf_counter() - t1:.1f} s oracle)", flush=True)
    mg, mo = np.mean(g_gpu), np.mean(g_ora)
    print(f"mean IGD gpu {mg:.6g} oracle {mo:.6g} ratio {mg / mo:.4f}")
    assert abs(mg - mo) <= 0.05 * mo, (g_gpu, g_ora)


def test_runs_are_deterministic(P):
    a = P.Run(1, 3, 40, 105, 105, seed=8)
    b = P.Run(1, 3, 40, 105, 105, seed=8)
    c = P.Run(1, 3, 40, 105, 105, seed=9)
    for r in (a, b, c):
        r.run(12)
    sa, sb, sc = a.get_state(), b.get_state(), c.get_state()
    for k in ("X", "F", "valid", "V", "gamma"):
        assert np.array_equal(sa[k], sb[k], equal_nan=True), k
    assert not np.array_equal(sa["X"], sc["X"])


def test_call_order_is_enforced(P):
    from paper_2404_01159_amd.rvea import RveaError, RVEA_ESTATE

    run = P.Run(2, 3, 12, 105, 105, seed=1)
    with pytest.raises(RveaError) as e:
        run.select()
    assert e.value.status == RVEA_ESTATE
    with pytest.raises(RveaError):
        run.adapt()
    run.step()
    with pytest.raises(RveaError):
        run.step()
    run.select()
    with pytest.raises(RveaError):
        run.select()
    run.adapt()
    run.generation()
    run.synchronize()


def test_kernel_timing_records_launches(P):
    run = P.Run(1, 3, 64, 105, 105, seed=1)
    run.set_timing(range(4))
    run.run(10)
    for k in range(3):
        ms, n = run.kernel_time(k)
        assert n == 10 and ms > 0
    ms, n = run.kernel_time(3)
    assert n == 1


def test_kernel_relaunch_timing_leaves_state(P):
    """rvea_time_kernels re-launches the hot kernels on the current state:
    the generation continues exactly as without it."""
    a = P.Run(1, 3, 60, 300, 300, seed=8, params=P.default_params(t_max=20))
    b = P.Run(1, 3, 60, 300, 300, seed=8, params=P.default_params(t_max=20))
    for r in (a, b):
        r.run(3)
        r.step()
    t = b.time_kernels(5)
    assert all(t[k] > 0 for k in ("offspring", "assoc", "rerank"))
    t = b.time_kernels(3)  # again in the same phase: its events come back to the pool
    assert all(t[k] > 0 for k in ("offspring", "assoc", "rerank"))
    for r in (a, b):
        r.select()
        r.adapt()
    sa, sb = a.get_state(), b.get_state()
    for k in ("X", "F", "valid", "V", "gamma", "t"):
        assert np.array_equal(sa[k], sb[k], equal_nan=True), k
    assert a.counters() == b.counters()
    with pytest.raises(P.RveaError):
        b.time_kernels(5)  # only between step and select
    a.close()
    b.close()


@pytest.mark.parametrize("shape", [(1, 3, 40, 1200, 1225), (2, 2, 30, 4000, 4096),
                                   (3, 5, 25, 1001, 1001)])
def test_autotuned_tiles_give_identical_runs(P, O, shape):
    """The association tile autotuner changes launch shapes only: a tuned run
    equals an untuned one bit for bit (adaptations included), and a tuned run
    still matches the oracle stage by stage."""
    problem, m, d, N, K = shape
    prm = P.default_params(t_max=30)
    a = P.Run(problem, m, d, N, K, seed=4, params=prm)
    b = P.Run(problem, m, d, N, K, seed=4, params=prm)
    t = b.autotune()
    assert t["rows_per_lane"] in (1, 2, 4) and t["chunk_vectors"] % 32 == 0
    assert t["candidates"] >= 6 and 0 < t["assoc_us"] <= t["default_us"]
    assert t["rerank_rows"] in (4, 8, 16) and 0 < t["rerank_us"] <= t["rerank_default_us"]
    assert t["gamma_rows_per_lane"] in (1, 2, 4) and t["gamma_chunk_vectors"] % 32 == 0
    assert 0 < t["gamma_us"] <= t["gamma_default_us"]
    a.run(12)
    b.run(12)
    sa, sb = a.get_state(), b.get_state()
    for k in ("X", "F", "valid", "V", "gamma", "t"):
        assert np.array_equal(sa[k], sb[k], equal_nan=True), k
    stats = lockstep(O, b, prm, 3, new_stats())
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
    b.close()
    a.close()


def test_graph_replays_match_eager(P):
    """Captured-graph generations equal eager ones, replay after replay, with
    eager work and synchronizations between the replays."""
    a = P.Run(1, 3, 200, 300, 300, seed=21, params=P.default_params(t_max=40))
    b = P.Run(1, 3, 200, 300, 300, seed=21, params=P.default_params(t_max=40))
    a.set_graphs(False)
    for chunk in (7, 1, 5, 12):
        a.run(chunk)
        b.run(chunk)
        sa, sb = a.get_state(), b.get_state()
        for k in ("X", "F", "valid", "V", "gamma", "t"):
            assert np.array_equal(sa[k], sb[k], equal_nan=True), (chunk, k)
        # eager generation on both in between the replays
        a.generation()
        b.generation()
        b.synchronize()
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa["X"], sb["X"]) and sa["t"] == sb["t"] == 29


def test_multi_generation_graphs_match_eager(P):
    """Graph launches of up to 16 generations, with the adaptation period
    longer than a launch (20), so the adapting generation sits at different
    positions of the captured runs, equal eager generations."""
    prm = P.default_params(t_max=200)
    a = P.Run(2, 3, 64, 120, 120, seed=5, params=prm)
    b = P.Run(2, 3, 64, 120, 120, seed=5, params=prm)
    a.set_graphs(False)
    b.prepare(23)
    for chunk in (23, 22, 16, 3):
        a.run(chunk)
        b.run(chunk)
        sa, sb = a.get_state(), b.get_state()
        for k in ("X", "F", "valid", "V", "gamma", "t"):
            assert np.array_equal(sa[k], sb[k], equal_nan=True), (chunk, k)
    assert sb["t"] == 64
    assert not np.array_equal(sb["V"], b.get_state()["V0"])  # adapted
