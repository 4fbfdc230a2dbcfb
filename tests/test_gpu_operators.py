"""The other reproduction operators (Sec. 4, Extensibility): DE/rand/1/bin,
PSO, CSO and random reproduction in place of SBX + polynomial mutation, HIP
path vs the oracle through the C ABI, generation by generation.

Genes and velocities are compared bit for bit: both sides take the same
binary64 additions, subtractions, products and clips in the same order from
the same binary32 inputs and round once, so there is no rounding straddle to
allow for.  Objectives within OBJ_RTOL (POLICY_RTOL for the rollouts), then
selection, the new population and the adaptation as for the genetic
operators (tests/parity.py); each survivor keeps the velocity of the row it
came from.
"""
import numpy as np
import pytest

import workloads as W
from parity import (POLICY_RTOL, check_after_offspring, new_stats, objectives_close,
                    ora_params)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OPS = ["de", "pso", "cso", "rand"]


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


def ora_op(O, prm):
    return O.op_params(prm.op, prm.op_a, prm.op_b)


def lockstep_op(P, O, run, prm, gens, stats, S=None):
    """gens generations of an operator run against the oracle; S is the
    policy problem's system (None for the test problems)."""
    problem, m, N, K, seed = run.problem, run.m, run.N, run.K, run.seed
    oprm = ora_params(O, prm)
    if S is not None:
        oprm = O.params(lq=S, alpha=prm.alpha, fr=prm.fr, t_max=prm.t_max, lb=prm.lb,
                        ub=prm.ub)
    opp = ora_op(O, prm)
    swarm = prm.op in (P.OP_PSO, P.OP_CSO)
    h = (N + 1) // 2
    for _ in range(gens):
        st = run.get_state()
        vel = run.get_velocities() if swarm else None
        t = st["t"] + 1
        print(f"op {prm.op} N={N} K={K} d={run.d} t={t}", flush=True)
        run.step()
        off = run.get_offspring()
        Xo, Vo = O.reproduce_op(oprm, opp, seed, t, st["X"], vel, st["valid"],
                                st["F"].astype(np.float64), N)
        bad = np.nonzero(off["X"].view(np.uint32) != Xo.view(np.uint32))
        assert len(bad[0]) == 0, f"genes differ at t={t}: first {bad[0][:5]}, {bad[1][:5]}"
        stats["genes"] += Xo.size
        if swarm:
            offv = run.get_velocities(offspring=True)
            assert np.array_equal(offv.view(np.uint32), Vo.view(np.uint32)), \
                f"velocities differ at t={t}"
        if S is not None:
            want = O.policy_evaluate(off["X"], S["x0"].shape[0], S["T"], S["A"], S["B"], S["x0"])
            objectives_close(off["F"], want, POLICY_RTOL)
        else:
            objectives_close(off["F"], O.evaluate(problem, m, off["X"]))
        pr = off["parents"]
        if prm.op == P.OP_CSO:
            # (winner, loser) per pair: the winner's copy is child p + ceil(N/2)
            fit = st["F"].astype(np.float64).sum(axis=1)
            assert np.all(st["valid"][pr.ravel()] == 1)
            w, lo = pr[:, 0], pr[:, 1]
            assert np.all((fit[w] < fit[lo]) | ((fit[w] == fit[lo]) & (w <= lo)))
            assert np.array_equal(off["X"][h:], st["X"][w[:N - h]])
        else:
            assert np.all(pr == -1)
        run.select()
        sel = run.get_selection()
        run.adapt()
        st2 = run.get_state()
        check_after_offspring(O, run, prm, st, off, sel, st2, stats)
        if swarm:
            vel2 = run.get_velocities()
            s = sel["surv"]
            ok = s >= 0
            Vm = np.vstack([vel, offv])
            assert np.array_equal(vel2[ok], Vm[s[ok]]) and not vel2[~ok].any()
    return stats


CASES = [  # problem, m, d, N, K, gens
    (1, 3, 100, 105, 105, 6),
    (2, 3, 1001, 51, 55, 5),    # odd N, several quads per lane and a ragged tail
    (3, 5, 37, 120, 126, 5),    # short rows: 16-lane segments
    (1, 2, 8, 9, 10, 8),        # tiny: 4-lane segments, population of a few members
]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("case", CASES, ids=lambda c: "p%d_m%d_d%d_N%d_K%d" % c[:5])
def test_operator_lockstep(P, O, op, case):
    problem, m, d, N, K, gens = case
    prm = P.default_params(op, t_max=10, fr=0.2)
    run = P.Run(problem, m, d, N, K, seed=17, params=prm)
    stats = lockstep_op(P, O, run, prm, gens, new_stats())
    assert stats["near_ties"] <= 1, stats
    run.close()


@pytest.mark.parametrize("op", ["de", "pso", "cso"])
def test_operator_parameters_reach_the_kernel(P, O, op):
    # non-default parameters, and for the swarms velocities set from the host
    kw = dict(de=dict(op_a=1.3, op_b=0.2), pso=dict(op_a=1.0, op_b=3.5), cso={})[op]
    prm = P.default_params(op, t_max=10, **kw)
    problem, m, d, N, K = 2, 3, 64, 45, 45
    run = P.Run(problem, m, d, N, K, seed=3, params=prm)
    if op != "de":
        V = W.rng(4).uniform(-0.3, 0.3, size=(K, d)).astype(np.float32)
        run.set_velocities(V)
        got = run.get_velocities()
        assert np.array_equal(got, V)  # every slot valid at creation (N = K)
    lockstep_op(P, O, run, prm, 3, new_stats())
    run.close()


@pytest.mark.parametrize("op", OPS)
def test_operator_policy_lockstep(P, O, op):
    S = dict(W.lq_system(2), T=3, sigma=0.1)
    prm = P.default_params(op, t_max=20, lb=-1.0, ub=1.0)
    run = P.Run(P.POLICY_LQ, 2, P.POLICY_D, 31, 40, seed=2, params=prm, system=S)
    lockstep_op(P, O, run, prm, 3, new_stats(), S=S)
    run.close()


@pytest.mark.parametrize("op", OPS)
def test_operator_graphs_match_eager(P, op):
    prm = P.default_params(op, t_max=30)
    a = P.Run(1, 3, 300, 105, 105, seed=9, params=prm)
    b = P.Run(1, 3, 300, 105, 105, seed=9, params=prm)
    a.set_graphs(True)
    a.run(7)
    a.run(5)
    for _ in range(12):
        b.generation()
    sa, sb = a.get_state(), b.get_state()
    for k in ("X", "F", "valid", "V", "gamma"):
        assert np.array_equal(sa[k], sb[k], equal_nan=True), k
    if op in ("pso", "cso"):
        assert np.array_equal(a.get_velocities(), b.get_velocities())
        assert np.array_equal(a.get_velocities(True), b.get_velocities(True))
    a.close()
    b.close()


@pytest.mark.parametrize("op", OPS)
def test_operator_full_size_generation(P, O, op):
    """One generation at the headline shape (m = 3, d = 500, N = K = 10,011):
    every offspring gene and velocity exact, objectives within OBJ_RTOL."""
    problem, m, d, N, K = 1, 3, 500, 10011, 10011
    prm = P.default_params(op)
    run = P.Run(problem, m, d, N, K, seed=1, params=prm)
    run.generation()  # a second generation reads non-zero velocities
    st = run.get_state()
    swarm = op in ("pso", "cso")
    vel = run.get_velocities() if swarm else None
    run.step()
    off = run.get_offspring()
    Xo, Vo = O.reproduce_op(ora_params(O, prm), ora_op(O, prm), 1, st["t"] + 1, st["X"], vel,
                            st["valid"], st["F"].astype(np.float64), N)
    assert np.array_equal(off["X"].view(np.uint32), Xo.view(np.uint32))
    if swarm:
        assert np.array_equal(run.get_velocities(True).view(np.uint32), Vo.view(np.uint32))
    objectives_close(off["F"], O.evaluate(problem, m, off["X"]))
    run.select()
    run.adapt()
    run.close()


def check_op_generation(P, O, run, prm, st, vel, stats):
    """One completed generation of an operator run (stepped alone or in a
    batch) against the oracle from its state before: genes and velocities
    bit for bit, objectives, the CSO pair report, then selection, the new
    population, the adaptation and the survivors' velocities."""
    N = run.N
    swarm = prm.op in (P.OP_PSO, P.OP_CSO)
    t = st["t"] + 1
    off = run.get_offspring()
    Xo, Vo = O.reproduce_op(ora_params(O, prm), ora_op(O, prm), run.seed, t, st["X"], vel,
                            st["valid"], st["F"].astype(np.float64), N)
    bad = np.nonzero(off["X"].view(np.uint32) != Xo.view(np.uint32))
    assert len(bad[0]) == 0, f"genes differ at t={t}: first {bad[0][:5]}, {bad[1][:5]}"
    stats["genes"] += Xo.size
    if swarm:
        offv = run.get_velocities(offspring=True)
        assert np.array_equal(offv.view(np.uint32), Vo.view(np.uint32)), \
            f"velocities differ at t={t}"
    objectives_close(off["F"], O.evaluate(run.problem, run.m, off["X"]))
    if prm.op == P.OP_CSO:
        h = (N + 1) // 2
        w = off["parents"][:, 0]
        assert np.array_equal(off["X"][h:], st["X"][w[:N - h]])
    sel = run.get_selection()
    st2 = run.get_state()
    check_after_offspring(O, run, prm, st, off, sel, st2, stats)
    if swarm:
        vel2 = run.get_velocities()
        s = sel["surv"]
        ok = s >= 0
        Vm = np.vstack([vel, offv])
        assert np.array_equal(vel2[ok], Vm[s[ok]]) and not vel2[~ok].any()


@pytest.mark.parametrize("graphs", [True, False])
def test_batched_operators_match_oracle(P, O, graphs):
    """Runs of every operator (and a genetic run) advanced together by one
    batch: every batched generation of every operator run against the
    oracle, stage by stage, from its state before the batch step."""
    specs = [("de", 1, 3, 100, 105, 105), ("pso", 2, 3, 1001, 51, 55),
             ("cso", 3, 5, 37, 120, 126), ("rand", 1, 2, 8, 9, 10),
             ("pso", 1, 3, 64, 90, 91), ("ga", 2, 3, 40, 105, 105)]
    runs, prms = [], []
    for op, problem, m, d, N, K in specs:
        prm = P.default_params(op, t_max=10, fr=0.2)
        runs.append(P.Run(problem, m, d, N, K, seed=23 + len(runs), params=prm))
        prms.append(prm)
    bt = P.Batch(8)
    bt.set_graphs(graphs)
    for r in runs:
        bt.admit(r)
    stats = new_stats()
    for tick in range(6):  # adaptations every second generation
        before = []
        for r, prm in zip(runs, prms):
            sw = prm.op in (P.OP_PSO, P.OP_CSO)
            before.append((r.get_state(), r.get_velocities() if sw else None))
        print(f"batched operators, tick {tick}", flush=True)
        bt.step()
        for r, prm, (st, vel) in zip(runs, prms, before):
            if prm.op != P.OP_GA:
                check_op_generation(P, O, r, prm, st, vel, stats)
    assert stats["near_ties"] <= 1 and stats["adaptations"] >= 5, stats
    for r in runs:
        bt.retire(r)
        r.close()
    bt.close()


def test_batched_operators_equal_alone(P):
    specs = [("de", 1, 3, 50, 105, 105), ("pso", 3, 3, 70, 91, 91), ("cso", 2, 2, 33, 40, 40),
             ("rand", 1, 3, 20, 21, 21)]
    alone, mixed = [], []
    for op, problem, m, d, N, K in specs:
        prm = P.default_params(op, t_max=20)
        alone.append(P.Run(problem, m, d, N, K, seed=7, params=prm))
        mixed.append(P.Run(problem, m, d, N, K, seed=7, params=prm))
    for r in alone:
        r.run(9)
    bt = P.Batch(4)
    for r in mixed:
        bt.admit(r)
    bt.step(9)
    bt.synchronize()
    for a, b in zip(alone, mixed):
        sa, sb = a.get_state(), b.get_state()
        for k in ("X", "F", "valid", "V", "gamma", "t"):
            assert np.array_equal(sa[k], sb[k], equal_nan=True), k
        if a.params.op in (P.OP_PSO, P.OP_CSO):
            assert np.array_equal(a.get_velocities(), b.get_velocities())
    for r in mixed:
        bt.retire(r)
    bt.close()
    for r in alone + mixed:
        r.close()


def test_velocities_only_for_swarms(P):
    g = P.Run(1, 3, 50, 105, 105, seed=1)
    with pytest.raises(P.RveaError):
        g.get_velocities()
    g.close()
