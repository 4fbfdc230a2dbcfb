"""Policy-rollout problem (Sec. 4.3's neuroevolution setting on a synthetic
linear system): HIP path vs the oracle through the C ABI.

Genes (Gaussian initialization, SBX and polynomial mutation on [-1, 1]) are
compared bit for bit, objectives within 1e-3 relative (bfloat16 matrix-core
products against the binary64 oracle that rounds the same operands), and
selection exactly from the GPU's merged objectives (tests/parity.py).
"""
import numpy as np
import pytest

import workloads as W
from parity import POLICY_RTOL, compare_selection, gene_mismatches, objectives_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

D = 6728


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


def system(seed=0, T=200, sigma=0.1):
    return dict(W.lq_system(seed), T=T, sigma=sigma)


def policy_params(P, **kw):
    kw.setdefault("lb", -1.0)
    kw.setdefault("ub", 1.0)
    return P.default_params(**kw)


def ora_params(O, prm, S):
    return O.params(lq=S, alpha=prm.alpha, fr=prm.fr, t_max=prm.t_max, eta_c=prm.eta_c,
                    eta_m=prm.eta_m, p_c=prm.p_c, p_m=prm.p_m, lb=prm.lb, ub=prm.ub)


def ora_eval(O, S, X):
    return O.policy_evaluate(X, S["x0"].shape[0], S["T"], S["A"], S["B"], S["x0"])


def lockstep(O, run, prm, S, gens, stats):
    N, K, seed = run.N, run.K, run.seed
    op = ora_params(O, prm, S)
    period = O.adapt_period(prm.fr, prm.t_max)
    for _ in range(gens):
        st = run.get_state()
        t = st["t"] + 1
        run.step()
        off = run.get_offspring()
        parents, _ = O.mate(seed, t, st["valid"], N)
        assert np.array_equal(off["parents"], parents), f"mating differs at t={t}"
        Xo, pre = O.reproduce(op, seed, t, st["X"], parents, N, with_pre=True)
        stats["straddles"] += gene_mismatches(off["X"], Xo, pre)
        stats["genes"] += Xo.size
        stats["worst"] = max(stats["worst"], objectives_close(off["F"], ora_eval(O, S, off["X"]),
                                                              POLICY_RTOL))
        run.select()
        sel = run.get_selection()
        Fm = np.vstack([st["F"], off["F"]]).astype(np.float64)
        mv = np.concatenate([st["valid"], np.ones(N, np.uint8)])
        ref = O.select(2, K, N, t, prm.t_max, prm.alpha, Fm, mv, st["V"], st["gamma"])
        stats["near_ties"] += compare_selection(sel, ref, K)
        run.adapt()
        st2 = run.get_state()
        s = sel["surv"]
        ok = s >= 0
        assert np.array_equal(st2["X"][ok], np.vstack([st["X"], off["X"]])[s[ok]])
        if t % period == 0:
            Vo, changed = O.adapt(st2["V0"], st2["F"].astype(np.float64), st2["valid"], st["V"])
            assert np.array_equal(st2["V"], Vo)
            stats["adaptations"] += int(changed)
    return stats


def new_stats():
    return dict(straddles=0, genes=0, near_ties=0, adaptations=0, worst=0.0)


@pytest.mark.parametrize("N,K,T", [(64, 64, 200), (30, 41, 7), (1, 2, 1)])
def test_policy_init_matches_oracle(P, O, N, K, T):
    S = system(1, T=T)
    run = P.Run(P.POLICY_LQ, 2, D, N, K, seed=5, params=policy_params(P), system=S)
    st = run.get_state()
    Xo, pre = O.init_gauss_rows(5, np.arange(N), D, 0.1, -1.0, 1.0, with_pre=True)
    assert gene_mismatches(st["X"][:N], Xo, pre) <= 1
    assert np.all(st["X"][N:] == 0) and np.array_equal(st["valid"], np.arange(K) < N)
    objectives_close(st["F"][:N], ora_eval(O, S, st["X"][:N]), POLICY_RTOL)
    assert np.all(np.isnan(st["F"][N:]))
    run.close()


@pytest.mark.parametrize("N,K,T,gens,seed", [(64, 64, 200, 6, 0), (31, 40, 3, 5, 2)])
def test_policy_generation_lockstep(P, O, N, K, T, gens, seed):
    S = system(seed, T=T)
    prm = policy_params(P, t_max=20)
    run = P.Run(P.POLICY_LQ, 2, D, N, K, seed=seed, params=prm, system=S)
    stats = lockstep(O, run, prm, S, gens, new_stats())
    assert stats["straddles"] <= max(2, 1e-6 * stats["genes"]), stats
    assert stats["near_ties"] <= 1, stats
    assert stats["adaptations"] >= 1, stats
    print(f"policy lockstep N={N} T={T}: worst objective rel err {stats['worst']:.2e}")
    run.close()


def test_policy_full_size_sampled(P, O):
    """4,096 policies, K = 4,096 (H = 4,095), 16 rollouts x 200 steps: one
    generation, outputs checked one by one on samples."""
    N = K = 4096
    seed = 0
    S = system(0)
    prm = policy_params(P, t_max=50)
    run = P.Run(P.POLICY_LQ, 2, D, N, K, seed=seed, params=prm, system=S)
    rng = np.random.default_rng(1)
    slots = np.sort(rng.choice(K, 32, replace=False))
    Xs, Fs = run.get_rows(slots)
    Xo, pre = O.init_gauss_rows(seed, slots, D, 0.1, -1.0, 1.0, with_pre=True)
    assert gene_mismatches(Xs, Xo, pre) <= 1
    objectives_close(Fs, ora_eval(O, S, Xs), POLICY_RTOL)
    st = run.get_state(genes=False)
    run.step()
    Pn = N // 2
    parents_all, _ = O.mate(seed, 1, st["valid"], N)
    pairs = np.sort(rng.choice(Pn, 16, replace=False))
    Xg1, Fg1 = run.get_rows(pairs, offspring=True)
    Xg2, Fg2 = run.get_rows(pairs + Pn, offspring=True)
    used = np.unique(parents_all[pairs].ravel())
    Xp, _ = run.get_rows(used)
    remap = {int(s_): i for i, s_ in enumerate(used)}
    table = np.zeros((Pn, 2), np.int32)
    table[pairs] = [[remap[int(a)], remap[int(b)]] for a, b in parents_all[pairs]]
    c1, c2 = O.reproduce_pairs(ora_params(O, prm, S), seed, 1, Xp, table, N, pairs)
    assert gene_mismatches(Xg1, c1) == 0 and gene_mismatches(Xg2, c2) == 0
    objectives_close(Fg1, ora_eval(O, S, Xg1), POLICY_RTOL)
    objectives_close(Fg2, ora_eval(O, S, Xg2), POLICY_RTOL)
    F_off = run.get_offspring(genes=False)["F"]
    run.select()
    sel = run.get_selection()
    Fm = np.vstack([st["F"], F_off]).astype(np.float64)
    z = Fm.min(axis=0)
    assert np.array_equal(sel["zstar"].astype(np.float64), z)
    V0 = O.unit_vectors(4095, 2)
    rows = np.sort(rng.choice(K + N, 256, replace=False))
    a, _, ap = O.assoc_rows(2, K, 1, prm.t_max, prm.alpha, Fm[rows], z, V0, st["gamma"])
    assert np.array_equal(sel["assoc"][rows], a)
    assert np.allclose(sel["apd"][rows], ap, rtol=1e-12, atol=0)
    run.close()


def test_policy_graph_replays_match_eager(P):
    S = system(3, T=20)
    prm = policy_params(P, t_max=30)
    a = P.Run(P.POLICY_LQ, 2, D, 48, 48, seed=7, params=prm, system=S)
    b = P.Run(P.POLICY_LQ, 2, D, 48, 48, seed=7, params=prm, system=S)
    a.set_graphs(False)
    for chunk in (4, 1, 6):
        a.run(chunk)
        b.run(chunk)
        sa, sb = a.get_state(), b.get_state()
        for k in ("X", "F", "valid", "V", "gamma", "t"):
            assert np.array_equal(sa[k], sb[k], equal_nan=True), (chunk, k)


def test_policy_rejections_and_timing(P):
    from paper_2404_01159_amd.rvea import (RVEA_EINVAL, RVEA_EUNSUPPORTED, RveaError,
                                           KERNEL_ROLLOUT)

    S = system(0, T=5)
    with pytest.raises(RveaError) as e:
        P.Run(P.POLICY_LQ, 2, D, 8, 8, params=policy_params(P))  # no system
    with pytest.raises(RveaError) as e:
        P.Run(P.POLICY_LQ, 2, D, 8, 8, params=policy_params(P),
              system=dict(S, x0=S["x0"][:8]))
    assert e.value.status == RVEA_EUNSUPPORTED
    with pytest.raises(RveaError) as e:
        P.Run(P.POLICY_LQ, 3, D, 10, 10, params=policy_params(P), system=S)
    assert e.value.status == RVEA_EINVAL
    run = P.Run(P.POLICY_LQ, 2, D, 16, 16, seed=1, params=policy_params(P), system=S)
    batch = P.Batch(2)
    with pytest.raises(RveaError) as e:
        batch.admit(run)
    assert e.value.status == RVEA_EUNSUPPORTED
    batch.close()
    run.set_timing([0, KERNEL_ROLLOUT])
    run.run(3)
    for k in (0, KERNEL_ROLLOUT):
        ms, n = run.kernel_time(k)
        assert n == 3 and ms > 0
    run.close()
