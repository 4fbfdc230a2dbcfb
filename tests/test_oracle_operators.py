"""Pins of the oracle's alternative reproduction operators (Sec. 4,
Extensibility): DE/rand/1/bin, PSO with inertia weight, CSO, and random
reproduction.

Each operator is pinned by what its definition fixes independently of the
oracle's code: special parameter values that reduce it to a copy (DE with
F = 0 takes donor genes verbatim; PSO with w = c = 0 copies the particle),
the geometry of the move (a PSO or CSO child with zero velocity lies on the
segment from the particle toward its leader or winner, never beyond it or
away from it), the crossover rate's frequency (a mutant gene with
probability CR + (1 - CR)/d), the distinctness of DE's donors (with four
members they are exactly the three that are not the target), the
competition's outcome (the winner copy has the smaller objective sum), the
uniform law of random reproduction (a Kolmogorov-Smirnov test against
U(lb, ub)), and the
generation's bookkeeping (each survivor keeps the velocity of the individual
it came from).
"""
import numpy as np
import pytest
from scipy import stats


def _pop(K, d, seed=0, lo=0.2, hi=0.8):
    rng = np.random.default_rng(seed)
    X = rng.uniform(lo, hi, size=(K, d)).astype(np.float32)
    F = rng.uniform(0.0, 1.0, size=(K, 3))
    return X, F


def test_de_donors_distinct_and_target_uniform(ora):
    K, d = 40, 16
    valid = np.ones(K, np.uint8)
    valid[::5] = 0
    members = np.nonzero(valid)[0]
    tg, jr = [], []
    for o in range(4000):
        t_, r1, r2, r3, j = ora.de_draws(seed=3, t=2, o=o, d=d, valid=valid)
        assert len({t_, r1, r2, r3}) == 4
        assert all(valid[x] for x in (t_, r1, r2, r3))
        tg.append(t_)
        jr.append(j)
    cnt = np.array([np.sum(np.array(tg) == s) for s in members])
    assert stats.chisquare(cnt).pvalue > 1e-4
    cj = np.bincount(jr, minlength=d)
    assert stats.chisquare(cj).pvalue > 1e-4


def test_de_four_members_use_all_others(ora):
    K, d = 9, 5
    valid = np.zeros(K, np.uint8)
    valid[[1, 4, 6, 8]] = 1
    for o in range(200):
        t_, r1, r2, r3, _ = ora.de_draws(seed=11, t=7, o=o, d=d, valid=valid)
        assert sorted((t_, r1, r2, r3)) == [1, 4, 6, 8]


def test_de_zero_scale_copies_donor_genes(ora):
    K, d, N = 30, 24, 200
    X, F = _pop(K, d)
    valid = np.ones(K, np.uint8)
    op = ora.op_params(ora.OP_DE, 0.0, 0.5)
    Xo, Vo = ora.reproduce_op(ora.params(), op, 5, 3, X, None, valid, F, N)
    assert not Vo.any()
    for o in range(N):
        t_, r1, _, _, j = ora.de_draws(5, 3, o, d, valid)
        assert Xo[o, j] == X[r1, j]
        assert np.all((Xo[o] == X[t_]) | (Xo[o] == X[r1]))


def test_de_crossover_rate(ora):
    K, d, N = 50, 200, 400
    X, F = _pop(K, d)
    valid = np.ones(K, np.uint8)
    for CR in (0.0, 0.3, 0.9):
        op = ora.op_params(ora.OP_DE, 0.0, CR)
        Xo, _ = ora.reproduce_op(ora.params(), op, 8, 1, X, None, valid, F, N)
        took = np.zeros((N, d), bool)
        for o in range(N):
            t_, r1, _, _, _ = ora.de_draws(8, 1, o, d, valid)
            took[o] = Xo[o] != X[t_]
        p = CR + (1.0 - CR) / d
        assert abs(took.mean() - p) < 6 * np.sqrt(p * (1 - p) / took.size) + 1e-12
        if CR == 0.0:
            assert np.all(took.sum(axis=1) == 1)


def test_de_mutant_direction_and_clip(ora):
    # two-valued population: rows at 0.25 or 0.75; with F = 1 and CR = 1 the
    # mutant x_r1 + (x_r2 - x_r3) takes values in {-0.25, 0.25, 0.75, 1.25},
    # clipped to the unit box
    K, d, N = 12, 8, 300
    X = np.where(np.arange(K)[:, None] % 2 == 0, 0.25, 0.75) * np.ones((1, d))
    X = X.astype(np.float32)
    F = np.zeros((K, 3))
    valid = np.ones(K, np.uint8)
    op = ora.op_params(ora.OP_DE, 1.0, 1.0)
    Xo, _ = ora.reproduce_op(ora.params(), op, 2, 9, X, None, valid, F, N)
    for o in range(N):
        _, r1, r2, r3, _ = ora.de_draws(2, 9, o, d, valid)
        want = min(max(float(X[r1, 0]) + float(X[r2, 0]) - float(X[r3, 0]), 0.0), 1.0)
        assert np.all(Xo[o] == np.float32(want))


def test_pso_copy_and_inertia(ora):
    K, d, N = 20, 10, 64
    X, F = _pop(K, d)
    rng = np.random.default_rng(4)
    Vel = rng.uniform(-0.1, 0.1, size=(K, d)).astype(np.float32)
    valid = np.ones(K, np.uint8)
    Xo, Vo = ora.reproduce_op(ora.params(), ora.op_params(ora.OP_PSO, 0.0, 0.0), 1, 1, X, Vel,
                              valid, F, N)
    assert not Vo.any()
    rows = [np.nonzero((X == Xo[o]).all(axis=1))[0] for o in range(N)]
    assert all(len(r) == 1 for r in rows)
    # w = 1, c = 0: each child is a member displaced by exactly its velocity
    Xo, Vo = ora.reproduce_op(ora.params(), ora.op_params(ora.OP_PSO, 1.0, 0.0), 1, 1, X, Vel,
                              valid, F, N)
    for o in range(N):
        i = [j for j in range(K) if np.array_equal(Vel[j], Vo[o])]
        assert len(i) == 1
        assert np.allclose(Xo[o], X[i[0]].astype(np.float64) + Vel[i[0]], atol=1e-7)


def _sel(ora, seed, u, t, i, n):
    """Index below n from word i of unit u's selection stream: the draw
    convention (Philox4x32-10 counter (i/4, u, t, 5) under the run seed, the
    top 32 bits of word * n)."""
    w = ora.philox([i // 4, u, t, 5], [seed & 0xffffffff, seed >> 32])[i % 4]
    return (int(w) * n) >> 32


def test_pso_moves_toward_leader(ora):
    # zero velocities: the child lies on the segment from the particle toward
    # x_i + c (x_l - x_i); with c = 1 the mean fraction of the way is E[r] = 1/2
    K, d, N = 9, 64, 600
    X, F = _pop(K, d, seed=2)
    valid = np.ones(K, np.uint8)
    Xo, Vo = ora.reproduce_op(ora.params(), ora.op_params(ora.OP_PSO, 0.7, 1.0), 6, 2, X, None,
                              valid, F, N)
    fr = []
    for o in range(N):
        i, l = _sel(ora, 6, o, 2, 0, K), _sel(ora, 6, o, 2, 1, K)
        diff = X[l].astype(np.float64) - X[i]
        assert np.allclose(Xo[o], X[i] + Vo[o].astype(np.float64), atol=1e-7)
        if i == l:
            assert not Vo[o].any()
            continue
        ok = np.abs(diff) > 1e-3
        f = Vo[o][ok] / diff[ok]
        assert np.all((f >= 0) & (f <= 1 + 1e-6))
        fr.extend(f.tolist())
    assert abs(np.mean(fr) - 0.5) < 0.01


def test_cso_winner_copy_and_loser_move(ora):
    K, d, N = 16, 12, 41
    X, F = _pop(K, d, seed=5)
    valid = np.ones(K, np.uint8)
    valid[3] = 0
    members = np.nonzero(valid)[0]
    rng = np.random.default_rng(1)
    Vel = rng.uniform(-0.05, 0.05, size=(K, d)).astype(np.float32)
    Xo, Vo = ora.reproduce_op(ora.params(), ora.op_params(ora.OP_CSO), 4, 6, X, Vel, valid, F, N)
    X0, V0 = ora.reproduce_op(ora.params(), ora.op_params(ora.OP_CSO), 4, 6, X, None, valid, F,
                              N)
    h = (N + 1) // 2
    fit = F.sum(axis=1)
    for p in range(h):
        a = members[_sel(ora, 4, p, 6, 0, len(members))]
        b = members[_sel(ora, 4, p, 6, 1, len(members))]
        w, l = (a, b) if (fit[a], a) <= (fit[b], b) else (b, a)
        if p + h < N:
            assert np.array_equal(Xo[p + h], X[w]) and np.array_equal(Vo[p + h], Vel[w])
        # with zero velocity the loser moves a fraction r2 in [0, 1) toward the winner
        diff = X[w].astype(np.float64) - X[l]
        assert np.allclose(X0[p], X[l] + V0[p].astype(np.float64), atol=1e-7)
        ok = np.abs(diff) > 1e-3
        f = V0[p][ok] / diff[ok]
        assert np.all((f >= 0) & (f <= 1 + 1e-6))
        # the velocity term adds r1 v_l with r1 in [0, 1): same sign as v_l, no larger
        extra = Vo[p].astype(np.float64) - V0[p]
        assert np.all(extra * Vel[l] >= -1e-7)
        assert np.all(np.abs(extra) <= np.abs(Vel[l]) + 1e-7)


def test_cso_tie_goes_to_lower_slot(ora):
    K, d, N = 8, 4, 64
    X, _ = _pop(K, d, seed=1)
    F = np.ones((K, 3))
    valid = np.ones(K, np.uint8)
    Xo, _ = ora.reproduce_op(ora.params(), ora.op_params(ora.OP_CSO), 1, 1, X, None, valid, F, N)
    h = N // 2
    for p in range(h):
        a, b = _sel(ora, 1, p, 1, 0, K), _sel(ora, 1, p, 1, 1, K)
        assert np.array_equal(Xo[p + h], X[min(a, b)])


def test_random_reproduction_is_uniform(ora):
    K, d, N = 10, 50, 400
    X, F = _pop(K, d)
    valid = np.ones(K, np.uint8)
    prm = ora.params(lb=-2.0, ub=3.0)
    Xo, _ = ora.reproduce_op(prm, ora.op_params(ora.OP_RAND), 7, 2, X, None, valid, F, N)
    v = Xo.astype(np.float64).ravel()
    assert v.min() >= -2.0 and v.max() < 3.0
    assert stats.kstest((v + 2.0) / 5.0, "uniform").pvalue > 1e-4
    Xo2, _ = ora.reproduce_op(prm, ora.op_params(ora.OP_RAND), 7, 3, X, None, valid, F, N)
    assert abs(np.corrcoef(Xo.ravel(), Xo2.ravel())[0, 1]) < 0.02


@pytest.mark.parametrize("op", ["DE", "PSO", "CSO", "RAND"])
def test_generation_keeps_survivor_velocities(ora, op):
    problem, m, d, N, K = 2, 3, 12, 20, 21
    prm = ora.params(t_max=10)
    st = ora.initial_state(problem, m, d, N, K, seed=3)
    Vel = np.zeros((K, d), np.float32)
    code = getattr(ora, "OP_" + op)
    o = ora.op_params(code, *( (0.5, 0.9) if op == "DE" else (0.5, 1.5) if op == "PSO" else ()))
    for t in range(1, 5):
        X0, V0v, F0 = st.X.copy(), Vel.copy(), st.F.copy()
        out = ora.generation_op(prm, o, problem, m, d, N, K, 3, t, st, Vel)
        for j, s in enumerate(out["surv"]):
            if s < 0:
                assert not st.valid[j]
                continue
            src_x = X0[s] if s < K else out["Xoff"][s - K]
            src_v = V0v[s] if s < K else out["Voff"][s - K]
            src_f = F0[s] if s < K else out["Foff"][s - K]
            assert np.array_equal(st.X[j], src_x)
            assert np.array_equal(Vel[j], src_v)
            assert np.array_equal(st.F[j], src_f)
        # the offspring's objectives are the problem's at their genes
        assert np.allclose(out["Foff"], ora.evaluate(problem, m, out["Xoff"]), rtol=0, atol=0)
