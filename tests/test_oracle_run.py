"""Whole-run checks of the oracle (Alg. 2): convergence toward the known
front, determinism, and that stepping generation by generation from a saved
state equals an uninterrupted run (checkpoint/resume)."""
import numpy as np
import pytest


def test_small_run_converges_to_the_sphere_front(ora):
    prm = ora.params()
    st = ora.run(prm, problem=2, m=3, d=12, N=105, K=105, seed=0, gens=100)
    F = st.F[st.valid == 1]
    assert len(F) > 80
    Fs = ora.front(2, 3, ora.front_H(3))
    igd = ora.igd(F, Fs)
    # 105 well-spread points on the unit sphere octant are ~0.05 from a dense sample
    assert igd < 0.08
    # the population has moved onto the front: sum f^2 close to 1
    assert np.median(np.abs((F**2).sum(1) - 1.0)) < 0.02


def test_run_is_deterministic_and_seeded(ora):
    prm = ora.params()
    a = ora.run(prm, 1, 3, 20, 21, 21, seed=5, gens=15)
    b = ora.run(prm, 1, 3, 20, 21, 21, seed=5, gens=15)
    c = ora.run(prm, 1, 3, 20, 21, 21, seed=6, gens=15)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.F, b.F, equal_nan=True)
    assert not np.array_equal(a.X, c.X)


def test_stepwise_equals_uninterrupted(ora):
    prm = ora.params(t_max=40)
    whole = ora.run(prm, 3, 3, 16, 28, 28, seed=9, gens=40)
    st = ora.initial_state(3, 3, 16, 28, 28, seed=9)
    adapted = []
    for t in range(1, 41):
        out = ora.generation(prm, 3, 3, 16, 28, 28, 9, t, st)
        adapted.append(out["adapted"])
        if t == 20:  # checkpoint: copy the state and resume from the copy
            st = ora.State(st.X, st.F, st.valid, st.V, st.V0, st.gamma)
    assert np.array_equal(st.X, whole.X)
    assert np.array_equal(st.F, whole.F, equal_nan=True)
    assert np.array_equal(st.V, whole.V) and np.array_equal(st.gamma, whole.gamma)
    assert [i + 1 for i, a in enumerate(adapted) if a] == [4 * k for k in range(1, 11)]


def test_population_smaller_than_vector_count(ora):
    prm = ora.params(t_max=10)
    st = ora.run(prm, 2, 3, 10, 30, 45, seed=1, gens=10)
    assert st.valid.sum() <= 45 and st.valid.sum() >= 10
