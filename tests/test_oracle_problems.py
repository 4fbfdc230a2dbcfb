"""Pins of the stand-in test problems and of IGD (Appendix C.2).

The problems are this repository's own (the paper does not define DTLZ);
they are pinned by hand-computed values at exactly representable inputs,
by the front identities (sum f = 1 for the linear front, sum f^2 = 1 for
the sphere front, when every distance variable is 1/2), and by invariances.
"""
import math

import numpy as np
import pytest


def ev(ora, problem, m, x):
    return ora.evaluate(problem, m, np.array([x], np.float32))[0]


def test_hand_values_sphere_unimodal(ora):
    f = ev(ora, 2, 2, [0.25, 0.5, 0.5])  # w = (1/4, 3/4), g = 0
    assert f == pytest.approx([1 / math.sqrt(10), 3 / math.sqrt(10)], rel=1e-15)
    f = ev(ora, 2, 2, [0.25, 1.0, 0.0])  # g = (4/2) * (1/4 + 1/4) = 1
    assert f == pytest.approx([2 / math.sqrt(10), 6 / math.sqrt(10)], rel=1e-15)


def test_hand_values_linear_multimodal(ora):
    # y = (0.625, 0.125) -> sorted spacings w = (0.125, 0.5, 0.375)
    # z = (0.75, 0.5): terms 10/16 + 2 sin^2(pi) = 0.625 and 0 -> g = 0.3125
    f = ev(ora, 1, 3, [0.625, 0.125, 0.75, 0.5])
    assert f == pytest.approx([0.1640625, 0.65625, 0.4921875], rel=1e-14)
    # z = (0.625, 0.5): 10/64 + 2 sin^2(pi/2) = 2.15625 -> g = 1.078125
    f = ev(ora, 1, 3, [0.625, 0.125, 0.625, 0.5])
    assert f == pytest.approx([0.259765625, 1.0390625, 0.779296875], rel=1e-14)


def test_hand_values_sphere_multimodal(ora):
    f = ev(ora, 3, 3, [0.625, 0.125, 0.625, 0.5])
    w = np.array([0.125, 0.5, 0.375])
    assert f == pytest.approx(2.078125 * w / np.linalg.norm(w), rel=1e-14)


@pytest.mark.parametrize("m", [2, 3, 5, 8])
@pytest.mark.parametrize("problem", [1, 2, 3])
def test_front_identity_at_distance_optimum(ora, problem, m):
    rng = np.random.default_rng(m * 10 + problem)
    d = m + 9
    X = rng.uniform(0, 1, size=(200, d)).astype(np.float32)
    X[:, m - 1:] = 0.5
    F = ora.evaluate(problem, m, X)
    assert F.min() >= 0
    if problem == 1:
        assert np.allclose(F.sum(1), 1.0, atol=1e-15)
    else:
        assert np.allclose((F**2).sum(1), 1.0, atol=1e-15)
    # away from the optimum the distance term lifts every point off the front
    X[:, -1] = 0.9
    G = ora.evaluate(problem, m, X)
    assert np.all(G >= F - 1e-15) and np.all(G.sum(1) > F.sum(1))


def test_position_variables_are_order_free(ora):
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, size=(50, 12)).astype(np.float32)
    Y = X.copy()
    Y[:, [0, 1, 2, 3]] = X[:, [3, 0, 2, 1]]
    assert np.array_equal(ora.evaluate(3, 5, X), ora.evaluate(3, 5, Y))


def test_bad_arguments(ora):
    with pytest.raises(ValueError):
        ora.evaluate(4, 3, np.zeros((2, 5), np.float32))
    with pytest.raises(ValueError):
        ora.evaluate(1, 3, np.zeros((2, 2), np.float32))


@pytest.mark.parametrize("problem,m", [(1, 3), (2, 3), (3, 2), (1, 2)])
def test_front_sample(ora, problem, m):
    H = ora.front_H(m)
    Fs = ora.front(problem, m, H)
    assert Fs.shape[0] >= 5000 and Fs.min() >= 0
    if problem == 1:
        assert np.allclose(Fs.sum(1), 1.0, atol=1e-15)
    else:
        assert np.allclose((Fs**2).sum(1), 1.0, atol=1e-15)


def test_igd_definition(ora):
    assert ora.igd(np.array([[3.0, 4.0]]), np.array([[0.0, 0.0]])) == pytest.approx(5.0)
    # two reference points, mean of the nearest distances
    F = np.array([[0.0, 0.0], [10.0, 0.0]])
    Fs = np.array([[1.0, 0.0], [10.0, 2.0]])
    assert ora.igd(F, Fs) == pytest.approx((1.0 + 2.0) / 2)
    Fs = ora.front(2, 3, 20)
    assert ora.igd(Fs, Fs) == 0.0
    rng = np.random.default_rng(0)
    A = Fs[rng.choice(len(Fs), 30, replace=False)]
    B = np.vstack([A, Fs[rng.choice(len(Fs), 60, replace=False)]])
    assert 0 < ora.igd(B, Fs) <= ora.igd(A, Fs)
