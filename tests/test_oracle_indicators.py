"""Oracle pins for the quality indicators: the App. C.2 hypervolume
(reference point ones on normalised objectives) and the expected utility
(mean over a weight set of the best utility -w.f').

The hypervolume is checked against closed forms (one box, two boxes, a
hand-worked three-box set), against two independent routes on small random
sets (inclusion-exclusion over every subset of boxes, and a sum over the cells
of the grid the points' coordinates span), and against the known volumes of
the fronts; the expected utility against its one-hot and single-point closed
forms and the front identity min over the simplex of w.f = min_k w_k."""
import itertools

import numpy as np
import pytest


def hv_inclusion_exclusion(P):
    """Union volume of the boxes [p, 1]: sum over non-empty subsets of
    (-1)^(|S|+1) times the volume of their intersection [max_S p, 1]."""
    n, m = P.shape
    tot = 0.0
    for r in range(1, n + 1):
        for S in itertools.combinations(range(n), r):
            corner = P[list(S)].max(axis=0)
            tot += (-1) ** (r + 1) * np.prod(np.clip(1.0 - corner, 0.0, None))
    return tot


def hv_grid(P):
    """Union volume as a sum over the cells of the grid spanned by the points'
    coordinates and 1: a cell is dominated when some point lies at or below its
    lower corner in every objective."""
    n, m = P.shape
    axes = [np.unique(np.concatenate([P[:, k], [1.0]])) for k in range(m)]
    tot = 0.0
    for idx in itertools.product(*[range(len(a) - 1) for a in axes]):
        lo = np.array([axes[k][i] for k, i in enumerate(idx)])
        hi = np.array([axes[k][i + 1] for k, i in enumerate(idx)])
        if np.any(np.all(P <= lo, axis=1)):
            tot += np.prod(hi - lo)
    return tot


@pytest.mark.parametrize("m", [2, 3])
def test_single_box(ora, m):
    p = np.array([[0.2, 0.3, 0.45][:m]])
    assert ora.hypervolume(p) == pytest.approx(np.prod(1 - p[0]), rel=1e-15)


def test_two_boxes(ora):
    a, b = np.array([0.1, 0.6, 0.3]), np.array([0.5, 0.2, 0.4])
    want = np.prod(1 - a) + np.prod(1 - b) - np.prod(1 - np.maximum(a, b))
    assert ora.hypervolume(np.vstack([a, b])) == pytest.approx(want, rel=1e-14)
    a2, b2 = a[:2], b[:2]
    want2 = np.prod(1 - a2) + np.prod(1 - b2) - np.prod(1 - np.maximum(a2, b2))
    assert ora.hypervolume(np.vstack([a2, b2])) == pytest.approx(want2, rel=1e-14)


def test_hand_worked_three_boxes(ora):
    # boxes of volume 1/4 each, every pairwise and the triple intersection the
    # cube [1/2, 1]^3 of volume 1/8: 3/4 - 3/8 + 1/8 = 1/2
    P = np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    assert ora.hypervolume(P) == pytest.approx(0.5, rel=1e-15)


@pytest.mark.parametrize("m,n,seed", [(2, 8, 0), (2, 10, 1), (3, 7, 2), (3, 9, 3), (3, 10, 4)])
def test_random_sets_two_routes(ora, m, n, seed):
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.0, 1.0, size=(n, m))
    P[rng.random(n) < 0.2] = np.round(P[0], 1)  # repeated coordinates
    hv = ora.hypervolume(P)
    assert hv == pytest.approx(hv_inclusion_exclusion(P), rel=1e-12, abs=1e-15)
    assert hv == pytest.approx(hv_grid(P), rel=1e-12, abs=1e-15)


def test_outside_dominated_invalid_and_scaling(ora):
    rng = np.random.default_rng(7)
    P = rng.uniform(0.0, 0.9, size=(20, 3))
    hv = ora.hypervolume(P)
    # points beyond the reference point add nothing; dominated ones neither
    Q = np.vstack([P, [[1.2, 0.1, 0.1], [0.95, 0.99, 1.0]], P[:5] + 0.05])
    assert ora.hypervolume(Q) == pytest.approx(hv, rel=1e-14)
    # rows marked invalid or non-finite are ignored
    R = np.vstack([P, [[0.0, 0.0, 0.0], [np.nan, 0.1, 0.1]]])
    valid = np.ones(len(R), np.uint8)
    valid[-2] = 0
    assert ora.hypervolume(R, valid) == pytest.approx(hv, rel=1e-14)
    # normalisation: (F - lo) / (hi - lo)
    lo, hi = np.array([1.0, -2.0, 0.5]), np.array([3.0, 2.0, 4.5])
    F = lo + P * (hi - lo)
    assert ora.hypervolume(F, lo=lo, hi=hi) == pytest.approx(hv, rel=1e-12)
    # order of the rows does not matter
    assert ora.hypervolume(P[::-1]) == pytest.approx(hv, rel=1e-14)


def test_front_volumes(ora):
    """Dense samples of the two front shapes approach the volume they bound
    in the unit cube from below: 1 - 1/6 above the plane sum f = 1, and
    1 - pi/6 outside the unit sphere's octant."""
    lin = [ora.hypervolume(ora.front(1, 3, H)) for H in (10, 30, 99)]
    sph = [ora.hypervolume(ora.front(2, 3, H)) for H in (10, 30, 99)]
    assert lin[0] < lin[1] < lin[2] < 5 / 6 and lin[2] > 5 / 6 - 0.02
    assert sph[0] < sph[1] < sph[2] < 1 - np.pi / 6 and sph[2] > 1 - np.pi / 6 - 0.02
    # m = 2: linear front f2 = 1 - f1 bounds 1/2, the quarter circle 1 - pi/4
    assert ora.hypervolume(ora.front(1, 2, 4999)) == pytest.approx(0.5, abs=2e-4)
    assert ora.hypervolume(ora.front(2, 2, 4999)) == pytest.approx(1 - np.pi / 4, abs=2e-4)


def test_expected_utility_closed_forms(ora):
    rng = np.random.default_rng(11)
    F = rng.uniform(0.0, 1.0, size=(40, 3))
    # one-hot weights: the best utility under e_k is -min_i f_ik
    W = np.eye(3)
    assert ora.expected_utility(F, W) == pytest.approx(-F.min(axis=0).mean(), rel=1e-14)
    # a single solution: its utility averaged over the weights
    W2 = ora.lattice(4, 3)
    assert ora.expected_utility(F[:1], W2) == pytest.approx(-(W2 @ F[0]).mean(), rel=1e-14)
    # a further solution never lowers it
    assert ora.expected_utility(F, W2) >= ora.expected_utility(F[:10], W2)
    # the linear front contains the simplex vertices, and w.f >= min_k w_k on
    # the simplex, so EU = -mean over w of min_k w_k
    Fs = ora.front(1, 3, 20)
    assert ora.expected_utility(Fs, W2) == pytest.approx(-W2.min(axis=1).mean(), rel=1e-14)
