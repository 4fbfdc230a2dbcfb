"""Pins of the reference-vector set (Alg. 2 input V_0) and gamma (Eq. 5).

Counts are the binomial C(H+m-1, m-1); the lattice is checked against
brute-force enumeration with itertools, and gamma against closed forms and
an angle computed by a different route (atan2 of cross and dot products).
"""
import itertools
import math

import numpy as np
import pytest


@pytest.mark.parametrize("H,m,K", [(13, 3, 105), (140, 3, 10011), (446, 3, 100128),
                                   (4095, 2, 4096), (8, 8, 6435), (19, 5, 8855), (1, 4, 4)])
def test_lattice_counts(ora, H, m, K):
    assert ora.lattice_count(H, m) == K == math.comb(H + m - 1, m - 1)


@pytest.mark.parametrize("H,m", [(13, 3), (4, 4), (6, 2), (3, 5), (1, 3)])
def test_lattice_equals_bruteforce_in_lexicographic_subset_order(ora, H, m):
    W = ora.lattice(H, m)
    # every composition of H into m non-negative parts, exactly once
    brute = sorted(c for c in itertools.product(range(H + 1), repeat=m) if sum(c) == H)
    got = sorted(tuple(int(round(x * H)) for x in row) for row in W)
    assert got == brute
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-15) and W.min() >= 0
    # row order follows itertools.combinations(1..H+m-1, m-1) (lexicographic)
    for row, comb in zip(W, itertools.combinations(range(1, H + m), m - 1)):
        cc = (0,) + comb + (H + m,)
        parts = [cc[i + 1] - cc[i] - 1 for i in range(m)]
        assert [int(round(x * H)) for x in row] == parts


def test_lattice_first_and_last_rows(ora):
    W = ora.lattice(13, 3)
    assert list(W[0]) == [0.0, 0.0, 1.0]
    assert list(W[-1]) == [1.0, 0.0, 0.0]


def test_unit_vectors(ora):
    V = ora.unit_vectors(140, 3)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0, atol=4e-16)
    assert V.min() >= 0.0
    # directions are those of the lattice
    W = ora.lattice(140, 3)
    cos = (V * W).sum(1) / np.linalg.norm(W, axis=1)
    assert np.allclose(cos, 1.0, atol=1e-15)


def test_gamma_closed_forms(ora):
    # H = 1: the coordinate axes, mutually orthogonal
    assert np.allclose(ora.gamma(ora.unit_vectors(1, 3)), math.pi / 2, atol=1e-15)
    # H = 2, m = 3: axes and the three edge midpoints; nearest is axis<->midpoint, 45 deg
    assert np.allclose(ora.gamma(ora.unit_vectors(2, 3)), math.pi / 4, atol=1e-15)
    # a single vector has no neighbour
    assert ora.gamma(np.array([[0.6, 0.8]]))[0] == pytest.approx(math.pi / 2)
    # exact duplicates are skipped
    g = ora.gamma(np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0]]))
    assert np.allclose(g, math.pi / 2)


def test_gamma_two_objectives_against_polar_angles(ora):
    H = 37
    V = ora.unit_vectors(H, 2)
    phi = np.arctan2(V[:, 1], V[:, 0])  # polar angle of each vector
    order = np.argsort(phi)
    ps = phi[order]
    gaps = np.diff(ps)
    want = np.empty(len(ps))
    want[0], want[-1] = gaps[0], gaps[-1]
    want[1:-1] = np.minimum(gaps[:-1], gaps[1:])
    got = ora.gamma(V)[order]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-14)


def test_gamma_bruteforce_random_vectors(ora):
    rng = np.random.default_rng(5)
    V = np.abs(rng.standard_normal((60, 3)))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    got = ora.gamma(V)
    for j in range(len(V)):
        best = math.inf
        for i in range(len(V)):
            if i == j:
                continue
            cr = np.linalg.norm(np.cross(V[i], V[j]))
            best = min(best, math.atan2(cr, float(V[i] @ V[j])))
        assert got[j] == pytest.approx(best, rel=1e-9)
